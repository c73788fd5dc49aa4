// FP32-bulk formal-solve kernels (FP32 profile, opacity, optical depth, source function
// and J accumulation; FP64 elimination) in every launch shape (formal_solve_kernels.h).
#include "formal_solve_kernels.h"

namespace nlte {

hipError_t launch_formal_solve_f32(const SolveArgs &a, const SolveConfig &cfg, hipStream_t s)
{
    return launch_fs_prec<true>(a, cfg, s);
}

size_t formal_solve_lds_f32(int lpl, int ns)
{
    switch (lpl) {
    case 1: return fs_lds_bytes<true, 1>(ns);
    case 2: return fs_lds_bytes<true, 2>(ns);
    case 3: return fs_lds_bytes<true, 3>(ns);
    case 4: return fs_lds_bytes<true, 4>(ns);
    default: return fs_lds_bytes<true, 5>(ns);
    }
}

}  // namespace nlte
