// FP64 formal-solve kernels: the line solve in every launch shape (formal_solve_kernels.h)
// and its band-operator variant.
#include "formal_solve_kernels.h"

namespace nlte {

hipError_t launch_formal_solve_f64(const SolveArgs &a, const SolveConfig &cfg, hipStream_t s)
{
    return launch_fs_prec<false>(a, cfg, s);
}

size_t formal_solve_lds_f64(int lpl, int ns)
{
    switch (lpl) {
    case 1: return fs_lds_bytes<false, 1>(ns);
    case 2: return fs_lds_bytes<false, 2>(ns);
    case 3: return fs_lds_bytes<false, 3>(ns);
    case 4: return fs_lds_bytes<false, 4>(ns);
    default: return fs_lds_bytes<false, 5>(ns);
    }
}

// Band-operator variant of the grid kernel: also the entries of the inverse system matrix
// between O and its neighbour nodes (Jb, Ld, Ln of SolveArgs).  LONG: the long-segment
// mode, profile recurrence and far-wing collapse (a collapsed last segment records a last
// step of weight 0, as its zero-opacity sub-steps would).
template <int LPL, bool LONG>
__global__ __launch_bounds__(64, 2) void k_formal_solve_band(SolveArgs a)
{
    extern __shared__ double fs_smem[];
    __shared__ double tab[16];
    auto *red = reinterpret_cast<double (*)[LPL][kWave]>(fs_smem);
    auto *rec = reinterpret_cast<NodeRec<double, 2 * LPL> *>(fs_smem + 3 * LPL * kWave);
    if (threadIdx.x < 16) tab[threadIdx.x] = kExp2Sixteenths[threadIdx.x];
    __syncthreads();
    const int64_t nb8 = (a.n_blocks + 7) / 8;
    const int64_t lb = (int64_t)(blockIdx.x & 7) * nb8 + (blockIdx.x >> 3);
    if (lb >= a.n_blocks) return;
    const int64_t O = lb / a.groups;
    solve_item<false, LPL, LONG, true>(a, O, (int)(lb - O * a.groups), rec, red, tab);
}

hipError_t launch_formal_solve_band(const SolveArgs &a, hipStream_t s)
{
    if (a.n_blocks == 0) return hipSuccess;
    const int lpl = a.lines_per_wave / a.ngrp;
    const int64_t nb8 = (a.n_blocks + 7) / 8;
    const dim3 grid((unsigned)(nb8 * 8));
    if (lpl == 1 && a.collapse)
        hipLaunchKernelGGL((k_formal_solve_band<1, true>), grid, dim3(kWave), (fs_lds_bytes<false, 1>(a.ns)), s, a);
    else if (lpl == 1)
        hipLaunchKernelGGL((k_formal_solve_band<1, false>), grid, dim3(kWave), (fs_lds_bytes<false, 1>(a.ns)), s, a);
    else if (lpl == 2 && a.collapse)
        hipLaunchKernelGGL((k_formal_solve_band<2, true>), grid, dim3(kWave), (fs_lds_bytes<false, 2>(a.ns)), s, a);
    else if (lpl == 2)
        hipLaunchKernelGGL((k_formal_solve_band<2, false>), grid, dim3(kWave), (fs_lds_bytes<false, 2>(a.ns)), s, a);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace nlte
