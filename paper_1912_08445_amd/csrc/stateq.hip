// Statistical equilibrium per point and the convergence reduction.
#include "rates.h"

namespace nlte {

// Assemble and solve the rate equations of one point (Eq. ourALI, diagonal ALO):
// u->l = A(1 - L) + B_ul Jeff + C_ul,  l->u = B_lu Jeff + C_lu; row 0 := conservation.
__device__ int solve_point(const SpeciesDev &sp, double T, double nh2, double ntot,
                           const double *Jrow, const double *Lrow, bool with_L, double *x)
{
    const int n = sp.n_lev;
    double M[kMaxLev * kMaxLev];
    double rhs[kMaxLev];
    rate_matrix(sp, T, nh2, ntot, Jrow, Lrow, with_L, M, rhs);
    // Gaussian elimination with partial pivoting
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (fabs(M[r * n + col]) > fabs(M[piv * n + col])) piv = r;
        if (M[piv * n + col] == 0.0) return -1;
        if (piv != col) {
            for (int c = 0; c < n; ++c) {
                double t = M[col * n + c];
                M[col * n + c] = M[piv * n + c];
                M[piv * n + c] = t;
            }
            double t = rhs[col];
            rhs[col] = rhs[piv];
            rhs[piv] = t;
        }
        for (int r = col + 1; r < n; ++r) {
            double f = M[r * n + col] / M[col * n + col];
            for (int c = col; c < n; ++c) M[r * n + c] -= f * M[col * n + c];
            rhs[r] -= f * rhs[col];
        }
    }
    for (int r = n - 1; r >= 0; --r) {
        double s = rhs[r];
        for (int c = r + 1; c < n; ++c) s -= M[r * n + c] * x[c];
        x[r] = s / M[r * n + r];
    }
    return 0;
}

__device__ __forceinline__ bool valid(int n, const double *x)
{
    for (int i = 0; i < n; ++i)
        if (!(x[i] > 0.0) || !isfinite(x[i])) return false;
    return true;
}

__global__ __launch_bounds__(256) void k_stateq(SpeciesDev sp, const CellRec *__restrict__ cell,
                                                const double *__restrict__ nh2,
                                                const double *__restrict__ Tg, int64_t P, int use_alo,
                                                const double *__restrict__ pops_old,
                                                const double *__restrict__ J,
                                                const double *__restrict__ Jeff,
                                                const double *__restrict__ L,
                                                double *__restrict__ pops_new,
                                                uint8_t *__restrict__ flags, ConvPartial *partials,
                                                const uint8_t *__restrict__ model_done,
                                                const int32_t *__restrict__ model_of,
                                                unsigned long long *__restrict__ model_change)
{
    __shared__ double s_max[256], s_sum[256];
    __shared__ int64_t s_cnt[256], s_fb[256], s_kept[256];
    __shared__ int s_one_model;
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (threadIdx.x == 0) s_one_model = block_in_one_model(model_of, P);
    double mx = 0.0, sum = 0.0;
    int64_t cnt = 0, fb = 0, kept = 0;
    const bool skip = p < P && model_done != nullptr && model_done[model_of[p]];
    if (skip) {
        // converged model: populations stay as they are
        for (int i = 0; i < sp.n_lev; ++i) pops_new[p * sp.n_lev + i] = pops_old[p * sp.n_lev + i];
        if (flags) flags[p] = 0;
    } else if (p < P) {
        const int n = sp.n_lev, nl = sp.n_lines;
        const double T = Tg[p], nh = nh2[p], nt = cell[p].ntot;
        double x[kMaxLev];
        uint8_t f = 0;
        const double *Jr = J + p * nl;
        const double *Er = use_alo ? Jeff + p * nl : Jr;
        if (solve_point(sp, T, nh, nt, Er, L + p * nl, use_alo != 0, x) != 0 || !valid(n, x)) {
            // Sec. 6.1: redo without the ALO, then keep the old populations
            f = 1;
            if (solve_point(sp, T, nh, nt, Jr, L + p * nl, false, x) != 0 || !valid(n, x)) {
                f = 2;
                for (int i = 0; i < n; ++i) x[i] = pops_old[p * n + i];
            }
        }
        for (int i = 0; i < n; ++i) {
            pops_new[p * n + i] = x[i];
            if (x[i] / nt > 1e-10) {
                double d = fabs(x[i] - pops_old[p * n + i]) / x[i];
                mx = fmax(mx, d);
                sum += d;
                ++cnt;
            }
        }
        if (flags) flags[p] = f;
        fb = (f == 1);
        kept = (f == 2);
    }
    const int t = threadIdx.x;
    s_max[t] = mx;
    s_sum[t] = sum;
    s_cnt[t] = cnt;
    s_fb[t] = fb;
    s_kept[t] = kept;
    __syncthreads();
    // per-model maximum (non-negative doubles order like their bit patterns): per point
    // only where the block straddles a model boundary, else once per block below
    if (model_change != nullptr && !s_one_model && cnt > 0)
        atomicMax(&model_change[model_of[p]], (unsigned long long)__double_as_longlong(mx));
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) {
            s_max[t] = fmax(s_max[t], s_max[t + w]);
            s_sum[t] += s_sum[t + w];
            s_cnt[t] += s_cnt[t + w];
            s_fb[t] += s_fb[t + w];
            s_kept[t] += s_kept[t + w];
        }
        __syncthreads();
    }
    if (t == 0 && model_change != nullptr && s_one_model && s_cnt[0] > 0)
        atomicMax(&model_change[model_of[blockIdx.x * (int64_t)blockDim.x]],
                  (unsigned long long)__double_as_longlong(s_max[0]));
    if (t == 0 && partials) {
        ConvPartial cp;
        cp.max_change = s_max[0];
        cp.sum_change = s_sum[0];
        cp.count = s_cnt[0];
        cp.n_fallback = s_fb[0];
        cp.n_kept = s_kept[0];
        partials[blockIdx.x] = cp;
    }
}

int64_t stateq_blocks(int64_t P) { return (P + 255) / 256; }

hipError_t launch_stateq(const SpeciesDev &sp, const CellRec *cell, const double *nh2,
                         const double *T, int64_t P, int use_alo, const double *pops_old,
                         const double *J, const double *Jeff, const double *L, double *pops_new,
                         uint8_t *flags, ConvPartial *partials, int64_t n_blocks,
                         const uint8_t *model_done, const int32_t *model_of,
                         unsigned long long *model_change, hipStream_t s)
{
    if (P == 0) return hipSuccess;
    hipLaunchKernelGGL(k_stateq, dim3((unsigned)n_blocks), dim3(256), 0, s, sp, cell, nh2, T, P,
                       use_alo, pops_old, J, Jeff, L, pops_new, flags, partials, model_done, model_of,
                       model_change);
    return hipGetLastError();
}

// Per-model convergence after an iteration: a model still iterating counts one more
// iteration, records its maximum relative change and stops once it is below tol.
__global__ void k_model_update(int n_models, const unsigned long long *__restrict__ change,
                               uint8_t *__restrict__ done, int32_t *__restrict__ iters,
                               double *__restrict__ last, double tol, int32_t *active)
{
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n_models || done[m]) return;
    iters[m] += 1;
    const double ch = __longlong_as_double((long long)change[m]);
    last[m] = ch;
    if (ch < tol)
        done[m] = 1;
    else
        atomicAdd(active, 1);
}

hipError_t launch_model_update(int n_models, unsigned long long *change, uint8_t *done, int32_t *iters,
                               double *last, double tol, int32_t *active, hipStream_t s)
{
    hipLaunchKernelGGL(k_model_update, dim3((n_models + 255) / 256), dim3(256), 0, s, n_models, change, done,
                       iters, last, tol, active);
    return hipGetLastError();
}

// Fill kernels (used instead of memset nodes so that the iteration can be captured).
__global__ void k_fill_u64(unsigned long long *p, int64_t n, unsigned long long v)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_fill_u8(uint8_t *p, int64_t n, uint8_t v)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

hipError_t launch_fill_u64(unsigned long long *p, int64_t n, unsigned long long v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

hipError_t launch_fill_u8(uint8_t *p, int64_t n, uint8_t v, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill_u8, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

// Deterministic final reduction of the per-block partials (one workgroup, fixed order).
__global__ __launch_bounds__(256) void k_conv_final(const ConvPartial *__restrict__ part, int64_t n,
                                                    ConvResult *out)
{
    __shared__ double s_max[256], s_sum[256];
    __shared__ int64_t s_cnt[256], s_fb[256], s_kept[256];
    const int t = threadIdx.x;
    double mx = 0.0, sum = 0.0;
    int64_t cnt = 0, fb = 0, kept = 0;
    for (int64_t i = t; i < n; i += 256) {
        mx = fmax(mx, part[i].max_change);
        sum += part[i].sum_change;
        cnt += part[i].count;
        fb += part[i].n_fallback;
        kept += part[i].n_kept;
    }
    s_max[t] = mx;
    s_sum[t] = sum;
    s_cnt[t] = cnt;
    s_fb[t] = fb;
    s_kept[t] = kept;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) {
            s_max[t] = fmax(s_max[t], s_max[t + w]);
            s_sum[t] += s_sum[t + w];
            s_cnt[t] += s_cnt[t + w];
            s_fb[t] += s_fb[t + w];
            s_kept[t] += s_kept[t + w];
        }
        __syncthreads();
    }
    if (t == 0) {
        ConvResult r;
        r.max_change = s_max[0];
        r.mean_change = s_cnt[0] ? s_sum[0] / (double)s_cnt[0] : 0.0;
        r.n_fallback = s_fb[0];
        r.n_kept = s_kept[0];
        *out = r;
    }
}

hipError_t launch_conv_final(const ConvPartial *partials, int64_t n, ConvResult *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_conv_final, dim3(1), dim3(256), 0, s, partials, n, out);
    return hipGetLastError();
}

}  // namespace nlte
