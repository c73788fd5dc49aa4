// Statistical equilibrium with the band ALO (Sec. 3.4): the rate equations of every point
// contain, besides its own populations, the new upper-level populations of the first
// cells of its walks (the cells the band of one node reaches).  For line (u -> lo) at
// point O the net downward rate is
//   n_u,O [A (1 - Ld) + B_ul Jb] - n_lo,O B_lu Jb - sum_r cpl_r n_u,c(r),
//   cpl_r = A (k_O / k_c) Ln_r,  k = h nu/4pi (n_lo B_lu - n_u B_ul) with the previous populations,
// so the system of all points is A = K + C with K the block diagonal of the points' own
// rate matrices and C the couplings.  It is solved by BiCGSTAB (van der Vorst 1992) on the
// block-Jacobi preconditioned system (I + K^-1 C) x = K^-1 b, starting from the uncoupled
// solution K^-1 b, with inner products weighted by 1 / n_tot^2 (fractional populations).
// Points of converged models are held fixed.  A model with a singular local matrix, or
// whose coupled solution has a population that is not positive and finite, takes the
// local (diagonal ALO) solve instead (Sec. 6.1); its couplings are left out of the
// coupled system, which is block diagonal over models.
#include "rates.h"

namespace nlte {

namespace {

constexpr int kBandThreads = 256;

// In-place LU factorisation with partial pivoting; false for a singular matrix.
__device__ inline bool lu_factor(int n, double *M, int *piv)
{
    for (int col = 0; col < n; ++col) {
        int p = col;
        for (int r = col + 1; r < n; ++r)
            if (fabs(M[r * n + col]) > fabs(M[p * n + col])) p = r;
        piv[col] = p;
        if (!(M[p * n + col] != 0.0)) return false;
        if (p != col)
            for (int c = 0; c < n; ++c) {
                const double t = M[col * n + c];
                M[col * n + c] = M[p * n + c];
                M[p * n + c] = t;
            }
        for (int r = col + 1; r < n; ++r) {
            const double f = M[r * n + col] / M[col * n + col];
            M[r * n + col] = f;
            for (int c = col + 1; c < n; ++c) M[r * n + c] -= f * M[col * n + c];
        }
    }
    return true;
}

__device__ inline void lu_solve(int n, const double *__restrict__ LU, const int32_t *__restrict__ piv, double *b)
{
    for (int col = 0; col < n; ++col) {
        const int p = piv[col];
        if (p != col) {
            const double t = b[col];
            b[col] = b[p];
            b[p] = t;
        }
        for (int r = col + 1; r < n; ++r) b[r] -= LU[r * n + col] * b[col];
    }
    for (int r = n - 1; r >= 0; --r) {
        double s = b[r];
        for (int c = r + 1; c < n; ++c) s -= LU[r * n + c] * b[c];
        b[r] = s / LU[r * n + r];
    }
}

}  // namespace

// First cell of the walk from every point along every ray (-1 for an empty walk).
__global__ void k_first_cells(const int64_t *__restrict__ roff, const int32_t *__restrict__ rcells, int64_t n,
                              int32_t *__restrict__ first)
{
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= n) return;
    first[q] = roff[q + 1] > roff[q] ? rcells[roff[q]] : -1;
}

hipError_t launch_first_cells(const int64_t *roff, const int32_t *rcells, int64_t n, int32_t *first, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_first_cells, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, roff, rcells, n, first);
    return hipGetLastError();
}

// Per point: LU factors of its own rate matrix (with the band diagonal Ld and Jb), the
// uncoupled solution x0 = K^-1 b, and the coupling coefficients to the first cells.
__global__ __launch_bounds__(kBandThreads) void k_band_setup(BandArgs b, SpeciesDev sp, const CellRec *__restrict__ cell,
                                                             const double *__restrict__ nh2,
                                                             const double *__restrict__ T,
                                                             const double *__restrict__ old)
{
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= b.P) return;
    const int n = sp.n_lev, nl = sp.n_lines, R = b.R;
    double M[kMaxLev * kMaxLev], rhs[kMaxLev];
    int pv[kMaxLev];
    const bool fixed = b.done != nullptr && b.done[b.model_of[p]];
    if (fixed) {
        for (int i = 0; i < n * n; ++i) M[i] = 0.0;
        for (int i = 0; i < n; ++i) {
            M[i * n + i] = 1.0;
            rhs[i] = old[p * n + i];
        }
    } else {
        rate_matrix(sp, T[p], nh2[p], cell[p].ntot, b.Jb + p * nl, b.Ld + p * nl, true, M, rhs);
    }
    if (!lu_factor(n, M, pv)) {
        atomicAdd(b.bad, 1ull);
        b.model_bad[b.model_of[p]] = 1;
        for (int i = 0; i < n * n; ++i) M[i] = (i % (n + 1) == 0) ? 1.0 : 0.0;
        for (int i = 0; i < n; ++i) {
            pv[i] = i;
            rhs[i] = old[p * n + i];
        }
    }
    for (int i = 0; i < n * n; ++i) b.LU[p * n * n + i] = M[i];
    for (int i = 0; i < n; ++i) b.piv[p * n + i] = pv[i];
    lu_solve(n, M, pv, rhs);
    for (int i = 0; i < n; ++i) b.x0[p * n + i] = rhs[i];
    for (int l = 0; l < nl; ++l) {
        const int u = sp.lu[l], lo = sp.ll[l];
        const double kO = sp.pre[l] * (old[p * n + lo] * sp.Blu[l] - old[p * n + u] * sp.Bul[l]);
        for (int r = 0; r < R; ++r) {
            const int32_t c = b.first[p * R + r];
            double k = 0.0;
            if (!fixed && c >= 0 && kO > 0.0) {
                const double kc = sp.pre[l] * (old[(int64_t)c * n + lo] * sp.Blu[l] - old[(int64_t)c * n + u] * sp.Bul[l]);
                if (kc > 0.0) k = sp.A[l] * (kO / kc) * b.Ln[(p * nl + l) * R + r];
            }
            b.cpl[(p * nl + l) * R + r] = k;
        }
    }
}

// Couplings of the points of models that take the local solve are dropped, so their rows
// read x = x0 and the coupled solve of the other models is unchanged.
__global__ __launch_bounds__(kBandThreads) void k_band_mask(BandArgs b, int n_lines)
{
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= b.P || !b.model_bad[b.model_of[p]]) return;
    for (int i = 0; i < n_lines * b.R; ++i) b.cpl[p * n_lines * b.R + i] = 0.0;
}

// w = y + K^-1 C y
__global__ __launch_bounds__(kBandThreads) void k_band_apply(BandArgs b, SpeciesDev sp, const double *__restrict__ y,
                                                             double *__restrict__ w)
{
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= b.P) return;
    const int n = sp.n_lev, nl = sp.n_lines, R = b.R;
    double cv[kMaxLev];
    for (int i = 0; i < n; ++i) cv[i] = 0.0;
    for (int l = 0; l < nl; ++l) {
        const int u = sp.lu[l], lo = sp.ll[l];
        for (int r = 0; r < R; ++r) {
            const double k = b.cpl[(p * nl + l) * R + r];
            if (k == 0.0) continue;
            const double v = k * y[(int64_t)b.first[p * R + r] * n + u];
            if (u != 0) cv[u] += v;
            if (lo != 0) cv[lo] -= v;
        }
    }
    lu_solve(n, b.LU + p * n * n, b.piv + p * n, cv);
    for (int i = 0; i < n; ++i) w[p * n + i] = y[p * n + i] + cv[i];
}

// Up to three inner products sum_p sum_i a[p,i] b[p,i] / ntot_p^2: per-block partial sums
// (fixed-order tree), then one block adds the partials in order.
__global__ __launch_bounds__(kBandThreads) void k_band_dots(DotArgs d, const CellRec *__restrict__ cell, int n, int64_t P,
                                                            double *__restrict__ part)
{
    __shared__ double red[3][kBandThreads];
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    double acc[3] = {0.0, 0.0, 0.0};
    if (p < P) {
        const double wgt = 1.0 / (cell[p].ntot * cell[p].ntot);
        for (int k = 0; k < d.nd; ++k) {
            double s = 0.0;
            for (int i = 0; i < n; ++i) s += d.a[k][p * n + i] * d.b[k][p * n + i];
            acc[k] = s * wgt;
        }
    }
    for (int k = 0; k < 3; ++k) red[k][threadIdx.x] = acc[k];
    __syncthreads();
    for (int w = kBandThreads / 2; w > 0; w >>= 1) {
        if (threadIdx.x < w)
            for (int k = 0; k < 3; ++k) red[k][threadIdx.x] += red[k][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 3) part[blockIdx.x * 3 + threadIdx.x] = red[threadIdx.x][0];
}

__global__ void k_band_dots_final(const double *__restrict__ part, int64_t nb, double *__restrict__ out)
{
    if (threadIdx.x >= 3) return;
    double s = 0.0;
    for (int64_t i = 0; i < nb; ++i) s += part[i * 3 + threadIdx.x];
    out[threadIdx.x] = s;
}

// out = a X + b Y (+ c Z)
__global__ void k_band_lin(double *__restrict__ out, double a, const double *__restrict__ X, double b,
                           const double *__restrict__ Y, double c, const double *__restrict__ Z, int64_t N)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= N) return;
    double v = a * X[i] + b * Y[i];
    if (Z) v += c * Z[i];
    out[i] = v;
}

// Models with a population that is not positive and finite.
__global__ void k_band_check_models(const double *__restrict__ x, int n, int64_t P,
                                    const int32_t *__restrict__ model_of, uint8_t *__restrict__ model_bad)
{
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= P) return;
    bool ok = true;
    for (int i = 0; i < n; ++i) ok = ok && x[p * n + i] > 0.0 && isfinite(x[p * n + i]);
    if (!ok) model_bad[model_of[p]] = 1;
}

// New populations: the band's, or the local solve's for models marked in model_bad
// (local and model_bad nullable: every model takes the band's); change statistics and
// per-model changes as the local solve reports them.
__global__ __launch_bounds__(256) void k_band_finish(const double *__restrict__ x, const double *__restrict__ local,
                                                     const uint8_t *__restrict__ model_bad,
                                                     const double *__restrict__ old,
                                                     const CellRec *__restrict__ cell, int n, int64_t P,
                                                     double *__restrict__ pops_new, uint8_t *__restrict__ flags,
                                                     ConvPartial *partials, const uint8_t *__restrict__ done,
                                                     const int32_t *__restrict__ model_of,
                                                     unsigned long long *__restrict__ model_change)
{
    __shared__ double s_max[256], s_sum[256];
    __shared__ int64_t s_cnt[256];
    __shared__ int s_one_model;
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (threadIdx.x == 0) s_one_model = block_in_one_model(model_of, P);
    double mx = 0.0, sum = 0.0;
    int64_t cnt = 0;
    if (p < P) {
        const bool fixed = done != nullptr && done[model_of[p]];
        const bool loc = model_bad != nullptr && model_bad[model_of[p]];
        const double *src = loc ? local : x;
        const double nt = cell[p].ntot;
        for (int i = 0; i < n; ++i) {
            const double v = fixed ? old[p * n + i] : src[p * n + i];
            pops_new[p * n + i] = v;
            if (!fixed && v / nt > 1e-10) {
                const double d = fabs(v - old[p * n + i]) / v;
                mx = fmax(mx, d);
                sum += d;
                ++cnt;
            }
        }
        if (flags && !loc) flags[p] = 0;   // the local solve has set its own
    }
    const int t = threadIdx.x;
    s_max[t] = mx;
    s_sum[t] = sum;
    s_cnt[t] = cnt;
    __syncthreads();
    if (model_change != nullptr && !s_one_model && cnt > 0)
        atomicMax(&model_change[model_of[p]], (unsigned long long)__double_as_longlong(mx));
    for (int w = 128; w > 0; w >>= 1) {
        if (t < w) {
            s_max[t] = fmax(s_max[t], s_max[t + w]);
            s_sum[t] += s_sum[t + w];
            s_cnt[t] += s_cnt[t + w];
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
        cp.n_fallback = 0;
        cp.n_kept = 0;
        partials[blockIdx.x] = cp;
    }
}

hipError_t launch_band_setup(const BandArgs &b, const SpeciesDev &sp, const CellRec *cell, const double *nh2,
                             const double *T, const double *old, hipStream_t s)
{
    if (b.P == 0) return hipSuccess;
    hipLaunchKernelGGL(k_band_setup, dim3((unsigned)((b.P + kBandThreads - 1) / kBandThreads)), dim3(kBandThreads), 0,
                       s, b, sp, cell, nh2, T, old);
    return hipGetLastError();
}

hipError_t launch_band_apply(const BandArgs &b, const SpeciesDev &sp, const double *y, double *w, hipStream_t s)
{
    if (b.P == 0) return hipSuccess;
    hipLaunchKernelGGL(k_band_apply, dim3((unsigned)((b.P + kBandThreads - 1) / kBandThreads)), dim3(kBandThreads), 0,
                       s, b, sp, y, w);
    return hipGetLastError();
}

int64_t band_dot_blocks(int64_t P) { return (P + kBandThreads - 1) / kBandThreads; }

hipError_t launch_band_dots(const DotArgs &d, const CellRec *cell, int n, int64_t P, double *part, double *out,
                            hipStream_t s)
{
    const int64_t nb = band_dot_blocks(P);
    hipLaunchKernelGGL(k_band_dots, dim3((unsigned)nb), dim3(kBandThreads), 0, s, d, cell, n, P, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_band_dots_final, dim3(1), dim3(64), 0, s, part, nb, out);
    return hipGetLastError();
}

hipError_t launch_band_lin(double *out, double a, const double *X, double b, const double *Y, double c,
                           const double *Z, int64_t N, hipStream_t s)
{
    if (N == 0) return hipSuccess;
    hipLaunchKernelGGL(k_band_lin, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, out, a, X, b, Y, c, Z, N);
    return hipGetLastError();
}

hipError_t launch_band_check_models(const double *x, int n, int64_t P, const int32_t *model_of, uint8_t *model_bad,
                                   hipStream_t s)
{
    if (P == 0) return hipSuccess;
    hipLaunchKernelGGL(k_band_check_models, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, x, n, P, model_of,
                       model_bad);
    return hipGetLastError();
}

hipError_t launch_band_mask(const BandArgs &b, int n_lines, hipStream_t s)
{
    if (b.P == 0) return hipSuccess;
    hipLaunchKernelGGL(k_band_mask, dim3((unsigned)((b.P + kBandThreads - 1) / kBandThreads)), dim3(kBandThreads), 0,
                       s, b, n_lines);
    return hipGetLastError();
}

hipError_t launch_band_finish(const double *x, const double *local, const uint8_t *model_bad, const double *old,
                              const CellRec *cell, int n, int64_t P, double *pops_new, uint8_t *flags,
                              ConvPartial *partials, const uint8_t *done, const int32_t *model_of,
                              unsigned long long *model_change, hipStream_t s)
{
    if (P == 0) return hipSuccess;
    hipLaunchKernelGGL(k_band_finish, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, x, local, model_bad, old,
                       cell, n, P, pops_new, flags, partials, done, model_of, model_change);
    return hipGetLastError();
}

}  // namespace nlte
