// Ng acceleration of the ALI (Sec. 3.4; Ng 1974, Olson, Auer & Buchler 1986).
//
// After every M regular iterations the populations of each model still iterating are
// replaced by sum_j a_j x_{n-j} (j = 0 .. M-2, sum a_j = 1), the combination of the last
// M - 1 iterates whose coefficients minimise || sum_j a_j (x_{n-j} - x_{n-j-1}) ||^2 over
// the fractional populations x / n_tot of all the model's points and levels (uniform
// weights).  With a_0 = 1 - sum_{j>0} a_j and d_j = r_j - r_0, r_j = x_{n-j} - x_{n-j-1},
// the normal equations are  sum_k (d_j . d_k) a_k = -(d_j . r_0),  j, k = 1 .. M-2.
// A point whose combination is not positive and finite keeps x_n.
#include "nlte_internal.h"

namespace nlte {

namespace {

constexpr int kNgThreads = 256;

__device__ inline int tri(int i, int j, int K) { return i * K - i * (i - 1) / 2 + (j - i); }  // i <= j

}  // namespace

// Block (m, c) accumulates the sums of model m over points off[m] + c*256 + t, strided by
// chunks*256, and writes them to part[(m * chunks + c) * NS + .]; NS = K(K+1)/2 + K.
__global__ __launch_bounds__(kNgThreads) void k_ng_dots(NgHist h, const CellRec *__restrict__ cell,
                                                        const int64_t *__restrict__ off, const uint8_t *__restrict__ done,
                                                        int n_lev, int chunks, double *__restrict__ part)
{
    __shared__ double red[kNgThreads];
    const int m = blockIdx.x / chunks, c = blockIdx.x % chunks;
    const int K = h.M - 2, NS = K * (K + 1) / 2 + K;
    double acc[kNgMaxSums];
    for (int s = 0; s < NS; ++s) acc[s] = 0.0;
    if (!done[m]) {
        for (int64_t p = off[m] + (int64_t)c * kNgThreads + threadIdx.x; p < off[m + 1];
             p += (int64_t)chunks * kNgThreads) {
            const double inv = 1.0 / cell[p].ntot;
            for (int i = 0; i < n_lev; ++i) {
                double f[kNgMaxM];
                for (int j = 0; j < h.M; ++j) f[j] = h.x[j][p * n_lev + i] * inv;  // newest first
                const double r0 = f[0] - f[1];
                double d[kNgMaxM];
                for (int j = 1; j <= K; ++j) d[j] = (f[j] - f[j + 1]) - r0;
                for (int j = 1; j <= K; ++j) {
                    for (int k = j; k <= K; ++k) acc[tri(j - 1, k - 1, K)] += d[j] * d[k];
                    acc[K * (K + 1) / 2 + j - 1] += d[j] * r0;
                }
            }
        }
    }
    // fixed-order tree over the block, one sum at a time
    for (int s = 0; s < NS; ++s) {
        red[threadIdx.x] = acc[s];
        __syncthreads();
        for (int w = kNgThreads / 2; w > 0; w >>= 1) {
            if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
            __syncthreads();
        }
        if (threadIdx.x == 0) part[(int64_t)blockIdx.x * NS + s] = red[0];
        __syncthreads();
    }
}

// One thread per model: chunk sums in order, then the normal equations by Gaussian
// elimination with partial pivoting.  A pivot below 1e-13 of the largest diagonal entry
// (or a non-finite one) marks the step singular: ok[m] = 0.  coef[m][0..M-2].
__global__ void k_ng_solve(const double *__restrict__ part, int n_models, int chunks, int M,
                           const uint8_t *__restrict__ done, double *__restrict__ coef, uint8_t *__restrict__ ok)
{
    const int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= n_models) return;
    const int K = M - 2, NS = K * (K + 1) / 2 + K;
    double s[kNgMaxSums];
    for (int k = 0; k < NS; ++k) s[k] = 0.0;
    for (int c = 0; c < chunks; ++c)
        for (int k = 0; k < NS; ++k) s[k] += part[((int64_t)m * chunks + c) * NS + k];
    double G[kNgMaxM][kNgMaxM + 1];
    double dmax = 0.0;
    for (int i = 0; i < K; ++i) {
        for (int j = 0; j < K; ++j) G[i][j] = s[i <= j ? tri(i, j, K) : tri(j, i, K)];
        G[i][K] = -s[K * (K + 1) / 2 + i];
        dmax = fmax(dmax, fabs(G[i][i]));
    }
    bool good = !done[m] && dmax > 0.0 && isfinite(dmax);
    for (int col = 0; col < K && good; ++col) {
        int piv = col;
        for (int r = col + 1; r < K; ++r)
            if (fabs(G[r][col]) > fabs(G[piv][col])) piv = r;
        if (!(fabs(G[piv][col]) > 1e-13 * dmax)) {
            good = false;
            break;
        }
        if (piv != col)
            for (int j = 0; j <= K; ++j) {
                const double t = G[col][j];
                G[col][j] = G[piv][j];
                G[piv][j] = t;
            }
        for (int r = col + 1; r < K; ++r) {
            const double f = G[r][col] / G[col][col];
            for (int j = col; j <= K; ++j) G[r][j] -= f * G[col][j];
        }
    }
    double a[kNgMaxM];
    if (good) {
        for (int i = K - 1; i >= 0; --i) {
            double v = G[i][K];
            for (int j = i + 1; j < K; ++j) v -= G[i][j] * a[j + 1];
            a[i + 1] = v / G[i][i];
        }
        double sum = 0.0;
        for (int j = 1; j <= K; ++j) sum += a[j];
        a[0] = 1.0 - sum;
        for (int j = 0; j <= K; ++j) good = good && isfinite(a[j]);
    }
    ok[m] = good ? 1 : 0;
    for (int j = 0; j <= K; ++j) coef[(int64_t)m * (M - 1) + j] = good ? a[j] : (j == 0 ? 1.0 : 0.0);
}

// One thread per point of an accepted model: out = sum_j a_j x_{n-j} where positive and
// finite, else unchanged (out holds x_n); rejected points are counted.
__global__ void k_ng_combine(NgHist h, const double *__restrict__ coef, const uint8_t *__restrict__ ok,
                             const int32_t *__restrict__ model_of, int n_lev, int64_t P, double *__restrict__ out,
                             unsigned long long *__restrict__ rejected)
{
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= P) return;
    const int m = model_of[p];
    if (!ok[m]) return;
    const double *a = coef + (int64_t)m * (h.M - 1);
    double v[kMaxLev];
    bool good = true;
    for (int i = 0; i < n_lev; ++i) {
        double s = 0.0;
        for (int j = 0; j < h.M - 1; ++j) s += a[j] * h.x[j][p * n_lev + i];
        v[i] = s;
        good = good && isfinite(s) && s > 0.0;
    }
    if (!good) {
        atomicAdd(rejected, 1ull);
        return;
    }
    for (int i = 0; i < n_lev; ++i) out[p * n_lev + i] = v[i];
}

int ng_chunks() { return 32; }

hipError_t launch_ng(const NgHist &h, const CellRec *cell, const int64_t *off, const uint8_t *done,
                     const int32_t *model_of, int n_models, int n_lev, int64_t P, double *part, double *coef,
                     uint8_t *ok, double *out, unsigned long long *rejected, hipStream_t s)
{
    const int chunks = ng_chunks();
    hipLaunchKernelGGL(k_ng_dots, dim3((unsigned)(n_models * chunks)), dim3(kNgThreads), 0, s, h, cell, off, done,
                       n_lev, chunks, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_ng_solve, dim3((unsigned)((n_models + 63) / 64)), dim3(64), 0, s, part, n_models, chunks,
                       h.M, done, coef, ok);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (P == 0) return hipSuccess;
    hipLaunchKernelGGL(k_ng_combine, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, h, coef, ok, model_of, n_lev,
                       P, out, rejected);
    return hipGetLastError();
}

}  // namespace nlte
