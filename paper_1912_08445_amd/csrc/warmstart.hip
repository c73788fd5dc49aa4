// Warm start of the accelerated Lambda iteration: per-point features of the local
// conditions and a small multilayer perceptron that maps them to starting level
// populations, predicted as departures from LTE.  This is not part of the paper's method, which only needs some initial
// populations for its iteration (Sec. 2.2.1, 3.4); the iteration itself still decides
// the result.
//
// Network: 8 -> 128 -> 128 -> 128 -> n_out (n_out <= 16), erf GELU after each hidden
// layer.  Parameters are one flat FP32 vector (master copy), matrices row-major
// [out][in] in the order W1 b1 W2 b2 W3 b3 W4 b4.  Products run on the matrix cores
// as v_mfma_f32_16x16x32_bf16: bfloat16 operands, FP32 accumulation.
//
// Operand layout used by every product (16x16 output tile, K = 32 per instruction):
//   lane l = 16 g + i (g = 0..3, i = 0..15); the A operand holds row i of the tile, the
//   B operand column i, and the four outputs of lane l are rows 4g .. 4g+3 of column i.
//   The eight K slots of lane group g carry the reduction indices
//       k(s, g, j) = 32 s + 16 (j / 4) + 4 g + (j % 4),   j = 0..7, K step s,
//   on both operands.  With this choice an output tile pair (2s, 2s+1) of one layer,
//   held as rows = features and columns = points, is exactly the B operand of K step s
//   of the next layer, so activations pass from layer to layer in registers.
#include "nlte_internal.h"

namespace nlte {

namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kHid = 128;

// Round to the nearest bfloat16, ties to even (finite inputs).
__device__ inline unsigned short bf16_bits(float x)
{
    unsigned u = __float_as_uint(x);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}

__device__ inline float bf16_value(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

struct Frag {
    unsigned short v[8];
};

__device__ inline bf16x8 as_bf16x8(const Frag &f) { return __builtin_bit_cast(bf16x8, f); }

__device__ inline f32x4 mfma(const Frag &a, const Frag &b, f32x4 c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(a), as_bf16x8(b), c, 0, 0, 0);
}

// GELU and its derivative from one exponential.  erf(x) for x >= 0 by Abramowitz &
// Stegun 7.1.26, erf(x) = 1 - t (a1 + t (a2 + t (a3 + t (a4 + t a5)))) e^{-x^2} with
// t = 1/(1 + p x) (absolute error below 1.5e-7, far under the bfloat16 rounding that
// follows); at x = |z|/sqrt 2 its Gaussian e^{-z^2/2} is also the derivative's:
//   gelu(z) = z (1 + erf(z/sqrt 2))/2,  gelu'(z) = (1 + erf(z/sqrt 2))/2 + z e^{-z^2/2}/sqrt(2 pi).
// 1 + erf is formed as q or 2 - q with q = 1 - erf(|x|), without cancellation for z < 0.
struct GeluPair {
    float h, dh;
};

__device__ inline GeluPair gelu_pair(float z)
{
    const float e = __builtin_amdgcn_exp2f(-0.72134752044448170f * (z * z));   // e^{-z^2/2}
    const float x = fabsf(z) * 0.70710678118654752f;
    const float t = __builtin_amdgcn_rcpf(fmaf(0.3275911f, x, 1.0f));
    float p = fmaf(1.061405429f, t, -1.453152027f);
    p = fmaf(p, t, 1.421413741f);
    p = fmaf(p, t, -0.284496736f);
    p = fmaf(p, t, 0.254829592f);
    const float q = (p * t) * e;
    const float one_p = z >= 0.0f ? 2.0f - q : q;
    return {0.5f * z * one_p, fmaf(z * e, 0.39894228040143268f, 0.5f * one_p)};
}

__device__ inline float gelu(float z) { return gelu_pair(z).h; }

// Reduction index of K slot j of lane group g in K step s.
__device__ inline int kslot(int s, int g, int j) { return 32 * s + 16 * (j >> 2) + 4 * g + (j & 3); }

// B operand of K step s from output tiles 2s and 2s+1 (FP32 values -> bfloat16).
__device__ inline Frag pack_pair(const f32x4 &lo, const f32x4 &hi)
{
    Frag f;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        f.v[j] = bf16_bits(lo[j]);
        f.v[4 + j] = bf16_bits(hi[j]);
    }
    return f;
}

__device__ inline Frag load_frag(const Frag *base, int idx, int lane) { return base[(int64_t)idx * 64 + lane]; }

}  // namespace

// ------------------------------------------------------------------------- features

// One wave per point.  F[p][0..7]: log10 n_H2, log10 T, log10 of the mean velocity
// gradient to the neighbours (floored at 1e-30 s^-1), and log10 of the minimum, quartiles
// and maximum over the rays of the H2 column along the cached walk (trapezoid in the
// projected distance, at least half a cell's column and 1 cm^-2).  Quantiles interpolate
// linearly between order statistics at position q (n_rays - 1).  The lanes take a ray's
// cells 64 at a time (coalesced reads of the walk cache), each forms its cell's trapezoid
// term with the previous cell's values from its neighbour lane, and the wave sums the
// terms.
__global__ __launch_bounds__(64) void k_features(const CellRec *__restrict__ cell,
                                                 const double *__restrict__ nh2,
                                                 const double *__restrict__ T,
                                                 const int32_t *__restrict__ nbr, int k,
                                                 const int64_t *__restrict__ roff,
                                                 const int32_t *__restrict__ rcells,
                                                 const double *__restrict__ dir, int R, int64_t P,
                                                 double *__restrict__ F)
{
    extern __shared__ double sh[];
    double *col = sh;
    double *srt = sh + R;
    const int64_t p = blockIdx.x;
    const int lane = threadIdx.x;
    if (p >= P) return;
    const double ox = cell[p].px, oy = cell[p].py, oz = cell[p].pz;
    // half a cell's column, the least a ray's column is taken to be (a walk with no cell
    // lies at the model's edge): n_H2 times half the mean distance to the neighbours
    double dsum = 0.0;
    int dcount = 0;
    for (int s = 0; s < k; ++s) {
        const int32_t m = nbr[p * k + s];
        if (m < 0) continue;
        const double dx = cell[m].px - ox, dy = cell[m].py - oy, dz = cell[m].pz - oz;
        dsum += sqrt((dx * dx + dy * dy) + dz * dz);
        ++dcount;
    }
    const double half_cell = dcount > 0 ? 0.5 * nh2[p] * (dsum / dcount) : 0.0;
    const double floor_col = half_cell > 1.0 ? half_cell : 1.0;

    const double n_O = nh2[p];
    for (int r = 0; r < R; ++r) {
        const double nx = dir[3 * r], ny = dir[3 * r + 1], nz = dir[3 * r + 2];
        const int64_t b = roff[p * R + r];
        const int L = (int)(roff[p * R + r + 1] - b);
        // trapezoid terms 0.5 (n_{i-1} + n_i)(Z_i - Z_{i-1}) from the point (n_O, Z = 0) on
        double acc = 0.0, n_carry = n_O, z_carry = 0.0;
        for (int i0 = 0; i0 < L; i0 += 64) {
            const int i = i0 + lane;
            double Z = 0.0, n_i = 0.0;
            if (i < L) {
                const int32_t c = rcells[b + i];
                const double dx = cell[c].px - ox, dy = cell[c].py - oy, dz = cell[c].pz - oz;
                Z = (dx * nx + dy * ny) + dz * nz;
                n_i = nh2[c];
            }
            double n_prev = __shfl_up(n_i, 1), z_prev = __shfl_up(Z, 1);
            if (lane == 0) {
                n_prev = n_carry;
                z_prev = z_carry;
            }
            if (i < L) acc += 0.5 * (n_prev + n_i) * (Z - z_prev);
            n_carry = __shfl(n_i, 63);
            z_carry = __shfl(Z, 63);
        }
        for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
        if (lane == 0) col[r] = acc > floor_col ? acc : floor_col;
    }
    __syncthreads();
    // order statistics: rank by value, equal values by ray index
    for (int r = lane; r < R; r += 64) {
        const double v = col[r];
        int rank = 0;
        for (int s = 0; s < R; ++s) {
            const double u = col[s];
            rank += (u < v) || (u == v && s < r);
        }
        srt[rank] = v;
    }
    __syncthreads();
    if (lane != 0) return;
    double *f = F + 8 * p;
    f[0] = log10(nh2[p]);
    f[1] = log10(T[p]);
    double gsum = 0.0;
    int gcount = 0;
    for (int s = 0; s < k; ++s) {
        const int32_t m = nbr[p * k + s];
        if (m < 0) continue;
        const double dvx = cell[m].vx - cell[p].vx, dvy = cell[m].vy - cell[p].vy, dvz = cell[m].vz - cell[p].vz;
        const double dx = cell[m].px - ox, dy = cell[m].py - oy, dz = cell[m].pz - oz;
        const double nv = sqrt((dvx * dvx + dvy * dvy) + dvz * dvz);
        const double nx = sqrt((dx * dx + dy * dy) + dz * dz);
        gsum += nv / nx;
        ++gcount;
    }
    const double g = gcount > 0 ? gsum / gcount : 0.0;
    f[2] = log10(g > 1e-30 ? g : 1e-30);
    const double qs[5] = {0.0, 0.25, 0.5, 0.75, 1.0};
    for (int j = 0; j < 5; ++j) {
        const double h = qs[j] * (R - 1);
        const int i = (int)floor(h);
        double v = srt[i];
        if (i + 1 < R) v = srt[i] + (h - i) * (srt[i + 1] - srt[i]);
        f[3 + j] = log10(v);
    }
}

hipError_t launch_features(const CellRec *cell, const double *nh2, const double *T, const int32_t *nbr,
                           int k, const int64_t *roff, const int32_t *rcells, const double *dir, int R,
                           int64_t P, double *F, hipStream_t s)
{
    if (P == 0) return hipSuccess;
    hipLaunchKernelGGL(k_features, dim3((unsigned)P), dim3(64), sizeof(double) * 2 * R, s, cell, nh2, T, nbr, k, roff, rcells, dir, R, P, F);
    return hipGetLastError();
}

// ------------------------------------------------------------------------- MLP

// Fragment counts: forward A operands (W, rows = outputs) per layer, then backward A
// operands (W transposed, rows = inputs) of layers 2..4.
//   forward:  L1 8 x 1, L2 8 x 4, L3 8 x 4, L4 1 x 4   (output tiles x K steps)
//   backward: L2 8 x 4, L3 8 x 4, L4 8 x 1
constexpr int kFwdBase[4] = {0, 8, 40, 72};
constexpr int kFwdFrags = 76;
constexpr int kBwdBase[4] = {0, 0, 32, 64};  // index by layer (1..3 used)
constexpr int kBwdFrags = 72;

int mlp_frag_count() { return kFwdFrags + kBwdFrags; }

// Pack the bfloat16 A operands from the FP32 master parameters.  One thread per
// (fragment, lane).
__global__ void k_mlp_pack(const float *__restrict__ theta, MlpDims d, Frag *__restrict__ frags)
{
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= (int64_t)(kFwdFrags + kBwdFrags) * 64) return;
    const int fi = (int)(t / 64), lane = (int)(t % 64);
    const int i = lane & 15, g = lane >> 4;
    Frag out;
    if (fi < kFwdFrags) {
        const int L = fi < 8 ? 0 : fi < 40 ? 1 : fi < 72 ? 2 : 3;
        const int KT = (L == 0) ? 1 : 4;
        const int local = fi - kFwdBase[L];
        const int mt = local / KT, s = local % KT;
        const int row = 16 * mt + i;
        for (int j = 0; j < 8; ++j) {
            const int kk = kslot(s, g, j);
            float w = 0.0f;
            if (row < d.out[L] && kk < d.in[L]) w = theta[d.w_off[L] + (int64_t)row * d.in[L] + kk];
            out.v[j] = bf16_bits(w);
        }
    } else {
        const int bi = fi - kFwdFrags;
        const int L = bi < 32 ? 1 : bi < 64 ? 2 : 3;
        const int KT = (L == 3) ? 1 : 4;
        const int local = bi - kBwdBase[L];
        const int mt = local / KT, s = local % KT;
        const int col = 16 * mt + i;  // input feature of layer L
        for (int j = 0; j < 8; ++j) {
            const int o = kslot(s, g, j);
            float w = 0.0f;
            if (o < d.out[L] && col < d.in[L]) w = theta[d.w_off[L] + (int64_t)o * d.in[L] + col];
            out.v[j] = bf16_bits(w);
        }
    }
    frags[t] = out;
}

hipError_t launch_mlp_pack(const float *theta, const MlpDims &d, void *frags, hipStream_t s)
{
    const int64_t n = (int64_t)(kFwdFrags + kBwdFrags) * 64;
    hipLaunchKernelGGL(k_mlp_pack, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, theta, d, (Frag *)frags);
    return hipGetLastError();
}

namespace {

// B operand of the first layer: standardised inputs of row `row` (zero beyond 8 inputs
// and for rows past the end).
__device__ inline Frag input_frag(const float *__restrict__ X, int64_t row, bool valid, int g)
{
    Frag f;
#pragma unroll
    for (int j = 0; j < 8; ++j) f.v[j] = 0;
    if (valid && g < 2) {
#pragma unroll
        for (int j = 0; j < 4; ++j) f.v[j] = bf16_bits(X[row * 8 + 4 * g + j]);
    }
    return f;
}

}  // namespace

// Inference: each wave evaluates NT tiles of 16 rows.  X [n][8] standardised inputs,
// Y [n][n_out] outputs (log10 fractional populations).
template <int NT>
__global__ __launch_bounds__(256) void k_mlp_forward(const Frag *__restrict__ fw, const float *__restrict__ theta,
                                                     MlpDims d, const float *__restrict__ X, int64_t n,
                                                     float *__restrict__ Y)
{
    const int lane = threadIdx.x & 63;
    const int64_t wave = blockIdx.x * (int64_t)(blockDim.x / 64) + (threadIdx.x >> 6);
    const int64_t row0 = wave * 16 * NT;
    if (row0 >= n) return;
    const int i = lane & 15, g = lane >> 4;
    Frag hb[NT][4];
    f32x4 acc[NT][8];
    // layer 1
    {
        Frag xb[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) {
            const int64_t row = row0 + 16 * t + i;
            xb[t] = input_frag(X, row, row < n, g);
        }
        const float *b1 = theta + d.b_off[0];
#pragma unroll
        for (int mt = 0; mt < 8; ++mt) {
            const Frag a = load_frag(fw, kFwdBase[0] + mt, lane);
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                f32x4 c = {0.f, 0.f, 0.f, 0.f};
                c = mfma(a, xb[t], c);
#pragma unroll
                for (int j = 0; j < 4; ++j) c[j] = gelu(c[j] + b1[16 * mt + 4 * g + j]);
                acc[t][mt] = c;
            }
        }
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int s = 0; s < 4; ++s) hb[t][s] = pack_pair(acc[t][2 * s], acc[t][2 * s + 1]);
    }
    // layers 2 and 3 (each layer's 32 weight operands requested together)
#pragma unroll
    for (int L = 1; L <= 2; ++L) {
        const float *bL = theta + d.b_off[L];
        Frag wL[32];
#pragma unroll
        for (int t = 0; t < 32; ++t) wL[t] = load_frag(fw, kFwdBase[L] + t, lane);
#pragma unroll
        for (int mt = 0; mt < 8; ++mt) {
            f32x4 c[NT];
#pragma unroll
            for (int t = 0; t < NT; ++t) c[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                const Frag a = wL[mt * 4 + s];
#pragma unroll
                for (int t = 0; t < NT; ++t) c[t] = mfma(a, hb[t][s], c[t]);
            }
#pragma unroll
            for (int t = 0; t < NT; ++t)
#pragma unroll
                for (int j = 0; j < 4; ++j) acc[t][mt][j] = gelu(c[t][j] + bL[16 * mt + 4 * g + j]);
        }
#pragma unroll
        for (int t = 0; t < NT; ++t)
#pragma unroll
            for (int s = 0; s < 4; ++s) hb[t][s] = pack_pair(acc[t][2 * s], acc[t][2 * s + 1]);
    }
    // output layer
    const float *b4 = theta + d.b_off[3];
    f32x4 c[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t) c[t] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < 4; ++s) {
        const Frag a = load_frag(fw, kFwdBase[3] + s, lane);
#pragma unroll
        for (int t = 0; t < NT; ++t) c[t] = mfma(a, hb[t][s], c[t]);
    }
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const int64_t row = row0 + 16 * t + i;
        if (row >= n) continue;
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int o = 4 * g + j;
            if (o < d.out[3]) Y[row * d.out[3] + o] = c[t][j] + b4[o];
        }
    }
}

hipError_t launch_mlp_forward(const void *frags, const float *theta, const MlpDims &d, const float *X,
                              int64_t n, float *Y, hipStream_t s)
{
    if (n == 0) return hipSuccess;
    constexpr int NT = 2;
    const int64_t waves = (n + 16 * NT - 1) / (16 * NT);
    const int64_t blocks = (waves + 3) / 4;
    hipLaunchKernelGGL(k_mlp_forward<NT>, dim3((unsigned)blocks), dim3(256), 0, s, (const Frag *)frags, theta, d,
                       X, n, Y);
    return hipGetLastError();
}

// ----------------------------------------------------------------- training
//
// One optimiser step is three launches:
//   k_mlp_fwdbwd  four waves per 16 batch rows: forward, loss and backward through every
//                 layer; each layer's input (bfloat16, as the products read it) and output
//                 gradient (FP32) go to global memory, feature-major with the batch rows
//                 contiguous (Ht [kHRows][ld], DZt [kDRows][ld], ld = batch rounded up to 32);
//   k_mlp_wgrad   the weight gradients dW_L = DZ_L^T H_L as products over the batch rows:
//                 one wave per (16 x 16 tile, chunk of rows), partial sums per chunk;
//   k_mlp_update  the chunks summed in order, Adam, and the new weights written into the
//                 bfloat16 operands of the forward and backward products.
// Rounding is where the single-kernel form had it: activations and output gradients are
// rounded to bfloat16 as product operands, the bias gradient sums the FP32 output gradients.

constexpr int kHRows = 16 + 3 * kHid;                              // feature rows of Ht
constexpr int kHOff[4] = {0, 16, 16 + kHid, 16 + 2 * kHid};        // input of layer L (8 inputs padded to 16)
constexpr int kDRows = 3 * kHid + 16;                              // feature rows of DZt
constexpr int kDOff[4] = {0, kHid, 2 * kHid, 3 * kHid};            // output gradient of layer L (n_out padded to 16)
// weight-gradient tiles (16 outputs x 16 inputs): L1 8 x 1, L2 8 x 8, L3 8 x 8, L4 1 x 8
constexpr int kTileBase[5] = {0, 8, 72, 136, 144};
constexpr int kTiles = 144;
constexpr int kChunkRows = 256;   // batch rows per weight-gradient chunk (more chunks up to kMaxChunks)
constexpr int kMaxChunks = 128;

// (rows padded to 32, row chunks) of a batch
__host__ __device__ inline int mlp_ld(int batch) { return (batch + 31) / 32 * 32; }
inline int mlp_chunks(int ld)
{
    const int c = (ld + kChunkRows - 1) / kChunkRows;
    return c < kMaxChunks ? c : kMaxChunks;
}

// Forward and backward of 16 batch rows by a workgroup of four waves: wave w computes
// output tiles 2w and 2w+1 of every 128-wide layer, whose packed pair is exactly K step w
// of the next product's B operand; the waves exchange those operands through LDS (two
// buffers used in turn, one barrier per exchange).  The output layer (one tile) is
// computed by every wave, so that each holds the output gradient; wave 0 alone writes it
// and the loss.  Every weight operand a wave needs (40 of them) is requested at the start
// and kept in registers while the workgroup takes tiles of 16 rows in grid stride.
__global__ __launch_bounds__(256) void k_mlp_fwdbwd(const Frag *__restrict__ frags, const float *__restrict__ theta,
                                                     MlpDims d, const float *__restrict__ X,
                                                     const float *__restrict__ Tg, int64_t n, int64_t start,
                                                     int batch, float gscale, unsigned short *__restrict__ Ht,
                                                     float *__restrict__ DZt, int ld, float *__restrict__ lpart)
{
    __shared__ Frag xch[2][4][64];
    const Frag *fw = frags;
    const Frag *bw = frags + (int64_t)kFwdFrags * 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int i = lane & 15, g = lane >> 4;

    // weight operands: forward layer 1 (tiles 2w, 2w+1), layers 2 and 3 (those tiles, K
    // steps 0..3), the output layer (K steps 0..3); backward of layers 4, 3, 2 (the wave's
    // tiles of W^T, one K step for layer 4, four otherwise)
    Frag f1[2], f2[8], f3[8], f4[4], g4[2], g3[8], g2[8];
#pragma unroll
    for (int t = 0; t < 2; ++t) f1[t] = load_frag(fw, kFwdBase[0] + 2 * w + t, lane);
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        f2[t] = load_frag(fw, kFwdBase[1] + 8 * w + t, lane);
        f3[t] = load_frag(fw, kFwdBase[2] + 8 * w + t, lane);
    }
#pragma unroll
    for (int t = 0; t < 4; ++t) f4[t] = load_frag(fw, kFwdBase[3] + t, lane);
#pragma unroll
    for (int t = 0; t < 2; ++t) g4[t] = load_frag(bw, kBwdBase[3] + 2 * w + t, lane);
#pragma unroll
    for (int t = 0; t < 8; ++t) {
        g3[t] = load_frag(bw, kBwdBase[2] + 8 * w + t, lane);
        g2[t] = load_frag(bw, kBwdBase[1] + 8 * w + t, lane);
    }
    int buf = 0;
    // exchange: this wave's packed pair in, the four K steps out
    auto exchange = [&](const Frag &mine, Frag (&all)[4]) {
        xch[buf][w][lane] = mine;
        __syncthreads();
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2) all[s2] = xch[buf][s2][lane];
        buf ^= 1;
    };

    // tiles of 16 rows, the workgroup's weights kept in registers from one to the next
    const int64_t n_tiles = ld / 16;
    for (int64_t tile = blockIdx.x; tile < n_tiles; tile += gridDim.x) {
        const int64_t b = tile * 16 + i;   // batch row: the tiles' column i
        const bool valid = b < batch;
        const int64_t row = valid ? (start + b) % n : 0;
        float tg[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
            const int o = 4 * g + j;
            tg[j] = (valid && o < d.out[3]) ? Tg[row * d.out[3] + o] : 0.0f;
        }

        const Frag xb = input_frag(X, row, valid, g);
        if (w == 0) {
#pragma unroll
            for (int j = 0; j < 4; ++j) Ht[(int64_t)(kHOff[0] + 4 * g + j) * ld + b] = xb.v[j];
        }
        // ---- forward
        f32x4 z[2];
        {
            const float *b1 = theta + d.b_off[0];
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                f32x4 c = {0.f, 0.f, 0.f, 0.f};
                c = mfma(f1[t], xb, c);
#pragma unroll
                for (int j = 0; j < 4; ++j) c[j] += b1[16 * (2 * w + t) + 4 * g + j];
                z[t] = c;
            }
        }
        f32x4 dg[3][2];   // GELU derivatives of the wave's tiles, hidden layers 1..3
        Frag hb[4];
#pragma unroll
        for (int L = 0; L < 3; ++L) {
            Frag mine;
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                const int mt = 2 * w + t;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const GeluPair q = gelu_pair(z[t][j]);
                    const unsigned short hv = bf16_bits(q.h);
                    Ht[(int64_t)(kHOff[L + 1] + 16 * mt + 4 * g + j) * ld + b] = hv;
                    mine.v[4 * t + j] = hv;
                    dg[L][t][j] = q.dh;
                }
            }
            exchange(mine, hb);
            if (L < 2) {
                const Frag *fl = L == 0 ? f2 : f3;
                const float *bL = theta + d.b_off[L + 1];
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    f32x4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int s2 = 0; s2 < 4; ++s2) c = mfma(fl[4 * t + s2], hb[s2], c);
#pragma unroll
                    for (int j = 0; j < 4; ++j) c[j] += bL[16 * (2 * w + t) + 4 * g + j];
                    z[t] = c;
                }
            }
        }
        // output layer (every wave) and loss (rows past the batch contribute zero gradients)
        f32x4 dz4;
        {
            f32x4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
            for (int s2 = 0; s2 < 4; ++s2) c = mfma(f4[s2], hb[s2], c);
            const float *b4 = theta + d.b_off[3];
            float sq = 0.0f;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int o = 4 * g + j;
                float e = 0.0f;
                if (valid && o < d.out[3]) e = (c[j] + b4[o]) - tg[j];
                sq += e * e;
                dz4[j] = gscale * e;
            }
            if (w == 0) {
#pragma unroll
                for (int off = 32; off >= 1; off >>= 1) sq += __shfl_xor(sq, off);
                if (lane == 0) lpart[tile] = sq;
#pragma unroll
                for (int j = 0; j < 4; ++j) DZt[(int64_t)(kDOff[3] + 4 * g + j) * ld + b] = dz4[j];
            }
        }
        // ---- backward: layer 4's output gradient to layer 3's (one K step), then layers 3, 2
        f32x4 dz[2];
        {
            const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
            const Frag db = pack_pair(dz4, zero);
#pragma unroll
            for (int t = 0; t < 2; ++t) {
                f32x4 c = {0.f, 0.f, 0.f, 0.f};
                c = mfma(g4[t], db, c);
#pragma unroll
                for (int j = 0; j < 4; ++j) dz[t][j] = c[j] * dg[2][t][j];
            }
        }
#pragma unroll
        for (int L = 2; L >= 0; --L) {
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int j = 0; j < 4; ++j) DZt[(int64_t)(kDOff[L] + 16 * (2 * w + t) + 4 * g + j) * ld + b] = dz[t][j];
            if (L > 0) {
                Frag db[4];
                exchange(pack_pair(dz[0], dz[1]), db);
                const Frag *gl = L == 2 ? g3 : g2;
#pragma unroll
                for (int t = 0; t < 2; ++t) {
                    f32x4 c = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
                    for (int s2 = 0; s2 < 4; ++s2) c = mfma(gl[4 * t + s2], db[s2], c);
#pragma unroll
                    for (int j = 0; j < 4; ++j) dz[t][j] = c[j] * dg[L - 1][t][j];
                }
            }
        }
    }
}

// Weight gradients of one 16 x 16 tile over one chunk of batch rows (blockIdx.x: tile,
// blockIdx.y: chunk).  The A operand is the output gradients (rounded to bfloat16), the
// B operand the layer's inputs; a lane loads its eight rows as two runs of four.  Tiles
// of the first input column also sum the FP32 output gradients for the bias.  gpart
// [chunks][n_params].
__global__ __launch_bounds__(64) void k_mlp_wgrad(MlpDims d, const unsigned short *__restrict__ Ht,
                                                   const float *__restrict__ DZt, int ld, int chunk,
                                                   float *__restrict__ gpart)
{
    const int tile = blockIdx.x, c = blockIdx.y;
    const int L = tile < kTileBase[1] ? 0 : tile < kTileBase[2] ? 1 : tile < kTileBase[3] ? 2 : 3;
    const int NT = L == 0 ? 1 : 8;
    const int local = tile - kTileBase[L];
    const int mt = local / NT, nt = local - mt * NT;
    const int lane = threadIdx.x;
    const int i = lane & 15, g = lane >> 4;
    const float *arow = DZt + (int64_t)(kDOff[L] + 16 * mt + i) * ld;
    const unsigned short *brow = Ht + (int64_t)(kHOff[L] + 16 * nt + i) * ld;
    const int r_beg = c * chunk, r_end = min(ld, r_beg + chunk);
    f32x4 acc = {0.f, 0.f, 0.f, 0.f};
    float bsum = 0.0f;
    // rows r0 + 16 q + 4 g + (0..3), q = 0, 1: the lane's eight K slots of one step
    struct Raw {
        float4 a0, a1;
        uint2 b0, b1;
    };
    auto fetch = [&](int r0) {
        Raw w;
        w.a0 = *reinterpret_cast<const float4 *>(arow + r0 + 4 * g);
        w.a1 = *reinterpret_cast<const float4 *>(arow + r0 + 16 + 4 * g);
        w.b0 = *reinterpret_cast<const uint2 *>(brow + r0 + 4 * g);
        w.b1 = *reinterpret_cast<const uint2 *>(brow + r0 + 16 + 4 * g);
        return w;
    };
    auto use = [&](const Raw &w) {
        Frag fa, fb;
        fa.v[0] = bf16_bits(w.a0.x);
        fa.v[1] = bf16_bits(w.a0.y);
        fa.v[2] = bf16_bits(w.a0.z);
        fa.v[3] = bf16_bits(w.a0.w);
        fa.v[4] = bf16_bits(w.a1.x);
        fa.v[5] = bf16_bits(w.a1.y);
        fa.v[6] = bf16_bits(w.a1.z);
        fa.v[7] = bf16_bits(w.a1.w);
        fb.v[0] = (unsigned short)(w.b0.x & 0xFFFFu);
        fb.v[1] = (unsigned short)(w.b0.x >> 16);
        fb.v[2] = (unsigned short)(w.b0.y & 0xFFFFu);
        fb.v[3] = (unsigned short)(w.b0.y >> 16);
        fb.v[4] = (unsigned short)(w.b1.x & 0xFFFFu);
        fb.v[5] = (unsigned short)(w.b1.x >> 16);
        fb.v[6] = (unsigned short)(w.b1.y & 0xFFFFu);
        fb.v[7] = (unsigned short)(w.b1.y >> 16);
        bsum += ((w.a0.x + w.a0.y) + (w.a0.z + w.a0.w)) + ((w.a1.x + w.a1.y) + (w.a1.z + w.a1.w));
        acc = mfma(fa, fb, acc);
    };
    int r0 = r_beg;
    // four steps' operands requested before the first of their products
    for (; r0 + 96 < r_end; r0 += 128) {
        const Raw w0 = fetch(r0), w1 = fetch(r0 + 32), w2 = fetch(r0 + 64), w3 = fetch(r0 + 96);
        use(w0);
        use(w1);
        use(w2);
        use(w3);
    }
    for (; r0 < r_end; r0 += 32) use(fetch(r0));
    float *gp = gpart + (int64_t)c * d.n_params;
    const int col = 16 * nt + i;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int o = 16 * mt + 4 * g + j;
        if (o < d.out[L] && col < d.in[L]) gp[d.w_off[L] + (int64_t)o * d.in[L] + col] = acc[j];
    }
    if (nt == 0) {
        // output 16 mt + i: the row sums of the four lane groups, in order
        const float t0 = __shfl(bsum, i), t1 = __shfl(bsum, 16 + i), t2 = __shfl(bsum, 32 + i),
                    t3 = __shfl(bsum, 48 + i);
        const int o = 16 * mt + i;
        if (g == 0 && o < d.out[L]) gp[d.b_off[L] + o] = ((t0 + t1) + t2) + t3;
    }
}

int mlp_train_ld(int batch) { return mlp_ld(batch); }
int mlp_train_chunks(int batch) { return mlp_chunks(mlp_ld(batch)); }
size_t mlp_train_ht_count(int batch) { return (size_t)kHRows * mlp_ld(batch); }
size_t mlp_train_dzt_count(int batch) { return (size_t)kDRows * mlp_ld(batch); }

hipError_t launch_mlp_train(const void *frags, const float *theta, const MlpDims &d, const float *X, const float *T,
                            int64_t n, int64_t start, int batch, unsigned short *Ht, float *DZt, float *gpart,
                            float *lpart, hipStream_t s)
{
    const int ld = mlp_ld(batch);
    const float gscale = (float)(2.0 / ((double)batch * d.out[3]));
    // up to 1024 workgroups (four per CU), each taking every 1024th tile of 16 rows
    const int grid = ld / 16 < 1024 ? ld / 16 : 1024;
    hipLaunchKernelGGL(k_mlp_fwdbwd, dim3((unsigned)grid), dim3(256), 0, s, (const Frag *)frags, theta, d, X, T,
                       n, start, batch, gscale, Ht, DZt, ld, lpart);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int S = mlp_chunks(ld);
    const int chunk = (ld / 32 + S - 1) / S * 32;
    hipLaunchKernelGGL(k_mlp_wgrad, dim3(kTiles, S), dim3(64), 0, s, d, (const unsigned short *)Ht,
                       (const float *)DZt, ld, chunk, gpart);
    return hipGetLastError();
}

// Sum the chunk partials in order; optionally write the gradient; with `update`, one
// Adam step (c1 = 1/(1 - beta1^t), c2 = 1/(1 - beta2^t)) and the new weight's bfloat16
// value written into its slot of the forward operands and, for layers 2-4, of the
// backward (transposed) operands; the slots are those k_mlp_pack fills, found by
// inverting its index map.  The first thread writes the batch loss (mean squared error).
__global__ void k_mlp_update(float *__restrict__ theta, float *__restrict__ m, float *__restrict__ v,
                             unsigned short *__restrict__ fslot, MlpDims d, const float *__restrict__ gpart, int S,
                             int update, float lr, float b1, float b2, float eps, float c1, float c2,
                             const float *__restrict__ lpart, int n_waves, float inv_count, float *__restrict__ loss,
                             float *__restrict__ grad_out)
{
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int64_t np = d.n_params;
    if (blockIdx.x == 0 && loss) {
        // the loss partials: thread t sums entries t, t + 256, ... in order, then a fixed tree
        __shared__ float red[256];
        float sacc = 0.0f;
        for (int w = threadIdx.x; w < n_waves; w += blockDim.x) sacc += lpart[w];
        red[threadIdx.x] = sacc;
        __syncthreads();
        for (int h = blockDim.x / 2; h > 0; h >>= 1) {
            if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
            __syncthreads();
        }
        if (threadIdx.x == 0) *loss = red[0] * inv_count;
    }
    if (p >= np) return;
    float gsum = 0.0f;
    for (int c = 0; c < S; ++c) gsum += gpart[(int64_t)c * np + p];
    if (grad_out) grad_out[p] = gsum;
    if (!update) return;
    const float mm = b1 * m[p] + (1.0f - b1) * gsum;
    const float vv = b2 * v[p] + (1.0f - b2) * gsum * gsum;
    m[p] = mm;
    v[p] = vv;
    const float t = theta[p] - lr * (mm * c1) / (sqrtf(vv * c2) + eps);
    theta[p] = t;
    int L = -1;
#pragma unroll
    for (int l = 0; l < 4; ++l)
        if (p >= d.w_off[l] && p < d.b_off[l]) L = l;
    if (L < 0) return;   // a bias: not in the packed operands
    const unsigned short tb = bf16_bits(t);
    const int o = (int)((p - d.w_off[L]) / d.in[L]);
    const int k = (int)((p - d.w_off[L]) - (int64_t)o * d.in[L]);
    {
        // forward operand: row o of tile mt, reduction index k = kslot(s, g, j)
        const int KT = L == 0 ? 1 : 4;
        const int s = k >> 5, r = k & 31;
        const int j = 4 * (r >> 4) + (r & 3), g = (r & 15) >> 2;
        const int fi = kFwdBase[L] + (o >> 4) * KT + s;
        fslot[((int64_t)fi * 64 + 16 * g + (o & 15)) * 8 + j] = tb;
    }
    if (L >= 1) {
        // backward operand: row k (the layer's input) of tile k / 16, reduction index o
        const int KT = L == 3 ? 1 : 4;
        const int s = o >> 5, r = o & 31;
        const int j = 4 * (r >> 4) + (r & 3), g = (r & 15) >> 2;
        const int fi = kFwdFrags + kBwdBase[L] + (k >> 4) * KT + s;
        fslot[((int64_t)fi * 64 + 16 * g + (k & 15)) * 8 + j] = tb;
    }
}

hipError_t launch_mlp_update(float *theta, float *m, float *v, void *frags, const MlpDims &d, const float *gpart,
                             int batch, int update, float lr, float b1, float b2, float eps, float c1, float c2,
                             const float *lpart, float inv_count, float *loss, float *grad_out, hipStream_t s)
{
    const int ld = mlp_ld(batch);
    const int64_t np = d.n_params;
    hipLaunchKernelGGL(k_mlp_update, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, s, theta, m, v,
                       (unsigned short *)frags, d, gpart, mlp_chunks(ld), update, lr, b1, b2, eps, c1, c2, lpart,
                       ld / 16, inv_count, loss, grad_out);
    return hipGetLastError();
}

// Standardised FP32 inputs from FP64 features.
__global__ void k_mlp_standardise(const double *__restrict__ F, MlpNorm nm, int64_t P, float *__restrict__ X)
{
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (t >= P * 8) return;
    const int f = (int)(t % 8);
    X[t] = (float)((F[t] - nm.mean[f]) / nm.std[f]);
}

hipError_t launch_mlp_standardise(const double *F, const MlpNorm &nm, int64_t P, float *X, hipStream_t s)
{
    if (P == 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_standardise, dim3((unsigned)((P * 8 + 255) / 256)), dim3(256), 0, s, F, nm, P, X);
    return hipGetLastError();
}

// Boltzmann fraction of level i at temperature T, floored at 1e-300.
__device__ inline double lte_fraction(const SpeciesDev &sp, double T, int i)
{
    const double kT = kKB * T;
    double Z = 0.0;
    for (int j = 0; j < sp.n_lev; ++j) Z += sp.g[j] * exp(-(sp.E[j] - sp.E[0]) / kT);
    const double f = sp.g[i] * exp(-(sp.E[i] - sp.E[0]) / kT) / Z;
    return f > 1e-300 ? f : 1e-300;
}

// Training targets: log10 of the departure from LTE, log10 (f_i / f_i^LTE), with the
// fractional population f_i = n_i / (abundance n_H2) floored at 1e-300.
__global__ void k_mlp_targets(SpeciesDev sp, const double *__restrict__ pops, const CellRec *__restrict__ cell,
                              const double *__restrict__ T, int64_t P, float *__restrict__ Tg)
{
    const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const int n_lev = sp.n_lev;
    if (t >= P * n_lev) return;
    const int64_t p = t / n_lev;
    const int i = (int)(t % n_lev);
    double f = pops[t] / cell[p].ntot;
    f = f > 1e-300 ? f : 1e-300;
    Tg[t] = (float)(log10(f) - log10(lte_fraction(sp, T[p], i)));
}

hipError_t launch_mlp_targets(const SpeciesDev &sp, const double *pops, const CellRec *cell, const double *T,
                              int64_t P, float *Tg, hipStream_t s)
{
    if (P == 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_targets, dim3((unsigned)((P * sp.n_lev + 255) / 256)), dim3(256), 0, s, sp, pops, cell,
                       T, P, Tg);
    return hipGetLastError();
}

// Populations from predicted departures y: n_i = ntot w_i / sum_j w_j with
// w_i = f_i^LTE 10^y_i (evaluated relative to the largest log10 w).  A point with a
// non-finite prediction keeps what pops already holds and is counted.
__global__ void k_mlp_populations(SpeciesDev sp, const float *__restrict__ Y, const CellRec *__restrict__ cell,
                                  const double *__restrict__ T, int64_t P, double *__restrict__ pops,
                                  unsigned long long *__restrict__ n_bad)
{
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= P) return;
    const int n_lev = sp.n_lev;
    double a[kMaxLev];
    double amax = -INFINITY;
    bool ok = true;
    for (int i = 0; i < n_lev; ++i) {
        const double y = (double)Y[p * n_lev + i];
        ok = ok && isfinite(y);
        a[i] = log10(lte_fraction(sp, T[p], i)) + y;
        amax = fmax(amax, a[i]);
    }
    if (!ok) {
        atomicAdd(n_bad, 1ull);
        return;
    }
    double sum = 0.0;
    for (int i = 0; i < n_lev; ++i) {
        a[i] = exp10(a[i] - amax);
        sum += a[i];
    }
    const double nt = cell[p].ntot;
    for (int i = 0; i < n_lev; ++i) pops[p * n_lev + i] = nt * a[i] / sum;
}

hipError_t launch_mlp_populations(const SpeciesDev &sp, const float *Y, const CellRec *cell, const double *T,
                                  int64_t P, double *pops, unsigned long long *n_bad, hipStream_t s)
{
    if (P == 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_populations, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, sp, Y, cell, T, P, pops,
                       n_bad);
    return hipGetLastError();
}

}  // namespace nlte
