// Per-point setup, LTE populations and the neighbour-graph ray walk.
//
// Everything here is compiled with -ffp-contract=off: the walk's comparisons and the
// line-width speeds feed integer decisions (the next cell, the number of velocity
// sub-steps) that must not depend on fused rounding.
#include <hipcub/hipcub.hpp>

#include <vector>

#include "nlte_internal.h"

namespace nlte {

// Sec. 2.2.1: v_th = sqrt(2kT/m); the line width is nu/c sqrt(v_th^2 + v_turb^2).
__global__ void k_setup_points(const double *__restrict__ pos, const double *__restrict__ vel,
                               const double *__restrict__ nh2, const double *__restrict__ T,
                               const double *__restrict__ vturb, const double *__restrict__ X,
                               double mass, int64_t P, CellRec *__restrict__ cell)
{
    int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= P) return;
    CellRec c;
    c.px = pos[3 * p];
    c.py = pos[3 * p + 1];
    c.pz = pos[3 * p + 2];
    c.vx = vel[3 * p];
    c.vy = vel[3 * p + 1];
    c.vz = vel[3 * p + 2];
    double vth2 = 2.0 * kKB * T[p] / mass;
    c.vw = sqrt(vth2 + vturb[p] * vturb[p]);
    c.ntot = X[p] * nh2[p];
    cell[p] = c;
}

hipError_t launch_setup_points(const double *pos, const double *vel, const double *nh2,
                               const double *T, const double *vturb, const double *X,
                               double mass, int64_t P, CellRec *cell, hipStream_t s)
{
    if (P == 0) return hipSuccess;
    int64_t blocks = (P + 255) / 256;
    hipLaunchKernelGGL(k_setup_points, dim3((unsigned)blocks), dim3(256), 0, s, pos, vel, nh2, T,
                       vturb, X, mass, P, cell);
    return hipGetLastError();
}

// Boltzmann populations at the local temperature, normalised to the species density.
__global__ void k_lte(SpeciesDev sp, const CellRec *__restrict__ cell, const double *__restrict__ T,
                      int64_t P, double *__restrict__ pops)
{
    int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= P) return;
    double kT = kKB * T[p];
    double Z = 0.0;
    for (int i = 0; i < sp.n_lev; ++i) Z += sp.g[i] * exp(-(sp.E[i] - sp.E[0]) / kT);
    double nt = cell[p].ntot;
    for (int i = 0; i < sp.n_lev; ++i)
        pops[p * sp.n_lev + i] = nt * sp.g[i] * exp(-(sp.E[i] - sp.E[0]) / kT) / Z;
}

hipError_t launch_lte(const SpeciesDev &sp, const CellRec *cell, const double *T, int64_t P,
                      double *pops, hipStream_t s)
{
    if (P == 0) return hipSuccess;
    hipLaunchKernelGGL(k_lte, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, sp, cell, T, P, pops);
    return hipGetLastError();
}

// Sec. 3.2 ray walk.  One thread per (origin point, ray).  From the current cell the
// walk moves to the neighbour whose projection Z on the ray exceeds the current one and
// whose squared distance q to the line through the origin is smallest (ties: lower
// index), and stops when no neighbour lies farther along the ray or at a flagged
// boundary point.  Z strictly increases, so at most P steps are taken.  A step reads the
// current cell's neighbour slots from the table (positions and indices side by side)
// rather than gathering each neighbour's record.
template <bool FILL>
__global__ void k_walk(const CellRec *__restrict__ cell, const NbrEntry *__restrict__ tab, int k,
                       const uint8_t *__restrict__ bnd, const double *__restrict__ dir, int n_rays,
                       int64_t P, int64_t *__restrict__ len_out, const int64_t *__restrict__ off,
                       int32_t *__restrict__ cells_out)
{
    int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= P * n_rays) return;
    int64_t O = q / n_rays;
    int r = (int)(q - O * n_rays);
    const double nx = dir[3 * r], ny = dir[3 * r + 1], nz = dir[3 * r + 2];
    const double ox = cell[O].px, oy = cell[O].py, oz = cell[O].pz;
    int64_t cur = O;
    double zcur = 0.0;
    int64_t len = 0;
    int64_t base = FILL ? off[q] : 0;
    for (int64_t step = 0; step < P; ++step) {
        if (cur != O && bnd != nullptr && bnd[cur]) break;
        int64_t best = -1;
        double bq = 0.0, bz = 0.0;
        for (int s = 0; s < k; ++s) {
            const NbrEntry e = tab[cur * k + s];
            const int32_t m = e.m;
            if (m < 0) continue;
            double dx = e.x - ox;
            double dy = e.y - oy;
            double dz = e.z - oz;
            double Z = (dx * nx + dy * ny) + dz * nz;
            if (!(Z > zcur)) continue;
            double qx = dx - Z * nx, qy = dy - Z * ny, qz = dz - Z * nz;
            double qq = (qx * qx + qy * qy) + qz * qz;
            if (best < 0 || qq < bq || (qq == bq && m < best)) {
                best = m;
                bq = qq;
                bz = Z;
            }
        }
        if (best < 0) break;
        if (FILL) cells_out[base + len] = (int32_t)best;
        ++len;
        cur = best;
        zcur = bz;
    }
    if (!FILL) len_out[q] = len;
}

__global__ void k_nbr_table(const CellRec *__restrict__ cell, const int32_t *__restrict__ nbr, int64_t n,
                            NbrEntry *__restrict__ tab)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t m = nbr[i];
    NbrEntry e;
    e.m = m;
    e.pad = 0;
    e.x = m >= 0 ? cell[m].px : 0.0;
    e.y = m >= 0 ? cell[m].py : 0.0;
    e.z = m >= 0 ? cell[m].pz : 0.0;
    tab[i] = e;
}

hipError_t launch_nbr_table(const CellRec *cell, const int32_t *nbr, int k, int64_t P, NbrEntry *tab, hipStream_t s)
{
    const int64_t n = P * k;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_nbr_table, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, cell, nbr, n, tab);
    return hipGetLastError();
}

hipError_t launch_walk_count(const CellRec *cell, const NbrEntry *tab, int k, const uint8_t *bnd,
                             const double *dir, int n_rays, int64_t P, int64_t *len, hipStream_t s)
{
    int64_t n = P * n_rays;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_walk<false>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, cell, tab,
                       k, bnd, dir, n_rays, P, len, nullptr, nullptr);
    return hipGetLastError();
}

hipError_t launch_walk_fill(const CellRec *cell, const NbrEntry *tab, int k, const uint8_t *bnd,
                            const double *dir, int n_rays, int64_t P, const int64_t *off,
                            int32_t *cells, hipStream_t s)
{
    int64_t n = P * n_rays;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_walk<true>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, cell, tab,
                       k, bnd, dir, n_rays, P, nullptr, off, cells);
    return hipGetLastError();
}

// In-place inclusive scan of lengths stored at [1..n] of an (n+1)-array whose [0] is 0,
// turning them into CSR offsets.  With tmp == nullptr only *tmp_bytes is set.
hipError_t scan_lengths(int64_t *arr, int64_t n, void *tmp, size_t *tmp_bytes, hipStream_t s)
{
    return hipcub::DeviceScan::InclusiveSum(tmp, *tmp_bytes, arr + 1, arr + 1, (int)n, s);
}

// Order of the points by decreasing cost (stable: equal costs keep increasing index).
hipError_t sort_by_cost(unsigned long long *cost, int32_t *order, int64_t P, hipStream_t s)
{
    unsigned long long *keys_out = nullptr;
    int32_t *idx_in = nullptr;
    hipError_t e = hipMalloc((void **)&keys_out, sizeof(unsigned long long) * P);
    if (e == hipSuccess) e = hipMalloc((void **)&idx_in, sizeof(int32_t) * P);
    if (e == hipSuccess) {
        std::vector<int32_t> h(P);
        for (int64_t i = 0; i < P; ++i) h[i] = (int32_t)i;
        e = hipMemcpy(idx_in, h.data(), sizeof(int32_t) * P, hipMemcpyHostToDevice);
    }
    size_t tmp_bytes = 0;
    if (e == hipSuccess)
        e = hipcub::DeviceRadixSort::SortPairsDescending(nullptr, tmp_bytes, cost, keys_out, idx_in, order, (int)P,
                                                         0, 64, s);
    void *tmp = nullptr;
    if (e == hipSuccess) e = hipMalloc(&tmp, tmp_bytes ? tmp_bytes : 1);
    if (e == hipSuccess)
        e = hipcub::DeviceRadixSort::SortPairsDescending(tmp, tmp_bytes, cost, keys_out, idx_in, order, (int)P, 0,
                                                         64, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (tmp) (void)hipFree(tmp);
    if (keys_out) (void)hipFree(keys_out);
    if (idx_in) (void)hipFree(idx_in);
    return e;
}

// Morton code of a point within its model's bounding box (box[m] = min x, y, z and
// extents): each coordinate quantised to q = floor((x - min) / extent * (2^21 - 1)) (0 for
// a flat extent), bits interleaved x, y, z from the most significant.
__global__ void k_morton(const CellRec *__restrict__ cell, const int32_t *__restrict__ model_of,
                         const double *__restrict__ box, int64_t P, unsigned long long *__restrict__ code)
{
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= P) return;
    const double *b = box + 6 * model_of[p];
    const double x[3] = {cell[p].px, cell[p].py, cell[p].pz};
    unsigned long long q[3];
    for (int d = 0; d < 3; ++d) {
        const double ext = b[3 + d];
        q[d] = ext > 0.0 ? (unsigned long long)floor((x[d] - b[d]) / ext * 2097151.0) : 0ull;
    }
    unsigned long long c = 0;
    for (int bit = 0; bit < 21; ++bit)
        for (int d = 0; d < 3; ++d) c |= ((q[d] >> bit) & 1ull) << (3 * bit + 2 - d);
    code[p] = c;
}

__global__ void k_iota(int32_t *__restrict__ v, int64_t n)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i < n) v[i] = (int32_t)i;
}

// Points of each model (offsets on the device) in Morton order, equal codes by index
// (the radix sort is stable).  Synchronises the stream.
hipError_t morton_order(const CellRec *cell, const int32_t *model_of, const double *box, const int64_t *off,
                        int n_models, int64_t P, int32_t *order, hipStream_t s)
{
    if (P == 0) return hipSuccess;
    unsigned long long *codes = nullptr, *codes_out = nullptr;
    int32_t *idx = nullptr;
    void *tmp = nullptr;
    size_t tmp_bytes = 0;
    hipError_t e = hipMalloc((void **)&codes, sizeof(unsigned long long) * P);
    if (e == hipSuccess) e = hipMalloc((void **)&codes_out, sizeof(unsigned long long) * P);
    if (e == hipSuccess) e = hipMalloc((void **)&idx, sizeof(int32_t) * P);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(k_morton, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, cell, model_of, box, P, codes);
        hipLaunchKernelGGL(k_iota, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, idx, P);
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = hipcub::DeviceSegmentedRadixSort::SortPairs(nullptr, tmp_bytes, codes, codes_out, idx, order, (int)P,
                                                         n_models, off, off + 1, 0, 63, s);
    if (e == hipSuccess) e = hipMalloc(&tmp, tmp_bytes ? tmp_bytes : 1);
    if (e == hipSuccess)
        e = hipcub::DeviceSegmentedRadixSort::SortPairs(tmp, tmp_bytes, codes, codes_out, idx, order, (int)P,
                                                         n_models, off, off + 1, 0, 63, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (tmp) (void)hipFree(tmp);
    if (codes) (void)hipFree(codes);
    if (codes_out) (void)hipFree(codes_out);
    if (idx) (void)hipFree(idx);
    return e;
}

}  // namespace nlte
