// Line coefficients and the ray-pair formal solve (the ALI hot loop).
//
// Discretisation (Sec. 3.3, no scattering): on the nodes of a ray pair the second-order
// equation d^2u/dtau^2 = u - S becomes the tridiagonal system
//   -A_i u_{i-1} + (1 + A_i + C_i) u_i - C_i u_{i+1} = S_i,
//   A_i = 2 / (D_-(D_- + D_+)),  C_i = 2 / (D_+(D_- + D_+)),
// with D_-+ the optical-depth steps on either side of node i, and second-order (Auer)
// boundary rows that bring in the incoming intensity at both ends.  The elimination of
// Rybicki & Hummer carries F_i = (1 + A_i F_{i-1}/(1 + F_{i-1})) / C_i.
//
// Both ends are eliminated toward the origin O of the pair, so each ray of the pair is
// one half-sweep from its far end to O.  Writing h_i = (D_- + D_+)/2 and
//   Q_i = F_i / (D_+ (1 + F_i)),   y_i = z_i / D_+
// (z_i the Rybicki-Hummer right-hand side), one elimination step becomes
//   T = h_i + Q_{i-1};  F_i = D_+ T;  E = 1/(1 + F_i);  Q_i = T E;  y_i = (S_i h_i + y_{i-1}) E
// with Q = 1, y = I_boundary, D_- = 0 before the first node, which is exactly the Auer
// boundary row.  No step divides by an optical depth.  The sweep carries Q and y as
// fractions N/D and Y/D (scaled by sqrt 2, which cancels at O), which turns each step
// into three multiply-adds of non-negative numbers with no division (see elim_step).
// At O the two halves combine into
//   u_O = (h_O S_O + y_f + y_b) / (h_O + Q_f + Q_b),   Lambda_OO = h_O / (h_O + Q_f + Q_b),
// and u_O - Lambda_OO S_O = (y_f + y_b) / (h_O + Q_f + Q_b) without cancellation.
//
// Mapping: see formal_solve_kernels.h (one wave per origin point and line block, lanes
// over frequencies and up to five lines per lane sharing the profile, ray segments staged
// in LDS).
#include "nlte_internal.h"

namespace nlte {

// ---------------------------------------------------------------- line coefficients

// Eq. (lines) without the profile, at line centre:
//   k_eta = (h nu/4 pi) n_u A_ul,  k_chi = (h nu/4 pi)(n_l B_lu - n_u B_ul),
// line-centre opacity kappa = k_chi / (sqrt(pi) dnu), dnu = nu v_w / c, S = k_eta / k_chi.
// Non-positive opacity (population inversion) is clamped to kappa = S = 0 and counted.
template <bool F32>
__global__ void k_line_coef(SpeciesDev sp, const CellRec *__restrict__ cell,
                            const double *__restrict__ pops, int64_t P, void *__restrict__ lc,
                            unsigned long long *__restrict__ maser)
{
    int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= P * sp.n_lines) return;
    int64_t p = q / sp.n_lines;
    int l = (int)(q - p * sp.n_lines);
    const double *n = pops + p * sp.n_lev;
    double nu_ = sp.nu[l];
    double pre = sp.pre[l];
    double nup = n[sp.lu[l]], nlo = n[sp.ll[l]];
    double keta = pre * nup * sp.A[l];
    double kchi = pre * (nlo * sp.Blu[l] - nup * sp.Bul[l]);
    double kap = 0.0, S = 0.0;
    if (kchi > 0.0) {
        double dnu = nu_ * cell[p].vw / kC;
        kap = kchi / (kSqrtPi * dnu);
        S = keta / kchi;
    } else if (maser) {
        atomicAdd(maser, 1ull);
    }
    if (F32)
        reinterpret_cast<float2 *>(lc)[q] = make_float2((float)kap, (float)S);
    else
        reinterpret_cast<double2 *>(lc)[q] = make_double2(kap, S);
}

hipError_t launch_line_coef(const SpeciesDev &sp, const CellRec *cell, const double *pops,
                            int64_t P, int fp32, void *lc, int64_t *maser_count, hipStream_t s)
{
    int64_t n = P * sp.n_lines;
    if (n == 0) return hipSuccess;
    dim3 grid((unsigned)((n + 255) / 256));
    auto *m = reinterpret_cast<unsigned long long *>(maser_count);
    if (fp32)
        hipLaunchKernelGGL(k_line_coef<true>, grid, dim3(256), 0, s, sp, cell, pops, P, lc, m);
    else
        hipLaunchKernelGGL(k_line_coef<false>, grid, dim3(256), 0, s, sp, cell, pops, P, lc, m);
    return hipGetLastError();
}

// ---------------------------------------------------------------- formal solve

// The kernels are templates in formal_solve_kernels.h, instantiated per precision in
// fs_fp64.hip and fs_fp32.hip (compiled in parallel).
hipError_t launch_formal_solve(const SolveArgs &a, const SolveConfig &cfg, int fp32, hipStream_t s)
{
    if (a.n_blocks == 0) return hipSuccess;
    return fp32 ? launch_formal_solve_f32(a, cfg, s) : launch_formal_solve_f64(a, cfg, s);
}

// Elimination steps per frequency over all half rays: the cells of every cached walk
// plus their velocity sub-steps, with the same sub-step rule as the sweep.  One thread
// per (point, ray); block sums are added atomically (integer, order-independent).
__global__ __launch_bounds__(256) void k_count_steps(SolveArgs a, unsigned long long *steps,
                                                     unsigned long long *point_cost)
{
    __shared__ unsigned long long part[256];
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    unsigned long long n = 0;
    if (q < a.P * a.n_rays) {
        const int64_t O = q / a.n_rays;
        const int ray = (int)(q - O * a.n_rays);
        const double nx = a.dir[3 * ray], ny = a.dir[3 * ray + 1], nz = a.dir[3 * ray + 2];
        const CellRec cO = a.cell[O];
        const int64_t beg = a.roff[q];
        const int L = (int)(a.roff[q + 1] - beg);
        double s_prev = 0.0, w_prev = cO.vw;   // start at O and walk outward
        for (int i = 0; i < L; ++i) {
            const CellRec c = a.cell[a.rcells[beg + i]];
            double dvx = c.vx - cO.vx, dvy = c.vy - cO.vy, dvz = c.vz - cO.vz;
            double sv = (dvx * nx + dvy * ny) + dvz * nz;
            double ds = fabs(sv - s_prev);
            double thr = a.f_sub * fmin(c.vw, w_prev);
            unsigned long long m = 1;
            if (ds > thr) {
                const double mr = ceil(ds / thr);
                m = mr < (double)kMaxSub ? (unsigned long long)mr : (unsigned long long)kMaxSub;
            }
            n += m;
            s_prev = sv;
            w_prev = c.vw;
        }
        if (point_cost != nullptr) atomicAdd(&point_cost[O], n + 1);
    }
    part[threadIdx.x] = n;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(steps, part[0]);
}

hipError_t launch_count_steps(const SolveArgs &a, int64_t *steps, unsigned long long *point_cost,
                              hipStream_t s)
{
    const int64_t n = a.P * a.n_rays;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_count_steps, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a,
                       reinterpret_cast<unsigned long long *>(steps), point_cost);
    return hipGetLastError();
}

}  // namespace nlte
