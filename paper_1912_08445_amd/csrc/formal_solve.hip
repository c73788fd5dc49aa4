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
// boundary row.  No step divides by an optical depth, so zero-opacity segments need no
// floor.  At O the two halves combine into
//   u_O = (h_O S_O + y_f + y_b) / (h_O + Q_f + Q_b),   Lambda_OO = h_O / (h_O + Q_f + Q_b),
// and u_O - Lambda_OO S_O = (y_f + y_b) / (h_O + Q_f + Q_b) without cancellation.
//
// Mapping: one workgroup = one wave = one origin point and up to 64 (line, frequency)
// items; all lanes walk the same nodes (uniform control flow), each with its own
// frequency.  The wave stages up to 64 cells of a ray at a time in LDS (position,
// velocity projection, Doppler coefficients, sub-step count, kappa and S of its lines);
// the sweep then reads them as broadcasts.  Velocity sub-steps interpolate the Doppler
// offset x, kappa and S linearly between cells in registers.
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

template <bool F32>
struct Bulk {
    using T = double;
    using T2 = double2;
};
template <>
struct Bulk<true> {
    using T = float;
    using T2 = float2;
};

// One staged node of a half ray.  (a, b) give the Doppler offset of a lane's frequency
// x_q at this node as x = a x_q - b; (dzh, m) describe the segment to the next node
// toward O: m sub-intervals of half-length dzh each.
template <typename T>
struct NodeRec {
    T a, b, dzh;
    T kap[2], S[2];
    int m;
};

struct HalfState {
    double Q, y, Dm;
};

__device__ __forceinline__ double rcp64(double d)
{
    // v_rcp_f64 refined by two Newton steps (d >= 1 here)
    double r = __builtin_amdgcn_rcp(d);
    double e = fma(-d, r, 1.0);
    r = fma(r, e, r);
    e = fma(-d, r, 1.0);
    return fma(r, e, r);
}

__device__ __forceinline__ double profile(double x) { return exp(-(x * x)); }
__device__ __forceinline__ float profile(float x)
{
    // e^{-x^2} = 2^{-x^2 log2 e} on the hardware exp2
    return __builtin_amdgcn_exp2f(-(x * x) * 1.44269504088896340736f);
}

template <bool F32>
__device__ __forceinline__ void elim_step(typename Bulk<F32>::T chi_t, typename Bulk<F32>::T S_t,
                                          typename Bulk<F32>::T dzh, typename Bulk<F32>::T &chi_prev,
                                          typename Bulk<F32>::T &S_e, HalfState &st, double floor)
{
    // trapezoid optical depth of the step, floored like the zero-opacity far wings
    double Dp = fmax((double)((chi_prev + chi_t) * dzh), floor);
    double h = 0.5 * (st.Dm + Dp);
    double Tt = h + st.Q;
    double F = Dp * Tt;
    double E = rcp64(1.0 + F);
    st.Q = Tt * E;
    st.y = fma((double)S_e, h, st.y) * E;
    st.Dm = Dp;
    chi_prev = chi_t;
    S_e = S_t;
}

// Half-sweep along ray `ray` from its far end to O for Doppler offset xq of this lane.
template <bool F32>
__device__ HalfState half_sweep(const SolveArgs &a, NodeRec<typename Bulk<F32>::T> *rec, int64_t O,
                                const CellRec &cO, int ray, typename Bulk<F32>::T xq, int slot,
                                int line0, int nlw, double ib)
{
    using T = typename Bulk<F32>::T;
    using T2 = typename Bulk<F32>::T2;
    const T2 *lc = reinterpret_cast<const T2 *>(a.lc);
    const int lane = threadIdx.x;
    HalfState st;
    st.Q = 1.0;
    st.y = ib;
    st.Dm = 0.0;
    const int64_t base = O * a.n_rays + ray;
    const int64_t beg = a.roff[base];
    const int L = (int)(a.roff[base + 1] - beg);
    if (L == 0) return st;
    const double nx = a.dir[3 * ray], ny = a.dir[3 * ray + 1], nz = a.dir[3 * ray + 2];
    T x_cur = 0, k_cur = 0, S_e = 0, chi_prev = 0;
    for (int b0 = 0; b0 < L; b0 += kWave - 1) {
        __syncthreads();
        // ---- stage nodes b0 .. b0+63 in sweep order (far end first, O last)
        const int s = b0 + lane;
        double Zs = 0.0, sv = 0.0, vw = 1.0;
        if (s <= L) {
            int64_t cidx = (s < L) ? (int64_t)a.rcells[beg + (L - 1 - s)] : O;
            const CellRec c = a.cell[cidx];
            double dx = c.px - cO.px, dy = c.py - cO.py, dz = c.pz - cO.pz;
            Zs = (dx * nx + dy * ny) + dz * nz;
            double dvx = c.vx - cO.vx, dvy = c.vy - cO.vy, dvz = c.vz - cO.vz;
            sv = (dvx * nx + dvy * ny) + dvz * nz;
            vw = c.vw;
            NodeRec<T> r;
            r.a = (T)(cO.vw / vw);
            r.b = (T)(sv / vw);
            T2 c0 = lc[cidx * a.n_lines + line0];
            r.kap[0] = c0.x;
            r.S[0] = c0.y;
            if (nlw > 1) {
                T2 c1 = lc[cidx * a.n_lines + line0 + 1];
                r.kap[1] = c1.x;
                r.S[1] = c1.y;
            } else {
                r.kap[1] = 0;
                r.S[1] = 0;
            }
            r.dzh = 0;
            r.m = 1;
            rec[lane] = r;
        }
        const double Zn = __shfl_down(Zs, 1), sn = __shfl_down(sv, 1), vwn = __shfl_down(vw, 1);
        if (s < L && lane < kWave - 1) {
            // velocity sub-steps (Sec. 3.2): split when the projected velocity changes by
            // more than f_sub of the smaller line-width speed
            double ds = fabs(sn - sv);
            double thr = a.f_sub * fmin(vw, vwn);
            int m = 1;
            if (ds > thr) {
                const double mr = ceil(ds / thr);
                m = mr < (double)kMaxSub ? (int)mr : kMaxSub;
            }
            rec[lane].m = m;
            rec[lane].dzh = (T)(0.5 * (Zs - Zn) / (double)m);
        }
        __syncthreads();
        // ---- sweep the staged segments
        const int nseg = min(kWave - 1, L - b0);
        if (b0 == 0) {
            x_cur = rec[0].a * xq - rec[0].b;
            k_cur = rec[0].kap[slot];
            S_e = rec[0].S[slot];
            chi_prev = k_cur * profile(x_cur);
        }
        for (int i = 0; i < nseg; ++i) {
            const int m = rec[i].m;
            const T dzh = rec[i].dzh;
            const T an = rec[i + 1].a, bn = rec[i + 1].b;
            const T kn = rec[i + 1].kap[slot], Sn = rec[i + 1].S[slot];
            const T xn = an * xq - bn;
            if (m > 1) {
                const T inv_m = (T)1 / (T)m;
                const T dx = (xn - x_cur) * inv_m, dk = (kn - k_cur) * inv_m, dS = (Sn - S_e) * inv_m;
                const T S0 = S_e;
                for (int j = 1; j < m; ++j) {
                    const T tj = (T)j;
                    const T xt = x_cur + tj * dx;
                    const T kt = k_cur + tj * dk;
                    const T St = S0 + tj * dS;
                    elim_step<F32>(kt * profile(xt), St, dzh, chi_prev, S_e, st, a.tau_floor);
                }
            }
            elim_step<F32>(kn * profile(xn), Sn, dzh, chi_prev, S_e, st, a.tau_floor);
            x_cur = xn;
            k_cur = kn;
        }
    }
    return st;
}

template <bool F32>
__global__ __launch_bounds__(64) void k_formal_solve(SolveArgs a)
{
    using T = typename Bulk<F32>::T;
    using T2 = typename Bulk<F32>::T2;
    using Acc = typename Bulk<F32>::T;
    __shared__ NodeRec<T> rec[kWave];
    __shared__ double red[3][kWave];
    const int lane = threadIdx.x;
    // Consecutive hardware workgroups go round-robin to the 8 XCDs; give each XCD a
    // contiguous range of origin points so that the cells their rays share stay in
    // that XCD's L2.
    const int64_t nb8 = (a.n_blocks + 7) / 8;
    const int64_t lb = (int64_t)(blockIdx.x & 7) * nb8 + (blockIdx.x >> 3);
    if (lb >= a.n_blocks) return;
    const int64_t O = lb / a.groups;
    const int g = (int)(lb - O * a.groups);

    int slot, nidx0, line, line0, nlw;
    bool active;
    if (a.lines_per_wave > 0) {
        slot = lane / a.n_q;
        nidx0 = lane - slot * a.n_q;
        line0 = g * a.lines_per_wave;
        line = line0 + slot;
        nlw = min(a.lines_per_wave, a.n_lines - line0);
        active = slot < a.lines_per_wave && line < a.n_lines;
    } else {
        slot = 0;
        nidx0 = lane;
        line0 = g;
        line = g;
        nlw = 1;
        active = true;
    }
    if (!active) {
        slot = 0;
        line = line0;
    }
    const T2 *lc = reinterpret_cast<const T2 *>(a.lc);
    const CellRec cO = a.cell[O];
    const double S_O = (double)lc[O * a.n_lines + line].y;
    const double ib = a.ibdy[line];
    Acc accJ = 0, accL = 0, accE = 0;
    for (int p = 0; p < a.n_pairs; ++p) {
        const int r = a.pair_r[p], rb = a.anti[r];
        for (int c = 0; c < a.fchunks; ++c) {
            const int nidx = (a.lines_per_wave > 0) ? nidx0 : c * kWave + lane;
            const bool act = active && nidx < a.n_q;
            const double xq = act ? a.qx[nidx] : 0.0;
            const double wq = act ? a.qw[nidx] : 0.0;
            // u pairs I(n, x) with I(-n, -x): the antipode sweeps at the mirrored offset
            HalfState hf = half_sweep<F32>(a, rec, O, cO, r, (T)xq, slot, line0, nlw, ib);
            HalfState hb = half_sweep<F32>(a, rec, O, cO, rb, (T)(-xq), slot, line0, nlw, ib);
            const double h = 0.5 * (hf.Dm + hb.Dm);
            const double inv = 1.0 / (h + hf.Q + hb.Q);
            const double yy = hf.y + hb.y;
            accJ += (Acc)(wq * (fma(h, S_O, yy) * inv));
            accL += (Acc)(wq * (h * inv));
            accE += (Acc)(wq * (yy * inv));
        }
    }
    red[0][lane] = (double)accJ;
    red[1][lane] = (double)accL;
    red[2][lane] = (double)accE;
    __syncthreads();
    if (a.lines_per_wave > 0) {
        if (lane < nlw) {
            Acc sJ = 0, sL = 0, sE = 0;
            for (int i = lane * a.n_q; i < (lane + 1) * a.n_q; ++i) {
                sJ += (Acc)red[0][i];
                sL += (Acc)red[1][i];
                sE += (Acc)red[2][i];
            }
            const int64_t o = O * a.n_lines + line0 + lane;
            a.J[o] = a.norm * (double)sJ;
            a.L[o] = a.norm * (double)sL;
            a.Jeff[o] = a.norm * (double)sE;
        }
    } else if (lane == 0) {
        Acc sJ = 0, sL = 0, sE = 0;
        for (int i = 0; i < kWave; ++i) {
            sJ += (Acc)red[0][i];
            sL += (Acc)red[1][i];
            sE += (Acc)red[2][i];
        }
        const int64_t o = O * a.n_lines + g;
        a.J[o] = a.norm * (double)sJ;
        a.L[o] = a.norm * (double)sL;
        a.Jeff[o] = a.norm * (double)sE;
    }
}

hipError_t launch_formal_solve(const SolveArgs &a, int fp32, hipStream_t s)
{
    if (a.n_blocks == 0) return hipSuccess;
    const int64_t nb8 = (a.n_blocks + 7) / 8;
    dim3 grid((unsigned)(nb8 * 8));
    if (fp32)
        hipLaunchKernelGGL(k_formal_solve<true>, grid, dim3(kWave), 0, s, a);
    else
        hipLaunchKernelGGL(k_formal_solve<false>, grid, dim3(kWave), 0, s, a);
    return hipGetLastError();
}

// Elimination steps per frequency over all half rays: the cells of every cached walk
// plus their velocity sub-steps, with the same sub-step rule as the sweep.  One thread
// per (point, ray); block sums are added atomically (integer, order-independent).
__global__ __launch_bounds__(256) void k_count_steps(SolveArgs a, unsigned long long *steps)
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
    }
    part[threadIdx.x] = n;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if (threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicAdd(steps, part[0]);
}

hipError_t launch_count_steps(const SolveArgs &a, int64_t *steps, hipStream_t s)
{
    const int64_t n = a.P * a.n_rays;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_count_steps, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, a,
                       reinterpret_cast<unsigned long long *>(steps));
    return hipGetLastError();
}

}  // namespace nlte
