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
// fractions N/D and Y/D, which turns each step into three multiply-adds of non-negative
// numbers with no division (see elim_step).  At O the two halves combine into
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
// x_q at this node as x = a x_q - b.  The segment to the next node toward O has m
// sub-intervals of half-length dzh; per sub-interval x changes by da x_q - db and kappa,
// S by dk, dS (per staged line); K is the restart interval of the profile recurrence.
template <typename T>
struct NodeRec {
    T a, b, dzh, da, db;
    T kap[2], S[2], dk[2], dS[2];
    int m, K;
};

// Elimination state of a half sweep in homogeneous form: the Rybicki-Hummer quantities
// Q = N / D and y = Y / D (see the file comment), and the previous optical-depth step.
struct HalfState {
    double N, D, Y, Dm;
};

// e^y for y <= 700 in FP64: y = n ln2 + r with |r| <= ln2/2 (two-part ln2), e^r by its
// degree-11 Taylor polynomial (truncation < 7e-15 relative), scaled by 2^n.  Results
// below the FP64 range come out as 0 through ldexp; no other special cases arise for
// the arguments used here (finite, at most 700).
__device__ __forceinline__ double exp_le700(double y)
{
    const double n = rint(y * 1.44269504088896338700);
    double r = fma(-n, 6.93147180369123816490e-01, y);
    r = fma(-n, 1.90821492927058770002e-10, r);
    double p = 2.50521083854417187751e-08;           // 1/11!
    p = fma(p, r, 2.75573192239858906526e-07);       // 1/10!
    p = fma(p, r, 2.75573192239858906526e-06);       // 1/9!
    p = fma(p, r, 2.48015873015873015873e-05);       // 1/8!
    p = fma(p, r, 1.98412698412698412698e-04);       // 1/7!
    p = fma(p, r, 1.38888888888888888889e-03);       // 1/6!
    p = fma(p, r, 8.33333333333333333333e-03);       // 1/5!
    p = fma(p, r, 4.16666666666666666667e-02);       // 1/4!
    p = fma(p, r, 1.66666666666666666667e-01);       // 1/3!
    p = fma(p, r, 0.5);
    p = fma(p, r, 1.0);
    p = fma(p, r, 1.0);
    const int ni = (int)fmax(n, -2200.0);
    return ldexp(p, ni);
}

__device__ __forceinline__ double profile(double x) { return exp_le700(-(x * x)); }
__device__ __forceinline__ float profile(float x)
{
    // e^{-x^2} = 2^{-x^2 log2 e} on the hardware exp2
    return __builtin_amdgcn_exp2f(-(x * x) * 1.44269504088896340736f);
}

// One elimination step: node with source S_e (between optical-depth steps Dm and Dp) is
// eliminated.  With h = (Dm + Dp)/2 the Rybicki-Hummer update
//   T = h + Q, E = 1/(1 + Dp T), Q' = T E, y' = (S h + y) E
// becomes, for Q = N/D and y = Y/D,
//   N' = N + h D,  Y' = Y + S h D,  D' = D + Dp N'
// (only products and sums of non-negative numbers).  RENORM rescales N, D, Y by the
// power of two that brings D into [0.5, 1), which is exact.
template <bool F32, bool RENORM>
__device__ __forceinline__ void elim_step(typename Bulk<F32>::T chi_t, typename Bulk<F32>::T S_t,
                                          typename Bulk<F32>::T dzh, typename Bulk<F32>::T &chi_prev,
                                          typename Bulk<F32>::T &S_e, HalfState &st)
{
    // trapezoid optical depth of the step; zero is allowed (nothing divides by it)
    const double Dp = (double)((chi_prev + chi_t) * dzh);
    const double hD = (0.5 * (st.Dm + Dp)) * st.D;
    st.N = st.N + hD;
    st.Y = fma((double)S_e, hD, st.Y);
    st.D = fma(Dp, st.N, st.D);
    st.Dm = Dp;
    chi_prev = chi_t;
    S_e = S_t;
    if (RENORM) {
        const int e = __builtin_amdgcn_frexp_exp(st.D);
        st.N = ldexp(st.N, -e);
        st.D = ldexp(st.D, -e);
        st.Y = ldexp(st.Y, -e);
    }
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
    st.N = 1.0;
    st.D = 1.0;
    st.Y = ib;
    st.Dm = 0.0;
    const int64_t base = O * a.n_rays + ray;
    const int64_t beg = a.roff[base];
    const int L = (int)(a.roff[base + 1] - beg);
    if (L == 0) return st;
    const double nx = a.dir[3 * ray], ny = a.dir[3 * ray + 1], nz = a.dir[3 * ray + 2];
    T x_cur = 0, k_cur = 0, S_e = 0, chi_prev = 0, g_cur = 0;
    for (int b0 = 0; b0 < L; b0 += kWave - 1) {
        __syncthreads();
        // ---- stage nodes b0 .. b0+63 in sweep order (far end first, O last)
        const int s = b0 + lane;
        double Zs = 0.0, sv = 0.0, vw = 1.0, an = 0.0, bn = 0.0;
        T k0 = 0, S0 = 0, k1 = 0, S1 = 0;
        if (s <= L) {
            int64_t cidx = (s < L) ? (int64_t)a.rcells[beg + (L - 1 - s)] : O;
            const CellRec c = a.cell[cidx];
            double dx = c.px - cO.px, dy = c.py - cO.py, dz = c.pz - cO.pz;
            Zs = (dx * nx + dy * ny) + dz * nz;
            double dvx = c.vx - cO.vx, dvy = c.vy - cO.vy, dvz = c.vz - cO.vz;
            sv = (dvx * nx + dvy * ny) + dvz * nz;
            vw = c.vw;
            an = cO.vw / vw;
            bn = sv / vw;
            T2 c0 = lc[cidx * a.n_lines + line0];
            k0 = c0.x;
            S0 = c0.y;
            if (nlw > 1) {
                T2 c1 = lc[cidx * a.n_lines + line0 + 1];
                k1 = c1.x;
                S1 = c1.y;
            }
        }
        const double Zn = __shfl_down(Zs, 1), sn = __shfl_down(sv, 1), vwn = __shfl_down(vw, 1);
        const double an1 = __shfl_down(an, 1), bn1 = __shfl_down(bn, 1);
        const T k0n = __shfl_down(k0, 1), S0n = __shfl_down(S0, 1);
        const T k1n = __shfl_down(k1, 1), S1n = __shfl_down(S1, 1);
        if (s <= L) {
            NodeRec<T> r;
            r.a = (T)an;
            r.b = (T)bn;
            r.kap[0] = k0;
            r.S[0] = S0;
            r.kap[1] = k1;
            r.S[1] = S1;
            r.m = 1;
            r.K = 64;
            r.dzh = 0;
            r.da = r.db = 0;
            r.dk[0] = r.dk[1] = r.dS[0] = r.dS[1] = 0;
            if (s < L && lane < kWave - 1) {
                // velocity sub-steps (Sec. 3.2): split when the projected velocity changes
                // by more than f_sub of the smaller line-width speed
                const double ds = fabs(sn - sv);
                const double thr = a.f_sub * fmin(vw, vwn);
                int m = 1;
                if (ds > thr) {
                    const double mr = ceil(ds / thr);
                    m = mr < (double)kMaxSub ? (int)mr : kMaxSub;
                }
                const double im = 1.0 / (double)m;
                r.m = m;
                r.dzh = (T)(0.5 * (Zs - Zn) * im);
                r.da = (T)((an1 - an) * im);
                r.db = (T)((bn1 - bn) * im);
                r.dk[0] = (T)((k0n - k0) * (T)im);
                r.dS[0] = (T)((S0n - S0) * (T)im);
                r.dk[1] = (T)((k1n - k1) * (T)im);
                r.dS[1] = (T)((S1n - S1) * (T)im);
                // bound on |dx| over every frequency of the quadrature; the recurrence of
                // the profile restarts after at most 16 widths of travel in x
                const double maxdx = (fabs(an1 - an) * a.xq_max + fabs(bn1 - bn)) * im;
                r.K = maxdx > 4.0 ? 0 : (maxdx > 0.25 ? (int)(16.0 / maxdx) : 64);
            }
            rec[lane] = r;
        }
        __syncthreads();
        // ---- sweep the staged segments
        const int nseg = min(kWave - 1, L - b0);
        if (b0 == 0) {
            x_cur = rec[0].a * xq - rec[0].b;
            k_cur = rec[0].kap[slot];
            S_e = rec[0].S[slot];
            g_cur = profile(x_cur);
            chi_prev = k_cur * g_cur;
        }
        for (int i = 0; i < nseg; ++i) {
            const int m = rec[i].m;
            const T dzh = rec[i].dzh;
            const T xn = rec[i + 1].a * xq - rec[i + 1].b;
            const T kn = rec[i + 1].kap[slot], Sn = rec[i + 1].S[slot];
            T gn;
            if (m == 1) {
                gn = profile(xn);
            } else {
                const T dx = rec[i].da * xq - rec[i].db;
                const T dk = rec[i].dk[slot], dS = rec[i].dS[slot];
                const int K = rec[i].K;
                if (F32 || K == 0) {
                    const T S0 = S_e;
                    for (int j = 1; j < m; ++j) {
                        const T tj = (T)j;
                        elim_step<F32, true>((k_cur + tj * dk) * profile(x_cur + tj * dx), S0 + tj * dS, dzh,
                                             chi_prev, S_e, st);
                    }
                } else {
                    // x is linear in the sub-step index j, so g_j = e^{-x_j^2} obeys
                    // g_{j+1} = g_j r_j, r_{j+1} = r_j c with r_j = e^{-2 x_j dx - dx^2} and
                    // c = e^{-2 dx^2}.  It starts from the exact value at the segment's
                    // first node and restarts from exact values every K sub-steps, K such
                    // that x moves by at most 16 widths in between: a value that
                    // underflowed (|x| > 27) cannot hide a profile above e^{-121}.
                    const double c = exp_le700(-2.0 * dx * dx);
                    double g = g_cur, r = exp_le700(fmin(-(2.0 * x_cur + dx) * dx, 700.0));
                    double kt = k_cur, St = S_e;
                    const double kc = k_cur, Sc = S_e;
                    for (int j0 = 0; j0 < m - 1; j0 += K) {
                        if (j0 > 0) {
                            const double xj = fma((double)j0, dx, x_cur);
                            g = exp_le700(-(xj * xj));
                            r = exp_le700(fmin(-(2.0 * xj + dx) * dx, 700.0));
                            kt = fma((double)j0, dk, kc);
                            St = fma((double)j0, dS, Sc);
                        }
                        const int j1 = min(j0 + K, m - 1);
                        int j = j0;
                        // groups of four steps, renormalised once: D grows by at most
                        // (1 + F)^4 in between, far from overflow for any optical-depth
                        // step below ~1e37
                        for (; j + 3 < j1; j += 4) {
#pragma unroll
                            for (int u = 0; u < 3; ++u) {
                                g *= r;
                                r *= c;
                                kt += dk;
                                St += dS;
                                elim_step<F32, false>(kt * g, St, dzh, chi_prev, S_e, st);
                            }
                            g *= r;
                            r *= c;
                            kt += dk;
                            St += dS;
                            elim_step<F32, true>(kt * g, St, dzh, chi_prev, S_e, st);
                        }
                        for (; j < j1; ++j) {
                            g *= r;
                            r *= c;
                            kt += dk;
                            St += dS;
                            elim_step<F32, true>(kt * g, St, dzh, chi_prev, S_e, st);
                        }
                    }
                }
                // the cell at the end of the segment gets its exact profile, so every
                // segment's recurrence starts from an exact value
                gn = profile(xn);
            }
            elim_step<F32, true>(kn * gn, Sn, dzh, chi_prev, S_e, st);
            x_cur = xn;
            k_cur = kn;
            g_cur = gn;
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
            const double idf = 1.0 / hf.D, idb = 1.0 / hb.D;
            const double h = 0.5 * (hf.Dm + hb.Dm);
            const double inv = 1.0 / (h + fma(hf.N, idf, hb.N * idb));
            const double yy = fma(hf.Y, idf, hb.Y * idb);
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
