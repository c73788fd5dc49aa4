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
// Mapping: one workgroup = one wave = one origin point and up to 64 (line, frequency)
// items; all lanes walk the same nodes (uniform control flow), each with its own
// frequency.  The wave stages up to 64 cells of a ray at a time in LDS (position,
// velocity projection, Doppler coefficients, sub-step count, kappa and S of its lines);
// the sweep then reads them as broadcasts.  Velocity sub-steps interpolate the Doppler
// offset x, kappa and S linearly between cells in registers.
#include "nlte_internal.h"
#include "device_math.h"

namespace nlte {

constexpr double kSqrt2 = 1.41421356237309504880;
constexpr double kInv2Sqrt2 = 0.35355339059327376220;  // 1 / (2 sqrt 2)

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

// A wave serves one origin point, one frequency per lane and NLW = 2 LPL lines: lanes
// [0, n_q) handle lines line0 .. line0+LPL-1 ("group" 0), lanes [n_q, 2 n_q) the next LPL
// lines (group 1).  The Doppler offset of a node depends on the frequency only (the line
// width is proportional to the line frequency), so the profile and its recurrence are
// shared by the LPL lines of a lane; only kappa, S and the elimination state are per line.

// One staged node of a half ray.  (a, b) give the Doppler offset of a lane's frequency
// x_q at this node as x = a x_q - b.  The segment to the next node toward O has m
// sub-intervals of length 2 sqrt(2) dzq; per sub-interval x changes by da x_q - db.  maxdx bounds
// |dx| over all frequencies, K is the restart interval of the profile recurrence (0:
// evaluate every profile directly).  kap, S: line-centre opacity and source function of
// the wave's lines.
template <typename T, int NLW>
struct NodeRec {
    T a, b, dzq, da, db, inv_m, maxdx;
    int m, K;
    T kap[NLW], S[NLW];
};

// Elimination state of a half sweep in homogeneous form: the Rybicki-Hummer quantities
// Q = N / (sqrt 2 D) and y = Y / (sqrt 2 D), and Hm = D_- / sqrt 2, the previous
// optical-depth step (see elim_step).
struct HalfState {
    double N, D, Y, Hm;
    double hd;   // weight h d of the last step (renormalised with the state): the share of the
    double Sl;   // last eliminated node's source Sl in Y (read by the band operator only)
};

__device__ __forceinline__ double profile(double x) { return exp_le700(-(x * x)); }
__device__ __forceinline__ float profile(float x)
{
    // e^{-x^2} = 2^{-x^2 log2 e} on the hardware exp2
    return __builtin_amdgcn_exp2f(-(x * x) * 1.44269504088896340736f);
}

// e^{-x^2} at a node of a wave's sweep (uniform control flow).  Beyond x^2 = 746 the FP64
// value above is exactly 0, so where every lane of the wave is that far in the wing the
// exponential is skipped without changing any result.  (The FP32 exponential is cheaper
// than the vote and branch, measured.)
__device__ __forceinline__ double profile_far(double x) { return __all(x * x > 746.0) ? 0.0 : profile(x); }
__device__ __forceinline__ float profile_far(float x) { return profile(x); }

// One elimination step.  The Rybicki-Hummer update with h = (D_- + D_+)/2 (mean of the
// trapezoid optical depths D_-, D_+ on either side of the node)
//   T = h + Q,  E = 1/(1 + D_+ T),  Q' = T E,  y' = (S h + y) E
// becomes, for Q = N/D and y = Y/D,
//   N' = N + h D,  Y' = Y + S h D,  D' = D + D_+ N'
// (products and sums of non-negative numbers only).  The node coefficients a are
// chi dz / (2 sqrt 2), so P = a_prev + a_t = D_+ / sqrt 2, and the state is carried as
// n = sqrt 2 N, y~ = sqrt 2 Y, d = D, which turns the update into
//   n' = n + (P_- + P) d,  y~' = y~ + S (P_- + P) d,  d' = d + P n'
// with no constant factors; Q = n/(sqrt 2 d), y = y~/(sqrt 2 d), and the factor sqrt 2
// cancels in every quantity formed at the origin.  RENORM rescales n, d, y~ by the power
// of two that brings d into [0.5, 1), which is exact.
template <bool F32, bool RENORM, bool TRACK = false>
__device__ __forceinline__ void elim_step(typename Bulk<F32>::T a_t, typename Bulk<F32>::T S_t,
                                          typename Bulk<F32>::T &a_prev, typename Bulk<F32>::T &S_e,
                                          HalfState &st)
{
    const double Pp = (double)(a_prev + a_t);
    const double hd = (st.Hm + Pp) * st.D;
    st.N = st.N + hd;
    st.Y = fma((double)S_e, hd, st.Y);
    st.D = fma(Pp, st.N, st.D);
    st.Hm = Pp;
    if (TRACK) {
        st.hd = hd;
        st.Sl = (double)S_e;
    }
    a_prev = a_t;
    S_e = S_t;
    if (RENORM) {
        const int e = __builtin_amdgcn_frexp_exp(st.D);
        st.N = ldexp(st.N, -e);
        st.D = ldexp(st.D, -e);
        st.Y = ldexp(st.Y, -e);
        if (TRACK) st.hd = ldexp(st.hd, -e);
    }
}

// Per-line state of a lane during a half sweep.
template <typename T, int LPL>
struct LineState {
    HalfState st[LPL];
    T k_cur[LPL], S_e[LPL], chi_cur[LPL];
    int m_last;   // sub-intervals of the last segment (the one ending at O)
};

// One recurrence step of all LPL lines: g <- g r, r <- r c (shared), then the linear
// kappa dz/4 and S of each line and its elimination step.
template <bool F32, int LPL, bool RENORM, bool TRACK = false>
__device__ __forceinline__ void recur_step(double &g, double &r, double c, double (&kq)[LPL],
                                           const double (&dkq)[LPL], double (&St)[LPL],
                                           const double (&dS)[LPL], typename Bulk<F32>::T (&a_prev)[LPL],
                                           LineState<typename Bulk<F32>::T, LPL> &ls)
{
    g *= r;
    r *= c;
#pragma unroll
    for (int l = 0; l < LPL; ++l) {
        kq[l] += dkq[l];
        St[l] += dS[l];
        elim_step<F32, RENORM, TRACK>(kq[l] * g, St[l], a_prev[l], ls.S_e[l], ls.st[l]);
    }
}

// Half-sweep along ray `ray` from its far end to O for Doppler offset xq of this lane.
// The result is left in ls.st (one HalfState per line of the lane).
// nexec counts the elimination steps the wave executes (a collapsed far-wing segment
// counts as one).
template <bool F32, int LPL, bool TRACK = false>
__device__ void half_sweep(const SolveArgs &a, NodeRec<typename Bulk<F32>::T, 2 * LPL> *rec, int64_t O,
                           const CellRec &cO, int ray, typename Bulk<F32>::T xq, int grp, int line0,
                           int nlw, const double (&ib)[LPL], LineState<typename Bulk<F32>::T, LPL> &ls,
                           int64_t &nexec)
{
    using T = typename Bulk<F32>::T;
    using T2 = typename Bulk<F32>::T2;
    constexpr int NLW = 2 * LPL;
    const T2 *lc = reinterpret_cast<const T2 *>(a.lc);
    const int lane = threadIdx.x;
#pragma unroll
    for (int l = 0; l < LPL; ++l) {
        // Q = 1, y = I_in at the far boundary (in the scaled state of elim_step)
        ls.st[l].N = kSqrt2;
        ls.st[l].D = 1.0;
        ls.st[l].Y = kSqrt2 * ib[l];
        ls.st[l].Hm = 0.0;
        if (TRACK) {
            ls.st[l].hd = 0.0;
            ls.st[l].Sl = 0.0;
        }
    }
    if (TRACK) ls.m_last = 1;
    const int64_t base = O * a.n_rays + ray;
    const int64_t beg = a.roff[base];
    const int L = (int)(a.roff[base + 1] - beg);
    if (L == 0) return;
    const double nx = a.dir[3 * ray], ny = a.dir[3 * ray + 1], nz = a.dir[3 * ray + 2];
    // x_cur, g_cur: Doppler offset and profile at the current node; travel bounds how far
    // x moved (any lane) since g was last evaluated exactly
    T x_cur = 0, g_cur = 0;
    double travel = 0.0;
    for (int b0 = 0; b0 < L; b0 += kWave - 1) {
        __syncthreads();
        // ---- stage nodes b0 .. b0+63 in sweep order (far end first, O last)
        const int s = b0 + lane;
        double Zs = 0.0, sv = 0.0, vw = 1.0, an = 0.0, bn = 0.0;
        int64_t cidx = O;
        if (s <= L) {
            cidx = (s < L) ? (int64_t)a.rcells[beg + (L - 1 - s)] : O;
            const CellRec c = a.cell[cidx];
            double dx = c.px - cO.px, dy = c.py - cO.py, dz = c.pz - cO.pz;
            Zs = (dx * nx + dy * ny) + dz * nz;
            double dvx = c.vx - cO.vx, dvy = c.vy - cO.vy, dvz = c.vz - cO.vz;
            sv = (dvx * nx + dvy * ny) + dvz * nz;
            vw = c.vw;
            an = cO.vw / vw;
            bn = sv / vw;
        }
        const double Zn = __shfl_down(Zs, 1), sn = __shfl_down(sv, 1), vwn = __shfl_down(vw, 1);
        const double an1 = __shfl_down(an, 1), bn1 = __shfl_down(bn, 1);
        if (s <= L) {
            NodeRec<T, NLW> r;
            r.a = (T)an;
            r.b = (T)bn;
#pragma unroll
            for (int l = 0; l < NLW; ++l) {
                T2 cl = l < nlw ? lc[cidx * a.n_lines + line0 + l] : T2{0, 0};
                r.kap[l] = cl.x;
                r.S[l] = cl.y;
            }
            r.m = 1;
            r.K = 64;
            r.dzq = 0;
            r.da = r.db = r.maxdx = 0;
            r.inv_m = 1;
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
                r.inv_m = (T)im;
                r.dzq = (T)(kInv2Sqrt2 * (Zs - Zn) * im);
                r.da = (T)((an1 - an) * im);
                r.db = (T)((bn1 - bn) * im);
                // bound on |dx| over every frequency of the quadrature; the recurrence of
                // the profile restarts after at most 16 widths of travel in x
                const double maxdx = (fabs(an1 - an) * a.xq_max + fabs(bn1 - bn)) * im;
                r.maxdx = (T)maxdx;
                r.K = maxdx > 4.0 ? 0 : (maxdx > 0.25 ? (int)(16.0 / maxdx) : 64);
            }
            rec[lane] = r;
        }
        __syncthreads();
        // ---- sweep the staged segments
        const int nseg = min(kWave - 1, L - b0);
        if (b0 == 0) {
            x_cur = rec[0].a * xq - rec[0].b;
            g_cur = profile(x_cur);
#pragma unroll
            for (int l = 0; l < LPL; ++l) {
                ls.k_cur[l] = rec[0].kap[grp * LPL + l];
                ls.S_e[l] = rec[0].S[grp * LPL + l];
                ls.chi_cur[l] = ls.k_cur[l] * g_cur;
            }
        }
        for (int i = 0; i < nseg; ++i) {
            const int m = rec[i].m;
            const T dzq = rec[i].dzq;
            const T xn = rec[i + 1].a * xq - rec[i + 1].b;
            T kn[LPL], Sn[LPL], a_prev[LPL];
#pragma unroll
            for (int l = 0; l < LPL; ++l) {
                kn[l] = rec[i + 1].kap[grp * LPL + l];
                Sn[l] = rec[i + 1].S[grp * LPL + l];
                a_prev[l] = ls.chi_cur[l] * dzq;
            }
            if (!TRACK && m > 1) {
                // Far wing: every lane beyond the range of its profile (exactly 0 past
                // x^2 = 750 in FP64, 105 in FP32) at both ends of the segment, on one side
                // of the line centre, and zero opacity at its first node.  Then every node of
                // the segment has zero opacity, the elimination steps after the first change
                // nothing, and one step with zero opacity and the end node's source leaves
                // the same state.  (A segment without sub-steps is one step anyway.)
                const T far2 = F32 ? (T)105 : (T)750;
                bool far = ((x_cur > (T)0) == (xn > (T)0)) && x_cur * x_cur > far2 && xn * xn > far2;
#pragma unroll
                for (int l = 0; l < LPL; ++l) far = far && ls.chi_cur[l] == (T)0;
                if (__all(far)) {
#pragma unroll
                    for (int l = 0; l < LPL; ++l) {
                        elim_step<F32, true, TRACK>((T)0, Sn[l], a_prev[l], ls.S_e[l], ls.st[l]);
                        ls.k_cur[l] = kn[l];
                        ls.chi_cur[l] = (T)0;
                    }
                    x_cur = xn;
                    g_cur = (T)0;
                    travel = 0.0;
                    ++nexec;
                    continue;
                }
            }
            nexec += m;
            T gn;
            if (m == 1) {
                gn = profile_far(xn);
                travel = 0.0;
            } else {
                const T im = rec[i].inv_m;
                const T dx = rec[i].da * xq - rec[i].db;
                const int K = rec[i].K;
                // direct evaluation where the recurrence would not pay for its two
                // exponentials (one sub-step node) or cannot be used (K == 0)
                if (F32 || K == 0 || m == 2) {
                    T S0[LPL], dk[LPL], dS[LPL];
#pragma unroll
                    for (int l = 0; l < LPL; ++l) {
                        S0[l] = ls.S_e[l];
                        dk[l] = (kn[l] - ls.k_cur[l]) * im;
                        dS[l] = (Sn[l] - S0[l]) * im;
                    }
                    for (int j = 1; j < m; ++j) {
                        const T tj = (T)j;
                        const T gq = profile_far(x_cur + tj * dx) * dzq;
#pragma unroll
                        for (int l = 0; l < LPL; ++l)
                            elim_step<F32, true, TRACK>((ls.k_cur[l] + tj * dk[l]) * gq, S0[l] + tj * dS[l], a_prev[l],
                                                 ls.S_e[l], ls.st[l]);
                    }
                    gn = profile_far(xn);
                    travel = 0.0;
                } else {
                    // x is linear in the sub-step index j, so g_j = e^{-x_j^2} obeys
                    // g_{j+1} = g_j r_j, r_{j+1} = r_j c with r_j = e^{-2 x_j dx - dx^2} and
                    // c = e^{-2 dx^2}.  Values are recomputed exactly whenever x may have
                    // moved by more than 16 widths since the last exact value, so one that
                    // underflowed (|x| > 27) cannot hide a profile above e^{-121}.
                    const double mdx = (double)rec[i].maxdx;
                    const double u2 = 2.0 * dx * dx;
                    const double c = mdx <= 0.5 ? exp_neg_small(u2) : exp_le700(-u2);
                    double kq0[LPL], dkq[LPL], Sc[LPL], dS[LPL], kq[LPL], St[LPL];
#pragma unroll
                    for (int l = 0; l < LPL; ++l) {
                        kq0[l] = (double)(ls.k_cur[l] * dzq);
                        dkq[l] = (double)((kn[l] - ls.k_cur[l]) * im * dzq);
                        Sc[l] = (double)ls.S_e[l];
                        dS[l] = (double)((Sn[l] - ls.S_e[l]) * im);
                        kq[l] = kq0[l];
                        St[l] = Sc[l];
                    }
                    double g = g_cur, r = exp_le700(fmin(-(2.0 * x_cur + dx) * dx, 700.0));
                    int budget = K;
                    if (mdx > 0.0) budget = (int)fminf((16.0f - (float)travel) * __builtin_amdgcn_rcpf((float)mdx),
                                                       (float)K);
                    if (budget < 1) {
                        g = profile((double)x_cur);
                        travel = 0.0;
                        budget = K;
                    }
                    int j = 0;
                    for (;;) {
                        const int jend = min(j + budget, m);
                        const int jint = min(jend, m - 1);
                        int jj = j;
                        for (; jj + 3 < jint; jj += 4) {
                            recur_step<F32, LPL, false, TRACK>(g, r, c, kq, dkq, St, dS, a_prev, ls);
                            recur_step<F32, LPL, false, TRACK>(g, r, c, kq, dkq, St, dS, a_prev, ls);
                            recur_step<F32, LPL, false, TRACK>(g, r, c, kq, dkq, St, dS, a_prev, ls);
                            recur_step<F32, LPL, true, TRACK>(g, r, c, kq, dkq, St, dS, a_prev, ls);
                        }
                        // the last 0-3 steps in straight-line code; the elimination step
                        // that follows renormalises, so at most seven steps pass between
                        // renormalisations
                        const int rem = jint - jj;
                        if (rem >= 2) {
                            recur_step<F32, LPL, false, TRACK>(g, r, c, kq, dkq, St, dS, a_prev, ls);
                            recur_step<F32, LPL, false, TRACK>(g, r, c, kq, dkq, St, dS, a_prev, ls);
                        }
                        if (rem & 1) recur_step<F32, LPL, false, TRACK>(g, r, c, kq, dkq, St, dS, a_prev, ls);
                        travel += mdx * (double)(jint - j);
                        j = jint;
                        if (jend == m) {
                            g *= r;          // the cell at the end of the segment
                            travel += mdx;
                            break;
                        }
                        const double xj = fma((double)j, dx, (double)x_cur);
                        g = exp_le700(-(xj * xj));
                        r = exp_le700(fmin(-(2.0 * xj + dx) * dx, 700.0));
#pragma unroll
                        for (int l = 0; l < LPL; ++l) {
                            kq[l] = fma((double)j, dkq[l], kq0[l]);
                            St[l] = fma((double)j, dS[l], Sc[l]);
                        }
                        travel = 0.0;
                        budget = K;
                    }
                    gn = g;
                }
            }
#pragma unroll
            for (int l = 0; l < LPL; ++l) {
                const T chi_n = kn[l] * gn;
                elim_step<F32, true, TRACK>(chi_n * dzq, Sn[l], a_prev[l], ls.S_e[l], ls.st[l]);
                ls.k_cur[l] = kn[l];
                ls.chi_cur[l] = chi_n;
            }
            x_cur = xn;
            g_cur = gn;
            if (TRACK) ls.m_last = m;
        }
    }
}

// All (line, frequency) work of one wave for origin point O and line block w, accumulated
// over every ray pair and written to J, L*, Jeff.  Points of models that already
// converged are skipped (their outputs are not needed).
template <bool F32, int LPL, bool BAND = false>
__device__ __forceinline__ void solve_item(const SolveArgs &a, int64_t O, int w,
                                           NodeRec<typename Bulk<F32>::T, 2 * LPL> *rec,
                                           double (*red)[LPL][kWave])
{
    using T = typename Bulk<F32>::T;
    using T2 = typename Bulk<F32>::T2;
    using Acc = typename Bulk<F32>::T;
    const int lane = threadIdx.x;
    if (a.model_done != nullptr && a.model_done[a.model_of[O]]) return;
    // lane -> (group, frequency); a wave owns lines line0 .. line0 + nlw - 1
    const int ngrp = a.lines_per_wave / LPL;     // 1 or 2 groups of lanes
    const int line0 = w * a.lines_per_wave;
    const int nlw = min(a.lines_per_wave, a.n_lines - line0);
    int grp, nidx0;
    if (a.fchunks == 1) {
        grp = lane / a.n_q;
        nidx0 = lane - grp * a.n_q;
    } else {
        grp = 0;
        nidx0 = lane;
    }
    const bool lane_ok = grp < ngrp;
    if (!lane_ok) grp = 0;
    const T2 *lc = reinterpret_cast<const T2 *>(a.lc);
    const CellRec cO = a.cell[O];
    double S_O[LPL], ib[LPL];
    bool lact[LPL];
#pragma unroll
    for (int l = 0; l < LPL; ++l) {
        const int li = grp * LPL + l;
        lact[l] = lane_ok && li < nlw;
        const int line = line0 + (li < nlw ? li : 0);
        S_O[l] = (double)lc[O * a.n_lines + line].y;
        ib[l] = a.ibdy[line];
    }
    Acc accJ[LPL], accL[LPL], accE[LPL];
    double accB[LPL], accD[LPL];   // band operator (BAND only): Jb and Ld
#pragma unroll
    for (int l = 0; l < LPL; ++l) {
        accJ[l] = accL[l] = accE[l] = 0;
        accB[l] = accD[l] = 0.0;
    }
    LineState<T, LPL> ls;
    unsigned long long my_exec = 0;   // executed node-frequency steps of this lane
    for (int p = 0; p < a.n_pairs; ++p) {
        const int r = a.pair_r[p], rb = a.anti[r];
        for (int c = 0; c < a.fchunks; ++c) {
            const int nidx = (a.fchunks == 1) ? nidx0 : c * kWave + lane;
            const bool act = lane_ok && nidx < a.n_q;
            const double xq = act ? a.qx[nidx] : 0.0;
            const double wq = act ? a.qw[nidx] : 0.0;
            // u pairs I(n, x) with I(-n, -x): the antipode sweeps at the mirrored offset
            int64_t nex = 0;
            half_sweep<F32, LPL, BAND>(a, rec, O, cO, r, (T)xq, grp, line0, nlw, ib, ls, nex);
            double Qf[LPL], yf[LPL], Hf[LPL], hdf[LPL], Sf[LPL];
            const int mf = BAND ? ls.m_last : 1;
#pragma unroll
            for (int l = 0; l < LPL; ++l) {
                const double id = 1.0 / ls.st[l].D;
                Qf[l] = ls.st[l].N * id;
                yf[l] = ls.st[l].Y * id;
                Hf[l] = ls.st[l].Hm;
                hdf[l] = ls.st[l].hd * id;
                Sf[l] = ls.st[l].Sl;
            }
            half_sweep<F32, LPL, BAND>(a, rec, O, cO, rb, (T)(-xq), grp, line0, nlw, ib, ls, nex);
            if (a.exec_steps != nullptr) {
                int nact = 0;
#pragma unroll
                for (int l = 0; l < LPL; ++l) nact += (lact[l] && act) ? 1 : 0;
                my_exec += (unsigned long long)nex * (unsigned long long)nact;
            }
            double nbf[LPL], nbb[LPL];
#pragma unroll
            for (int l = 0; l < LPL; ++l) {
                const double id = 1.0 / ls.st[l].D;
                const double h = Hf[l] + ls.st[l].Hm;
                const double inv = 1.0 / (h + fma(ls.st[l].N, id, Qf[l]));
                const double yy = fma(ls.st[l].Y, id, yf[l]);
                accJ[l] += (Acc)(wq * (fma(h, S_O[l], yy) * inv));
                accL[l] += (Acc)(wq * (h * inv));
                accE[l] += (Acc)(wq * (yy * inv));
                if (BAND) {
                    // (T^-1)_{O, neighbour} on either side: the neighbour's share of y
                    // over the combine's denominator; a neighbour at fraction 1/m of the
                    // segment toward the first cell interpolates O's own source by 1 - 1/m
                    const double tf = hdf[l] * inv, tb = ls.st[l].hd * id * inv;
                    const double imf = 1.0 / (double)mf, imb = 1.0 / (double)ls.m_last;
                    accB[l] += wq * (yy * inv - tf * Sf[l] - tb * ls.st[l].Sl);
                    accD[l] += wq * (h * inv + (1.0 - imf) * tf + (1.0 - imb) * tb);
                    nbf[l] = wq * tf * imf;
                    nbb[l] = wq * tb * imb;
                }
            }
            if (BAND) {
                // couplings to the first cells along r and rb, summed over this wave's
                // frequencies in a fixed order
#pragma unroll
                for (int l = 0; l < LPL; ++l) {
                    red[0][l][lane] = lact[l] && act ? nbf[l] : 0.0;
                    red[1][l][lane] = lact[l] && act ? nbb[l] : 0.0;
                }
                __syncthreads();
                if (lane < nlw) {
                    const int g = lane / LPL, l = lane - g * LPL;
                    const int n0 = (a.fchunks == 1) ? g * a.n_q : 0;
                    const int n1 = (a.fchunks == 1) ? n0 + a.n_q : kWave;
                    double sf = 0.0, sb = 0.0;
                    for (int i = n0; i < n1; ++i) {
                        sf += red[0][l][i];
                        sb += red[1][l][i];
                    }
                    const int64_t o = (O * a.n_lines + line0 + lane) * a.n_rays;
                    if (c == 0) {
                        a.Ln[o + r] = a.norm * sf;
                        a.Ln[o + rb] = a.norm * sb;
                    } else {
                        a.Ln[o + r] += a.norm * sf;
                        a.Ln[o + rb] += a.norm * sb;
                    }
                }
                __syncthreads();
            }
        }
    }
    if (a.exec_steps != nullptr) {
        for (int o = kWave / 2; o > 0; o >>= 1) my_exec += __shfl_xor(my_exec, o);
        if (lane == 0) atomicAdd(a.exec_steps, my_exec);
    }
#pragma unroll
    for (int l = 0; l < LPL; ++l) {
        red[0][l][lane] = lact[l] ? (double)accJ[l] : 0.0;
        red[1][l][lane] = lact[l] ? (double)accL[l] : 0.0;
        red[2][l][lane] = lact[l] ? (double)accE[l] : 0.0;
    }
    __syncthreads();
    // lane t < nlw sums line t over the frequencies of its group in a fixed order
    if (lane < nlw) {
        const int g = lane / LPL, l = lane - g * LPL;
        const int n0 = (a.fchunks == 1) ? g * a.n_q : 0;
        const int n1 = (a.fchunks == 1) ? n0 + a.n_q : kWave;
        Acc sJ = 0, sL = 0, sE = 0;
        for (int i = n0; i < n1; ++i) {
            sJ += (Acc)red[0][l][i];
            sL += (Acc)red[1][l][i];
            sE += (Acc)red[2][l][i];
        }
        const int64_t o = O * a.n_lines + line0 + lane;
        a.J[o] = a.norm * (double)sJ;
        a.L[o] = a.norm * (double)sL;
        a.Jeff[o] = a.norm * (double)sE;
    }
    if (BAND) {
        __syncthreads();
#pragma unroll
        for (int l = 0; l < LPL; ++l) {
            red[0][l][lane] = lact[l] ? accB[l] : 0.0;
            red[1][l][lane] = lact[l] ? accD[l] : 0.0;
        }
        __syncthreads();
        if (lane < nlw) {
            const int g = lane / LPL, l = lane - g * LPL;
            const int n0 = (a.fchunks == 1) ? g * a.n_q : 0;
            const int n1 = (a.fchunks == 1) ? n0 + a.n_q : kWave;
            double sB = 0.0, sD = 0.0;
            for (int i = n0; i < n1; ++i) {
                sB += red[0][l][i];
                sD += red[1][l][i];
            }
            const int64_t o = O * a.n_lines + line0 + lane;
            a.Jb[o] = a.norm * sB;
            a.Ld[o] = a.norm * sD;
        }
    }
}

// Grid form: one workgroup per (point, line block).  Consecutive hardware workgroups go
// round-robin to the 8 XCDs; each XCD gets a contiguous range of origin points so that
// the cells their rays share stay in that XCD's L2.  HIGH asks for at least 3 waves per
// SIMD (4 with one line per lane): measured on the 50,000-point outflow model this beats
// the compiler's default register budget (two waves) although a few bytes of the sweep's
// live values then go to scratch.
template <bool F32, int LPL, bool HIGH>
__global__ __launch_bounds__(64, HIGH ? (LPL == 1 ? 4 : 3) : 1) void k_formal_solve(SolveArgs a)
{
    __shared__ NodeRec<typename Bulk<F32>::T, 2 * LPL> rec[kWave];
    __shared__ double red[3][LPL][kWave];
    const int64_t nb8 = (a.n_blocks + 7) / 8;
    const int64_t lb = (int64_t)(blockIdx.x & 7) * nb8 + (blockIdx.x >> 3);
    if (lb >= a.n_blocks) return;
    const int64_t O = lb / a.groups;
    solve_item<F32, LPL>(a, O, (int)(lb - O * a.groups), rec, red);
}

// Persistent form: a fixed grid of workgroups takes (point, line block) items from an
// atomic counter in the order a.order gives (points by decreasing cached step count, so
// the longest items start first and the tail is short).  Every workgroup leaves the loop
// once the counter has passed the last item.
template <bool F32, int LPL, bool HIGH>
__global__ __launch_bounds__(64, HIGH ? (LPL == 1 ? 4 : 3) : 1) void k_formal_solve_queue(SolveArgs a)
{
    __shared__ NodeRec<typename Bulk<F32>::T, 2 * LPL> rec[kWave];
    __shared__ double red[3][LPL][kWave];
    __shared__ unsigned long long item_s;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) item_s = atomicAdd(a.work_counter, 1ull);
        __syncthreads();
        const int64_t item = (int64_t)item_s;
        if (item >= a.n_blocks) break;
        const int64_t rank = item / a.groups;
        solve_item<F32, LPL>(a, (int64_t)a.order[rank], (int)(item - rank * a.groups), rec, red);
    }
}

// Band-operator variant of the FP64 grid kernel: also the entries of the inverse system
// matrix between O and its neighbour nodes (Jb, Ld, Ln of SolveArgs).
template <int LPL>
__global__ __launch_bounds__(64, 1) void k_formal_solve_band(SolveArgs a)
{
    __shared__ NodeRec<double, 2 * LPL> rec[kWave];
    __shared__ double red[3][LPL][kWave];
    const int64_t nb8 = (a.n_blocks + 7) / 8;
    const int64_t lb = (int64_t)(blockIdx.x & 7) * nb8 + (blockIdx.x >> 3);
    if (lb >= a.n_blocks) return;
    const int64_t O = lb / a.groups;
    solve_item<false, LPL, true>(a, O, (int)(lb - O * a.groups), rec, red);
}

hipError_t launch_formal_solve_band(const SolveArgs &a, hipStream_t s)
{
    if (a.n_blocks == 0) return hipSuccess;
    const int lpl = a.lines_per_wave / ((a.fchunks == 1 && 2 * a.n_q <= kWave) ? 2 : 1);
    const int64_t nb8 = (a.n_blocks + 7) / 8;
    if (lpl == 1)
        hipLaunchKernelGGL(k_formal_solve_band<1>, dim3((unsigned)(nb8 * 8)), dim3(kWave), 0, s, a);
    else if (lpl == 2)
        hipLaunchKernelGGL(k_formal_solve_band<2>, dim3((unsigned)(nb8 * 8)), dim3(kWave), 0, s, a);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

template <bool F32, int LPL, bool HIGH>
hipError_t launch_variant(const SolveArgs &a, int persistent, int n_wg, hipStream_t s)
{
    if (persistent) {
        hipLaunchKernelGGL((k_formal_solve_queue<F32, LPL, HIGH>), dim3(n_wg), dim3(kWave), 0, s, a);
    } else {
        const int64_t nb8 = (a.n_blocks + 7) / 8;
        hipLaunchKernelGGL((k_formal_solve<F32, LPL, HIGH>), dim3((unsigned)(nb8 * 8)), dim3(kWave), 0, s, a);
    }
    return hipGetLastError();
}

template <bool F32>
hipError_t launch_fs(const SolveArgs &a, const SolveConfig &cfg, hipStream_t s)
{
    const int lpl = a.lines_per_wave / ((a.fchunks == 1 && 2 * a.n_q <= kWave) ? 2 : 1);
    if (lpl == 1)
        return cfg.high_occupancy ? launch_variant<F32, 1, true>(a, cfg.persistent, cfg.n_wg, s)
                                  : launch_variant<F32, 1, false>(a, cfg.persistent, cfg.n_wg, s);
    if (lpl == 2)
        return cfg.high_occupancy ? launch_variant<F32, 2, true>(a, cfg.persistent, cfg.n_wg, s)
                                  : launch_variant<F32, 2, false>(a, cfg.persistent, cfg.n_wg, s);
    // three lines per lane only in the FP32 form: its state fits 3 waves per SIMD without
    // spills, where the FP64 one would not
    if (F32 && lpl == 3)
        return cfg.high_occupancy ? launch_variant<true, 3, true>(a, cfg.persistent, cfg.n_wg, s)
                                  : launch_variant<true, 3, false>(a, cfg.persistent, cfg.n_wg, s);
    return hipErrorInvalidValue;
}

hipError_t launch_formal_solve(const SolveArgs &a, const SolveConfig &cfg, int fp32, hipStream_t s)
{
    if (a.n_blocks == 0) return hipSuccess;
    return fp32 ? launch_fs<true>(a, cfg, s) : launch_fs<false>(a, cfg, s);
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
