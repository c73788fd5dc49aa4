// Ray-pair formal solve (the ALI hot loop): device templates shared by the per-precision
// instantiation units fs_fp64.hip and fs_fp32.hip.  The discretisation and the
// elimination are described at the top of formal_solve.hip.
//
// Mapping: one workgroup = one wave = one origin point and up to 64 (line, frequency)
// items; lanes [0, n_q) take lines line0 .. line0+LPL-1 ("group" 0), lanes [n_q, 2 n_q)
// the next LPL lines (group 1), one frequency per lane.  The Doppler offset of a node
// depends on the frequency only (line widths are proportional to the line frequency), so
// the LPL lines of a lane share its profile evaluation and its recurrence; with up to
// five lines per lane a point's nine lines take a single wave, which stages each ray
// segment and evaluates each profile once.  All lanes walk the same nodes (uniform control
// flow).  The wave stages `ns` nodes of a ray at a time in LDS (position, velocity
// projection, Doppler coefficients, sub-step count and increments, kappa and S of its
// lines); the sweep reads them as broadcasts.
#pragma once
#include "device_math.h"
#include "nlte_internal.h"

namespace nlte {

constexpr double kSqrt2 = 1.41421356237309504880;
constexpr double kInv2Sqrt2 = 0.35355339059327376220;  // 1 / (2 sqrt 2)
// The elimination state only grows (see elim_step); it is rescaled by a power of two once
// any line's D passes 2^300, checked after every node (every second node in the short
// mode's segment loop) and at least every fourth sub-step, which leaves room for steps
// with D_+ up to about 2^70 before the FP64 range ends.
// Power-of-two rescaling is exact, so when it happens does not change any result.
constexpr double kRenormAbove = 2.0370359763344861e90;   // 2^300

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
// sub-intervals of length 2 sqrt(2) dzq; per sub-interval x changes by da x_q - db.  maxdx
// bounds |dx| over all frequencies, K is the restart interval of the profile recurrence
// (0: evaluate every profile directly) in the long-segment mode and, in the short mode,
// which has no recurrence, the number of segments without sub-steps from this node on.  kap, S: line-centre opacity and source function
// of the wave's lines.
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
    double hd;   // weight h d of the last step (rescaled with the state): the share of the
    double Sl;   // last eliminated node's source Sl in Y (read by the band operator only)
};

// e^{-x^2}: FP64 by the table-driven exponential (tab: 2^{j/16} in LDS); FP32 on the
// hardware exp2, e^{-x^2} = 2^{-x^2 log2 e}.
__device__ __forceinline__ double profile(double x, const double *tab) { return exp_tab16(-(x * x), tab); }
__device__ __forceinline__ float profile(float x, const double *)
{
    return __builtin_amdgcn_exp2f(-(x * x) * 1.44269504088896340736f);
}

// e^{-x^2} at a node of a wave's sweep (uniform control flow).  Beyond x^2 = 746 the FP64
// value above is exactly 0, so where every lane of the wave is that far in the wing the
// exponential is skipped without changing any result.  (The FP32 exponential is cheaper
// than the vote and branch, measured.)
__device__ __forceinline__ double profile_far(double x, const double *tab)
{
    return __all(x * x > 746.0) ? 0.0 : profile(x, tab);
}
__device__ __forceinline__ float profile_far(float x, const double *tab) { return profile(x, tab); }

template <bool TRACK>
__device__ __forceinline__ void rescale(HalfState &st)
{
    const int e = __builtin_amdgcn_frexp_exp(st.D);
    st.N = ldexp(st.N, -e);
    st.D = ldexp(st.D, -e);
    st.Y = ldexp(st.Y, -e);
    if (TRACK) st.hd = ldexp(st.hd, -e);
}

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
    if (RENORM) rescale<TRACK>(st);
}

// Per-line state of a lane during a half sweep.
// (The opacity at the current node is k_cur g_cur, recomputed where needed: the same
// product the node's step used, so the same bits.)
template <typename T, int LPL>
struct LineState {
    HalfState st[LPL];
    T k_cur[LPL], S_e[LPL];
    int m_last;   // sub-intervals of the last segment (the one ending at O)
};

// A compiler barrier: LDS values read after it are loaded again instead of being kept in
// registers across the code before it (it emits no instruction).
__device__ __forceinline__ void reload_fence() { __atomic_signal_fence(__ATOMIC_SEQ_CST); }

// Rescale the lanes whose state passed 2^500 (in any of their lines).
template <int LPL, bool TRACK, typename T>
__device__ __forceinline__ void rescale_if_big(LineState<T, LPL> &ls)
{
    bool big = false;
#pragma unroll
    for (int l = 0; l < LPL; ++l) big = big || ls.st[l].D > kRenormAbove;
    if (big) {
#pragma unroll
        for (int l = 0; l < LPL; ++l) rescale<TRACK>(ls.st[l]);
    }
}

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

// The elimination step of elim_step with the segment's P = D_+ / sqrt 2 given and the
// source S_row of the row being eliminated; nothing is carried to the next step but the
// state (the lean form of the sweeps without the band operator's record).
__device__ __forceinline__ void elim_p(double Pp, double S_row, HalfState &st)
{
    const double hd = (st.Hm + Pp) * st.D;
    st.N = st.N + hd;
    st.Y = fma(S_row, hd, st.Y);
    st.D = fma(Pp, st.N, st.D);
    st.Hm = Pp;
}

// short_node skips the profile's exponential where the whole wave is beyond its range
// if SHORT_VOTE is set.  It is not: the vote is a wave-wide branch on a vector result at
// every node, whose wait costs more than the exponentials it saves on a disc.  For the
// same reason the segment loop checks for rescaling after every second node only (every
// fourth measured slower: its extra test costs more than the check), and tests for the
// end of a run on a scalar count taken at the run's start rather than on the next staged
// record (disc10 FP64 sweep 5.50 -> 4.90 s for the three together).
constexpr bool SHORT_VOTE = false;

// One segment without sub-steps, to staged node r1 (the segment's dzq given): the
// profile g1 of this lane at r1, r1's kappa and S of the lane's lines (k1, S1), and every
// line's step with P = (kappa_0 g0 + kappa_1 g1) dzq and the row source S0 (in FP32 formed
// as the general path forms it, so that both segment modes give the same bits).  A loop over
// segments that calls this twice per iteration with the (g, k, S) sets swapped copies no
// registers between segments.
template <bool F32, int LPL, bool CHECK = true>
__device__ __forceinline__ void short_node(const NodeRec<typename Bulk<F32>::T, 2 * LPL> &r1,
                                           typename Bulk<F32>::T dzq, typename Bulk<F32>::T xq,
                                           const double *tab, int grp, typename Bulk<F32>::T g0,
                                           typename Bulk<F32>::T &g1, const typename Bulk<F32>::T (&k0)[LPL],
                                           typename Bulk<F32>::T (&k1)[LPL], const typename Bulk<F32>::T (&S0)[LPL],
                                           typename Bulk<F32>::T (&S1)[LPL], LineState<typename Bulk<F32>::T, LPL> &ls)
{
    using T = typename Bulk<F32>::T;
    const T xn = r1.a * xq - r1.b;
    if constexpr (SHORT_VOTE)
        g1 = profile_far(xn, tab);
    else
        g1 = profile(xn, tab);
#pragma unroll
    for (int l = 0; l < LPL; ++l) {
        const int c = grp * LPL + l;
        k1[l] = r1.kap[c];
        S1[l] = r1.S[c];
        T Pp;
        if constexpr (F32)
            Pp = (k0[l] * g0) * dzq + (k1[l] * g1) * dzq;   // as the general path forms it, bit for bit
        else
            Pp = fma(k0[l], g0, k1[l] * g1) * dzq;
        elim_p((double)Pp, (double)S0[l], ls.st[l]);
    }
    if (CHECK) rescale_if_big<LPL, false>(ls);
}

// The profile at a sub-step node: with the far-wing vote in the long-segment mode, without
// it in the short mode (whose segments are rarely all in the far wing; the vote's branch
// costs more there than the exponentials it saves).
template <bool COLLAPSE, typename T>
__device__ __forceinline__ T profile_sub(T x, const double *tab)
{
    if constexpr (COLLAPSE)
        return profile_far(x, tab);
    else
        return profile(x, tab);
}

// Runs of segments without sub-steps take the loop of short_node (not in the long-segment
// mode, whose far-wing collapse measured faster without it).
template <bool F32, bool COLLAPSE>
constexpr bool SHORT_LOOP = !COLLAPSE;
// Sub-step segments: the form of the loop that alternates two sets of optical depths
// (LEAN) or the one that carries a_prev and S_e through elim_step.
template <bool F32, bool COLLAPSE>
constexpr bool LEAN_SUBSTEPS = true;

// Half-sweep along ray `ray` from its far end to O for Doppler offset xq of this lane.
// The result is left in ls.st (one HalfState per line of the lane).  nexec counts the
// elimination steps the wave executes (a collapsed far-wing segment counts as one).
// COLLAPSE: eliminate far-wing sub-step segments in one step (see below).
template <bool F32, int LPL, bool COLLAPSE, bool TRACK = false>
__device__ __forceinline__ void half_sweep(const SolveArgs &a, NodeRec<typename Bulk<F32>::T, 2 * LPL> *rec,
                                          const double *tab, int64_t O, int ray,
                                          typename Bulk<F32>::T xq, int grp, int line0, int nlw,
                                          LineState<typename Bulk<F32>::T, LPL> &ls, int64_t &nexec)
{
    using T = typename Bulk<F32>::T;
    using T2 = typename Bulk<F32>::T2;
    constexpr int NLW = 2 * LPL;
    const T2 *lc = reinterpret_cast<const T2 *>(a.lc);
    const int lane = threadIdx.x;
    const int ns = a.ns;   // nodes staged per round (2..64)
#pragma unroll
    for (int l = 0; l < LPL; ++l) {
        // Q = 1, y = I_in at the far boundary (in the scaled state of elim_step)
        const int li = grp * LPL + l;
        ls.st[l].N = kSqrt2;
        ls.st[l].D = 1.0;
        ls.st[l].Y = kSqrt2 * a.ibdy[line0 + (li < nlw ? li : 0)];
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
    // x_cur, g_cur: Doppler offset and profile at the current node; travel bounds how far
    // x moved (any lane) since g was last evaluated exactly
    T x_cur = 0, g_cur = 0;
    double travel = 0.0;
    for (int b0 = 0; b0 < L; b0 += ns - 1) {
        __syncthreads();
        // ---- stage nodes b0 .. b0+ns-1 in sweep order (far end first, O last)
        const int s = b0 + lane;
        double Zs = 0.0, sv = 0.0, vw = 1.0, an = 0.0, bn = 0.0;
        int64_t cidx = O;
        const bool load = lane < ns && s <= L;
        if (load) {
            cidx = (s < L) ? (int64_t)a.rcells[beg + (L - 1 - s)] : O;
            const CellRec c = a.cell[cidx];
            // O's record and the ray's direction are read again for each staging round (from
            // the caches) rather than held in registers through the sweep
            reload_fence();
            const CellRec cO = a.cell[O];
            const double nx = a.dir[3 * ray], ny = a.dir[3 * ray + 1], nz = a.dir[3 * ray + 2];
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
        int m_seg = 1;   // sub-intervals of this lane's segment (1 where it has none)
        if (load) {
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
            if (s < L && lane < ns - 1) {
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
                m_seg = m;
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
        if (!COLLAPSE) {
            // short mode has no recurrence: K holds the number of segments without sub-steps
            // from this node on within the round (the trailing zeros of the wave's mask of
            // segments with sub-steps or past the round's last)
            const int nseg_r = min(ns - 1, L - b0);
            const unsigned long long brk = __ballot(!(lane < nseg_r && m_seg == 1));
            if (load) rec[lane].K = (int)__builtin_ctzll(brk >> lane);
        }
        __syncthreads();
        // ---- sweep the staged segments
        const int nseg = min(ns - 1, L - b0);
        if (b0 == 0) {
            x_cur = rec[0].a * xq - rec[0].b;
            g_cur = profile(x_cur, tab);
#pragma unroll
            for (int l = 0; l < LPL; ++l) {
                ls.k_cur[l] = rec[0].kap[grp * LPL + l];
                ls.S_e[l] = rec[0].S[grp * LPL + l];
            }
        }
        for (int i = 0; i < nseg; ++i) {
            if (!TRACK && SHORT_LOOP<F32, COLLAPSE> && rec[i].m == 1) {
                // a run of segments without sub-steps (most of a disc's rays): one profile
                // evaluation per node and one step per line (short_node), two segments per
                // iteration so that the node values alternate between the A and B sets
                T gA = g_cur, gB = 0;
                T kA[LPL], kB[LPL], SA[LPL], SB[LPL];
#pragma unroll
                for (int l = 0; l < LPL; ++l) {
                    kA[l] = ls.k_cur[l];
                    SA[l] = ls.S_e[l];
                }
                // the run's length is known at its start (>= 1): the test between segments is on a
                // scalar count, not on the next record
                int run = rec[i].K;
                // two segments per iteration (the sets alternate A -> B -> A ...); the state is
                // checked for rescaling after the second and where the run ends
                for (;;) {
                    short_node<F32, LPL, false>(rec[i + 1], rec[i].dzq, xq, tab, grp, gA, gB, kA, kB, SA, SB, ls);
                    ++nexec;
                    ++i;
                    if (--run == 0) {
                        rescale_if_big<LPL, false>(ls);
                        gA = gB;
#pragma unroll
                        for (int l = 0; l < LPL; ++l) {
                            kA[l] = kB[l];
                            SA[l] = SB[l];
                        }
                        break;
                    }
                    short_node<F32, LPL, false>(rec[i + 1], rec[i].dzq, xq, tab, grp, gB, gA, kB, kA, SB, SA, ls);
                    ++nexec;
                    ++i;
                    rescale_if_big<LPL, false>(ls);
                    if (--run == 0) break;
                }
                g_cur = gA;
                x_cur = rec[i].a * xq - rec[i].b;   // the same bits as the last xn
#pragma unroll
                for (int l = 0; l < LPL; ++l) {
                    ls.k_cur[l] = kA[l];
                    ls.S_e[l] = SA[l];
                }
                travel = 0.0;
                if (i >= nseg) break;
            }
            if (TRACK && !F32 && !COLLAPSE && rec[i].m == 1) {
                // a run of segments without sub-steps (most of a disc's rays): one step per
                // node with the profile evaluated there, in a loop of its own (FP64 short-
                // segment mode; the FP32 form, whose exponential is one instruction, and the
                // long-segment mode measured faster without it)
                do {
                    const T dzq = rec[i].dzq;
                    const T xn = rec[i + 1].a * xq - rec[i + 1].b;
                    const T gn = profile_far(xn, tab);
#pragma unroll
                    for (int l = 0; l < LPL; ++l) {
                        const T kn = rec[i + 1].kap[grp * LPL + l];
                        T a_prev = (ls.k_cur[l] * g_cur) * dzq;
                        const T chi_n = kn * gn;
                        elim_step<F32, false, TRACK>(chi_n * dzq, rec[i + 1].S[grp * LPL + l], a_prev, ls.S_e[l],
                                                     ls.st[l]);
                        ls.k_cur[l] = kn;
                    }
                    rescale_if_big<LPL, TRACK>(ls);
                    x_cur = xn;
                    g_cur = gn;
                    ++nexec;
                    ++i;
                } while (i < nseg && rec[i].m == 1);
                travel = 0.0;
                if (TRACK) ls.m_last = 1;
                if (i >= nseg) break;
            }
            const int m = rec[i].m;
            const T dzq = rec[i].dzq;
            const T xn = rec[i + 1].a * xq - rec[i + 1].b;
            // kn, Sn: the end node's data for the sub-step increments; read again (after a
            // reload_fence) for the end node's own step, so they are not held meanwhile
            T kn[LPL], Sn[LPL], a_prev[LPL];
#pragma unroll
            for (int l = 0; l < LPL; ++l) {
                kn[l] = rec[i + 1].kap[grp * LPL + l];
                Sn[l] = rec[i + 1].S[grp * LPL + l];
                a_prev[l] = (ls.k_cur[l] * g_cur) * dzq;
            }
            if (COLLAPSE && m > 1) {
                // Far wing: every lane beyond the range of its profile (exactly 0 past
                // x^2 = 750 in FP64, 105 in FP32) at both ends of the segment, on one side
                // of the line centre, and zero opacity at its first node.  Then every node of
                // the segment has zero opacity, the elimination steps after the first change
                // nothing, and one step with zero opacity and the end node's source leaves
                // the same state.  (A segment without sub-steps is one step anyway.)  The
                // band operator's record of the last step: its weight is 0 (zero optical
                // depth on both sides of the last sub-step node), so that node's source does
                // not enter the neighbour entry.
                const T far2 = F32 ? (T)105 : (T)750;
                bool far = ((x_cur > (T)0) == (xn > (T)0)) && x_cur * x_cur > far2 && xn * xn > far2;
#pragma unroll
                for (int l = 0; l < LPL; ++l) far = far && ls.k_cur[l] * g_cur == (T)0;
                if (__all(far)) {
#pragma unroll
                    for (int l = 0; l < LPL; ++l) {
                        elim_step<F32, false, TRACK>((T)0, Sn[l], a_prev[l], ls.S_e[l], ls.st[l]);
                        ls.k_cur[l] = kn[l];
                        if (TRACK) {
                            ls.st[l].hd = 0.0;
                            ls.st[l].Sl = 0.0;
                        }
                    }
                    if (TRACK) ls.m_last = m;
                    rescale_if_big<LPL, TRACK>(ls);
                    x_cur = xn;
                    g_cur = (T)0;
                    travel = 0.0;
                    ++nexec;
                    continue;
                }
            }
            nexec += m;
            T gn;
            {
                const T im = rec[i].inv_m;
                const T dx = rec[i].da * xq - rec[i].db;
                const int K = rec[i].K;
                // direct evaluation where the recurrence would not pay for its two
                // exponentials (no or one sub-step node) or cannot be used (K == 0)
                if (!TRACK && LEAN_SUBSTEPS<F32, COLLAPSE> && (F32 || !COLLAPSE || K == 0 || m <= 2)) {
                    // sub-node j: x = x_cur + j dx, kappa and S linear in j; two sub-nodes per
                    // iteration, the step's P formed from the optical depths a at both ends
                    // (alternating between a_prev and aB) and the row's S recomputed from j, so
                    // that nothing else is carried from one sub-step to the next
                    T S0[LPL], dk[LPL], dS[LPL], aB[LPL];
#pragma unroll
                    for (int l = 0; l < LPL; ++l) {
                        S0[l] = ls.S_e[l];
                        dk[l] = (kn[l] - ls.k_cur[l]) * im;
                        dS[l] = (Sn[l] - S0[l]) * im;
                    }
                    int j = 1;
                    for (; j + 1 < m; j += 2) {
                        const T t1 = (T)j, t2 = (T)(j + 1);
                        const T g1 = profile_sub<COLLAPSE>(fma(t1, dx, x_cur), tab) * dzq;
#pragma unroll
                        for (int l = 0; l < LPL; ++l) {
                            aB[l] = fma(t1, dk[l], ls.k_cur[l]) * g1;
                            elim_p((double)(a_prev[l] + aB[l]), (double)fma(t1 - (T)1, dS[l], S0[l]), ls.st[l]);
                        }
                        const T g2 = profile_sub<COLLAPSE>(fma(t2, dx, x_cur), tab) * dzq;
#pragma unroll
                        for (int l = 0; l < LPL; ++l) {
                            a_prev[l] = fma(t2, dk[l], ls.k_cur[l]) * g2;
                            elim_p((double)(aB[l] + a_prev[l]), (double)fma(t1, dS[l], S0[l]), ls.st[l]);
                        }
                        if (((j + 1) & 3) == 0) rescale_if_big<LPL, false>(ls);   // (the end node checks too)
                    }
                    if (j < m) {
                        const T t1 = (T)j;
                        const T g1 = profile_sub<COLLAPSE>(fma(t1, dx, x_cur), tab) * dzq;
#pragma unroll
                        for (int l = 0; l < LPL; ++l) {
                            aB[l] = fma(t1, dk[l], ls.k_cur[l]) * g1;
                            elim_p((double)(a_prev[l] + aB[l]), (double)fma(t1 - (T)1, dS[l], S0[l]), ls.st[l]);
                            a_prev[l] = aB[l];
                        }
                    }
                    // the source of the last sub-node, whose row the end node's step eliminates
#pragma unroll
                    for (int l = 0; l < LPL; ++l) ls.S_e[l] = fma((T)(m - 1), dS[l], S0[l]);
                    gn = profile_sub<COLLAPSE>(xn, tab);
                    travel = 0.0;
                } else if ((TRACK || !LEAN_SUBSTEPS<F32, COLLAPSE>) && (F32 || !COLLAPSE || K == 0 || m <= 2)) {
                    T S0[LPL], dk[LPL], dS[LPL];
#pragma unroll
                    for (int l = 0; l < LPL; ++l) {
                        S0[l] = ls.S_e[l];
                        dk[l] = (kn[l] - ls.k_cur[l]) * im;
                        dS[l] = (Sn[l] - S0[l]) * im;
                    }
                    for (int j = 1; j < m; ++j) {
                        const T tj = (T)j;
                        const T gq = profile_far(x_cur + tj * dx, tab) * dzq;
#pragma unroll
                        for (int l = 0; l < LPL; ++l)
                            elim_step<F32, false, TRACK>((ls.k_cur[l] + tj * dk[l]) * gq, S0[l] + tj * dS[l],
                                                         a_prev[l], ls.S_e[l], ls.st[l]);
                        if ((j & 3) == 0) rescale_if_big<LPL, TRACK>(ls);   // (the end node checks too)
                    }
                    gn = profile_far(xn, tab);
                    travel = 0.0;
                } else {
                    // x is linear in the sub-step index j, so g_j = e^{-x_j^2} obeys
                    // g_{j+1} = g_j r_j, r_{j+1} = r_j c with r_j = e^{-2 x_j dx - dx^2} and
                    // c = e^{-2 dx^2}.  Values are recomputed exactly whenever x may have
                    // moved by more than 16 widths since the last exact value, so one that
                    // underflowed (|x| > 27) cannot hide a profile above e^{-121}.
                    const double mdx = (double)rec[i].maxdx;
                    const double u2 = 2.0 * dx * dx;
                    const double c = mdx <= 0.5 ? exp_neg_small(u2) : exp_tab16(-u2, tab);
                    // (kq starts at kappa dzq of the segment's first node, which k_cur keeps
                    // until the segment ends, so restarts recompute it instead of holding it)
                    // (restarts take S of the segment's first node from LDS again: S_e held it
                    // when the segment began)
                    double dkq[LPL], dS[LPL], kq[LPL], St[LPL];
#pragma unroll
                    for (int l = 0; l < LPL; ++l) {
                        dkq[l] = (double)((kn[l] - ls.k_cur[l]) * im * dzq);
                        dS[l] = (double)((Sn[l] - ls.S_e[l]) * im);
                        kq[l] = (double)(ls.k_cur[l] * dzq);
                        St[l] = (double)ls.S_e[l];
                    }
                    double g = g_cur, r = exp_tab16(fmin(-(2.0 * x_cur + dx) * dx, 700.0), tab);
                    int budget = K;
                    if (mdx > 0.0) budget = (int)fminf((16.0f - (float)travel) * __builtin_amdgcn_rcpf((float)mdx),
                                                       (float)K);
                    if (budget < 1) {
                        g = profile((double)x_cur, tab);
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
                        // the last 0-3 steps in straight-line code (checked for rescaling
                        // after the segment's end node)
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
                        rescale_if_big<LPL, TRACK>(ls);
                        const double xj = fma((double)j, dx, (double)x_cur);
                        g = exp_tab16(-(xj * xj), tab);
                        r = exp_tab16(fmin(-(2.0 * xj + dx) * dx, 700.0), tab);
                        reload_fence();
#pragma unroll
                        for (int l = 0; l < LPL; ++l) {
                            kq[l] = fma((double)j, dkq[l], (double)(ls.k_cur[l] * dzq));
                            St[l] = fma((double)j, dS[l], (double)rec[i].S[grp * LPL + l]);
                        }
                        travel = 0.0;
                        budget = K;
                    }
                    gn = g;
                }
            }
            reload_fence();
#pragma unroll
            for (int l = 0; l < LPL; ++l) {
                const T kn_e = rec[i + 1].kap[grp * LPL + l];
                const T chi_n = kn_e * gn;
                elim_step<F32, false, TRACK>(chi_n * dzq, rec[i + 1].S[grp * LPL + l], a_prev[l], ls.S_e[l],
                                             ls.st[l]);
                ls.k_cur[l] = kn_e;
            }
            rescale_if_big<LPL, TRACK>(ls);
            x_cur = xn;
            g_cur = gn;
            if (TRACK) ls.m_last = m;
        }
    }
}

// All (line, frequency) work of one wave for origin point O and line block w, accumulated
// over every ray pair and written to J, L*, Jeff.  Points of models that already
// converged are skipped (their outputs are not needed).
// Lanes: with two groups, group g takes lanes 32 g .. 32 g + n_q - 1 (one frequency each)
// and lines line0 + g LPL ...; with one group, lanes 0..63 take frequencies c 64 + lane of
// chunk c.
// red: LDS rows [3][LPL][64].  Each lane keeps the first half sweep's Q, y and last
// optical-depth step in its column until the second half sweep ends (freeing registers in
// the sweep); then the lanes write their contributions to J, L* and Jeff of each line
// there, and lane q LPL + l of each group sums row (q, l) over the group's frequencies in
// index order and adds it to its one accumulator (one register, not three per line).
template <bool F32, int LPL, bool COLLAPSE, bool BAND = false>
__device__ __forceinline__ void solve_item(const SolveArgs &a, int64_t O, int w,
                                           NodeRec<typename Bulk<F32>::T, 2 * LPL> *rec,
                                           double (*red)[LPL][kWave], const double *tab)
{
    using T = typename Bulk<F32>::T;
    using T2 = typename Bulk<F32>::T2;
    using Acc = typename Bulk<F32>::T;
    const int lane = threadIdx.x;
    if (a.model_done != nullptr && a.model_done[a.model_of[O]]) return;
    // lane -> (group, frequency); a wave owns lines line0 .. line0 + nlw - 1
    const int ngrp = a.ngrp;
    const int width = ngrp == 2 ? 32 : kWave;    // lanes per group
    const int line0 = w * a.lines_per_wave;
    const int nlw = min(a.lines_per_wave, a.n_lines - line0);
    const int grp = ngrp == 2 ? lane >> 5 : 0;
    const int sub = lane & (width - 1);           // lane within its group
    const T2 *lc = reinterpret_cast<const T2 *>(a.lc);
    bool lact[LPL];
#pragma unroll
    for (int l = 0; l < LPL; ++l) lact[l] = grp * LPL + l < nlw;
    const int nfq = ngrp == 2 ? a.n_q : min(kWave, a.n_q);   // frequencies of a group (per chunk)
    const int col0 = grp * width;                             // first lane of the group
    // lane col0 + q LPL + l (q < 3) accumulates quantity q (J, L*, Jeff) of line l; with
    // BAND lanes col0 + 3 LPL + q LPL + l (q < 2) accumulate Jb and Ld
    Acc acc = 0;
    const int rq = sub / LPL, rl = sub - rq * LPL;   // the row this lane sums
    LineState<T, LPL> ls;
    unsigned long long my_exec = 0;   // executed node-frequency steps of this lane
    for (int p = 0; p < a.n_pairs; ++p) {
        const int r = a.pair_r[p], rb = a.anti[r];
        for (int c = 0; c < a.fchunks; ++c) {
            const int nidx = (a.fchunks == 1) ? sub : c * kWave + lane;
            const bool act = nidx < a.n_q;
            const double xq = act ? a.qx[nidx] : 0.0;
            const double wq = act ? a.qw[nidx] : 0.0;
            // u pairs I(n, x) with I(-n, -x): the antipode sweeps at the mirrored offset
            int64_t nex = 0;
            double hdf[LPL], Sf[LPL];
            int mf = 1;
            // the two halves (unrolled: measured faster than one compiled sweep in a loop)
#pragma unroll
            for (int half = 0; half < 2; ++half) {
                half_sweep<F32, LPL, COLLAPSE, BAND>(a, rec, tab, O, half ? rb : r, (T)(half ? -xq : xq), grp,
                                                     line0, nlw, ls, nex);
                if (half) break;
                if (BAND) mf = ls.m_last;
#pragma unroll
                for (int l = 0; l < LPL; ++l) {
                    const double id = 1.0 / ls.st[l].D;
                    red[0][l][lane] = ls.st[l].N * id;   // Q of the first half
                    red[1][l][lane] = ls.st[l].Y * id;   // y
                    red[2][l][lane] = ls.st[l].Hm;       // its last optical-depth step / sqrt 2
                    if (BAND) {
                        hdf[l] = ls.st[l].hd * id;
                        Sf[l] = ls.st[l].Sl;
                    }
                }
            }
            if (a.exec_steps != nullptr && act) {
                int nact = 0;
#pragma unroll
                for (int l = 0; l < LPL; ++l) nact += lact[l] ? 1 : 0;
                my_exec += (unsigned long long)nex * (unsigned long long)nact;
            }
            double vB[LPL], vD[LPL], nbf[LPL], nbb[LPL];
            double vJ[LPL], vL[LPL], vE[LPL];
#pragma unroll
            for (int l = 0; l < LPL; ++l) {
                const int li = grp * LPL + l;
                const double S_O = (double)lc[O * a.n_lines + line0 + (li < nlw ? li : 0)].y;
                const double id = 1.0 / ls.st[l].D;
                const double h = red[2][l][lane] + ls.st[l].Hm;
                const double inv = 1.0 / (h + fma(ls.st[l].N, id, red[0][l][lane]));
                const double yy = fma(ls.st[l].Y, id, red[1][l][lane]);
                const bool on = act && lact[l];
                vJ[l] = on ? wq * (fma(h, S_O, yy) * inv) : 0.0;
                vL[l] = on ? wq * (h * inv) : 0.0;
                vE[l] = on ? wq * (yy * inv) : 0.0;
                if (BAND) {
                    // (T^-1)_{O, neighbour} on either side: the neighbour's share of y
                    // over the combine's denominator; a neighbour at fraction 1/m of the
                    // segment toward the first cell interpolates O's own source by 1 - 1/m
                    const double tf = hdf[l] * inv, tb = ls.st[l].hd * id * inv;
                    const double imf = 1.0 / (double)mf, imb = 1.0 / (double)ls.m_last;
                    vB[l] = on ? wq * (yy * inv - tf * Sf[l] - tb * ls.st[l].Sl) : 0.0;
                    vD[l] = on ? wq * (h * inv + (1.0 - imf) * tf + (1.0 - imb) * tb) : 0.0;
                    nbf[l] = on ? wq * tf * imf : 0.0;
                    nbb[l] = on ? wq * tb * imb : 0.0;
                }
            }
            // sums over the group's frequencies (the rows' first-half values are consumed)
            __syncthreads();
#pragma unroll
            for (int l = 0; l < LPL; ++l) {
                red[0][l][lane] = vJ[l];
                red[1][l][lane] = vL[l];
                red[2][l][lane] = vE[l];
            }
            __syncthreads();
            if (sub < 3 * LPL) {
                Acc sum = 0;
                for (int i = 0; i < nfq; ++i) sum += (Acc)red[rq][rl][col0 + i];
                acc += sum;
            }
            if (BAND) {
                __syncthreads();
#pragma unroll
                for (int l = 0; l < LPL; ++l) {
                    red[0][l][lane] = vB[l];
                    red[1][l][lane] = vD[l];
                }
                __syncthreads();
                if (sub >= 3 * LPL && sub < 5 * LPL) {
                    const int q = (sub - 3 * LPL) / LPL, l = sub - 3 * LPL - q * LPL;
                    double sum = 0.0;
                    for (int i = 0; i < nfq; ++i) sum += red[q][l][col0 + i];
                    acc += (Acc)sum;
                }
                // couplings to the first cells along r and rb, per line summed over this
                // group's frequencies (fixed order)
                __syncthreads();
#pragma unroll
                for (int l = 0; l < LPL; ++l) {
                    red[0][l][lane] = nbf[l];
                    red[1][l][lane] = nbb[l];
                }
                __syncthreads();
                if (sub < 2 * LPL) {
                    const int q = sub / LPL, l = sub - q * LPL;
                    if (lact[l]) {
                        double sum = 0.0;
                        for (int i = 0; i < nfq; ++i) sum += red[q][l][col0 + i];
                        const int64_t o = (O * a.n_lines + line0 + grp * LPL + l) * a.n_rays + (q ? rb : r);
                        if (c == 0)
                            a.Ln[o] = a.norm * sum;
                        else
                            a.Ln[o] += a.norm * sum;
                    }
                }
            }
        }
    }
    if (a.exec_steps != nullptr) {
        for (int o = kWave / 2; o > 0; o >>= 1) my_exec += __shfl_xor(my_exec, o);
        if (lane == 0) atomicAdd(a.exec_steps, my_exec);
    }
    if (sub < (BAND ? 5 : 3) * LPL && rl < LPL) {
        const int q = sub / LPL, l = sub - q * LPL, li = grp * LPL + l;
        if (li < nlw) {
            const int64_t o = O * a.n_lines + line0 + li;
            double *out = q == 0 ? a.J : q == 1 ? a.L : q == 2 ? a.Jeff : q == 3 ? a.Jb : a.Ld;
            out[o] = a.norm * (double)acc;
        }
    }
}

// Dynamic LDS of a formal-solve workgroup: the rows [3][LPL][64] (FP64), then ns staged
// nodes.
template <bool F32, int LPL>
constexpr size_t fs_rows_bytes()
{
    return sizeof(double) * 3 * LPL * kWave;
}
template <bool F32, int LPL>
constexpr size_t fs_lds_bytes(int ns)
{
    return fs_rows_bytes<F32, LPL>() + (size_t)ns * sizeof(NodeRec<typename Bulk<F32>::T, 2 * LPL>);
}

// Work items are (point, line block); a workgroup takes a.tile consecutive items at a time.
// Grid form: one workgroup per tile of items; consecutive hardware workgroups go
// round-robin to the 8 XCDs and each XCD gets a contiguous range of origin points, so
// that the cells their rays share stay in that XCD's L2.  Persistent form (a.persistent):
// a fixed grid of workgroups takes tiles from an atomic counter in the order a.order gives
// (points by decreasing cached step count, so the longest items start first and the tail
// is short); every workgroup leaves the loop once the counter has passed the last item.
// W: waves per SIMD the register budget is built for.
template <bool F32, int LPL, int W, bool COLLAPSE>
__global__ __launch_bounds__(64, W) void k_formal_solve(SolveArgs a)
{
    extern __shared__ double fs_smem[];
    __shared__ double tab[16];
    auto *red = reinterpret_cast<double (*)[LPL][kWave]>(fs_smem);
    auto *rec = reinterpret_cast<NodeRec<typename Bulk<F32>::T, 2 * LPL> *>(fs_smem + 3 * LPL * kWave);
    if (!F32) {
        if (threadIdx.x < 16) tab[threadIdx.x] = kExp2Sixteenths[threadIdx.x];
        __syncthreads();
    }
    // one call site for both forms (the sweep is compiled once): a grid workgroup takes
    // its own item and stops
    // a workgroup takes a.tile consecutive items at a time
    __shared__ unsigned long long item_s;
    const int64_t tile = a.tile;
    int64_t first;
    if (a.persistent) {
        if (threadIdx.x == 0) item_s = atomicAdd(a.work_counter, (unsigned long long)tile);
        __syncthreads();
        first = (int64_t)item_s;
    } else {
        const int64_t n_tiles = (a.n_blocks + tile - 1) / tile;
        const int64_t nb8 = (n_tiles + 7) / 8;
        first = ((int64_t)(blockIdx.x & 7) * nb8 + (blockIdx.x >> 3)) * tile;
    }
    while (first < a.n_blocks) {
        const int64_t last = first + tile < a.n_blocks ? first + tile : a.n_blocks;
        for (int64_t item = first; item < last; ++item) {
            const int64_t rank = item / a.groups;
            const int64_t O = a.persistent ? (int64_t)a.order[rank] : rank;
            solve_item<F32, LPL, COLLAPSE>(a, O, (int)(item - rank * a.groups), rec, red, tab);
        }
        if (!a.persistent) break;
        __syncthreads();
        if (threadIdx.x == 0) item_s = atomicAdd(a.work_counter, (unsigned long long)tile);
        __syncthreads();
        first = (int64_t)item_s;
    }
}

template <bool F32, int LPL, int W, bool COLLAPSE>
hipError_t launch_fs_variant(const SolveArgs &a, int n_wg, hipStream_t s)
{
    const size_t lds = fs_lds_bytes<F32, LPL>(a.ns);
    const int64_t n_tiles = (a.n_blocks + a.tile - 1) / a.tile;
    const unsigned grid = a.persistent ? (unsigned)n_wg : (unsigned)(((n_tiles + 7) / 8) * 8);
    hipLaunchKernelGGL((k_formal_solve<F32, LPL, W, COLLAPSE>), dim3(grid), dim3(kWave), lds, s, a);
    return hipGetLastError();
}

template <bool F32, int LPL>
hipError_t launch_fs_lpl(const SolveArgs &a, const SolveConfig &cfg, hipStream_t s)
{
    if (a.waves == 3)
        return a.collapse ? launch_fs_variant<F32, LPL, 3, true>(a, cfg.n_wg, s)
                          : launch_fs_variant<F32, LPL, 3, false>(a, cfg.n_wg, s);
    if (a.waves == 1)
        return a.collapse ? launch_fs_variant<F32, LPL, 1, true>(a, cfg.n_wg, s)
                          : launch_fs_variant<F32, LPL, 1, false>(a, cfg.n_wg, s);
    return a.collapse ? launch_fs_variant<F32, LPL, 2, true>(a, cfg.n_wg, s)
                      : launch_fs_variant<F32, LPL, 2, false>(a, cfg.n_wg, s);
}

template <bool F32>
hipError_t launch_fs_prec(const SolveArgs &a, const SolveConfig &cfg, hipStream_t s)
{
    switch (a.lines_per_wave / a.ngrp) {
    case 1: return launch_fs_lpl<F32, 1>(a, cfg, s);
    case 2: return launch_fs_lpl<F32, 2>(a, cfg, s);
    case 3: return launch_fs_lpl<F32, 3>(a, cfg, s);
    case 4: return launch_fs_lpl<F32, 4>(a, cfg, s);
    case 5: return launch_fs_lpl<F32, 5>(a, cfg, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace nlte
