// Formal solve with scattering: both equations of the generalised Feautrier form
// (Sec. 3.3, Eq. GFE) for a scattering opacity chi_s(n) = chi_s + chi_dip . n, grey over
// a line's frequencies (chi^+ = chi_s, chi^- = chi_dip . n), scattering coherently in
// each point's comoving frame with the reciprocal redistribution
// chi_s(n) chi_s(n')/(4 pi chi_s), so that the emissivity into n is chi_s(n) Jw with Jw
// the mean intensity weighted by w(n') = chi_s(n')/chi_s, and with the right-hand sides
// from the previous iteration's Jw (Sec. 3.3: the Psi terms are evaluated with the
// previous solution).  Jw is J_nu when chi_dip = 0.
//
// At a node the photon of the sweep's own direction has comoving offset -y (y = a x - b
// for the lane's x), the opposite one +y; with chi^- along the sweep direction cm,
// chi_t = chi_line + chi_s, r = chi_s/chi_t and rm = cm/chi_t:
//   S+ = S + r (Jbar - S) + rm dJ,   sigma~ = r dJ + rm Jbar   (Psi^-/chi_t, sweep direction),
// Jbar = (Jw(-y) + Jw(y))/2, dJ = (Jw(-y) - Jw(y))/2.  The interior rows of the u-equation
// gain -d sigma/dtau as the central difference over the two neighbours, those of the
// v-equation -d S+/dtau; the boundary rows the half-node values.  Both equations share the
// matrix, so one elimination carries two particular solutions (y for u, yv for v).
// chi^- enters through the integrating factor e^M, M = int chi^- ds along the sweep: the
// transformed pair has chi^- = 0 and sources e^M S+, e^M sigma; the elimination keeps its
// particular solutions and held sources in the frame of the current node (M = 0 there), so
// each step multiplies them by e^{-dM} of its sub-interval (trapezoid of chi^-), and at the
// origin the frames of both halves coincide.
// J(y) is linear in y between the quadrature offsets (constant beyond them; the offset is
// located once for both end cells of a sub-step segment, by its arithmetic position on an
// evenly spaced quadrature, where -y mirrors +y, and by bisection otherwise); velocity
// sub-steps interpolate chi_s and the end cells' J linearly in t at their own offset.
// The elimination carries sigma~ / sqrt 2, the form in which it enters the scaled rows.
//
// One workgroup per point and line (two lines, in lanes 0-31 and 32-63, when n_q <= 32),
// one lane per frequency (n_q <= 256 lanes).  Each lane
// eliminates both halves of every ray pair from the far ends toward the origin in the
// division-free scaled state of the line formal solve (n, d, y~, yv~ with node coefficients
// chi dz/(2 sqrt 2)) in FP64, and combines them at the origin.  The block stages up to 24
// nodes of a half ray at a time in LDS (cell records, the lines' coefficients, their J_nu
// rows, and the sub-step segments between them).  Inside a sub-step segment the line
// profile follows the multiplicative recurrence of the line formal solve (exact restarts
// after at most 16 widths of travel) and, on an evenly spaced quadrature, the position
// of +-y advances by a constant; the state is renormalised at every cell node and every
// fourth sub-step.  With isotropic scattering two kinds of sub-step segment take shorter
// forms: where every lane's lookups clamp, Jw is linear along the segment and the node values
// come from the running Jbar - S and dJ; in the far wing (no line opacity) every node value
// is linear in the sub-node index, so from the third sub-node on the differences across the
// eliminated node are constants.  Besides J, L* (times chi_line/chi_t) and Jeff it returns Jw at the
// quadrature offsets from u and v at the origin: I(n, x) = u(x) + v(x) and
// I(-n, x) = u(-x) - v(-x) for the pair representative n, weighted by w(+-n) of the origin.
#include <type_traits>

#include "nlte_internal.h"
#include "device_math.h"

namespace nlte {

namespace {

constexpr int kScatMaxQ = 256;
constexpr int kChunk = 24;   // nodes staged per round
constexpr double kSq2 = 1.41421356237309504880;
constexpr double kISq2 = 0.70710678118654752440;

// Position of offset y on an arbitrary ascending quadrature: J(y) = row[i0] + t (row[i1] -
// row[i0]) with qx[i0] <= y < qx[i1], or i0 = i1 at the outermost offset beyond which J is
// constant (bisection).
struct QPos {
    int i0, i1;
    double t;
};

__device__ inline QPos locate(const double *qx, int nq, double y)
{
    QPos p;
    if (!(y > qx[0])) {   // also a NaN offset: no read outside the row
        p.i0 = p.i1 = 0;
        p.t = 0.0;
        return p;
    }
    if (!(y < qx[nq - 1])) {
        p.i0 = p.i1 = nq - 1;
        p.t = 0.0;
        return p;
    }
    int lo = 0, hi = nq - 1;   // qx[lo] <= y < qx[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (qx[mid] <= y)
            lo = mid;
        else
            hi = mid;
    }
    p.i0 = lo;
    p.i1 = lo + 1;
    p.t = (y - qx[lo]) / (qx[lo + 1] - qx[lo]);
    return p;
}

__device__ __forceinline__ double j_at(const double *__restrict__ row, const QPos &p)
{
    const double r0 = row[p.i0];
    return fma(p.t, row[p.i1] - r0, r0);
}

// Evenly spaced quadrature (n_q >= 2): u = (y - x_0)/h in grid steps, clamped to
// [0, n_q - 1]; J(y) = row[i] + t (row[i+1] - row[i]) with i = min(floor u, n_q - 2) and
// t = u - i.  On the symmetric grid -y sits at n_q - 1 - u, which is interval n_q - 2 - i
// at fraction 1 - t (the same value as its own floor at a knot, where the interpolant is
// continuous, and the grid's end values at the clamped ends).
struct UPair {
    int ip, im;
    double tp, tm;
};

__device__ __forceinline__ UPair upos(double u, double top, int lo_max)
{
    const double uc = fmin(fmax(u, 0.0), top);   // a NaN position becomes 0: no read outside the row
    UPair q;
    q.ip = min((int)uc, lo_max);
    q.tp = uc - (double)q.ip;
    q.im = lo_max - q.ip;
    q.tm = 1.0 - q.tp;
    return q;
}

__device__ __forceinline__ double j_u(const double *__restrict__ row, int i, double t)
{
    const double r0 = row[i];
    return fma(t, row[i + 1] - r0, r0);
}

// Quadrature geometry for the lookups.
struct QGeo {
    const double *qx;   // in LDS
    int nq, lo_max;
    double top, inv_h;
    double mx0;         // -x_0 / h
};

// Where an offset y is looked up: its grid position u on an evenly spaced quadrature,
// else y itself (bisection).
template <bool UNI>
__device__ __forceinline__ double qpos(const QGeo &g, double y)
{
    if constexpr (UNI)
        return fma(y, g.inv_h, g.mx0);
    else
        return y;
}

// J(y) and J(-y) of one row at lookup position pos = qpos(y).
template <bool UNI>
__device__ __forceinline__ void j_node(const QGeo &g, const double *row, double pos, double &jp, double &jm)
{
    if constexpr (UNI) {
        const UPair q = upos(pos, g.top, g.lo_max);
        jp = j_u(row, q.ip, q.tp);
        jm = j_u(row, q.im, q.tm);
    } else {
        jp = j_at(row, locate(g.qx, g.nq, pos));
        jm = j_at(row, locate(g.qx, g.nq, -pos));
    }
}

// J(y) and J(-y) at a sub-step node (lookup position pos = qpos(y)): the two end cells'
// rows at the node's own offset, interpolated linearly at fraction tt of the segment.
template <bool UNI>
__device__ __forceinline__ void j_sub(const QGeo &g, const double *rp, const double *rq, double pos, double tt,
                                      double &jp, double &jm)
{
    double ap, bp, am, bm;
    if constexpr (UNI) {
        const UPair q = upos(pos, g.top, g.lo_max);
        ap = j_u(rp, q.ip, q.tp);
        bp = j_u(rq, q.ip, q.tp);
        am = j_u(rp, q.im, q.tm);
        bm = j_u(rq, q.im, q.tm);
    } else {
        const QPos lp = locate(g.qx, g.nq, pos), lm = locate(g.qx, g.nq, -pos);
        ap = j_at(rp, lp);
        bp = j_at(rq, lp);
        am = j_at(rp, lm);
        bm = j_at(rq, lm);
    }
    jp = fma(tt, bp - ap, ap);
    jm = fma(tt, bm - am, am);
}

// Staged node of a half ray in sweep order (far end first, O last): projection Z, projected
// velocity s and line-width speed relative to O, Doppler coefficients y = a x - b, and per
// line slot the line-centre opacity, source function, scattering opacity and J_nu row.
struct SNode {
    double Z, s, vw, a, b;
    double kap[2], S[2], cs[2], cm[2];   // cm: chi^- along the sweep direction
    const double *jrow[2];
};

// Segment from a staged node to the next: m sub-intervals of optical-depth weight
// hz = (Z - Z_next)/(2 sqrt 2 m), per sub-interval increments of the Doppler coefficients
// and of kappa, S and chi_s; maxdx bounds |dy| over the quadrature (imdx = 1/maxdx, 0 for
// none), K is the restart interval of the profile recurrence (0: direct evaluation).
// With an odd opacity: per sub-interval the increment dcm of cm, the path length ds, and
// the frame factor e^{-dM} of the first sub-interval (f0) and its ratio between successive
// ones (rho), dM = ds (cm_j + cm_{j+1})/2 being linear in the sub-interval index.
struct SSeg {
    double hz, da, db, im, maxdx, imdx, ds;
    double dk[2], dS[2], dcs[2], dcm[2], f0[2], rho[2];
    int m, K;
};

// Node quantities at the lane's frequency: total opacity, S+ and sq = sigma~ / sqrt 2.
struct NodeVal {
    double chit, Sp, sq;
};

// S+ = S + r (Jbar - S) + rm dJ and sigma~ = r dJ + rm Jbar with r = chi_s/chi_t, the
// scattering share, and rm = cm/chi_t (safe for denormal far-wing opacities; cm = 0
// wherever chi_s = 0).  Without scattering r = 0, so S+ is the line's S also where the line
// opacity has underflowed to zero: the value does not jump where the profile underflows.
template <bool ANISO>
__device__ __forceinline__ NodeVal node_val(double cl, double cs, double cm, double S, double jp, double jm)
{
    NodeVal v;
    v.chit = cl + cs;
    // 1/chit: the hardware estimate and one Newton step (relative error below 3e-15, measured
    // over 2^22 inputs spread over 1e-30..1e30)
    double ic = __builtin_amdgcn_rcp(v.chit);
    ic = fma(ic, fma(-v.chit, ic, 1.0), ic);
    ic = cs > 0.0 ? ic : 0.0;   // chit >= cs > 0
    const double r = cs * ic;
    v.Sp = fma(0.5 * r, jp + jm, fma(-r, S, S));
    v.sq = (0.5 * kISq2 * r) * (jm - jp);
    if (ANISO) {
        const double rm = cm * ic;
        v.Sp = fma(0.5 * rm, jm - jp, v.Sp);
        v.sq = fma(0.5 * kISq2 * rm, jp + jm, v.sq);
    }
    return v;
}

// The same where Jw is linear along a segment (its lookups clamp), from the running
// D = Jbar - S and Q = (Jw(-y) - Jw(y)) / (2 sqrt 2), themselves linear in the sub-node index:
// S+ = S + r D, sigma~ / sqrt 2 = r Q (isotropic scattering).
__device__ __forceinline__ NodeVal node_val_lin(double chit, double cs, double S, double D, double Q)
{
    NodeVal v;
    v.chit = chit;
    double ic = __builtin_amdgcn_rcp(chit);
    ic = fma(ic, fma(-chit, ic, 1.0), ic);
    ic = cs > 0.0 ? ic : 0.0;
    const double r = cs * ic;
    v.Sp = fma(r, D, S);
    v.sq = r * Q;
    return v;
}

// e^{-y^2} by the table-driven exponential (tab: 2^{j/16} in LDS).
__device__ __forceinline__ double profile(double y, const double *tab) { return exp_tab16(-(y * y), tab); }

// Elimination state of a half sweep and the last node reached (chit, Sp, sq), with sq_pp
// and Sp_pp the sq and Sp of the node before it (virtual -sq, -Sp at the far end); y is
// the particular solution of the u-equation, yv that of the v-equation divided by sqrt 2
// (which leaves a factor 1/2 as its only constant).
struct HalfState {
    double n, d, y, yv, Pm;
    double chit, Sp, sq, sq_pp, Sp_pp;
};

__device__ __forceinline__ void start(HalfState &h, const NodeVal &first, double I_in)
{
    h.n = kSq2;
    h.d = 1.0;
    h.y = kSq2 * I_in;
    h.yv = I_in;
    h.Pm = 0.0;
    h.chit = first.chit;
    h.Sp = first.Sp;
    h.sq = first.sq;
    h.sq_pp = -first.sq;
    h.Sp_pp = -first.Sp;
}

// Move the state into the frame of the next node: the particular solutions and the held
// sources times e^{-dM} of the sub-interval.
template <bool ANISO>
__device__ __forceinline__ void reframe(HalfState &h, double f)
{
    if (ANISO) {
        h.y *= f;
        h.yv *= f;
        h.Sp *= f;
        h.sq *= f;
        h.sq_pp *= f;
        h.Sp_pp *= f;
    }
}

// Eliminate the last node, stepping to node v over a sub-interval with optical-depth
// weight P (the trapezoid chi dz / sqrt 2).
template <bool RENORM>
__device__ __forceinline__ void step_p(HalfState &h, const NodeVal &v, double P)
{
    const double hd = (h.Pm + P) * h.d;
    h.n += hd;
    h.y = fma(h.sq_pp - v.sq, h.d, fma(h.Sp, hd, h.y));   // y + S+ h d - (sigma~ - sigma~_pp) d / sqrt 2
    // (yv + sigma~ h d - (S+ - S+_pp) d / sqrt 2) / sqrt 2
    h.yv = fma((h.Sp_pp - v.Sp) * 0.5, h.d, fma(h.sq, hd, h.yv));
    h.d = fma(P, h.n, h.d);
    h.Pm = P;
    h.sq_pp = h.sq;
    h.Sp_pp = h.Sp;
    h.chit = v.chit;
    h.Sp = v.Sp;
    h.sq = v.sq;
    if (RENORM) {
        const int ex = __builtin_amdgcn_frexp_exp(h.d);
        h.n = ldexp(h.n, -ex);
        h.d = ldexp(h.d, -ex);
        h.y = ldexp(h.y, -ex);
        h.yv = ldexp(h.yv, -ex);
    }
}

// The same over a sub-interval of weight hz per unit of the two nodes' total opacities.
template <bool RENORM>
__device__ __forceinline__ void step(HalfState &h, const NodeVal &v, double hz)
{
    step_p<RENORM>(h, v, (h.chit + v.chit) * hz);
}

// Running values of a lane inside a recurrence segment (pos: the lookup position; f: the
// frame factor of the next sub-interval).
struct SubRun {
    double g, r, kq, cs, cm, S, pos, tt, f;
    double D, Q;   // clamped lookups, isotropic: node_val_lin's D and Q
};

// Jw end values of a segment whose lookups clamp: +y lookups a + t da, -y lookups a_m + t da_m.
struct JEnds {
    double ap, dap, am, dam;
    double dD, dQ;   // per sub-interval changes of node_val_lin's D and Q
};

template <bool UNI, bool ANISO, bool CLAMP, bool RENORM>
__device__ __forceinline__ void sub_step(HalfState &h, SubRun &w, double c, double dk, double dcs, double dcm,
                                         double dS, double dpos, double im, double rho, const QGeo &qg,
                                         const double *rp, const double *rq, const JEnds &je, double hz)
{
    w.g *= w.r;
    w.r *= c;
    w.kq += dk;
    w.cs += dcs;
    w.S += dS;
    if constexpr (CLAMP && !ANISO) {
        w.D += je.dD;
        w.Q += je.dQ;
        step<RENORM>(h, node_val_lin(fma(w.kq, w.g, w.cs), w.cs, w.S, w.D, w.Q), hz);
        return;
    }
    w.tt += im;
    if (ANISO) w.cm += dcm;
    double jp, jm;
    if constexpr (CLAMP) {
        jp = fma(w.tt, je.dap, je.ap);
        jm = fma(w.tt, je.dam, je.am);
    } else {
        w.pos += dpos;
        j_sub<UNI>(qg, rp, rq, w.pos, w.tt, jp, jm);
    }
    const NodeVal v = node_val<ANISO>(w.kq * w.g, w.cs, w.cm, w.S, jp, jm);
    reframe<ANISO>(h, w.f);
    if (ANISO) w.f *= rho;
    step<RENORM>(h, v, hz);
}

// e^{-x} for the frame factors, with x kept where the factor and its inverse are finite.
__device__ __forceinline__ double frame_exp(double x) { return exp_le700(fmin(fmax(-x, -700.0), 700.0)); }

// Half sweep along `ray` (lane offset x in that ray's frame, line slot gs of the `per`
// staged lines line0 ..) from the far end of its walk to O; on return h holds O's node,
// in O's frame.  jr receives the staged nodes' J_nu rows, [node][slot][n_q].
template <bool UNI, bool ANISO>
__device__ void half(const ScatArgs &a, const QGeo &qg, const double *tab, SNode *nd, SSeg *sgm, double *jr, int per, int64_t O,
                     const CellRec &cO, int ray, double x, bool live, int line0, int gs, double I_in,
                     double xq_max, HalfState &h)
{
    const int t = threadIdx.x;
    const double nx = a.dir[3 * ray], ny = a.dir[3 * ray + 1], nz = a.dir[3 * ray + 2];
    const int64_t beg = a.roff[O * a.n_rays + ray];
    const int L = (int)(a.roff[O * a.n_rays + ray + 1] - beg);   // cells; nodes 0 .. L (O)
    const double2 *lc = reinterpret_cast<const double2 *>(a.lc);
    const int rl = per * a.n_q, cslot = t / a.n_q, cq = t - cslot * a.n_q;
    double y_cur = 0.0, g_cur = 0.0, kap_cur = 0.0, cs_cur = 0.0, cm_cur = 0.0, S_cur = 0.0, travel = 0.0;
    const double *row_cur = nullptr;
    for (int b0 = 0;; b0 += kChunk - 1) {
        __syncthreads();
        // ---- stage nodes b0 .. b0 + kChunk - 1
        const int sidx = b0 + t;
        if (t < kChunk && sidx <= L) {
            const int64_t c = sidx < L ? (int64_t)a.rcells[beg + (L - 1 - sidx)] : O;
            const CellRec cc = a.cell[c];
            SNode v;
            const double dx = cc.px - cO.px, dy = cc.py - cO.py, dz = cc.pz - cO.pz;
            v.Z = (dx * nx + dy * ny) + dz * nz;
            const double dvx = cc.vx - cO.vx, dvy = cc.vy - cO.vy, dvz = cc.vz - cO.vz;
            v.s = (dvx * nx + dvy * ny) + dvz * nz;
            v.vw = cc.vw;
            v.a = cO.vw / cc.vw;
            v.b = v.s / cc.vw;
#pragma unroll
            for (int l = 0; l < 2; ++l) {
                const int ln = min(line0 + l, a.n_lines - 1);
                const double2 k = lc[c * a.n_lines + ln];
                v.kap[l] = k.x;
                v.S[l] = k.y;
                v.cs[l] = a.chi_sca[c * a.n_lines + ln];
                v.cm[l] = 0.0;
                if (ANISO) {
                    // the sweep runs toward O, against the ray's direction
                    const double *dp = a.chi_dip + 3 * (c * a.n_lines + ln);
                    v.cm[l] = -((dp[0] * nx + dp[1] * ny) + dp[2] * nz);
                }
                v.jrow[l] = a.Jin + (c * a.n_lines + ln) * a.n_q;
            }
            nd[t] = v;
        }
        __syncthreads();
        if (t < kChunk - 1 && sidx < L) {
            const SNode &p = nd[t], &q = nd[t + 1];
            // velocity sub-steps (Sec. 3.2): split when the projected velocity changes by
            // more than f_sub of the smaller line-width speed
            const double ds = fabs(q.s - p.s);
            const double thr = a.f_sub * fmin(p.vw, q.vw);
            int m = 1;
            if (ds > thr) {
                const double mr = ceil(ds / thr);
                m = mr < (double)kMaxSub ? (int)mr : kMaxSub;
            }
            SSeg e;
            e.m = m;
            e.im = 1.0 / (double)m;
            e.hz = 0.5 * kISq2 * (p.Z - q.Z) * e.im;
            e.ds = (p.Z - q.Z) * e.im;
            e.da = (q.a - p.a) * e.im;
            e.db = (q.b - p.b) * e.im;
#pragma unroll
            for (int l = 0; l < 2; ++l) {
                e.dk[l] = (q.kap[l] - p.kap[l]) * e.im;
                e.dS[l] = (q.S[l] - p.S[l]) * e.im;
                e.dcs[l] = (q.cs[l] - p.cs[l]) * e.im;
                e.dcm[l] = 0.0;
                e.f0[l] = e.rho[l] = 1.0;
                if (ANISO) {
                    e.dcm[l] = (q.cm[l] - p.cm[l]) * e.im;
                    e.f0[l] = frame_exp(e.ds * fma(0.5, e.dcm[l], p.cm[l]));
                    e.rho[l] = frame_exp(e.ds * e.dcm[l]);
                }
            }
            e.maxdx = (fabs(q.a - p.a) * xq_max + fabs(q.b - p.b)) * e.im;
            e.imdx = e.maxdx > 0.0 ? 1.0 / e.maxdx : 0.0;
            e.K = e.maxdx > 4.0 ? 0 : (e.maxdx > 0.25 ? (int)(16.0 / e.maxdx) : 64);
            sgm[t] = e;
        }
        if (t < rl) {
            // the staged nodes' J_nu rows: lane t copies entry cq of slot cslot of every node
            // (a row set per * n_q never exceeds the block)
            const int nst = min(kChunk, L - b0 + 1);
            for (int node = 0; node < nst; ++node) jr[node * rl + t] = nd[node].jrow[cslot][cq];
        }
        __syncthreads();
        // ---- sweep the staged segments
        row_cur = jr + gs * a.n_q;   // node 0 of the chunk
        if (b0 == 0) {
            y_cur = nd[0].a * x - nd[0].b;
            g_cur = profile(y_cur, tab);
            kap_cur = nd[0].kap[gs];
            cs_cur = nd[0].cs[gs];
            cm_cur = nd[0].cm[gs];
            S_cur = nd[0].S[gs];
            double jp, jm;
            j_node<UNI>(qg, row_cur, qpos<UNI>(qg, y_cur), jp, jm);
            start(h, node_val<ANISO>(kap_cur * g_cur, cs_cur, cm_cur, S_cur, jp, jm), I_in);
        }
        const int nseg = min(kChunk - 1, L - b0);
        for (int i = 0; i < nseg; ++i) {
            const int m = sgm[i].m;
            const double hz = sgm[i].hz;
            const double kap_n = nd[i + 1].kap[gs], cs_n = nd[i + 1].cs[gs], S_n = nd[i + 1].S[gs];
            const double cm_n = nd[i + 1].cm[gs];
            const double *row_n = jr + ((i + 1) * per + gs) * a.n_q;
            const double y_n = nd[i + 1].a * x - nd[i + 1].b;
            double g_n;
            double f = ANISO ? sgm[i].f0[gs] : 1.0;   // frame factor of the next sub-interval
            int end_lookup = -1;   // >= 0: the end node's lookups clamp (+y at this row index)
            if (m == 1) {
                g_n = profile(y_n, tab);
                travel = 0.0;
            } else {
                const double dy = sgm[i].da * x - sgm[i].db;
                const double dk = sgm[i].dk[gs], dS = sgm[i].dS[gs], dcs = sgm[i].dcs[gs], im = sgm[i].im;
                const double dcm = ANISO ? sgm[i].dcm[gs] : 0.0, rho = ANISO ? sgm[i].rho[gs] : 1.0;
                const double mdx = sgm[i].maxdx, imdx = sgm[i].imdx;
                const int K = sgm[i].K;
                // Every lane's offsets beyond the quadrature on one side over the whole
                // segment (x is linear in the sub-step index): both lookups clamp to the end
                // values of the rows, so Jw of a sub-node is linear in its fraction t
                bool clampJ;
                if constexpr (UNI) {
                    const double pc = qpos<UNI>(qg, y_cur), pn = qpos<UNI>(qg, y_n);
                    clampJ = (pc >= qg.top && pn >= qg.top) || (pc <= 0.0 && pn <= 0.0);
                } else {
                    const double lo = qg.qx[0], hi = qg.qx[qg.nq - 1];
                    clampJ = (y_cur >= hi && y_n >= hi) || (y_cur <= lo && y_n <= lo);
                }
                clampJ = __all(clampJ || !live);   // (lanes without a frequency do not vote)
                if (clampJ) end_lookup = y_cur > 0.0 ? qg.nq - 1 : 0;
                // (lookup of +y at ep, of -y at em; the rows' end values and their changes over t)
                const int ep = y_cur > 0.0 ? qg.nq - 1 : 0, em = qg.nq - 1 - ep;
                const double ap = row_cur[ep], am = row_cur[em];
                const double dap = row_n[ep] - ap, dam = row_n[em] - am;
                // far wing besides: e^{-y^2} is 0 in FP64 at every sub-node (no line opacity)
                const bool far = clampJ && __all(!live || (((y_cur > 0.0) == (y_n > 0.0)) && y_cur * y_cur > 750.0 &&
                                                           y_n * y_n > 750.0));
                auto sweep = [&](auto clamp_tag) {
                    constexpr bool CLAMP = decltype(clamp_tag)::value;
                    if (K == 0 || m == 2) {
                        for (int j = 1; j < m; ++j) {
                            const double fj = (double)j;
                            const double yj = fma(fj, dy, y_cur);
                            double jp, jm;
                            if constexpr (CLAMP) {
                                jp = fma(fj * im, dap, ap);
                                jm = fma(fj * im, dam, am);
                            } else {
                                j_sub<UNI>(qg, row_cur, row_n, qpos<UNI>(qg, yj), fj * im, jp, jm);
                            }
                            const NodeVal v = node_val<ANISO>(fma(fj, dk, kap_cur) * profile(yj, tab), fma(fj, dcs, cs_cur),
                                                              fma(fj, dcm, cm_cur), fma(fj, dS, S_cur), jp, jm);
                            reframe<ANISO>(h, f);
                            if (ANISO) f *= rho;
                            step<true>(h, v, hz);
                        }
                        g_n = profile(y_n, tab);
                        travel = 0.0;
                        return;
                    }
                    // g_{j+1} = g_j r_j, r_{j+1} = r_j c with r_j = e^{-2 y_j dy - dy^2} and
                    // c = e^{-2 dy^2}; exact values again whenever y may have moved by more
                    // than 16 widths since the last exact one, so that an underflowed value
                    // (|y| > 27) cannot hide a profile above e^{-121}
                    const double u2 = 2.0 * dy * dy;
                    const double c = mdx <= 0.5 ? exp_neg_small(u2) : exp_le700(-u2);
                    // (D and Q of node_val_lin at the segment's start and their changes)
                    const double D0 = fma(0.5, ap + am, -S_cur), Q0 = (0.5 * kISq2) * (am - ap);
                    const JEnds je{ap, dap, am, dam, fma(0.5 * im, dap + dam, -dS), (0.5 * kISq2 * im) * (dam - dap)};
                    SubRun w;
                    w.g = g_cur;
                    w.r = exp_tab16(fmin(-(2.0 * y_cur + dy) * dy, 700.0), tab);
                    w.kq = kap_cur;
                    w.cs = cs_cur;
                    w.cm = cm_cur;
                    w.S = S_cur;
                    w.pos = qpos<UNI>(qg, y_cur);
                    w.tt = 0.0;
                    w.f = f;
                    w.D = D0;
                    w.Q = Q0;
                    const double dpos = UNI ? dy * qg.inv_h : dy;
                    int budget = K;
                    if (mdx > 0.0) budget = (int)fmin((16.0 - travel) * imdx, (double)K);
                    if (budget < 1) {
                        w.g = profile(y_cur, tab);
                        travel = 0.0;
                        budget = K;
                    }
                    int j = 0;
                    for (;;) {
                        const int jend = min(j + budget, m);
                        const int jint = min(jend, m - 1);
                        int jj = j;
                        for (; jj + 3 < jint; jj += 4) {
                            sub_step<UNI, ANISO, CLAMP, false>(h, w, c, dk, dcs, dcm, dS, dpos, im, rho, qg, row_cur, row_n, je, hz);
                            sub_step<UNI, ANISO, CLAMP, false>(h, w, c, dk, dcs, dcm, dS, dpos, im, rho, qg, row_cur, row_n, je, hz);
                            sub_step<UNI, ANISO, CLAMP, false>(h, w, c, dk, dcs, dcm, dS, dpos, im, rho, qg, row_cur, row_n, je, hz);
                            sub_step<UNI, ANISO, CLAMP, true>(h, w, c, dk, dcs, dcm, dS, dpos, im, rho, qg, row_cur, row_n, je, hz);
                        }
                        // the last 0-3 steps; the cell node's step that follows renormalises,
                        // so at most seven steps pass between renormalisations
                        const int rem = jint - jj;
                        if (rem >= 2) {
                            sub_step<UNI, ANISO, CLAMP, false>(h, w, c, dk, dcs, dcm, dS, dpos, im, rho, qg, row_cur, row_n, je, hz);
                            sub_step<UNI, ANISO, CLAMP, false>(h, w, c, dk, dcs, dcm, dS, dpos, im, rho, qg, row_cur, row_n, je, hz);
                        }
                        if (rem & 1)
                            sub_step<UNI, ANISO, CLAMP, false>(h, w, c, dk, dcs, dcm, dS, dpos, im, rho, qg, row_cur, row_n, je, hz);
                        travel += mdx * (double)(jint - j);
                        j = jint;
                        if (jend == m) {
                            w.g *= w.r;   // the cell node at the end of the segment
                            travel += mdx;
                            break;
                        }
                        const double fj = (double)j;
                        const double yj = fma(fj, dy, y_cur);
                        w.pos = qpos<UNI>(qg, yj);
                        w.g = profile(yj, tab);
                        w.r = exp_tab16(fmin(-(2.0 * yj + dy) * dy, 700.0), tab);
                        w.kq = fma(fj, dk, kap_cur);
                        w.cs = fma(fj, dcs, cs_cur);
                        w.S = fma(fj, dS, S_cur);
                        w.tt = fj * im;
                        w.D = fma(fj, je.dD, D0);
                        w.Q = fma(fj, je.dQ, Q0);
                        if (ANISO) {
                            w.cm = fma(fj, dcm, cm_cur);
                            w.f = frame_exp(sgm[i].ds * fma(fj + 0.5, dcm, cm_cur));
                        }
                        travel = 0.0;
                        budget = K;
                    }
                    g_n = w.g;
                    f = w.f;
                };
                if (far) {
                    // no line opacity anywhere in the segment: each sub-node is the scattering
                    // term alone, S+ = Jbar and sigma~ = dJ (sqrt 2 sq), linear in the sub-node
                    // index like Jw and chi_s (r = 1 wherever chi_s > 0: at every sub-node when
                    // either end has scattering, linear interpolation keeping it positive);
                    // without scattering at either end, S+ = S (no opacity, r = 0) and sigma~ = 0
                    const double on = (cs_cur > 0.0 || nd[i + 1].cs[gs] > 0.0) ? 1.0 : 0.0;
                    const double Sp0 = on > 0.0 ? 0.5 * (ap + am) : S_cur, dSp = on > 0.0 ? (0.5 * im) * (dap + dam) : dS;
                    const double sq0 = (0.5 * kISq2 * on) * (am - ap), dsq = (0.5 * kISq2 * on * im) * (dam - dap);
                    // the sub-interval ending at sub-node j has P = (chi_{j-1} + chi_j) hz, linear in j
                    const double dP = 2.0 * dcs * hz, P0 = (2.0 * cs_cur - dcs) * hz;
                    auto far_step = [&](int j, auto renorm_tag) {
                        const double fj = (double)j;
                        NodeVal v;
                        v.chit = fma(fj, dcs, cs_cur);
                        v.Sp = fma(fj, dSp, Sp0);
                        v.sq = fma(fj, dsq, sq0);
                        if (ANISO) {
                            const double cm = fma(fj, dcm, cm_cur);
                            const double jb = fma(fj * im, dap + dam, ap + am), dj = fma(fj * im, dam - dap, am - ap);
                            const double rm = v.chit > 0.0 ? cm * rcp_refined(v.chit) : 0.0;
                            v.Sp = fma(0.5 * rm, dj, v.Sp);
                            v.sq = fma(0.5 * kISq2 * rm, jb, v.sq);
                        }
                        reframe<ANISO>(h, f);
                        if (ANISO) f *= rho;
                        step_p<decltype(renorm_tag)::value>(h, v, fma(fj, dP, P0));
                    };
                    if constexpr (ANISO) {
                        int j = 1;
                        for (; j + 3 < m; j += 4) {
                            far_step(j, std::false_type{});
                            far_step(j + 1, std::false_type{});
                            far_step(j + 2, std::false_type{});
                            far_step(j + 3, std::true_type{});
                        }
                        for (; j < m; ++j) far_step(j, std::false_type{});
                    } else {
                        // sub-nodes 1 and 2 by the general step: their central differences reach
                        // back to the cell node, whose values need not lie on the line
                        far_step(1, std::false_type{});
                        if (m > 2) far_step(2, std::false_type{});
                        if (m > 3) {
                            // from sub-node 3 on both neighbours of the eliminated sub-node lie on
                            // the line: the sigma~ and S+ differences across it are the constants
                            // -2 dsq and -2 dSp (the v-equation takes half the latter, cv), and
                            // P_{j-1} + P_j grows by 2 dP per sub-node
                            double n = h.n, d = h.d, y = h.y, yv = h.yv, Sh = h.Sp, qh = h.sq;
                            const double cy = -2.0 * dsq, cv = -dSp, dQ = 2.0 * dP, Q0 = fma(2.0, P0, -dP);
                            double fj = 3.0;
                            auto lean = [&](auto renorm_tag) {
                                const double hd = fma(fj, dQ, Q0) * d;
                                n += hd;
                                y = fma(Sh, hd, fma(cy, d, y));
                                yv = fma(qh, hd, fma(cv, d, yv));
                                d = fma(fma(fj, dP, P0), n, d);
                                Sh = fma(fj, dSp, Sp0);
                                qh = fma(fj, dsq, sq0);
                                fj += 1.0;
                                if (decltype(renorm_tag)::value) {
                                    const int ex = __builtin_amdgcn_frexp_exp(d);
                                    n = ldexp(n, -ex);
                                    d = ldexp(d, -ex);
                                    y = ldexp(y, -ex);
                                    yv = ldexp(yv, -ex);
                                }
                            };
                            int j = 3;
                            for (; j + 3 < m; j += 4) {
                                lean(std::false_type{});
                                lean(std::false_type{});
                                lean(std::false_type{});
                                lean(std::true_type{});
                            }
                            for (; j < m; ++j) lean(std::false_type{});
                            // the state after sub-node m - 1, as the general step leaves it
                            const double fl = (double)(m - 1);
                            h.n = n;
                            h.d = d;
                            h.y = y;
                            h.yv = yv;
                            h.Pm = fma(fl, dP, P0);
                            h.chit = fma(fl, dcs, cs_cur);
                            h.Sp = Sh;
                            h.sq = qh;
                            h.Sp_pp = fma(fl - 1.0, dSp, Sp0);
                            h.sq_pp = fma(fl - 1.0, dsq, sq0);
                        }
                    }
                    g_n = 0.0;   // e^{-y_n^2} underflows too
                    travel = 0.0;
                } else if (clampJ) {
                    sweep(std::true_type{});
                } else {
                    sweep(std::false_type{});
                }
            }
            double jp, jm;
            if (end_lookup >= 0) {
                jp = row_n[end_lookup];
                jm = row_n[qg.nq - 1 - end_lookup];
            } else {
                j_node<UNI>(qg, row_n, qpos<UNI>(qg, y_n), jp, jm);
            }
            const NodeVal vn = node_val<ANISO>(kap_n * g_n, cs_n, cm_n, S_n, jp, jm);
            reframe<ANISO>(h, f);
            step<true>(h, vn, hz);
            y_cur = y_n;
            g_cur = g_n;
            kap_cur = kap_n;
            cs_cur = cs_n;
            cm_cur = cm_n;
            S_cur = S_n;
            row_cur = row_n;
        }
        if (b0 + kChunk - 1 >= L) break;
    }
}

}  // namespace

// Every form is held to two waves per SIMD: the isotropic one on an evenly spaced quadrature
// then needs no spill (at three it spills and runs slower); the others spill (45 to 83 VGPRs)
// and still run a third or more faster than at one wave (outflow5 sweeps: with a dipole
// 336 -> 225 ms; on 24 Gauss-Hermite offsets 491 -> 275 ms, with a dipole 567 -> 346 ms).
template <bool UNI, bool ANISO>
__global__ __launch_bounds__(kScatMaxQ, 2) void k_formal_solve_scat(ScatArgs a)
{
    extern __shared__ double smem[];
    // lanes: with n_q <= 32 two lines per wave (lanes 32 g + frequency), else one line
    const int nq = a.n_q, t = threadIdx.x, nt = blockDim.x;
    double *s_tab = smem;        // [16] 2^{j/16} for the exponential
    double *s_qx = smem + 16;
    SNode *nd = reinterpret_cast<SNode *>(smem + 16 + nq);
    SSeg *sgm = reinterpret_cast<SSeg *>(nd + kChunk);
    double *jr = reinterpret_cast<double *>(sgm + kChunk);   // [kChunk][per][n_q]
    double *s_red = smem + 16 + nq;   // after the sweeps: [5][nt] over the staging area
    const int per = nq <= 32 ? 2 : 1;
    const int groups = (a.n_lines + per - 1) / per;
    const int64_t O = blockIdx.x / groups;
    const int line0 = (int)(blockIdx.x - O * groups) * per;
    const int g = per == 2 ? t >> 5 : 0;
    const int fi = t - 32 * g;
    const int line = line0 + g;
    const bool act = fi < nq && line < a.n_lines;
    const int lc_line = line < a.n_lines ? line : a.n_lines - 1;
    const int64_t row = O * a.n_lines + lc_line;
    if (a.model_done != nullptr && a.model_done[a.model_of[O]]) {
        // converged model: its J_nu carries over unchanged
        if (act) a.Jout[row * nq + fi] = a.Jin[row * nq + fi];
        return;
    }
    if (t < nq) s_qx[t] = a.qx[t];
    if (t < 16) s_tab[t] = kExp2Sixteenths[t];
    __syncthreads();
    QGeo qg;
    qg.qx = s_qx;
    qg.nq = nq;
    qg.lo_max = nq - 2;
    qg.top = (double)(nq - 1);
    qg.inv_h = a.q_inv_h;
    qg.mx0 = -s_qx[0] * a.q_inv_h;
    const double xq_max = fmax(fabs(s_qx[0]), fabs(s_qx[nq - 1]));
    const double x = fi < nq ? s_qx[fi] : 0.0;
    const double w = act ? a.qw[fi] : 0.0;
    const CellRec cO = a.cell[O];
    const double I_in = a.ibdy[lc_line];
    const double2 lcO = reinterpret_cast<const double2 *>(a.lc)[row];
    // direction weights of the re-emitted field at O: w(+-n) = 1 +- e . n, e = chi_dip/chi_s
    double ex = 0.0, ey = 0.0, ez = 0.0;
    if (ANISO) {
        const double cs = a.chi_sca[row];
        if (cs > 0.0) {
            const double *dp = a.chi_dip + 3 * row;
            ex = dp[0] / cs;
            ey = dp[1] / cs;
            ez = dp[2] / cs;
        }
    }
    double accJ = 0.0, accL = 0.0, accE = 0.0, jp = 0.0, jm = 0.0;
    for (int p = 0; p < a.n_pairs; ++p) {
        const int r = a.pair_r[p], rb = a.anti[r];
        HalfState f, b;
        half<UNI, ANISO>(a, qg, s_tab, nd, sgm, jr, per, O, cO, r, x, act, line0, g, I_in, xq_max, f);
        half<UNI, ANISO>(a, qg, s_tab, nd, sgm, jr, per, O, cO, rb, -x, act, line0, g, I_in, xq_max, b);
        // combine at O: h u + (Q_f u - y_f) + (Q_b u - y_b) = h R_O (scaled rows)
        const double idf = 1.0 / f.d, idb = 1.0 / b.d;
        const double h = f.Pm + b.Pm;
        const double yy = f.y * idf + b.y * idb;
        const double sgO = f.sq_pp + b.sq_pp;
        const double inv = 1.0 / (h + f.n * idf + b.n * idb);
        const double u = (h * f.Sp + yy + sgO) * inv;
        // line part of O's own source, for L* and Jeff (Eq. ALO)
        const double clO = lcO.x * profile(x, s_tab);
        const double ratio = f.chit > 0.0 ? clO / f.chit : 1.0;   // all of it without opacity
        accJ += w * u;
        accL += w * (h * inv) * ratio;
        accE += w * ((h * (f.Sp - ratio * lcO.y) + yy + sgO) * inv);
        // v along n = ray r, the sweep direction of half b, from the v-equation: the same
        // combine with b's particular solution and f's with the sign of the other
        // orientation, sigma~_O (b's) in place of S+_O and the S+ difference across O
        const double v = kSq2 * ((h * b.sq + (b.yv * idb - f.yv * idf) + (b.Sp_pp - f.Sp_pp) * 0.5) * inv);
        double wp = 1.0, wm = 1.0;
        if (ANISO) {
            const double en = (ex * a.dir[3 * r] + ey * a.dir[3 * r + 1]) + ez * a.dir[3 * r + 2];
            wp += en;
            wm -= en;
        }
        jp += wp * (u + v);
        jm += wm * (u - v);
    }
    __syncthreads();   // the staging area becomes the reduction area
    s_red[t] = act ? accJ : 0.0;
    s_red[nt + t] = act ? accL : 0.0;
    s_red[2 * nt + t] = act ? accE : 0.0;
    s_red[3 * nt + t] = jp;
    s_red[4 * nt + t] = jm;
    __syncthreads();
    const int base = 32 * g;
    if (fi == 0 && line < a.n_lines) {
        double sJ = 0.0, sL = 0.0, sE = 0.0;
        for (int i = 0; i < nq; ++i) {
            sJ += s_red[base + i];
            sL += s_red[nt + base + i];
            sE += s_red[2 * nt + base + i];
        }
        a.J[row] = a.norm * sJ;
        a.L[row] = a.norm * sL;
        a.Jeff[row] = a.norm * sE;
    }
    if (act) a.Jout[row * nq + fi] = (s_red[3 * nt + t] + s_red[4 * nt + base + nq - 1 - fi]) * a.inv_rays;
}

// J_nu of the first scattering iteration: the boundary intensity of each line everywhere.
__global__ void k_jnu_start(const double *__restrict__ ibdy, int64_t n, int n_lines, int n_q, double *__restrict__ jnu)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (i >= n) return;
    jnu[i] = ibdy[(i / n_q) % n_lines];
}

hipError_t launch_jnu_start(const double *ibdy, int64_t P, int n_lines, int n_q, double *jnu, hipStream_t s)
{
    const int64_t n = P * n_lines * n_q;
    if (n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_jnu_start, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, ibdy, n, n_lines, n_q, jnu);
    return hipGetLastError();
}

hipError_t launch_formal_solve_scat(const ScatArgs &a, hipStream_t s)
{
    if (a.P == 0) return hipSuccess;
    if (a.n_q < 1 || a.n_q > kScatMaxQ) return hipErrorInvalidValue;
    if (a.q_uniform && a.n_q < 2) return hipErrorInvalidValue;
    const int per = a.n_q <= 32 ? 2 : 1;
    const int threads = per == 2 ? kWave : (a.n_q + kWave - 1) / kWave * kWave;
    const int64_t groups = (a.n_lines + per - 1) / per;
    const size_t stage = kChunk * (sizeof(SNode) + sizeof(SSeg) + sizeof(double) * (size_t)per * a.n_q);
    const size_t red = 5 * sizeof(double) * (size_t)threads;
    const size_t shmem = sizeof(double) * (16 + (size_t)a.n_q) + (stage > red ? stage : red);
    const dim3 grid((unsigned)(a.P * groups));
    if (a.chi_dip != nullptr) {
        if (a.q_uniform)
            hipLaunchKernelGGL((k_formal_solve_scat<true, true>), grid, dim3(threads), shmem, s, a);
        else
            hipLaunchKernelGGL((k_formal_solve_scat<false, true>), grid, dim3(threads), shmem, s, a);
    } else {
        if (a.q_uniform)
            hipLaunchKernelGGL((k_formal_solve_scat<true, false>), grid, dim3(threads), shmem, s, a);
        else
            hipLaunchKernelGGL((k_formal_solve_scat<false, false>), grid, dim3(threads), shmem, s, a);
    }
    return hipGetLastError();
}

}  // namespace nlte
