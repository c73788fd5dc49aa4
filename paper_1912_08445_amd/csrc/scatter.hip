// Formal solve with scattering: the u-equation of the generalised Feautrier form
// (Sec. 3.3, Eq. GFE) for an isotropic scattering opacity chi_s (chi^- = 0), grey over a
// line's frequencies, scattering coherently and isotropically in each point's comoving
// frame, with the right-hand sides from the previous iteration's mean intensity J_nu
// (Sec. 3.3: the Psi terms are evaluated with the previous solution).
//
// At a node whose comoving offset is y (line widths of that node) the photon of the
// sweep's own direction sees chi_s J(y) and the one of the opposite direction chi_s J(-y),
// so with chi_t = chi_line + chi_s
//   S+ = (chi_line S + chi_s (J(y) + J(-y))/2) / chi_t,
//   sigma~ = chi_s (J(-y) - J(y))/2 / chi_t   (Psi^-/chi_t along the sweep direction),
// and the interior rows of the second-order system gain -d sigma/dtau as the central
// difference over the two neighbours; the boundary rows gain the half-node value of sigma.
// J(y) is linear in y between the quadrature offsets (constant beyond them; the offset is
// located once for both end cells of a sub-step segment, by direct index on an evenly
// spaced quadrature and by bisection otherwise); velocity
// sub-steps interpolate chi_s and the end cells' J linearly in t at their own offset.
//
// One workgroup per point and line (two lines, in lanes 0-31 and 32-63, when n_q <= 32),
// one lane per frequency (n_q <= 256 lanes).  Each lane
// eliminates both halves of every ray pair from the far ends toward the origin in the
// division-free scaled state of the line formal solve (n, d, y~ with node coefficients
// chi dz/(2 sqrt 2)), FP64 with a direct exponential at every node, and combines them at
// the origin.  Besides J, L* (times chi_line/chi_t) and Jeff it returns J_nu at the
// quadrature offsets from u and the flux-like v at the origin: I(n, x) = u(x) + v(x) and
// I(-n, x) = u(-x) - v(-x) for the pair representative n.
#include "nlte_internal.h"
#include "device_math.h"

namespace nlte {

namespace {

constexpr int kScatMaxQ = 256;
constexpr double kSq2 = 1.41421356237309504880;
constexpr double kISq2 = 0.70710678118654752440;

// Position of offset y on the quadrature: J(y) = row[i0] + t (row[i1] - row[i0]) with
// qx[i0] <= y < qx[i1], or i0 = i1 at the outermost offset beyond which J is constant.
struct QPos {
    int i0, i1;
    double t;
};

struct QGrid {
    const double *qx;   // in LDS
    int nq;
    bool uniform;       // evenly spaced: direct index, then at most a step of fix-up
    double x0, inv_h;
};

__device__ inline QPos locate(const QGrid &g, double y)
{
    const double *qx = g.qx;
    const int nq = g.nq;
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
    int lo;
    if (g.uniform) {
        lo = (int)floor((y - g.x0) * g.inv_h);
        lo = lo < 0 ? 0 : (lo > nq - 2 ? nq - 2 : lo);
        while (lo > 0 && qx[lo] > y) --lo;
        while (lo < nq - 2 && qx[lo + 1] <= y) ++lo;
    } else {
        lo = 0;
        int hi = nq - 1;   // qx[lo] <= y < qx[hi]
        while (hi - lo > 1) {
            const int mid = (lo + hi) >> 1;
            if (qx[mid] <= y)
                lo = mid;
            else
                hi = mid;
        }
    }
    p.i0 = lo;
    p.i1 = lo + 1;
    p.t = g.uniform ? (y - qx[lo]) * g.inv_h : (y - qx[lo]) / (qx[lo + 1] - qx[lo]);
    return p;
}

__device__ inline double j_at(const double *__restrict__ row, const QPos &p)
{
    const double r0 = row[p.i0];
    return r0 + p.t * (row[p.i1] - r0);
}

// Base node of a half sweep in the walk frame of its ray.
struct Base {
    double Z, s, vw, a, b, kap, S, cs;
    const double *jrow;
};

__device__ inline Base base_node(const ScatArgs &a, const CellRec &cO, int64_t c, double nx, double ny, double nz,
                                 int line)
{
    const CellRec cc = a.cell[c];
    Base d;
    const double dx = cc.px - cO.px, dy = cc.py - cO.py, dz = cc.pz - cO.pz;
    d.Z = (dx * nx + dy * ny) + dz * nz;
    const double dvx = cc.vx - cO.vx, dvy = cc.vy - cO.vy, dvz = cc.vz - cO.vz;
    d.s = (dvx * nx + dvy * ny) + dvz * nz;
    d.vw = cc.vw;
    d.a = cO.vw / cc.vw;
    d.b = d.s / cc.vw;
    const double2 lc = reinterpret_cast<const double2 *>(a.lc)[c * a.n_lines + line];
    d.kap = lc.x;
    d.S = lc.y;
    d.cs = a.chi_sca[c * a.n_lines + line];
    d.jrow = a.Jin + (c * a.n_lines + line) * a.n_q;
    return d;
}

// Node quantities at the lane's frequency: total opacity, S+ and sigma~.
struct NodeVal {
    double Z, chit, Sp, sg;
};

// S+ = S + r (Jbar - S) and sigma~ = r (J(-y) - J(y))/2 with r = chi_s/chi_t, the
// scattering share (one division, safe for denormal far-wing opacities).
__device__ inline NodeVal node_val(double Z, double cl, double cs, double S, double jp, double jm)
{
    NodeVal v;
    v.Z = Z;
    v.chit = cl + cs;
    const double r = cs > 0.0 ? cs * rcp_refined(v.chit) : 0.0;   // chit >= cs > 0
    v.Sp = v.chit > 0.0 ? S + r * (0.5 * (jp + jm) - S) : 0.0;
    v.sg = r * 0.5 * (jm - jp);
    return v;
}

__device__ inline NodeVal eval_base(const Base &d, double x, const QGrid &g)
{
    const double y = d.a * x - d.b;
    const double cl = d.kap * exp(-(y * y));
    const double jp = j_at(d.jrow, locate(g, y)), jm = j_at(d.jrow, locate(g, -y));
    return node_val(d.Z, cl, d.cs, d.S, jp, jm);
}

// Sub-step node at fraction t from base p toward base q.
__device__ inline NodeVal eval_sub(const Base &p, const Base &q, double t, double x, const QGrid &g)
{
    const double aa = p.a + t * (q.a - p.a), bb = p.b + t * (q.b - p.b);
    const double y = aa * x - bb;
    const double cl = (p.kap + t * (q.kap - p.kap)) * exp(-(y * y));
    const double cs = (1.0 - t) * p.cs + t * q.cs;
    const double S = p.S + t * (q.S - p.S);
    const QPos lp = locate(g, y), lm = locate(g, -y);
    const double jp = (1.0 - t) * j_at(p.jrow, lp) + t * j_at(q.jrow, lp);
    const double jm = (1.0 - t) * j_at(p.jrow, lm) + t * j_at(q.jrow, lm);
    return node_val(p.Z + t * (q.Z - p.Z), cl, cs, S, jp, jm);
}

// Elimination state of a half sweep; `prev` is the last node reached.
struct HalfState {
    double n, d, y, Pm;
    NodeVal prev;
    double sg_pp;   // sigma~ of the node before prev (virtual -sigma~ at the far end)
};

__device__ inline void start(HalfState &h, const NodeVal &first, double I_in)
{
    h.n = kSq2;
    h.d = 1.0;
    h.y = kSq2 * I_in;
    h.Pm = 0.0;
    h.prev = first;
    h.sg_pp = -first.sg;
}

// Eliminate h.prev, stepping to node cur.
__device__ inline void step(HalfState &h, const NodeVal &cur)
{
    const double P = 0.5 * (h.prev.chit + cur.chit) * (h.prev.Z - cur.Z) * kISq2;
    const double hd = (h.Pm + P) * h.d;
    h.n += hd;
    h.y = h.y + h.prev.Sp * hd - (cur.sg - h.sg_pp) * h.d * kISq2;
    h.d = fma(P, h.n, h.d);
    h.Pm = P;
    const int ex = __builtin_amdgcn_frexp_exp(h.d);
    h.n = ldexp(h.n, -ex);
    h.d = ldexp(h.d, -ex);
    h.y = ldexp(h.y, -ex);
    h.sg_pp = h.prev.sg;
    h.prev = cur;
}

// Half sweep along `ray` (lane offset x in that ray's frame) from the far end of its
// walk to O; on return h.prev is O's node.
__device__ inline void half(const ScatArgs &a, const QGrid &g, int64_t O, const CellRec &cO, int ray, double x,
                            int line, double I_in, HalfState &h)
{
    const double nx = a.dir[3 * ray], ny = a.dir[3 * ray + 1], nz = a.dir[3 * ray + 2];
    const int64_t beg = a.roff[O * a.n_rays + ray], end = a.roff[O * a.n_rays + ray + 1];
    Base prev = base_node(a, cO, end > beg ? (int64_t)a.rcells[end - 1] : O, nx, ny, nz, line);
    start(h, eval_base(prev, x, g), I_in);
    for (int64_t i = end - 1; i >= beg; --i) {
        const Base cur = base_node(a, cO, i > beg ? (int64_t)a.rcells[i - 1] : O, nx, ny, nz, line);
        // velocity sub-steps (Sec. 3.2): split when the projected velocity changes by more
        // than f_sub of the smaller line-width speed
        const double ds = fabs(cur.s - prev.s);
        const double thr = a.f_sub * fmin(prev.vw, cur.vw);
        int m = 1;
        if (ds > thr) {
            const double mr = ceil(ds / thr);
            m = mr < (double)kMaxSub ? (int)mr : kMaxSub;
        }
        if (m > 1) {
            const double inv_m = 1.0 / (double)m;
            for (int j = 1; j < m; ++j) step(h, eval_sub(prev, cur, (double)j * inv_m, x, g));
        }
        step(h, eval_base(cur, x, g));
        prev = cur;
    }
}

}  // namespace

__global__ __launch_bounds__(kScatMaxQ) void k_formal_solve_scat(ScatArgs a)
{
    __shared__ double s_qx[kScatMaxQ];
    __shared__ double s_red[3][kScatMaxQ];
    __shared__ double s_jp[kScatMaxQ], s_jm[kScatMaxQ];
    // lanes: with n_q <= 32 two lines per wave (lanes 32 g + frequency), else one line
    const int nq = a.n_q, t = threadIdx.x;
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
    __syncthreads();
    QGrid qg;
    qg.qx = s_qx;
    qg.nq = nq;
    qg.uniform = a.q_uniform != 0;
    qg.x0 = s_qx[0];
    qg.inv_h = a.q_inv_h;
    const double x = fi < nq ? s_qx[fi] : 0.0;
    const double w = act ? a.qw[fi] : 0.0;
    const CellRec cO = a.cell[O];
    const double I_in = a.ibdy[lc_line];
    const double2 lcO = reinterpret_cast<const double2 *>(a.lc)[row];
    double accJ = 0.0, accL = 0.0, accE = 0.0, jp = 0.0, jm = 0.0;
    for (int p = 0; p < a.n_pairs; ++p) {
        const int r = a.pair_r[p], rb = a.anti[r];
        HalfState f, b;
        half(a, qg, O, cO, r, x, lc_line, I_in, f);
        half(a, qg, O, cO, rb, -x, lc_line, I_in, b);
        // combine at O: h u + (Q_f u - y_f) + (Q_b u - y_b) = h R_O (scaled rows)
        const double idf = 1.0 / f.d, idb = 1.0 / b.d;
        const double h = f.Pm + b.Pm;
        const double yy = f.y * idf + b.y * idb;
        const double sgO = (f.sg_pp + b.sg_pp) * kISq2;
        const double inv = 1.0 / (h + f.n * idf + b.n * idb);
        const double u = (h * f.prev.Sp + yy + sgO) * inv;
        // line part of O's own source, for L* and Jeff (Eq. ALO)
        const double clO = lcO.x * exp_le700(-(x * x));
        const double ratio = f.prev.chit > 0.0 ? clO / f.prev.chit : 1.0;   // all of it without opacity
        accJ += w * u;
        accL += w * (h * inv) * ratio;
        accE += w * ((h * (f.prev.Sp - ratio * lcO.y) + yy + sgO) * inv);
        // v along n = ray r: the half-node fluxes (u_O - u_nb)/dtau on each side from the
        // elimination state, with sigma at the half nodes, interpolated in tau to O
        const double fl_f = (f.n * u - f.y) * idf * kISq2 - 0.5 * (f.sg_pp + f.prev.sg);
        const double fl_b = (b.n * u - b.y) * idb * kISq2 - 0.5 * (b.sg_pp + b.prev.sg);
        const double v = h > 0.0 ? (b.Pm * fl_f - f.Pm * fl_b) / h : 0.5 * (fl_f - fl_b);
        jp += u + v;
        jm += u - v;
    }
    s_red[0][t] = act ? accJ : 0.0;
    s_red[1][t] = act ? accL : 0.0;
    s_red[2][t] = act ? accE : 0.0;
    s_jp[t] = jp;
    s_jm[t] = jm;
    __syncthreads();
    const int base = 32 * g;
    if (fi == 0 && line < a.n_lines) {
        double sJ = 0.0, sL = 0.0, sE = 0.0;
        for (int i = 0; i < nq; ++i) {
            sJ += s_red[0][base + i];
            sL += s_red[1][base + i];
            sE += s_red[2][base + i];
        }
        a.J[row] = a.norm * sJ;
        a.L[row] = a.norm * sL;
        a.Jeff[row] = a.norm * sE;
    }
    if (act) a.Jout[row * nq + fi] = (s_jp[t] + s_jm[base + nq - 1 - fi]) * a.inv_rays;
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
    const int per = a.n_q <= 32 ? 2 : 1;
    const int threads = per == 2 ? kWave : (a.n_q + kWave - 1) / kWave * kWave;
    const int64_t groups = (a.n_lines + per - 1) / per;
    hipLaunchKernelGGL(k_formal_solve_scat, dim3((unsigned)(a.P * groups)), dim3(threads), 0, s, a);
    return hipGetLastError();
}

}  // namespace nlte
