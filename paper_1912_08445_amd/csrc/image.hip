// Images of the model (Sec. 3.5): the intensity leaving the model along an image
// direction n at the far end of the ray pair through every point, at observer-frame
// channel velocities v.  The pixel of point O sits at O's projection on the plane
// orthogonal to n.
//
// Along the pair (the cached walk of the antipode from its far end to O, then the walk
// of n outward) the profile offset at node k is x_k = (v - n.v_k)/v_w,k.  The
// second-order system of the pair (Sec. 3.3) is eliminated from the upwind end to the
// emergent end E, which plays the part of the origin with an empty far side, so that
//   u_E = (h_E S_E + y + I_in) / (h_E + Q + 1),   I_out = 2 u_E - I_in
// (u = (I(n) + I(-n))/2 with the CMB entering at E).  The elimination uses the
// division-free scaled state of the formal solve (n, d, y~ with Q = n/(sqrt 2 d),
// y = y~/(sqrt 2 d), P = D_+/sqrt 2) in FP64; velocity sub-steps interpolate z, the
// Doppler coefficients, kappa and S linearly as in the formal solve.
//
// One wave per point and block of 64 channels, one channel per lane.  The wave stages up
// to 64 nodes of the pair at a time in LDS (gathered by the lanes together) and sweeps
// them with uniform control flow.  Inside a sub-step segment the offset is linear in the
// step index, so e^{-x^2} follows the multiplicative recurrence g <- g r, r <- r c with
// exact restarts after at most 16 widths of travel; cell nodes and short segments
// evaluate the exponential directly.  The state is renormalised by a power of two at
// every cell node and every fourth sub-step.
#include "nlte_internal.h"
#include "device_math.h"

namespace nlte {

namespace {

constexpr double kSqrt2i = 1.41421356237309504880;
constexpr double kInvSqrt2 = 0.70710678118654752440;

// Staged base node (sweep order): projection z on n relative to O, Doppler coefficients
// x = a x_O - b in O's frame, line coefficients, projected velocity s and line-width speed.
struct ImgNode {
    double z, a, b, kap, S, s, vw;
};

// Segment from a staged node to the next: m sub-intervals of optical-depth weight
// hz = (z_next - z)/(2 sqrt 2 m); per sub-interval the offset changes by da x_O - db and
// kappa hz by dkq, S by dS.  maxdx bounds |dx| over the block's channels, K is the
// restart interval of the profile recurrence (0: direct evaluation).
struct ImgSeg {
    double hz, da, db, dkq, dS, maxdx;
    int m, K;
};

// e^{-x^2}; the argument is clamped where the result is 0 in FP64 anyway, so that any
// finite channel velocity stays inside the exponential's range.
__device__ __forceinline__ double profile(double x) { return exp_le700(fmax(-(x * x), -800.0)); }

struct Elim {
    double n, d, y, Pm;   // scaled elimination state and the previous step's P
    double q, S;          // chi hz and S of the last node
};

template <bool RENORM>
__device__ __forceinline__ void elim(Elim &e, double q, double S)
{
    const double P = e.q + q;
    const double hd = (e.Pm + P) * e.d;
    e.n += hd;
    e.y = fma(e.S, hd, e.y);
    e.d = fma(P, e.n, e.d);
    e.Pm = P;
    e.q = q;
    e.S = S;
    if (RENORM) {
        const int ex = __builtin_amdgcn_frexp_exp(e.d);
        e.n = ldexp(e.n, -ex);
        e.d = ldexp(e.d, -ex);
        e.y = ldexp(e.y, -ex);
    }
}

template <bool RENORM>
__device__ __forceinline__ void recur(Elim &e, double &g, double &r, double c, double &kq, double dkq, double &St,
                                      double dS)
{
    g *= r;
    r *= c;
    kq += dkq;
    St += dS;
    elim<RENORM>(e, kq * g, St);
}

}  // namespace

__global__ __launch_bounds__(64) void k_image(ImageArgs a)
{
    __shared__ ImgNode nd[kWave];
    __shared__ ImgSeg sg[kWave];
    const int chunks = (a.n_ch + kWave - 1) / kWave;
    const int64_t O = blockIdx.x / chunks;
    const int lane = threadIdx.x;
    const int ch = (int)(blockIdx.x % chunks) * kWave + lane;
    if (O >= a.P) return;
    const bool act = ch < a.n_ch;
    const double nx = a.dir[3 * a.ray], ny = a.dir[3 * a.ray + 1], nz = a.dir[3 * a.ray + 2];
    const CellRec cO = a.cell[O];
    const double xO = act ? (a.v_ch[ch] - ((cO.vx * nx + cO.vy * ny) + cO.vz * nz)) / cO.vw : 0.0;
    double xmax = fabs(xO);
    for (int o = kWave / 2; o > 0; o >>= 1) xmax = fmax(xmax, __shfl_xor(xmax, o));
    const double2 *lc = reinterpret_cast<const double2 *>(a.lc);

    // base nodes in sweep order: the antipode's walk from its far end, O, the walk along n
    const int rb = a.anti[a.ray];
    const int64_t bb = a.roff[O * a.n_rays + rb], be = a.roff[O * a.n_rays + rb + 1];
    const int64_t fb = a.roff[O * a.n_rays + a.ray];
    const int nb = (int)(be - bb);
    const int Ls = nb + (int)(a.roff[O * a.n_rays + a.ray + 1] - fb);   // segments

    Elim e;
    e.n = kSqrt2i;
    e.d = 1.0;
    e.y = kSqrt2i * a.I_in;
    e.Pm = 0.0;
    e.q = 0.0;
    e.S = 0.0;
    double x_cur = 0.0, g_cur = 0.0, chi_cur = 0.0, kap_cur = 0.0, travel = 0.0;
    for (int b0 = 0; b0 < Ls; b0 += kWave - 1) {
        __syncthreads();
        // ---- stage nodes b0 .. b0 + 63
        const int sidx = b0 + lane;
        if (sidx <= Ls) {
            const int64_t c = sidx < nb ? (int64_t)a.rcells[be - 1 - sidx]
                                        : (sidx == nb ? O : (int64_t)a.rcells[fb + (sidx - nb - 1)]);
            const CellRec cc = a.cell[c];
            ImgNode v;
            const double dx = cc.px - cO.px, dy = cc.py - cO.py, dz = cc.pz - cO.pz;
            v.z = (dx * nx + dy * ny) + dz * nz;
            const double dvx = cc.vx - cO.vx, dvy = cc.vy - cO.vy, dvz = cc.vz - cO.vz;
            v.s = (dvx * nx + dvy * ny) + dvz * nz;
            v.vw = cc.vw;
            v.a = cO.vw / cc.vw;
            v.b = v.s / cc.vw;
            const double2 k = lc[c * a.n_lines + a.line];
            v.kap = k.x;
            v.S = k.y;
            nd[lane] = v;
        }
        __syncthreads();
        if (sidx < Ls && lane < kWave - 1) {
            const ImgNode p = nd[lane], q = nd[lane + 1];
            // velocity sub-steps (Sec. 3.2): split when the projected velocity changes by
            // more than f_sub of the smaller line-width speed
            const double ds = fabs(q.s - p.s);
            const double thr = a.f_sub * fmin(p.vw, q.vw);
            int m = 1;
            if (ds > thr) {
                const double mr = ceil(ds / thr);
                m = mr < (double)kMaxSub ? (int)mr : kMaxSub;
            }
            const double im = 1.0 / (double)m;
            ImgSeg t;
            t.m = m;
            t.hz = 0.5 * kInvSqrt2 * (q.z - p.z) * im;
            t.da = (q.a - p.a) * im;
            t.db = (q.b - p.b) * im;
            t.dkq = (q.kap - p.kap) * im * t.hz;
            t.dS = (q.S - p.S) * im;
            t.maxdx = (fabs(q.a - p.a) * xmax + fabs(q.b - p.b)) * im;
            t.K = t.maxdx > 4.0 ? 0 : (t.maxdx > 0.25 ? (int)(16.0 / t.maxdx) : 64);
            sg[lane] = t;
        }
        __syncthreads();
        // ---- sweep the staged segments
        const int nseg = min(kWave - 1, Ls - b0);
        if (b0 == 0) {
            x_cur = nd[0].a * xO - nd[0].b;
            g_cur = profile(x_cur);
            kap_cur = nd[0].kap;
            chi_cur = kap_cur * g_cur;
            e.S = nd[0].S;
        }
        for (int i = 0; i < nseg; ++i) {
            const ImgSeg t = sg[i];
            const double kn = nd[i + 1].kap, Sn = nd[i + 1].S;
            const double xn = nd[i + 1].a * xO - nd[i + 1].b;
            const double hz = t.hz;
            e.q = chi_cur * hz;   // the last node's weight in this segment's steps
            double gn;
            if (t.m == 1) {
                gn = profile(xn);
                travel = 0.0;
            } else {
                const double dx = t.da * xO - t.db;
                const double kq0 = kap_cur * hz, S0 = e.S;
                if (t.K == 0 || t.m == 2) {
                    for (int j = 1; j < t.m; ++j) {
                        const double fj = (double)j;
                        elim<true>(e, fma(fj, t.dkq, kq0) * profile(fma(fj, dx, x_cur)), fma(fj, t.dS, S0));
                    }
                    gn = profile(xn);
                    travel = 0.0;
                } else {
                    // g_{j+1} = g_j r_j, r_{j+1} = r_j c with r_j = e^{-2 x_j dx - dx^2} and
                    // c = e^{-2 dx^2}; exact values again whenever x may have moved by more
                    // than 16 widths since the last exact one, so that an underflowed value
                    // (|x| > 27) cannot hide a profile above e^{-121}
                    const double u2 = 2.0 * dx * dx;
                    const double c = t.maxdx <= 0.5 ? exp_neg_small(u2) : exp_le700(-u2);
                    double g = g_cur;
                    double r = exp_le700(fmax(fmin(-(2.0 * x_cur + dx) * dx, 700.0), -800.0));
                    double kq = kq0, St = S0;
                    int budget = t.K;
                    if (t.maxdx > 0.0) budget = (int)fmin((16.0 - travel) / t.maxdx, (double)t.K);
                    if (budget < 1) {
                        g = profile(x_cur);
                        travel = 0.0;
                        budget = t.K;
                    }
                    const int m = t.m;
                    int j = 0;
                    for (;;) {
                        const int jend = min(j + budget, m);
                        const int jint = min(jend, m - 1);
                        int jj = j;
                        for (; jj + 3 < jint; jj += 4) {
                            recur<false>(e, g, r, c, kq, t.dkq, St, t.dS);
                            recur<false>(e, g, r, c, kq, t.dkq, St, t.dS);
                            recur<false>(e, g, r, c, kq, t.dkq, St, t.dS);
                            recur<true>(e, g, r, c, kq, t.dkq, St, t.dS);
                        }
                        // the last 0-3 steps; the cell node's step that follows renormalises,
                        // so at most seven steps pass between renormalisations
                        const int rem = jint - jj;
                        if (rem >= 2) {
                            recur<false>(e, g, r, c, kq, t.dkq, St, t.dS);
                            recur<false>(e, g, r, c, kq, t.dkq, St, t.dS);
                        }
                        if (rem & 1) recur<false>(e, g, r, c, kq, t.dkq, St, t.dS);
                        travel += t.maxdx * (double)(jint - j);
                        j = jint;
                        if (jend == m) {
                            g *= r;   // the cell node at the end of the segment
                            travel += t.maxdx;
                            break;
                        }
                        const double xj = fma((double)j, dx, x_cur);
                        g = profile(xj);
                        r = exp_le700(fmax(fmin(-(2.0 * xj + dx) * dx, 700.0), -800.0));
                        kq = fma((double)j, t.dkq, kq0);
                        St = fma((double)j, t.dS, S0);
                        travel = 0.0;
                        budget = t.K;
                    }
                    gn = g;
                }
            }
            elim<true>(e, kn * gn * hz, Sn);
            x_cur = xn;
            g_cur = gn;
            kap_cur = kn;
            chi_cur = kn * gn;
        }
    }
    // the last node is the emergent end: its far side is empty (Q = 1, y = I_in)
    const double id = 1.0 / e.d;
    const double u = (e.Pm * e.S + e.y * id + kSqrt2i * a.I_in) / (e.Pm + e.n * id + kSqrt2i);
    if (act) a.I[O * a.n_ch + ch] = 2.0 * u - a.I_in;
}

// Image-plane coordinates (x . e1, x . e2) of every point.
__global__ void k_image_plane(const CellRec *__restrict__ cell, double3 e1, double3 e2, int64_t P,
                              double *__restrict__ xy)
{
    const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (p >= P) return;
    const CellRec c = cell[p];
    xy[2 * p] = (c.px * e1.x + c.py * e1.y) + c.pz * e1.z;
    xy[2 * p + 1] = (c.px * e2.x + c.py * e2.y) + c.pz * e2.z;
}

hipError_t launch_image(const ImageArgs &a, hipStream_t s)
{
    if (a.P == 0) return hipSuccess;
    const int64_t chunks = (a.n_ch + 63) / 64;
    hipLaunchKernelGGL(k_image, dim3((unsigned)(a.P * chunks)), dim3(64), 0, s, a);
    return hipGetLastError();
}

hipError_t launch_image_plane(const CellRec *cell, double3 e1, double3 e2, int64_t P, double *xy, hipStream_t s)
{
    if (P == 0) return hipSuccess;
    hipLaunchKernelGGL(k_image_plane, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, s, cell, e1, e2, P, xy);
    return hipGetLastError();
}

}  // namespace nlte
