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
// y = y~/(sqrt 2 d), P = D_+/sqrt 2), evaluated in FP64 with a direct exponential at
// every node; velocity sub-steps interpolate z, the Doppler coefficients, kappa and S
// linearly as in the formal solve.
#include "nlte_internal.h"

namespace nlte {

namespace {

constexpr double kSqrt2i = 1.41421356237309504880;
constexpr double kInvSqrt2 = 0.70710678118654752440;

struct Node {
    double z, a, b, kap, S, vw, s;
};

// Base node: cell c seen from O along direction n (z and velocity projection relative to
// O, Doppler coefficients in O's frame, coefficients of `line`).
__device__ inline Node base_node(const ImageArgs &a, const CellRec &cO, int64_t c, double nx, double ny, double nz)
{
    const CellRec cc = a.cell[c];
    Node d;
    const double dx = cc.px - cO.px, dy = cc.py - cO.py, dz = cc.pz - cO.pz;
    d.z = (dx * nx + dy * ny) + dz * nz;
    const double dvx = cc.vx - cO.vx, dvy = cc.vy - cO.vy, dvz = cc.vz - cO.vz;
    d.s = (dvx * nx + dvy * ny) + dvz * nz;
    d.vw = cc.vw;
    d.a = cO.vw / cc.vw;
    d.b = d.s / cc.vw;
    const double2 lc = reinterpret_cast<const double2 *>(a.lc)[c * a.n_lines + a.line];
    d.kap = lc.x;
    d.S = lc.y;
    return d;
}

struct Elim {
    double n, d, y, Pm;   // scaled elimination state and the previous step's P
    double chi, z, S;     // values at the last node
};

__device__ inline void step(Elim &e, double chi, double z, double S)
{
    const double P = 0.5 * (e.chi + chi) * (z - e.z) * kInvSqrt2;
    const double hd = (e.Pm + P) * e.d;
    e.n += hd;
    e.y = fma(e.S, hd, e.y);
    e.d = fma(P, e.n, e.d);
    e.Pm = P;
    const int ex = __builtin_amdgcn_frexp_exp(e.d);
    e.n = ldexp(e.n, -ex);
    e.d = ldexp(e.d, -ex);
    e.y = ldexp(e.y, -ex);
    e.chi = chi;
    e.z = z;
    e.S = S;
}

// Visit node (with the sub-steps of the segment from the previous base node).
__device__ inline void visit(const ImageArgs &a, Elim &e, bool &first, Node &prev, const Node &cur, double xO)
{
    if (first) {
        const double x = cur.a * xO - cur.b;
        e.chi = cur.kap * exp(-(x * x));
        e.z = cur.z;
        e.S = cur.S;
        first = false;
        prev = cur;
        return;
    }
    // velocity sub-steps: split when the projected velocity changes by more than f_sub
    // of the smaller line-width speed
    const double ds = fabs(cur.s - prev.s);
    const double thr = a.f_sub * fmin(prev.vw, cur.vw);
    int m = 1;
    if (ds > thr) {
        const double mr = ceil(ds / thr);
        m = mr < (double)kMaxSub ? (int)mr : kMaxSub;
    }
    for (int j = 1; j < m; ++j) {
        const double t = (double)j / (double)m;
        const double z = prev.z + t * (cur.z - prev.z);
        const double aa = prev.a + t * (cur.a - prev.a);
        const double bb = prev.b + t * (cur.b - prev.b);
        const double k = prev.kap + t * (cur.kap - prev.kap);
        const double S = prev.S + t * (cur.S - prev.S);
        const double x = aa * xO - bb;
        step(e, k * exp(-(x * x)), z, S);
    }
    const double x = cur.a * xO - cur.b;
    step(e, cur.kap * exp(-(x * x)), cur.z, cur.S);
    prev = cur;
}

}  // namespace

__global__ __launch_bounds__(64) void k_image(ImageArgs a)
{
    const int chunks = (a.n_ch + 63) / 64;
    const int64_t O = blockIdx.x / chunks;
    const int ch = (int)(blockIdx.x % chunks) * 64 + threadIdx.x;
    if (O >= a.P) return;
    const bool act = ch < a.n_ch;
    const double nx = a.dir[3 * a.ray], ny = a.dir[3 * a.ray + 1], nz = a.dir[3 * a.ray + 2];
    const CellRec cO = a.cell[O];
    const double xO = act ? (a.v_ch[ch] - ((cO.vx * nx + cO.vy * ny) + cO.vz * nz)) / cO.vw : 0.0;
    Elim e;
    e.n = kSqrt2i;
    e.d = 1.0;
    e.y = kSqrt2i * a.I_in;
    e.Pm = 0.0;
    bool first = true;
    Node prev{};
    // upwind half: the antipode's walk from its far end toward O
    const int rb = a.anti[a.ray];
    const int64_t bb = a.roff[O * a.n_rays + rb], be = a.roff[O * a.n_rays + rb + 1];
    for (int64_t i = be - 1; i >= bb; --i) visit(a, e, first, prev, base_node(a, cO, a.rcells[i], nx, ny, nz), xO);
    visit(a, e, first, prev, base_node(a, cO, O, nx, ny, nz), xO);
    // downwind half: the walk along n from O outward
    const int64_t fb = a.roff[O * a.n_rays + a.ray], fe = a.roff[O * a.n_rays + a.ray + 1];
    for (int64_t i = fb; i < fe; ++i) visit(a, e, first, prev, base_node(a, cO, a.rcells[i], nx, ny, nz), xO);
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

hipError_t launch_image(const ImageArgs &a, double3 e1, double3 e2, double *xy, hipStream_t s)
{
    if (a.P == 0) return hipSuccess;
    const int64_t chunks = (a.n_ch + 63) / 64;
    hipLaunchKernelGGL(k_image, dim3((unsigned)(a.P * chunks)), dim3(64), 0, s, a);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || xy == nullptr) return e;
    hipLaunchKernelGGL(k_image_plane, dim3((unsigned)((a.P + 255) / 256)), dim3(256), 0, s, a.cell, e1, e2, a.P, xy);
    return hipGetLastError();
}

}  // namespace nlte
