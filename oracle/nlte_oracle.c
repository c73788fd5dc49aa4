/*
 * Plain FP64 CPU oracle for the non-LTE line radiative-transfer hot path of
 * De Ceuster et al., "Magritte I: non-LTE atomic and molecular line modelling".
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct reference the
 * HIP library is checked against.  Only the test suite, the smoke entry point and
 * the benchmark's CPU-baseline leg may build, load or call it.  It shares no source
 * with the HIP library and the library never calls it.
 *
 * What it computes, step by step, each citing the passage it follows:
 *   setup        line width (Sec. 2.2.1), collision rates with detailed balance
 *                (Sec. 2.2.1), LTE populations;
 *   walk         the neighbour-graph ray tracer (Sec. 3.2);
 *   pair nodes   the ray pair with on-the-fly velocity sub-steps (Sec. 3.1.1, 3.2);
 *   solve        the second-order (Feautrier) equation on a ray pair with Auer
 *                boundary rows, solved by forward elimination in the Rybicki-Hummer
 *                form and back-substitution (Sec. 3.3);
 *   accumulate   J, the Lambda-operator diagonal L* and J_eff (Sec. 2.2.1, 3.1.3, 3.4);
 *   stateq       the linearised statistical equilibrium with the diagonal ALO
 *                (Sec. 2.2.1, 3.4) and the positivity fallback (Sec. 6.1);
 *   ali          the accelerated Lambda iteration loop (Sec. 2.2.1, 3.4).
 *
 * Compiled with -O2 -ffp-contract=off -fno-fast-math so that every floating-point
 * decision (walk comparisons, sub-step counts) is taken with IEEE double arithmetic in
 * the written order.  OpenMP parallelises over origin points only.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "nlte_oracle.h"

#ifdef _OPENMP
#include <omp.h>
#endif

/* CGS constants (SI-exact values) */
#define OR_H 6.62607015e-27
#define OR_KB 1.380649e-16
#define OR_C 2.99792458e10
#define OR_PI 3.14159265358979323846
#define OR_SQRTPI 1.77245385090551602730

struct or_ctx {
    /* species */
    int n_lev, n_lines, n_coll, n_T;
    double *E, *g, mass;
    int32_t *lu, *ll;
    double *A, *nu, *Bul, *Blu;
    int32_t *cu, *cl;
    double *Ttab, *Ktab;
    /* model */
    int64_t P;
    int k;
    double *pos, *vel, *nh2, *T, *vturb, *X;
    int32_t *nbr;
    uint8_t *bnd;
    /* rays */
    int n_rays, n_pairs;
    double *dir;
    int32_t *anti, *pair_r;
    /* quadrature */
    int nq;
    double *qx, *qw;
    /* parameters */
    double t_cmb, f_sub, tau_floor;
    int use_alo;
    /* derived per point */
    double *vw, *ntot;
};

static void *dup(const void *src, size_t bytes)
{
    if (!src || bytes == 0) return NULL;
    void *p = malloc(bytes);
    memcpy(p, src, bytes);
    return p;
}

or_ctx *or_create(void)
{
    or_ctx *c = (or_ctx *)calloc(1, sizeof(or_ctx));
    c->t_cmb = 2.725;
    c->f_sub = 0.25;
    c->tau_floor = 1e-100; /* guards A_i, C_i against zero optical depth; effect < 1e-90 */
    c->use_alo = 1;
    return c;
}

void or_destroy(or_ctx *c)
{
    if (!c) return;
    void *ps[] = {c->E, c->g, c->lu, c->ll, c->A, c->nu, c->Bul, c->Blu, c->cu, c->cl, c->Ttab,
                  c->Ktab, c->pos, c->vel, c->nh2, c->T, c->vturb, c->X, c->nbr, c->bnd,
                  c->dir, c->anti, c->pair_r, c->qx, c->qw, c->vw, c->ntot};
    for (size_t i = 0; i < sizeof(ps) / sizeof(ps[0]); ++i) free(ps[i]);
    free(c);
}

/* Einstein B coefficients from A, with J in intensity units (textbook relations; the
 * paper uses A and B without relating them, Sec. 2.2.1). */
int or_set_species(or_ctx *c, int n_lev, const double *E, const double *g, double mass,
                   int n_lines, const int32_t *up, const int32_t *lo, const double *A,
                   int n_coll, const int32_t *cup, const int32_t *clo, int n_T,
                   const double *Ttab, const double *Ktab)
{
    c->n_lev = n_lev;
    c->n_lines = n_lines;
    c->n_coll = n_coll;
    c->n_T = n_T;
    c->mass = mass;
    c->E = dup(E, sizeof(double) * n_lev);
    c->g = dup(g, sizeof(double) * n_lev);
    c->lu = dup(up, sizeof(int32_t) * n_lines);
    c->ll = dup(lo, sizeof(int32_t) * n_lines);
    c->A = dup(A, sizeof(double) * n_lines);
    c->nu = malloc(sizeof(double) * n_lines);
    c->Bul = malloc(sizeof(double) * n_lines);
    c->Blu = malloc(sizeof(double) * n_lines);
    for (int l = 0; l < n_lines; ++l) {
        double nu = (E[up[l]] - E[lo[l]]) / OR_H;
        c->nu[l] = nu;
        c->Bul[l] = A[l] * OR_C * OR_C / (2.0 * OR_H * nu * nu * nu);
        c->Blu[l] = (g[up[l]] / g[lo[l]]) * c->Bul[l];
    }
    c->cu = dup(cup, sizeof(int32_t) * n_coll);
    c->cl = dup(clo, sizeof(int32_t) * n_coll);
    c->Ttab = dup(Ttab, sizeof(double) * n_T);
    c->Ktab = dup(Ktab, sizeof(double) * (size_t)n_coll * n_T);
    return 0;
}

int or_set_model(or_ctx *c, int64_t P, const double *pos, const double *vel, const double *nh2,
                 const double *T, const double *vturb, const double *X, int k, const int32_t *nbr,
                 const uint8_t *bnd)
{
    c->P = P;
    c->k = k;
    c->pos = dup(pos, sizeof(double) * 3 * P);
    c->vel = dup(vel, sizeof(double) * 3 * P);
    c->nh2 = dup(nh2, sizeof(double) * P);
    c->T = dup(T, sizeof(double) * P);
    c->vturb = dup(vturb, sizeof(double) * P);
    c->X = dup(X, sizeof(double) * P);
    c->nbr = dup(nbr, sizeof(int32_t) * k * P);
    c->bnd = bnd ? dup(bnd, P) : NULL;
    /* Sec. 2.2.1: line width from thermal plus turbulent speed, v_th = sqrt(2kT/m). */
    c->vw = malloc(sizeof(double) * P);
    c->ntot = malloc(sizeof(double) * P);
    for (int64_t p = 0; p < P; ++p) {
        double vth2 = 2.0 * OR_KB * T[p] / c->mass;
        c->vw[p] = sqrt(vth2 + vturb[p] * vturb[p]);
        c->ntot[p] = X[p] * nh2[p];
    }
    return 0;
}

/* Directions must come in antipodal pairs; the pair representative is the lower index. */
int or_set_rays(or_ctx *c, int n_rays, const double *dir)
{
    c->n_rays = n_rays;
    c->dir = dup(dir, sizeof(double) * 3 * n_rays);
    c->anti = malloc(sizeof(int32_t) * n_rays);
    c->pair_r = malloc(sizeof(int32_t) * n_rays);
    c->n_pairs = 0;
    for (int r = 0; r < n_rays; ++r) {
        c->anti[r] = -1;
        for (int s = 0; s < n_rays; ++s) {
            double e = fabs(dir[3 * r] + dir[3 * s]) + fabs(dir[3 * r + 1] + dir[3 * s + 1]) +
                       fabs(dir[3 * r + 2] + dir[3 * s + 2]);
            if (e < 1e-12) c->anti[r] = s;
        }
        if (c->anti[r] < 0) return -1;
    }
    for (int r = 0; r < n_rays; ++r)
        if (r < c->anti[r]) c->pair_r[c->n_pairs++] = r;
    return c->n_pairs;
}

int or_set_quadrature(or_ctx *c, int nq, const double *x, const double *w)
{
    c->nq = nq;
    c->qx = dup(x, sizeof(double) * nq);
    c->qw = dup(w, sizeof(double) * nq);
    return 0;
}

void or_set_params(or_ctx *c, double t_cmb, double f_sub, double tau_floor, int use_alo)
{
    c->t_cmb = t_cmb;
    c->f_sub = f_sub;
    c->tau_floor = tau_floor;
    c->use_alo = use_alo;
}

int or_n_pairs(const or_ctx *c) { return c->n_pairs; }

void or_line_width_speed(const or_ctx *c, double *vw)
{
    memcpy(vw, c->vw, sizeof(double) * c->P);
}

/* Planck function at frequency nu and temperature T (intensity units). */
double or_planck(double nu, double T)
{
    return 2.0 * OR_H * nu * nu * nu / (OR_C * OR_C) / expm1(OR_H * nu / (OR_KB * T));
}

/* ------------------------------------------------------------------ setup */

/* H2 collisional de-excitation coefficient, linear in T between table points and
 * clamped at the table ends (tabulated data, Sec. 2.2.1). */
static double coll_K(const or_ctx *c, int ic, double T)
{
    const double *Tt = c->Ttab, *K = c->Ktab + (size_t)ic * c->n_T;
    if (T <= Tt[0]) return K[0];
    if (T >= Tt[c->n_T - 1]) return K[c->n_T - 1];
    int j = 0;
    while (j + 2 < c->n_T && !(T < Tt[j + 1])) ++j;
    return K[j] + (K[j + 1] - K[j]) * (T - Tt[j]) / (Tt[j + 1] - Tt[j]);
}

/* Collisional rates for point p: C_ul = K_ul(T) n_H2 and the excitation rate by
 * detailed balance C_lu = C_ul (g_u/g_l) exp(-(E_u - E_l)/kT).  The paper prints the
 * exponent with a positive sign (Sec. 2.2.1); only the negative sign gives Boltzmann
 * populations in thermal equilibrium, which the tests check. */
void or_coll_rates(const or_ctx *c, int64_t p, double *Cul, double *Clu)
{
    double T = c->T[p];
    for (int ic = 0; ic < c->n_coll; ++ic) {
        int u = c->cu[ic], l = c->cl[ic];
        double cul = coll_K(c, ic, T) * c->nh2[p];
        Cul[ic] = cul;
        Clu[ic] = cul * (c->g[u] / c->g[l]) * exp(-(c->E[u] - c->E[l]) / (OR_KB * T));
    }
}

/* Boltzmann populations at the local temperature, normalised to X n_H2. */
void or_lte(const or_ctx *c, double *pops)
{
    int nl = c->n_lev;
    for (int64_t p = 0; p < c->P; ++p) {
        double T = c->T[p], Z = 0.0;
        for (int i = 0; i < nl; ++i) Z += c->g[i] * exp(-(c->E[i] - c->E[0]) / (OR_KB * T));
        for (int i = 0; i < nl; ++i)
            pops[p * nl + i] = c->ntot[p] * c->g[i] * exp(-(c->E[i] - c->E[0]) / (OR_KB * T)) / Z;
    }
}

/* Eq. (2) line emissivity and opacity without the profile, at line centre frequency:
 *   k_eta = (h nu / 4 pi) n_u A_ul,  k_chi = (h nu / 4 pi) (n_l B_lu - n_u B_ul),
 * and the line-centre opacity kappa = k_chi / (sqrt(pi) dnu) with dnu = nu v_w / c
 * (Gaussian profile, Sec. 2.2.1), S = k_eta / k_chi.  Negative opacities (masers) are
 * clamped to zero opacity and zero source. */
static void line_coefs(const or_ctx *c, const double *pops, int64_t p, int l, double *kappa,
                       double *S)
{
    int u = c->lu[l], lo = c->ll[l];
    double nu = c->nu[l];
    const double *n = pops + p * c->n_lev;
    double pre = OR_H * nu / (4.0 * OR_PI);
    double keta = pre * n[u] * c->A[l];
    double kchi = pre * (n[lo] * c->Blu[l] - n[u] * c->Bul[l]);
    if (!(kchi > 0.0)) {
        *kappa = 0.0;
        *S = 0.0;
        return;
    }
    double dnu = nu * c->vw[p] / OR_C;
    *kappa = kchi / (OR_SQRTPI * dnu);
    *S = keta / kchi;
}

/* ------------------------------------------------------------------ ray walk */

/* Sec. 3.2: from the current cell, step to the neighbour whose projection on the ray
 * lies farther than the current one and which lies closest to the ray; repeat until no
 * such neighbour exists or a flagged boundary point is reached.  Distances to the ray
 * are measured to the line through the origin O.  Exact ties go to the lower index. */
int or_walk(const or_ctx *c, int64_t O, int ray, int32_t *cells, double *Zs, int cap)
{
    const double *n = c->dir + 3 * ray;
    const double ox = c->pos[3 * O], oy = c->pos[3 * O + 1], oz = c->pos[3 * O + 2];
    int64_t cur = O;
    double Zcur = 0.0;
    int len = 0;
    for (;;) {
        if (cur != O && c->bnd && c->bnd[cur]) break;
        int64_t best = -1;
        double bq = 0.0, bZ = 0.0;
        for (int s = 0; s < c->k; ++s) {
            int32_t m = c->nbr[cur * c->k + s];
            if (m < 0) continue;
            double dx = c->pos[3 * (int64_t)m] - ox;
            double dy = c->pos[3 * (int64_t)m + 1] - oy;
            double dz = c->pos[3 * (int64_t)m + 2] - oz;
            double Z = (dx * n[0] + dy * n[1]) + dz * n[2];
            if (!(Z > Zcur)) continue;
            double qx = dx - Z * n[0], qy = dy - Z * n[1], qz = dz - Z * n[2];
            double q = (qx * qx + qy * qy) + qz * qz;
            if (best < 0 || q < bq || (q == bq && m < best)) {
                best = m;
                bq = q;
                bZ = Z;
            }
        }
        if (best < 0) break;
        if (len < cap) {
            cells[len] = (int32_t)best;
            if (Zs) Zs[len] = bZ;
        }
        ++len;
        cur = best;
        Zcur = bZ;
    }
    return len;
}

/* ------------------------------------------------------------------ ray pair */

/* Velocity projection of cell q relative to O along direction n. */
static double vproj(const or_ctx *c, int64_t O, int64_t q, const double *n)
{
    double dx = c->vel[3 * q] - c->vel[3 * O];
    double dy = c->vel[3 * q + 1] - c->vel[3 * O + 1];
    double dz = c->vel[3 * q + 2] - c->vel[3 * O + 2];
    return (dx * n[0] + dy * n[1]) + dz * n[2];
}

/* Number of sub-intervals a segment is split into (Sec. 3.1.1, 3.2): the projected
 * velocity may change by at most f_sub times the smaller of the two line-width speeds
 * between consecutive nodes. */
static int n_sub(double f, double s0, double s1, double w0, double w1)
{
    double ds = fabs(s1 - s0);
    double thr = f * fmin(w0, w1);
    if (!(ds > thr)) return 1;
    double m = ceil(ds / thr);
    return m < 1048576.0 ? (int)m : 1048576; /* cap of 2^20 sub-intervals per segment */
}

/*
 * Assemble the nodes of the ray pair (ray r and its antipode) through O, with
 * coordinates z along ray r: reversed walk of the antipode (z = -Z), O (z = 0), walk
 * of r (z = Z).  Per node: a = v_w(O)/v_w, b = s/v_w with s the velocity projection
 * on ray r relative to O (each half computes its projection with its own direction and
 * ray r's frame uses minus the antipode's), plus kappa and S per line.  A segment whose
 * projected-velocity step exceeds f_sub of the smaller width is split into m equal
 * parts; inserted nodes interpolate z, a, b, kappa and S linearly.
 *
 * Returns the node count (or the count needed if cap is too small); *io receives the
 * index of O.  kap and S are [node][line].
 */
static int pair_nodes_src(const or_ctx *c, const double *pops, int64_t O, int pair, int cap,
                          double *z, double *a, double *b, double *kap, double *S, int64_t *c_lo,
                          int64_t *c_hi, double *t_hi, int *io);

int or_pair_nodes(const or_ctx *c, const double *pops, int64_t O, int pair, int cap, double *z,
                  double *a, double *b, double *kap, double *S, int *io)
{
    return pair_nodes_src(c, pops, O, pair, cap, z, a, b, kap, S, NULL, NULL, NULL, io);
}

/* As or_pair_nodes; c_lo, c_hi, t_hi (nullable) receive for every node the base cells it
 * lies between (lower and higher z) and its fraction t of the way from c_lo to c_hi (a
 * base node is its own c_lo = c_hi with t = 0). */
static int pair_nodes_src(const or_ctx *c, const double *pops, int64_t O, int pair, int cap,
                          double *z, double *a, double *b, double *kap, double *S, int64_t *c_lo,
                          int64_t *c_hi, double *t_hi, int *io)
{
    int r = c->pair_r[pair], rb = c->anti[r];
    int nl = c->n_lines;
    int Lf = or_walk(c, O, r, NULL, NULL, 0);
    int Lb = or_walk(c, O, rb, NULL, NULL, 0);
    int32_t *cf = malloc(sizeof(int32_t) * (Lf + 1)), *cb = malloc(sizeof(int32_t) * (Lb + 1));
    double *Zf = malloc(sizeof(double) * (Lf + 1)), *Zb = malloc(sizeof(double) * (Lb + 1));
    or_walk(c, O, r, cf, Zf, Lf);
    or_walk(c, O, rb, cb, Zb, Lb);
    int nb = Lb + 1 + Lf;
    /* base nodes */
    int64_t *cell = malloc(sizeof(int64_t) * nb);
    double *bz = malloc(sizeof(double) * nb), *bs = malloc(sizeof(double) * nb);
    for (int i = 0; i < Lb; ++i) {
        int j = Lb - 1 - i;
        cell[i] = cb[j];
        bz[i] = -Zb[j];
        bs[i] = -vproj(c, O, cb[j], c->dir + 3 * rb);
    }
    cell[Lb] = O;
    bz[Lb] = 0.0;
    bs[Lb] = 0.0;
    for (int i = 0; i < Lf; ++i) {
        cell[Lb + 1 + i] = cf[i];
        bz[Lb + 1 + i] = Zf[i];
        bs[Lb + 1 + i] = vproj(c, O, cf[i], c->dir + 3 * r);
    }
    /* count nodes with sub-steps */
    int total = 1, obase = -1;
    for (int i = 0; i + 1 < nb; ++i)
        total += n_sub(c->f_sub, bs[i], bs[i + 1], c->vw[cell[i]], c->vw[cell[i + 1]]);
    if (total > cap) {
        free(cf); free(cb); free(Zf); free(Zb); free(cell); free(bz); free(bs);
        return total;
    }
    double vwO = c->vw[O];
    double *bk = malloc(sizeof(double) * nl * 2);
    int w = 0;
    for (int i = 0; i < nb; ++i) {
        double ai = vwO / c->vw[cell[i]], bi = bs[i] / c->vw[cell[i]];
        if (i == Lb) obase = w;
        z[w] = bz[i];
        a[w] = ai;
        b[w] = bi;
        if (c_lo) {
            c_lo[w] = c_hi[w] = cell[i];
            t_hi[w] = 0.0;
        }
        for (int l = 0; l < nl; ++l) line_coefs(c, pops, cell[i], l, &kap[w * nl + l], &S[w * nl + l]);
        ++w;
        if (i + 1 == nb) break;
        int m = n_sub(c->f_sub, bs[i], bs[i + 1], c->vw[cell[i]], c->vw[cell[i + 1]]);
        if (m > 1) {
            double a1 = vwO / c->vw[cell[i + 1]], b1 = bs[i + 1] / c->vw[cell[i + 1]];
            for (int l = 0; l < nl; ++l) line_coefs(c, pops, cell[i + 1], l, &bk[2 * l], &bk[2 * l + 1]);
            for (int j = 1; j < m; ++j) {
                double t = (double)j / (double)m;
                z[w] = bz[i] + t * (bz[i + 1] - bz[i]);
                a[w] = ai + t * (a1 - ai);
                b[w] = bi + t * (b1 - bi);
                if (c_lo) {
                    c_lo[w] = cell[i];
                    c_hi[w] = cell[i + 1];
                    t_hi[w] = t;
                }
                for (int l = 0; l < nl; ++l) {
                    double k0 = kap[(w - j) * nl + l], s0 = S[(w - j) * nl + l];
                    kap[w * nl + l] = k0 + t * (bk[2 * l] - k0);
                    S[w * nl + l] = s0 + t * (bk[2 * l + 1] - s0);
                }
                ++w;
            }
        }
    }
    *io = obase;
    free(bk); free(cf); free(cb); free(Zf); free(Zb); free(cell); free(bz); free(bs);
    return total;
}

/* ------------------------------------------------------------------ Feautrier solve */

/*
 * Tridiagonal system of the second-order transfer equation d^2u/dtau^2 = u - S on N
 * nodes (Sec. 3.3, no scattering), rows  -A_i u_{i-1} + (H_i + A_i + C_i) u_i - C_i u_{i+1} = R_i:
 *   interior  A_i = 2/(dt_-(dt_- + dt_+)), C_i = 2/(dt_+(dt_- + dt_+)), H_i = 1, R_i = S_i;
 *   ends      second-order (Auer) boundary rows for incoming intensity I:
 *             A or C = 2/dt^2 toward the interior, H = 1 + 2/dt, R = S + (2/dt) I.
 * Solved by the Rybicki-Hummer forward elimination F_i = (H_i + A_i F_{i-1}/(1+F_{i-1}))/C_i,
 * z_i = (R_i + A_i z_{i-1})/(C_i(1+F_i)) and back-substitution u_i = z_i + u_{i+1}/(1+F_i).
 */
static void rh_solve(int N, const double *Ac, const double *Cc, const double *Hc, const double *R,
                     double *F, double *zz, double *u)
{
    F[0] = Hc[0] / Cc[0];
    zz[0] = R[0] / (Cc[0] * (1.0 + F[0]));
    for (int i = 1; i < N - 1; ++i) {
        F[i] = (Hc[i] + Ac[i] * F[i - 1] / (1.0 + F[i - 1])) / Cc[i];
        zz[i] = (R[i] + Ac[i] * zz[i - 1]) / (Cc[i] * (1.0 + F[i]));
    }
    int L = N - 1;
    u[L] = (R[L] + Ac[L] * zz[L - 1]) / (Hc[L] + Ac[L] * F[L - 1] / (1.0 + F[L - 1]));
    for (int i = L - 1; i >= 0; --i) u[i] = zz[i] + u[i + 1] / (1.0 + F[i]);
}

/*
 * Solve one ray pair at one frequency given nodal z, chi, S and the incoming boundary
 * intensities I_lo (entering at node 0 along +z) and I_hi (entering at node N-1).
 * Outputs at node o: u_o, the diagonal Lambda_oo of the inverse system matrix, and
 * ueff_o = u_o - Lambda_oo S_o obtained by solving with S_o removed from the right-hand
 * side (the contribution of all other nodes).  u_all (nullable) receives u at all nodes.
 * A single node (no neighbours either way) sees only the boundary: u = (I_lo + I_hi)/2.
 */
void or_solve_ray(int N, const double *z, const double *chi, const double *S, double I_lo,
                  double I_hi, int o, double tau_floor, double *u_o, double *lam_o,
                  double *ueff_o, double *u_all)
{
    if (N == 1) {
        *u_o = 0.5 * (I_lo + I_hi);
        *lam_o = 0.0;
        *ueff_o = *u_o;
        if (u_all) u_all[0] = *u_o;
        return;
    }
    double *dt = malloc(sizeof(double) * N);
    double *Ac = calloc(N, sizeof(double)), *Cc = calloc(N, sizeof(double));
    double *Hc = malloc(sizeof(double) * N), *R = malloc(sizeof(double) * N);
    double *F = malloc(sizeof(double) * N), *zz = malloc(sizeof(double) * N);
    double *u = malloc(sizeof(double) * N);
    for (int i = 0; i + 1 < N; ++i) {
        double d = 0.5 * (chi[i] + chi[i + 1]) * (z[i + 1] - z[i]);
        dt[i] = d > tau_floor ? d : tau_floor;
    }
    for (int i = 0; i < N; ++i) {
        Hc[i] = 1.0;
        R[i] = S[i];
    }
    Cc[0] = 2.0 / (dt[0] * dt[0]);
    Hc[0] = 1.0 + 2.0 / dt[0];
    R[0] = S[0] + 2.0 / dt[0] * I_lo;
    for (int i = 1; i < N - 1; ++i) {
        Ac[i] = 2.0 / (dt[i - 1] * (dt[i - 1] + dt[i]));
        Cc[i] = 2.0 / (dt[i] * (dt[i - 1] + dt[i]));
    }
    Ac[N - 1] = 2.0 / (dt[N - 2] * dt[N - 2]);
    Hc[N - 1] = 1.0 + 2.0 / dt[N - 2];
    R[N - 1] = S[N - 1] + 2.0 / dt[N - 2] * I_hi;

    rh_solve(N, Ac, Cc, Hc, R, F, zz, u);
    *u_o = u[o];
    if (u_all) memcpy(u_all, u, sizeof(double) * N);
    /* diagonal of the inverse: solve with the unit vector at o */
    double *e = calloc(N, sizeof(double));
    e[o] = 1.0;
    rh_solve(N, Ac, Cc, Hc, e, F, zz, u);
    *lam_o = u[o];
    /* all contributions except the node's own source */
    R[o] -= S[o];
    rh_solve(N, Ac, Cc, Hc, R, F, zz, u);
    *ueff_o = u[o];
    free(e); free(dt); free(Ac); free(Cc); free(Hc); free(R); free(F); free(zz); free(u);
}

/* ------------------------------------------------------------------ formal solve */

/*
 * J, L* and J_eff at the selected origin points for populations pops:
 *   J_l     = (2/N_rays) sum_pairs sum_n w_n u_o         (Eq. meanIntensity with the
 *             ray average of Sec. 3.1.3; u pairs I(n, x) with I(-n, -x), and the
 *             symmetric quadrature makes the pair sum equal the sum over all rays),
 *   L_l     = (2/N_rays) sum_pairs sum_n w_n Lambda_oo   (diagonal ALO, Sec. 3.4),
 *   Jeff_l  = (2/N_rays) sum_pairs sum_n w_n ueff_o      (Eq. ourJeff: J - L*[S]).
 * Frequencies are nu_l + x_n dnu_l(O); the profile at node k is evaluated at
 * x_k = a_k x_n - b_k in units of the local width.  Boundary intensity: CMB at the
 * line centre frequency on both ends.
 */
void or_formal_solve(const or_ctx *c, const double *pops, int64_t n_sel, const int64_t *sel,
                     double *J, double *Jeff, double *L)
{
    int nl = c->n_lines, nq = c->nq;
    double norm = 2.0 / (double)c->n_rays;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t s = 0; s < n_sel; ++s) {
        int64_t O = sel ? sel[s] : s;
        double *Js = calloc(nl, sizeof(double)), *Ls = calloc(nl, sizeof(double));
        double *Es = calloc(nl, sizeof(double));
        for (int p = 0; p < c->n_pairs; ++p) {
            int io;
            int N = or_pair_nodes(c, pops, O, p, 0, NULL, NULL, NULL, NULL, NULL, &io);
            double *z = malloc(sizeof(double) * N), *a = malloc(sizeof(double) * N);
            double *b = malloc(sizeof(double) * N);
            double *kap = malloc(sizeof(double) * N * nl), *S = malloc(sizeof(double) * N * nl);
            or_pair_nodes(c, pops, O, p, N, z, a, b, kap, S, &io);
            double *chi = malloc(sizeof(double) * N), *Sl = malloc(sizeof(double) * N);
            for (int l = 0; l < nl; ++l) {
                double Ib = or_planck(c->nu[l], c->t_cmb);
                for (int i = 0; i < N; ++i) Sl[i] = S[i * nl + l];
                for (int n = 0; n < nq; ++n) {
                    for (int i = 0; i < N; ++i) {
                        double x = a[i] * c->qx[n] - b[i];
                        chi[i] = kap[i * nl + l] * exp(-x * x);
                    }
                    double u, lam, ue;
                    or_solve_ray(N, z, chi, Sl, Ib, Ib, io, c->tau_floor, &u, &lam, &ue, NULL);
                    Js[l] += c->qw[n] * u;
                    Ls[l] += c->qw[n] * lam;
                    Es[l] += c->qw[n] * ue;
                }
            }
            free(z); free(a); free(b); free(kap); free(S); free(chi); free(Sl);
        }
        for (int l = 0; l < nl; ++l) {
            J[s * nl + l] = norm * Js[l];
            L[s * nl + l] = norm * Ls[l];
            Jeff[s * nl + l] = norm * Es[l];
        }
        free(Js); free(Ls); free(Es);
    }
}

/* ------------------------------------------------------------------ statistical equilibrium */

/* Gaussian elimination with partial pivoting on the dense n x n system M x = rhs. */
static int gauss_solve(int n, double *M, double *rhs, double *x)
{
    for (int col = 0; col < n; ++col) {
        int piv = col;
        for (int r = col + 1; r < n; ++r)
            if (fabs(M[r * n + col]) > fabs(M[piv * n + col])) piv = r;
        if (M[piv * n + col] == 0.0) return -1;
        if (piv != col) {
            for (int j = 0; j < n; ++j) {
                double t = M[col * n + j];
                M[col * n + j] = M[piv * n + j];
                M[piv * n + j] = t;
            }
            double t = rhs[col];
            rhs[col] = rhs[piv];
            rhs[piv] = t;
        }
        for (int r = col + 1; r < n; ++r) {
            double f = M[r * n + col] / M[col * n + col];
            for (int j = col; j < n; ++j) M[r * n + j] -= f * M[col * n + j];
            rhs[r] -= f * rhs[col];
        }
    }
    for (int r = n - 1; r >= 0; --r) {
        double s = rhs[r];
        for (int j = r + 1; j < n; ++j) s -= M[r * n + j] * x[j];
        x[r] = s / M[r * n + r];
    }
    return 0;
}

/*
 * Level populations of point p from Eq. (ourALI) with the diagonal ALO:
 *   rate u->l = A_ul (1 - L_l) + B_ul Jeff_l + C_ul,   rate l->u = B_lu Jeff_l + C_lu,
 *   sum_j n_j P_ji - n_i sum_j P_ij = 0 for every level, with the first level's
 *   equation replaced by sum_i n_i = X n_H2.
 */
static int stateq_point(const or_ctx *c, int64_t p, const double *Jl, const double *Jeffl,
                        const double *Ll, double *out)
{
    int n = c->n_lev;
    double *P = calloc(n * n, sizeof(double)), *M = malloc(sizeof(double) * n * n);
    double *rhs = calloc(n, sizeof(double));
    double *Cul = malloc(sizeof(double) * (c->n_coll + 1)), *Clu = malloc(sizeof(double) * (c->n_coll + 1));
    (void)Jl;
    for (int l = 0; l < c->n_lines; ++l) {
        int u = c->lu[l], lo = c->ll[l];
        P[u * n + lo] += c->A[l] * (1.0 - Ll[l]) + c->Bul[l] * Jeffl[l];
        P[lo * n + u] += c->Blu[l] * Jeffl[l];
    }
    or_coll_rates(c, p, Cul, Clu);
    for (int ic = 0; ic < c->n_coll; ++ic) {
        int u = c->cu[ic], lo = c->cl[ic];
        P[u * n + lo] += Cul[ic];
        P[lo * n + u] += Clu[ic];
    }
    for (int i = 0; i < n; ++i) {
        double out_i = 0.0;
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            M[i * n + j] = P[j * n + i];
            out_i += P[i * n + j];
        }
        M[i * n + i] = -out_i;
    }
    for (int j = 0; j < n; ++j) M[j] = 1.0;
    rhs[0] = c->ntot[p];
    int rc = gauss_solve(n, M, rhs, out);
    free(P); free(M); free(rhs); free(Cul); free(Clu);
    return rc;
}

static int pops_valid(int n, const double *x)
{
    for (int i = 0; i < n; ++i)
        if (!(x[i] > 0.0) || !isfinite(x[i])) return 0;
    return 1;
}

/*
 * Statistical equilibrium at every point.  Validity check (Sec. 6.1): if the ALO
 * solution has a non-positive or non-finite population, solve again without the ALO
 * (L = 0, Jeff = J, plain Lambda iteration); if that fails too, keep the previous
 * populations.  flags: 0 ok, 1 fell back to plain Lambda, 2 kept previous.
 */
void or_stateq(const or_ctx *c, const double *pops_old, const double *J, const double *Jeff,
               const double *L, double *pops_new, uint8_t *flags)
{
    int nl = c->n_lines, n = c->n_lev;
#pragma omp parallel for schedule(static)
    for (int64_t p = 0; p < c->P; ++p) {
        double *zero = calloc(nl, sizeof(double));
        const double *Lp = c->use_alo ? L + p * nl : zero;
        const double *Ep = c->use_alo ? Jeff + p * nl : J + p * nl;
        double *x = pops_new + p * n;
        uint8_t f = 0;
        if (stateq_point(c, p, J + p * nl, Ep, Lp, x) != 0 || !pops_valid(n, x)) {
            f = 1;
            if (stateq_point(c, p, J + p * nl, J + p * nl, zero, x) != 0 || !pops_valid(n, x)) {
                f = 2;
                memcpy(x, pops_old + p * n, sizeof(double) * n);
            }
        }
        if (flags) flags[p] = f;
        free(zero);
    }
}

/* Convergence measure: max over points and levels with n_i/n_tot > 1e-10 of
 * |n_new - n_old| / n_new; the mean over the same entries goes to *mean. */
double or_rel_change(const or_ctx *c, const double *old, const double *nw, double *mean)
{
    double mx = 0.0, sum = 0.0;
    int64_t cnt = 0;
    for (int64_t p = 0; p < c->P; ++p)
        for (int i = 0; i < c->n_lev; ++i) {
            double v = nw[p * c->n_lev + i];
            if (!(v / c->ntot[p] > 1e-10)) continue;
            double d = fabs(v - old[p * c->n_lev + i]) / v;
            if (d > mx) mx = d;
            sum += d;
            ++cnt;
        }
    if (mean) *mean = cnt ? sum / (double)cnt : 0.0;
    return mx;
}

/* Accelerated Lambda iteration (Sec. 2.2.1, 3.4): formal solve with the previous
 * populations, then statistical equilibrium, until the relative change drops below tol
 * or max_iter iterations ran.  Returns the iteration count; max_change[it] holds the
 * change of each iteration. */
int or_run_ali(const or_ctx *c, const double *pops_init, double *pops_out, int max_iter, double tol,
               double *max_change)
{
    int64_t P = c->P;
    int nl = c->n_lines, n = c->n_lev;
    double *J = malloc(sizeof(double) * P * nl), *Je = malloc(sizeof(double) * P * nl);
    double *L = malloc(sizeof(double) * P * nl), *nw = malloc(sizeof(double) * P * n);
    if (pops_init)
        memcpy(pops_out, pops_init, sizeof(double) * P * n);
    else
        or_lte(c, pops_out);
    int it = 0;
    while (it < max_iter) {
        or_formal_solve(c, pops_out, P, NULL, J, Je, L);
        or_stateq(c, pops_out, J, Je, L, nw, NULL);
        double ch = or_rel_change(c, pops_out, nw, NULL);
        memcpy(pops_out, nw, sizeof(double) * P * n);
        if (max_change) max_change[it] = ch;
        ++it;
        if (ch < tol) break;
    }
    free(J); free(Je); free(L); free(nw);
    return it;
}

/* Every (point, ray) walk in CSR form, rays of a point consecutive: off [P*n_rays+1],
 * cells [off[P*n_rays]] (pass cells = NULL to get the offsets and the total only). */
int64_t or_walk_all(const or_ctx *c, int64_t *off, int32_t *cells)
{
    int64_t n = c->P * c->n_rays;
    off[0] = 0;
    for (int64_t q = 0; q < n; ++q)
        off[q + 1] = off[q] + or_walk(c, q / c->n_rays, (int)(q % c->n_rays), NULL, NULL, 0);
    if (cells) {
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t q = 0; q < n; ++q)
            or_walk(c, q / c->n_rays, (int)(q % c->n_rays), cells + off[q], NULL,
                    (int)(off[q + 1] - off[q]));
    }
    return off[n];
}

/* ------------------------------------------------------------------ warm-start features */

static int cmp_double(const void *a, const void *b)
{
    double x = *(const double *)a, y = *(const double *)b;
    return (x > y) - (x < y);
}

/* Inputs of the warm-start surrogate (not part of the paper's method; they describe
 * the local conditions its starting populations are predicted from).  Per point p,
 * F[p][0..7]:
 *   0  log10 n_H2,   1  log10 T,
 *   2  log10 max(g, 1e-30) with g the mean over p's valid neighbours m of
 *      |v_m - v_p| / |x_m - x_p| (0 without neighbours),
 *   3..7  log10 of the minimum, lower quartile, median, upper quartile and maximum over
 *      all rays of the H2 column N from p to the end of its walk (Sec. 3.2): the
 *      trapezoid sum of n_H2 over the projected distances between consecutive cells,
 *      starting at p with projection 0, and at least half a cell's column,
 *      n_H2(p) d / 2 with d the mean distance to p's valid neighbours (a walk with no
 *      cell, at the model's edge, takes that), and at least 1 cm^-2.  A quantile at q
 *      is the linear interpolation between order statistics at position q (n_rays - 1). */
void or_features(const or_ctx *c, double *F)
{
    const int R = c->n_rays;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t p = 0; p < c->P; ++p) {
        double *f = F + 8 * p;
        f[0] = log10(c->nh2[p]);
        f[1] = log10(c->T[p]);
        double gsum = 0.0, dsum = 0.0;
        int gcount = 0;
        for (int s = 0; s < c->k; ++s) {
            int32_t m = c->nbr[p * c->k + s];
            if (m < 0) continue;
            double dv[3], dx[3];
            for (int d = 0; d < 3; ++d) {
                dv[d] = c->vel[3 * (int64_t)m + d] - c->vel[3 * p + d];
                dx[d] = c->pos[3 * (int64_t)m + d] - c->pos[3 * p + d];
            }
            double nv = sqrt((dv[0] * dv[0] + dv[1] * dv[1]) + dv[2] * dv[2]);
            double nx = sqrt((dx[0] * dx[0] + dx[1] * dx[1]) + dx[2] * dx[2]);
            gsum += nv / nx;
            dsum += nx;
            ++gcount;
        }
        double g = gcount > 0 ? gsum / gcount : 0.0;
        f[2] = log10(g > 1e-30 ? g : 1e-30);
        double half_cell = gcount > 0 ? 0.5 * c->nh2[p] * (dsum / gcount) : 0.0;
        double floor_col = half_cell > 1.0 ? half_cell : 1.0;

        double *col = malloc(sizeof(double) * R);
        for (int r = 0; r < R; ++r) {
            int len = or_walk(c, p, r, NULL, NULL, 0);
            int32_t *cells = malloc(sizeof(int32_t) * (len > 0 ? len : 1));
            double *Zs = malloc(sizeof(double) * (len > 0 ? len : 1));
            or_walk(c, p, r, cells, Zs, len);
            double N = 0.0, n_prev = c->nh2[p], z_prev = 0.0;
            for (int i = 0; i < len; ++i) {
                double n_i = c->nh2[cells[i]];
                N += 0.5 * (n_prev + n_i) * (Zs[i] - z_prev);
                n_prev = n_i;
                z_prev = Zs[i];
            }
            col[r] = N > floor_col ? N : floor_col;
            free(cells);
            free(Zs);
        }
        qsort(col, R, sizeof(double), cmp_double);
        static const double qs[5] = {0.0, 0.25, 0.5, 0.75, 1.0};
        for (int j = 0; j < 5; ++j) {
            double h = qs[j] * (R - 1);
            int i = (int)floor(h);
            double v = col[i];
            if (i + 1 < R) v = col[i] + (h - i) * (col[i + 1] - col[i]);
            f[3 + j] = log10(v);
        }
        free(col);
    }
}

/* ------------------------------------------------------------------ band ALO */

/* or_solve_ray plus the entries (T^-1)_{o,o-1} and (T^-1)_{o,o+1} of the inverse system
 * matrix (0 where the neighbour node does not exist), from solves with unit right-hand
 * sides at o-1 and o+1. */
static void solve_ray_band(int N, const double *z, const double *chi, const double *S, double I_lo,
                           double I_hi, int o, double tau_floor, double *u_o, double *lam_o,
                           double *ueff_o, double *tm, double *tp)
{
    or_solve_ray(N, z, chi, S, I_lo, I_hi, o, tau_floor, u_o, lam_o, ueff_o, NULL);
    *tm = *tp = 0.0;
    if (N == 1) return;
    double *u = malloc(sizeof(double) * N), *zero = calloc(N, sizeof(double));
    for (int side = -1; side <= 1; side += 2) {
        int j = o + side;
        if (j < 0 || j >= N) continue;
        /* T u = e_j with no incoming intensity: the source-free system with S = e_j */
        double *e = calloc(N, sizeof(double));
        e[j] = 1.0;
        double uo, lo_, ue_;
        or_solve_ray(N, z, chi, e, 0.0, 0.0, o, tau_floor, &uo, &lo_, &ue_, u);
        if (side < 0) *tm = uo; else *tp = uo;
        free(e);
    }
    free(u);
    free(zero);
}

/* Band ALO of width one node (Sec. 3.4: the diagonal band of the matrix representation
 * of the Lambda operator; here the origin node and its neighbour on each side of every
 * ray pair).  Per selected point and line, besides J, Jeff and L of or_formal_solve:
 *   Ld     L plus the average of (1 - t)(T^-1)_{o,o+-1}: a neighbour node at fraction t of
 *          the first segment toward the first cell c of the walk carries the source
 *          function (1 - t) S_O + t S_c (t = 1 when the neighbour is the cell itself),
 *   Ln[r]  the average of t (T^-1)_{o,o+-1} for the neighbour node along ray r: the
 *          coupling to the first cell of the walk along r (0 without one),
 *   Jb     Jeff minus the average of (T^-1)_{o,o+-1} S_{o+-1}: J without the band's share.
 * Averages are (2/N_rays) sum over pairs and frequencies with the weights w_n, as for L.
 * Ln is [n_sel][n_lines][n_rays]. */
void or_formal_solve_band(const or_ctx *c, const double *pops, int64_t n_sel, const int64_t *sel,
                          double *J, double *Jeff, double *L, double *Jb, double *Ld, double *Ln)
{
    int nl = c->n_lines, nq = c->nq, R = c->n_rays;
    double norm = 2.0 / (double)R;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t s = 0; s < n_sel; ++s) {
        int64_t O = sel ? sel[s] : s;
        double *Js = calloc(nl, sizeof(double)), *Ls = calloc(nl, sizeof(double));
        double *Es = calloc(nl, sizeof(double)), *Bs = calloc(nl, sizeof(double));
        double *Ds = calloc(nl, sizeof(double)), *Ns = calloc((size_t)nl * R, sizeof(double));
        for (int p = 0; p < c->n_pairs; ++p) {
            int r = c->pair_r[p], rb = c->anti[r];
            int io;
            int N = or_pair_nodes(c, pops, O, p, 0, NULL, NULL, NULL, NULL, NULL, &io);
            double *z = malloc(sizeof(double) * N), *a = malloc(sizeof(double) * N);
            double *b = malloc(sizeof(double) * N);
            double *kap = malloc(sizeof(double) * N * nl), *S = malloc(sizeof(double) * N * nl);
            or_pair_nodes(c, pops, O, p, N, z, a, b, kap, S, &io);
            /* fractions of the first segments at which the neighbour nodes lie */
            double tf = 1.0, tb = 1.0;
            int32_t c1;
            if (or_walk(c, O, r, &c1, NULL, 1) > 0)
                tf = 1.0 / n_sub(c->f_sub, 0.0, vproj(c, O, c1, c->dir + 3 * r), c->vw[O], c->vw[c1]);
            if (or_walk(c, O, rb, &c1, NULL, 1) > 0)
                tb = 1.0 / n_sub(c->f_sub, 0.0, vproj(c, O, c1, c->dir + 3 * rb), c->vw[O], c->vw[c1]);
            double *chi = malloc(sizeof(double) * N), *Sl = malloc(sizeof(double) * N);
            for (int l = 0; l < nl; ++l) {
                double Ib = or_planck(c->nu[l], c->t_cmb);
                for (int i = 0; i < N; ++i) Sl[i] = S[i * nl + l];
                for (int n = 0; n < nq; ++n) {
                    for (int i = 0; i < N; ++i) {
                        double x = a[i] * c->qx[n] - b[i];
                        chi[i] = kap[i * nl + l] * exp(-x * x);
                    }
                    double u, lam, ue, tm, tp;
                    solve_ray_band(N, z, chi, Sl, Ib, Ib, io, c->tau_floor, &u, &lam, &ue, &tm, &tp);
                    double w = c->qw[n];
                    Js[l] += w * u;
                    Ls[l] += w * lam;
                    Es[l] += w * ue;
                    double band = 0.0;
                    if (io > 0) band += tm * Sl[io - 1];
                    if (io + 1 < N) band += tp * Sl[io + 1];
                    Bs[l] += w * (ue - band);
                    Ds[l] += w * (lam + (1.0 - tb) * tm + (1.0 - tf) * tp);
                    Ns[(size_t)l * R + r] += w * tf * tp;
                    Ns[(size_t)l * R + rb] += w * tb * tm;
                }
            }
            free(z); free(a); free(b); free(kap); free(S); free(chi); free(Sl);
        }
        for (int l = 0; l < nl; ++l) {
            J[s * nl + l] = norm * Js[l];
            L[s * nl + l] = norm * Ls[l];
            Jeff[s * nl + l] = norm * Es[l];
            Jb[s * nl + l] = norm * Bs[l];
            Ld[s * nl + l] = norm * Ds[l];
            for (int q = 0; q < R; ++q) Ln[((size_t)s * nl + l) * R + q] = norm * Ns[(size_t)l * R + q];
        }
        free(Js); free(Ls); free(Es); free(Bs); free(Ds); free(Ns);
    }
}

/* ------------------------------------------------------------------ scattering */

/*
 * Generalised Feautrier equations on a ray pair (Sec. 3.3, Eq. RTE2 and GFE) with known
 * (previous-iteration) right-hand sides, per node: the total opacity chi = chi_line + chi^+,
 * the odd part of the scattering opacity chim = chi^- along +z (NULL: zero), and
 * Splus = (eta + Psi^+)/(chi + chi^+), sigma = Psi^-/(chi + chi^+).  With dtau = chi dz and
 * mu = chi^-/chi, the operator of Eq. GFE is D = d/dtau + mu, and the first-order pair of
 * Eq. RTE2 reads
 *     D u = sigma - v,    D v = Splus - u.
 * The integrating factor e^M, M(z) = int_{z_o}^{z} chi^- dz' (trapezoid over the nodes, so
 * M_o = 0), makes D e^{-M} = e^{-M} d/dtau exactly: u~ = e^M u and v~ = e^M v obey the pair
 * with mu = 0 and sources e^M Splus, e^M sigma, and the incoming intensities become
 * e^{M_0} I_lo and e^{M_N-1} I_hi.  At the origin u~ = u and v~ = v.  (|M| <= the optical
 * depth from o, since |chi^-| <= chi^+; beyond |M| = 700 the factors leave the FP64 range
 * and the function returns -2.)
 * The transformed pair is discretised with half-node values: from du/dtau = sigma - v,
 * v_{i+1/2} = (sigma_i + sigma_{i+1})/2 - (u_{i+1} - u_i)/dt_{i+1/2}, and integrating
 * dv/dtau = Splus - u over the nodes' cells gives the rows
 *     -A_i u_{i-1} + (1 + A_i + C_i) u_i - C_i u_{i+1} = R_i,
 *     R_i = Splus_i - (sigma_{i+1} - sigma_{i-1})/(dt_- + dt_+),
 * A_i = 2/(dt_-(dt_- + dt_+)), C_i = 2/(dt_+(dt_- + dt_+)); the boundary rows (incoming
 * I_lo along +z at node 0, I_hi along -z at node N-1: v_0 = I_lo - u_0, v_{N-1} = u_{N-1} -
 * I_hi, half-cell integration) have C_0 = A_{N-1} = 2/dt^2 and
 *     R_0 = Splus_0 + (2/dt)(I_lo - (sigma_0 + sigma_1)/2),
 *     R_{N-1} = Splus_{N-1} + (2/dt)(I_hi + (sigma_{N-2} + sigma_{N-1})/2).
 * The second equation of Eq. GFE, (1 - D^2) v = sigma - D Splus, is the same pair with the
 * roles of Splus and sigma exchanged (half-node u from dv/dtau, cells integrating du/dtau,
 * u_0 = I_lo - v_0, u_{N-1} = I_hi + v_{N-1}): the same matrix with
 *     Rv_i = sigma_i - (Splus_{i+1} - Splus_{i-1})/(dt_- + dt_+),
 *     Rv_0 = sigma_0 + (2/dt)(I_lo - (Splus_0 + Splus_1)/2),
 *     Rv_{N-1} = sigma_{N-1} + (2/dt)((Splus_{N-2} + Splus_{N-1})/2 - I_hi).
 * With chim = NULL and sigma = 0 the u rows are exactly those of or_solve_ray.
 * Both right-hand sides go through one Rybicki-Hummer elimination from both ends toward o
 * (F, z from node 0, G, w from node N-1) and the two-sided combine at o.  Outputs at node
 * o: u_o, Lambda_oo (diagonal of the inverse), ueff_o (u with `own` removed from R_o) and
 * v_o = (I(+z) - I(-z))/2; a single node has u = (I_lo + I_hi)/2, v = (I_lo - I_hi)/2.
 */
int or_solve_ray_gen(int N, const double *z, const double *chi, const double *chim, const double *Splus,
                     const double *sigma, double I_lo, double I_hi, int o, double tau_floor, double own,
                     double *u_o, double *lam_o, double *ueff_o, double *v_o)
{
    if (N == 1) {
        *u_o = 0.5 * (I_lo + I_hi);
        *lam_o = 0.0;
        *ueff_o = *u_o;
        *v_o = 0.5 * (I_lo - I_hi);
        return 0;
    }
    double *E = malloc(sizeof(double) * N), *Sp = malloc(sizeof(double) * N), *sg = malloc(sizeof(double) * N);
    /* integrating factor e^M, M_o = 0 */
    double M = 0.0;
    int bad = 0;
    E[o] = 1.0;
    for (int i = o + 1; i < N; ++i) {
        if (chim) M += 0.5 * (chim[i - 1] + chim[i]) * (z[i] - z[i - 1]);
        if (fabs(M) > 700.0) bad = 1;
        E[i] = exp(M);
    }
    M = 0.0;
    for (int i = o - 1; i >= 0; --i) {
        if (chim) M -= 0.5 * (chim[i] + chim[i + 1]) * (z[i + 1] - z[i]);
        if (fabs(M) > 700.0) bad = 1;
        E[i] = exp(M);
    }
    if (bad) {
        free(E); free(Sp); free(sg);
        return -2;
    }
    for (int i = 0; i < N; ++i) {
        Sp[i] = E[i] * Splus[i];
        sg[i] = E[i] * sigma[i];
    }
    I_lo *= E[0];
    I_hi *= E[N - 1];

    double *dt = malloc(sizeof(double) * N);
    double *Ac = calloc(N, sizeof(double)), *Cc = calloc(N, sizeof(double));
    double *Hc = malloc(sizeof(double) * N), *R = malloc(sizeof(double) * N), *Rv = malloc(sizeof(double) * N);
    double *F = malloc(sizeof(double) * N), *zz = malloc(sizeof(double) * N), *zv = malloc(sizeof(double) * N);
    double *G = malloc(sizeof(double) * N), *ww = malloc(sizeof(double) * N), *wv = malloc(sizeof(double) * N);
    for (int i = 0; i + 1 < N; ++i) {
        double d = 0.5 * (chi[i] + chi[i + 1]) * (z[i + 1] - z[i]);
        dt[i] = d > tau_floor ? d : tau_floor;
    }
    for (int i = 0; i < N; ++i) Hc[i] = 1.0;
    Cc[0] = 2.0 / (dt[0] * dt[0]);
    Hc[0] = 1.0 + 2.0 / dt[0];
    R[0] = Sp[0] + 2.0 / dt[0] * (I_lo - 0.5 * (sg[0] + sg[1]));
    Rv[0] = sg[0] + 2.0 / dt[0] * (I_lo - 0.5 * (Sp[0] + Sp[1]));
    for (int i = 1; i < N - 1; ++i) {
        Ac[i] = 2.0 / (dt[i - 1] * (dt[i - 1] + dt[i]));
        Cc[i] = 2.0 / (dt[i] * (dt[i - 1] + dt[i]));
        R[i] = Sp[i] - (sg[i + 1] - sg[i - 1]) / (dt[i - 1] + dt[i]);
        Rv[i] = sg[i] - (Sp[i + 1] - Sp[i - 1]) / (dt[i - 1] + dt[i]);
    }
    Ac[N - 1] = 2.0 / (dt[N - 2] * dt[N - 2]);
    Hc[N - 1] = 1.0 + 2.0 / dt[N - 2];
    R[N - 1] = Sp[N - 1] + 2.0 / dt[N - 2] * (I_hi + 0.5 * (sg[N - 2] + sg[N - 1]));
    Rv[N - 1] = sg[N - 1] + 2.0 / dt[N - 2] * (0.5 * (Sp[N - 2] + Sp[N - 1]) - I_hi);

    /* Rybicki-Hummer elimination from both ends toward o: x_{i-1} = zz_{i-1} + x_i/(1 + F_{i-1})
     * below o and x_{i+1} = ww_{i+1} + x_i/(1 + G_{i+1}) above it (zz, ww for u; zv, wv for v) */
    for (int i = 0; i < o; ++i) {
        double q = i > 0 ? Ac[i] * F[i - 1] / (1.0 + F[i - 1]) : 0.0;
        F[i] = (Hc[i] + q) / Cc[i];
        zz[i] = (R[i] + (i > 0 ? Ac[i] * zz[i - 1] : 0.0)) / (Cc[i] * (1.0 + F[i]));
        zv[i] = (Rv[i] + (i > 0 ? Ac[i] * zv[i - 1] : 0.0)) / (Cc[i] * (1.0 + F[i]));
    }
    for (int i = N - 1; i > o; --i) {
        double q = i < N - 1 ? Cc[i] * G[i + 1] / (1.0 + G[i + 1]) : 0.0;
        G[i] = (Hc[i] + q) / Ac[i];
        ww[i] = (R[i] + (i < N - 1 ? Cc[i] * ww[i + 1] : 0.0)) / (Ac[i] * (1.0 + G[i]));
        wv[i] = (Rv[i] + (i < N - 1 ? Cc[i] * wv[i + 1] : 0.0)) / (Ac[i] * (1.0 + G[i]));
    }
    double den = Hc[o], num = R[o], numv = Rv[o];
    if (o > 0) {
        den += Ac[o] * F[o - 1] / (1.0 + F[o - 1]);
        num += Ac[o] * zz[o - 1];
        numv += Ac[o] * zv[o - 1];
    }
    if (o < N - 1) {
        den += Cc[o] * G[o + 1] / (1.0 + G[o + 1]);
        num += Cc[o] * ww[o + 1];
        numv += Cc[o] * wv[o + 1];
    }
    *u_o = num / den;
    *lam_o = 1.0 / den;
    *ueff_o = (num - own) / den;
    *v_o = numv / den;
    free(E); free(Sp); free(sg);
    free(dt); free(Ac); free(Cc); free(Hc); free(R); free(Rv); free(F); free(zz); free(zv);
    free(G); free(ww); free(wv);
    return 0;
}

/* J_nu of point q, line l at offset x (in q's line widths, q's frame): linear in x
 * between the quadrature offsets (ascending), constant beyond the outermost ones. */
static double jnu_at(const or_ctx *c, const double *Jnu, int64_t q, int l, double x)
{
    const double *row = Jnu + ((size_t)q * c->n_lines + l) * c->nq;
    int nq = c->nq;
    if (x <= c->qx[0]) return row[0];
    if (x >= c->qx[nq - 1]) return row[nq - 1];
    int i = 0;
    while (c->qx[i + 1] <= x) ++i;
    double t = (x - c->qx[i]) / (c->qx[i + 1] - c->qx[i]);
    return row[i] + t * (row[i + 1] - row[i]);
}

/*
 * Formal solve with scattering (Sec. 2.1 Eq. RTE, 3.3, 3.4).  The scattering opacity of
 * direction n is chi_sca + chi_dip . n (cm^-1; chi_sca [P][n_lines], chi_dip
 * [P][n_lines][3] or NULL for zero, |chi_dip| <= chi_sca so that it is nowhere negative),
 * grey over each line's frequencies, so chi^+ = chi_sca and chi^- = chi_dip . n.  The
 * scattering is coherent in the comoving frame of the scatterer, with the redistribution
 * Phi(n, n') = chi_s(n) chi_s(n') / (4 pi chi_sca) (chi_s(n) the opacity of direction n):
 * the radiation removed from every direction is re-emitted in all (energy is conserved,
 * int Phi dOmega = chi_s(n')), and I = B solves every direction in thermal equilibrium
 * (int Phi dOmega' = chi_s(n)).  At offset y (widths, the scatterer's frame) the
 * emissivity into n is then chi_s(n) Jw(y), Jw = (1/4pi) int w(n') I(n', y) dOmega' with
 * w(n) = chi_s(n)/chi_sca = 1 + (chi_dip . n)/chi_sca (w = 1 where chi_sca = 0; Jw is the
 * mean intensity J_nu when chi_dip = 0).  Jw comes from the previous iteration (Jnu_in
 * [P][n_lines][n_q], at the quadrature offsets, interpolated by jnu_at).  The pair at lane
 * offset x joins I(n, x) and I(-n, -x); at a node whose offset is y = a x - b, with
 * chi^- = chi_dip . n there, the two directions receive (chi_sca + chi^-) Jw(y) and
 * (chi_sca - chi^-) Jw(-y), and Psi^+-, the half sum and half difference of these, give
 * with chi_tot = chi_line + chi_sca:  Splus = (chi_line S + Psi^+)/chi_tot,
 * sigma = Psi^-/chi_tot (where chi_tot = 0, Splus = S, the limit as the line opacity
 * vanishes without scattering, and sigma = 0).  Velocity sub-steps interpolate
 * chi_sca, chi_dip . n and the Jw of the segment's end cells linearly in t, at the
 * sub-step's own offset.  Per selected point and line:
 *   J     (2/N_rays) sum_pairs sum_n w_n u_o,
 *   L     (2/N_rays) sum sum w_n Lambda_oo chi_line,o/chi_tot,o     (Eq. ALO),
 *   Jeff  (2/N_rays) sum sum w_n (u_o - Lambda_oo (chi_line,o/chi_tot,o) S_o),
 *         with the share chi_line,o/chi_tot,o taken as 1 where chi_tot,o = 0,
 *   Jnu_out[n] = (1/N_rays) sum over pairs of w_o(n) I(n, x_n) + w_o(-n) I(-n, x_n), with
 *         I(n, x) = u(x) + v(x) and I(-n, x) = u(-x) - v(-x) (the mirrored offset), u and v
 *         from the two equations of Eq. GFE (or_solve_ray_gen).
 * Returns -1 unless the quadrature is ascending (and, as always, symmetric), -3 if some
 * |chi_dip| exceeds chi_sca (by more than 1e-12 relative), -2 if a ray leaves the range
 * of or_solve_ray_gen's integrating factor.
 */
int or_formal_solve_scat(const or_ctx *c, const double *pops, const double *chi_sca, const double *chi_dip,
                         const double *Jnu_in, int64_t n_sel, const int64_t *sel, double *J,
                         double *Jeff, double *L, double *Jnu_out)
{
    int nl = c->n_lines, nq = c->nq;
    for (int n = 0; n + 1 < nq; ++n)
        if (!(c->qx[n] < c->qx[n + 1])) return -1;
    if (chi_dip)
        for (int64_t i = 0; i < c->P * nl; ++i) {
            const double *d = chi_dip + 3 * i;
            if (!(sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]) <= chi_sca[i] * (1.0 + 1e-12))) return -3;
        }
    double norm = 2.0 / (double)c->n_rays;
    int status = 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t s = 0; s < n_sel; ++s) {
        int64_t O = sel ? sel[s] : s;
        double *Js = calloc(nl, sizeof(double)), *Ls = calloc(nl, sizeof(double));
        double *Es = calloc(nl, sizeof(double));
        double *Jp = calloc((size_t)nl * nq, sizeof(double)), *Jm = calloc((size_t)nl * nq, sizeof(double));
        for (int p = 0; p < c->n_pairs; ++p) {
            int io;
            int N = pair_nodes_src(c, pops, O, p, 0, NULL, NULL, NULL, NULL, NULL, NULL, NULL, NULL, &io);
            double *z = malloc(sizeof(double) * N), *a = malloc(sizeof(double) * N);
            double *b = malloc(sizeof(double) * N), *th = malloc(sizeof(double) * N);
            int64_t *clo = malloc(sizeof(int64_t) * N), *chh = malloc(sizeof(int64_t) * N);
            double *kap = malloc(sizeof(double) * N * nl), *S = malloc(sizeof(double) * N * nl);
            pair_nodes_src(c, pops, O, p, N, z, a, b, kap, S, clo, chh, th, &io);
            double *ct = malloc(sizeof(double) * N), *Sp = malloc(sizeof(double) * N);
            double *sg = malloc(sizeof(double) * N), *cm = malloc(sizeof(double) * N);
            const double *nr = c->dir + 3 * c->pair_r[p];   /* +z of the pair's nodes */
            for (int l = 0; l < nl; ++l) {
                double Ib = or_planck(c->nu[l], c->t_cmb);
                /* chi^- along +z at every node, and the weights of the two directions at O */
                double wp = 1.0, wm = 1.0;
                for (int i = 0; i < N; ++i) {
                    double t = th[i], mlo = 0.0, mhi = 0.0;
                    if (chi_dip) {
                        const double *dl = chi_dip + 3 * (clo[i] * nl + l), *dh = chi_dip + 3 * (chh[i] * nl + l);
                        mlo = dl[0] * nr[0] + dl[1] * nr[1] + dl[2] * nr[2];
                        mhi = dh[0] * nr[0] + dh[1] * nr[1] + dh[2] * nr[2];
                    }
                    cm[i] = (1.0 - t) * mlo + t * mhi;
                }
                if (chi_sca[O * nl + l] > 0.0) {
                    wp = 1.0 + cm[io] / chi_sca[O * nl + l];
                    wm = 1.0 - cm[io] / chi_sca[O * nl + l];
                }
                for (int n = 0; n < nq; ++n) {
                    double clO = 0.0, ctO = 0.0;
                    for (int i = 0; i < N; ++i) {
                        double y = a[i] * c->qx[n] - b[i];
                        double cl = kap[i * nl + l] * exp(-y * y);
                        double t = th[i];
                        double cs = (1.0 - t) * chi_sca[clo[i] * nl + l] + t * chi_sca[chh[i] * nl + l];
                        double jp = (1.0 - t) * jnu_at(c, Jnu_in, clo[i], l, y) + t * jnu_at(c, Jnu_in, chh[i], l, y);
                        double jm = (1.0 - t) * jnu_at(c, Jnu_in, clo[i], l, -y) + t * jnu_at(c, Jnu_in, chh[i], l, -y);
                        /* emissivities into +z (offset y) and -z (offset -y) */
                        double psi_p = (cs + cm[i]) * jp, psi_m = (cs - cm[i]) * jm;
                        double tot = cl + cs;
                        ct[i] = tot;
                        /* (chi_line S + Psi^+)/chi_tot as (chi_line/chi_tot) S + Psi^+/chi_tot: the
                         * same value, but chi_line S does not underflow where the line opacity is
                         * denormal (without scattering the share is then exactly 1); with no
                         * opacity at all the line's S, the limit as its opacity goes to zero, as
                         * in the line-only solve */
                        double share_i = tot > 0.0 ? cl / tot : 1.0;
                        Sp[i] = share_i * S[i * nl + l] + (tot > 0.0 ? 0.5 * (psi_p + psi_m) / tot : 0.0);
                        sg[i] = tot > 0.0 ? 0.5 * (psi_p - psi_m) / tot : 0.0;
                        if (i == io) {
                            clO = cl;
                            ctO = tot;
                        }
                    }
                    /* the line's share of O's source; all of it where O has no opacity at all
                     * (as in the line-only solve) */
                    double share = ctO > 0.0 ? clO / ctO : 1.0;
                    double own = share * S[io * nl + l];
                    double u, lam, ue, v;
                    if (or_solve_ray_gen(N, z, ct, chi_dip ? cm : NULL, Sp, sg, Ib, Ib, io, c->tau_floor, own, &u,
                                         &lam, &ue, &v) != 0) {
#pragma omp atomic write
                        status = -2;
                    }
                    double w = c->qw[n];
                    Js[l] += w * u;
                    Ls[l] += w * lam * share;
                    Es[l] += w * ue;
                    Jp[(size_t)l * nq + n] += wp * (u + v);
                    Jm[(size_t)l * nq + n] += wm * (u - v);
                }
            }
            free(z); free(a); free(b); free(th); free(clo); free(chh); free(kap); free(S);
            free(ct); free(Sp); free(sg); free(cm);
        }
        for (int l = 0; l < nl; ++l) {
            J[s * nl + l] = norm * Js[l];
            L[s * nl + l] = norm * Ls[l];
            Jeff[s * nl + l] = norm * Es[l];
            for (int n = 0; n < nq; ++n)
                Jnu_out[((size_t)s * nl + l) * nq + n] =
                    (Jp[(size_t)l * nq + n] + Jm[(size_t)l * nq + (nq - 1 - n)]) / (double)c->n_rays;
        }
        free(Js); free(Ls); free(Es); free(Jp); free(Jm);
    }
    return status;
}

/* Threads of the OpenMP loops over origin points (timing runs). */
void or_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
