/*
 * nlte.h -- C ABI of the MI355X (gfx950) non-LTE line radiative-transfer library.
 *
 * The library implements the hot path of the accelerated Lambda iteration (ALI) of
 * De Ceuster et al., "Magritte I: non-LTE atomic and molecular line modelling":
 * rays traced over a point cloud with nearest-neighbour lists (Sec. 3.2), the
 * second-order (Feautrier) transfer equation solved on every antipodal ray pair at
 * every Doppler-shifted line frequency (Sec. 3.3), accumulation of the mean intensity
 * J and of the diagonal approximate Lambda operator (Sec. 2.2.1, 3.4), and the
 * per-point statistical-equilibrium update that consumes them (Eq. ourALI).
 *
 * Conventions
 *   - CGS units; arrays are dense and row-major; indices are 0-based.
 *   - The caller owns every buffer.  The library copies what it keeps and never
 *     retains or frees a caller pointer.  Host-pointer calls copy in and out and return
 *     when the results are in the caller's buffers.  *_dev calls take device pointers
 *     and a hipStream_t (passed as void*, NULL = the context's own stream); they only
 *     enqueue work, so the caller synchronises that stream before reading results.  The
 *     context's own stream is a blocking stream: it is ordered with the legacy default
 *     (null) stream both ways, so work that a caller enqueues on the null stream before
 *     or after a call with NULL is ordered with that call's work.
 *   - Return codes: NLTE_OK (0); errors are negative, warnings positive.  After any
 *     non-zero code nlte_last_error() describes it.  No C++ exception crosses the ABI.
 *   - A context is bound to one HIP device and is not thread-safe: use one context per
 *     host thread.  Calls must follow the order create -> set_species -> set_model(s)
 *     -> set_rays -> set_quadrature -> [set_params] -> trace -> compute calls;
 *     NLTE_E_STATE reports a call made before its prerequisites.
 */
#ifndef NLTE_H
#define NLTE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct nlte_ctx nlte_ctx;
typedef int nlte_status;

#define NLTE_OK 0
#define NLTE_E_INVALID_ARG (-1) /* an argument is out of range, non-finite or inconsistent */
#define NLTE_E_STATE (-2)       /* a prerequisite call is missing */
#define NLTE_E_OOM (-3)         /* device or host allocation failed */
#define NLTE_E_HIP (-4)         /* a HIP runtime call failed */
#define NLTE_W_NOT_CONVERGED 1  /* ALI stopped at max_iter above tol */
#define NLTE_W_NONPHYSICAL 2    /* some points fell back or kept their old populations */

/* Arithmetic used by the formal solve. */
#define NLTE_PREC_FP64 0      /* every step in FP64 */
#define NLTE_PREC_FP32_BULK 1 /* FP32 profile, opacity, optical depth, source function and
                                 J accumulation; FP64 Feautrier elimination and stat-eq */

typedef struct {
    double t_cmb;     /* boundary (CMB) temperature [K]; incoming intensity B_nu(t_cmb) at the
                         line-centre frequency on both ends of every ray pair (Sec. 4.1). 2.725 */
    double f_sub;     /* velocity sub-step fraction: a segment whose projected velocity
                         changes by more than f_sub times the smaller line-width speed of its
                         two ends is split into equal parts (Sec. 3.1.1, 3.2).  0.25 */
    double tol;       /* ALI stops when the maximum relative population change is below tol */
    int max_iter;     /* ALI iteration cap */
    int use_alo;      /* 1: diagonal ALO (Sec. 3.4); 0: plain Lambda iteration */
    int precision;    /* NLTE_PREC_* */
    int profile;      /* 1: time every kernel with HIP events (nlte_kernel_stats); the ALI
                         then launches kernels one by one instead of replaying a graph */
    int use_graph;    /* 1: capture one ALI iteration as a hipGraph and replay it.  1 */
    int lines_per_lane; /* formal-solve lines per lane, 1..5 (0 = by rule: the fewest waves per
                           point, then the fewest lines per lane); the lines of a lane share
                           its profile evaluations.  0 */
    int waves_per_simd; /* formal-solve register budget: 1, 2 or 3 waves per SIMD (1: the whole
                           register file, 512 with the accumulation registers; 3: 168);
                           0 = by rule (3 in the FP32 form and up to two lines per lane in
                           FP64, else 2).  0 */
    int persistent;   /* 1: persistent formal solve taking points from a work queue in
                         decreasing order of their cached step counts; 0: one workgroup per
                         tile of points in index order (XCD-contiguous).  1 */
    int ng_every;     /* Ng acceleration (Sec. 3.4): after every ng_every regular ALI
                         iterations each model still iterating takes the combination of its
                         last ng_every - 1 iterates, summing to one, that minimises the same
                         combination of successive changes in the fractional populations
                         (uniform weights); points where it is not positive keep the newest
                         iterate.  0 = off, else 3..8 (the paper's default is 4).  0 */
    int alo_band;     /* 1: band ALO of one node on each side of the origin (Sec. 3.4; see
                         nlte_formal_solve_band), the coupled rate equations of all points
                         solved together each iteration; a model whose band populations are
                         not all positive takes the local (diagonal) solve (Sec. 6.1).
                         FP64 formal solve whatever the precision; no graph replay.  Needs
                         use_alo.  0 */
    int long_segments; /* velocity sub-step segments (Sec. 3.2) in the formal solve: 1 = long
                         segments: along a segment's sub-steps the line profile follows a
                         multiplicative recurrence, and a segment that lies beyond the
                         profile's range for every frequency of a wave is eliminated in one
                         step (it has no opacity); 0 = short segments: every sub-step node
                         evaluates its profile; -1 = by the trace (long when the cached walks
                         average more than two elimination steps per cell).  The two agree
                         to rounding.  -1 */
    int stage_nodes;  /* ray nodes a formal-solve wave stages in LDS at a time, 2..64 (0 = by
                         rule: the most that keep the register budget's occupancy).  0 */
    int tile_points;  /* formal-solve work items (point, line block) a workgroup takes at a time,
                         1..16 (0 = 1): the grid launch gives each workgroup that many
                         consecutive items, the persistent launch takes that many from the
                         queue per atomic.  Results do not depend on it.  0 */
} nlte_params;

/* Defaults listed above; max_iter 50, tol 1e-4, use_alo 1, precision FP64, profile 0, ng_every 0,
 * alo_band 0, long_segments -1, stage_nodes 0, tile_points 0. */
void nlte_default_params(nlte_params *p);

typedef struct {
    int iterations;          /* ALI iterations performed */
    int converged;           /* 1 if the last change was below tol */
    double max_change[1024]; /* per-iteration max relative change over the models still
                                iterating (first min(iters,1024)) */
    double mean_change[1024];/* per-iteration mean relative change over the same entries */
    int64_t n_models_converged; /* models whose change fell below tol */
    int64_t n_fallback;      /* stat-eq solves that fell back to plain Lambda (last iteration) */
    int64_t n_kept;          /* points that kept their previous populations (last iteration) */
    int64_t n_maser;         /* (point, line) pairs with non-positive opacity (last iteration) */
    double ms_total;         /* wall time of the iteration loop [ms] */
    int n_ng_steps;          /* Ng extrapolations applied (ng_every > 0) */
    int64_t n_ng_rejected;   /* points that kept the newest iterate in those steps */
    int n_band;              /* iterations in which at least one model kept the band ALO's
                                populations (alo_band) */
} nlte_ali_report;

/* ---------------------------------------------------------------- context */

/* Create a context on HIP device `hip_device`.  *out receives the handle. */
nlte_status nlte_create(nlte_ctx **out, int hip_device);
/* Free the context and every device buffer it owns.  NULL is allowed.  Waits first for
 * all work on the context's device, so that work which a *_dev call enqueued on a caller's
 * stream and which reads the context's buffers has finished before they are freed. */
void nlte_destroy(nlte_ctx *ctx);
/* Text of the last error or warning on this context (valid until the next call). */
const char *nlte_last_error(const nlte_ctx *ctx);

/* ---------------------------------------------------------------- inputs */

/*
 * Species (Sec. 2.2.1).  n_lev levels with energies E [erg] and statistical weights g;
 * species mass [g] for the thermal speed sqrt(2kT/m).  n_lines radiative lines
 * up[l] -> lo[l] (E[up] > E[lo]) with Einstein A_ul [s^-1]; line frequency
 * nu = (E_up - E_lo)/h, B_ul = A_ul c^2/(2 h nu^3), B_lu = (g_up/g_lo) B_ul.
 * n_coll collisional pairs c_up[c] -> c_lo[c] with H2 de-excitation coefficients
 * K_ul[c][t] [cm^3 s^-1] tabulated at n_T strictly increasing temperatures T_K[t],
 * interpolated linearly in T and clamped at the ends; excitation follows from
 * detailed balance C_lu = C_ul (g_u/g_l) exp(-(E_u - E_l)/kT).
 * Limits: 2 <= n_lev <= 16, 1 <= n_lines <= 32, 0 <= n_coll <= 256, 1 <= n_T <= 256.
 */
nlte_status nlte_set_species(nlte_ctx *ctx, int n_lev, const double *E, const double *g,
                             double mass, int n_lines, const int32_t *up, const int32_t *lo,
                             const double *A_ul, int n_coll, const int32_t *c_up,
                             const int32_t *c_lo, int n_T, const double *T_K,
                             const double *K_ul);

/*
 * Model(s): the point cloud with nearest-neighbour lists (Sec. 3.1.1).  n_models models
 * are stored back to back; model m owns points offsets[m] .. offsets[m+1]-1, with
 * offsets [n_models+1] required, offsets[0] = 0 and P = offsets[n_models] (one model:
 * {0, P}).  Must follow nlte_set_species (which invalidates a previous model, since the
 * line widths depend on the species mass).  Per point: pos [P][3] cm, vel [P][3] cm/s,
 * n_h2 [P] cm^-3, T [P] K, v_turb [P] cm/s, abundance [P] (species per H2);
 * nbr [P][k] neighbour indices local to the point's model, -1 = unused slot (no self
 * references).  boundary (nullable) [P]: 1 marks points where rays end (Sec. 3.1.1).
 * Invalidates a previous trace.
 */
nlte_status nlte_set_models(nlte_ctx *ctx, int n_models, const int64_t *offsets,
                            const double *pos, const double *vel, const double *n_h2,
                            const double *T, const double *v_turb, const double *abundance,
                            int k, const int32_t *nbr, const uint8_t *boundary);

/*
 * Ray directions (Sec. 3.1.3): n_rays unit vectors [n][3] forming antipodal pairs
 * (every direction's negative is in the set within 1e-12).  The pair representative is
 * the lower index; n_rays <= 1024.  Invalidates a previous trace.
 */
nlte_status nlte_set_rays(nlte_ctx *ctx, int n_rays, const double *dir);

/*
 * The 12 nside^2 HEALPix pixel centres (Sec. 3.1.3: rays along the centres of HEALPix
 * pixels; RING scheme of Gorski et al. 2005, ring by ring from the north pole) as the
 * ray set, nside 1..9 (up to 972 rays); as nlte_set_rays otherwise.
 */
nlte_status nlte_set_rays_healpix(nlte_ctx *ctx, int nside);

/* The current ray set: *n_rays (nullable) and, if dir is not NULL, the directions
 * [n_rays][3] (host memory of the caller).  E_STATE before any rays are set. */
nlte_status nlte_get_rays(nlte_ctx *ctx, int *n_rays, double *dir);

/*
 * Frequency quadrature (Sec. 3.1.2): offsets x[n] in units of the local line width and
 * weights w[n] against the normalised profile, symmetric (x[n] = -x[N-1-n],
 * w[n] = w[N-1-n] within 1e-12) with sum w = 1 within 1e-12.  1 <= n_q <= 256.
 */
nlte_status nlte_set_quadrature(nlte_ctx *ctx, int n_q, const double *x, const double *w);

nlte_status nlte_set_params(nlte_ctx *ctx, const nlte_params *p);

/* ---------------------------------------------------------------- ray walk */

/*
 * Trace every (point, ray) once (Sec. 3.2): from the current cell step to the neighbour
 * whose projection on the ray lies farther than the current one and which is closest
 * to the line through the origin point; stop when no such neighbour exists or at a
 * flagged boundary point.  Exact distance ties go to the lower point index.  The cell
 * lists are cached on the device for all later sweeps.
 */
nlte_status nlte_trace(nlte_ctx *ctx);

/* Cells met by ray `ray` from global point `point`, nearest first.  Copies up to cap
 * indices (model-local, like nbr) into cells; *len receives the full length.  The velocity
 * sub-step counts of the segments between them (Sec. 3.2) are not part of the cache: every
 * sweep recomputes them from the cell records (the same FP64 decision as the walk's), so
 * there is no per-segment count to return; nlte_get_point_cost gives their sum per point. */
nlte_status nlte_get_ray(nlte_ctx *ctx, int64_t point, int ray, int32_t *cells, int cap,
                         int *len);

/* Processing order of the points (set by nlte_set_models): within each model, by the
 * Morton code of the coordinates quantised to 21 bits over the model's bounding box,
 * q = floor((x - min) / (max - min) * (2^21 - 1)) (0 for a flat extent), bits interleaved
 * x, y, z from the most significant; equal codes in index order.  perm [P]: the global
 * index of the point at each position: the order in which points would be split into
 * contiguous shards across devices.  (The formal solve on one device keeps index order,
 * which measured as fast or faster; results do not depend on the order.) */
nlte_status nlte_get_order(nlte_ctx *ctx, int64_t *perm);

/* Total cached cells over all (point, ray), the longest ray, and the number of
 * elimination steps one frequency of one line takes over all half rays (cells plus
 * velocity sub-steps); any output pointer may be NULL. */
nlte_status nlte_trace_stats(nlte_ctx *ctx, int64_t *total_cells, int *max_len,
                             int64_t *total_steps);

/* Work per origin point as the trace counts it (Sec. 3.2 walks with the velocity
 * sub-steps of Sec. 3.2.1): for each point, the sum over its rays of the ray's elimination
 * steps for one frequency of one line (one per cached cell, or that cell's number of
 * sub-steps) plus one.  cost [P] (host).  The persistent formal solve hands out points in
 * decreasing order of this cost. */
nlte_status nlte_get_point_cost(nlte_ctx *ctx, int64_t *cost);

/* Per-point line-width speed sqrt(2kT/m + v_turb^2) [cm/s] as the kernels use it. */
nlte_status nlte_get_line_width_speed(nlte_ctx *ctx, double *vw);

/* ---------------------------------------------------------------- one ALI step */

/* Boltzmann populations at the local temperature, scaled to abundance * n_h2.
 * pops [P][n_lev]. */
nlte_status nlte_lte(nlte_ctx *ctx, double *pops);
nlte_status nlte_lte_dev(nlte_ctx *ctx, double *d_pops, void *stream);

/*
 * One formal-solve sweep with populations pops [P][n_lev]:
 *   J    [P][n_lines]  mean intensity in the line (Eq. meanIntensity, ray average of
 *                      Sec. 3.1.3, u pairs I(n, x) with I(-n, -x)),
 *   Jeff [P][n_lines]  J - L*[S], the part of J not produced by the point's own source
 *                      function (Eq. ourJeff),
 *   Lstar[P][n_lines]  diagonal of the line-averaged Lambda operator (Eq. ALO).
 */
nlte_status nlte_formal_solve(nlte_ctx *ctx, const double *pops, double *J, double *Jeff,
                              double *Lstar);
nlte_status nlte_formal_solve_dev(nlte_ctx *ctx, const double *d_pops, double *d_J,
                                  double *d_Jeff, double *d_Lstar, void *stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation): nlte_formal_solve_dev with the same
 * arguments, results and kernels, which allocates nothing.  Its scratch (the per-(point,
 * line) opacity and source staging and the work-queue counter) lives in a fixed array of
 * 64 MiB in the library's device code, one per GPU, held until the process ends, instead
 * of the context's buffers.  It takes P * n_lines <= 4,194,288 in FP64 (8,388,576 in the
 * FP32 form); larger models get NLTE_E_INVALID_ARG (use nlte_formal_solve_dev).  Every
 * call on one GPU shares that GPU's array, from any context: calls that overlap on one GPU
 * (two streams, two threads) race and must be ordered by the caller.  The counter is
 * cleared by a kernel on `stream` at each call (no memset node), so the call can be
 * captured.  No kernel timing or step counting (params.profile is ignored).
 */
nlte_status nlte_formal_solve_noalloc_dev(nlte_ctx *ctx, const double *d_pops, double *d_J,
                                          double *d_Jeff, double *d_Lstar, void *stream);

/*
 * Statistical equilibrium (Eq. ourALI with the diagonal ALO): per point the rates
 * u->l = A(1 - L*) + B_ul Jeff + C_ul and l->u = B_lu Jeff + C_lu, the first level's
 * equation replaced by sum_i n_i = abundance * n_h2, solved by Gaussian elimination
 * with partial pivoting.  A solution with a non-positive or non-finite population is
 * redone without the ALO (L* = 0, Jeff = J); if that also fails the point keeps
 * pops_old (Sec. 6.1).  flags [P] (nullable): 0 ok, 1 fell back, 2 kept old.
 * With use_alo = 0 the plain Lambda-iteration rates are used directly.
 */
nlte_status nlte_stateq(nlte_ctx *ctx, const double *pops_old, const double *J,
                        const double *Jeff, const double *Lstar, double *pops_new,
                        uint8_t *flags);
nlte_status nlte_stateq_dev(nlte_ctx *ctx, const double *d_pops_old, const double *d_J,
                            const double *d_Jeff, const double *d_Lstar, double *d_pops_new,
                            uint8_t *d_flags, void *stream);

/*
 * Band ALO (Sec. 3.4: the diagonal band of the matrix representation of the Lambda
 * operator), one node on each side of the origin of every ray pair.  With T the pair's
 * system matrix, (T^-1)_{O,O+-1} is the weight of the neighbour node's source function in
 * u_O.  A neighbour node at fraction t of the first segment toward the first cell c of the
 * walk (t = 1 when it is c) carries (1 - t) S_O + t S_c.  Per point and line, averaged over
 * rays and frequencies like L*:
 *   Ld [P][n_lines]          L* plus the (1 - t) shares,
 *   Ln [P][n_lines][n_rays]  the t shares, coupling to the first cell of the walk along
 *                            each ray (0 without one),
 *   Jb [P][n_lines]          Jeff minus the band's contribution of the current source
 *                            functions.
 * J, Jeff, Lstar as nlte_formal_solve.  All arrays host memory of the caller.  FP64
 * whatever the precision setting; lines_per_lane above 2 is taken as 2.
 */
nlte_status nlte_formal_solve_band(nlte_ctx *ctx, const double *pops, double *J, double *Jeff,
                                   double *Lstar, double *Jb, double *Ld, double *Ln);

/*
 * Statistical equilibrium with the band ALO: the rate equations of all points together,
 * per point as nlte_stateq with L* := Ld and Jeff := Jb, plus for every line (u -> l) and
 * ray the coupling -A (k_O / k_c) Ln n_u,c of the first cell c in the net downward rate
 * (k = h nu/4pi (n_l B_lu - n_u B_ul) with pops_old; no coupling where either k is not
 * positive).  Solved by BiCGSTAB preconditioned with the points' own rate matrices, from
 * their uncoupled solution, to a weighted relative residual of 1e-13.  Per model: a model
 * with a singular local matrix, or with a population that is not positive and finite,
 * takes the local solve of nlte_stateq with J, Jeff, Lstar (Sec. 6.1), the others keep the
 * band's populations; if the solver fails, every model takes the local solve.
 * *band_used (nullable): the number of models that kept the band's populations;
 * *solver_iterations (nullable): solver steps.  Host arrays; needs use_alo.
 */
nlte_status nlte_stateq_band(nlte_ctx *ctx, const double *pops_old, const double *J,
                             const double *Jeff, const double *Lstar, const double *Jb,
                             const double *Ld, const double *Ln, double *pops_new, int *band_used,
                             int *solver_iterations);

/*
 * Scattering (Sec. 2.1 Eq. RTE; Sec. 3.3 Eq. RTE2, GFE).  chi_sca [P][n_lines] (cm^-1, >= 0,
 * host, copied) is the scattering opacity, grey over each line's frequencies, isotropic
 * unless nlte_set_scattering_dipole adds an odd part.  Scattering is coherent in the
 * comoving frame of each point.  The formal solve then solves both equations of the
 * generalised Feautrier form (u and the flux-like v) with chi^+ = chi_sca and the Psi^+-
 * terms of the previous iteration's field (the paper's iterative treatment of the
 * coupling), and returns the new field [P][n_lines][n_q] (at the quadrature offsets, in
 * each point's frame and line widths) from u and v at the origin: the mean intensity
 * J_nu, or with a dipole the weighted mean Jw described there.  L* and Jeff take the
 * line's share chi_line/(chi_line + chi_sca) of the origin's source (Eq. ALO).  With
 * scattering set, nlte_run_ali uses this solve (FP64 whatever the precision setting, not
 * graph-captured), starting from the boundary intensity of each line.  Needs an ascending
 * quadrature (E_INVALID_ARG otherwise); does not combine with alo_band.  NULL clears it
 * (and the dipole); nlte_set_species and nlte_set_models clear both, and every call clears
 * the dipole.
 */
nlte_status nlte_set_scattering(nlte_ctx *ctx, const double *chi_sca);

/*
 * Direction-dependent scattering opacity (Sec. 2.1, 3.3: chi^- != 0): chi_dip
 * [P][n_lines][3] (cm^-1, host, copied) makes the opacity of direction n
 * chi_sca + chi_dip . n, so chi^+ = chi_sca and chi^- = chi_dip . n along each ray pair.
 * |chi_dip| <= chi_sca (1 + 1e-12) at every point and line (E_INVALID_ARG otherwise: a
 * negative opacity).  The scattered radiation is redistributed reciprocally,
 * Phi(n, n') = chi_s(n) chi_s(n') / (4 pi chi_sca): energy is conserved and I = B solves
 * every direction in thermal equilibrium.  The emissivity into n is then chi_s(n) Jw, with
 * Jw = (1/4pi) int (chi_s(n')/chi_sca) I(n') dOmega' the weighted mean intensity that the
 * scattering field holds (J_nu without a dipole).  chi^- enters the ray-pair solve through
 * the integrating factor e^{int chi^- ds}; an odd part that changes a ray's e-folding by
 * more than 700 within one sub-step is clamped there.  NULL removes the odd part.
 * E_STATE unless nlte_set_scattering set opacities.
 */
nlte_status nlte_set_scattering_dipole(nlte_ctx *ctx, const double *chi_dip);

/* One formal solve with scattering driven by jnu_in (host arrays, [P][n_lines][n_q]):
 * J, Jeff, Lstar [P][n_lines] and jnu_out. */
nlte_status nlte_formal_solve_scat(nlte_ctx *ctx, const double *pops, const double *jnu_in,
                                   double *J, double *Jeff, double *Lstar, double *jnu_out);
/* Device-pointer variant on `stream` (hipStream_t; NULL = the context's stream);
 * jnu_in and jnu_out must not alias. */
nlte_status nlte_formal_solve_scat_dev(nlte_ctx *ctx, const double *d_pops, const double *d_jnu_in,
                                       double *d_J, double *d_Jeff, double *d_Lstar,
                                       double *d_jnu_out, void *stream);
/* The scattering field (J_nu, or Jw with a dipole) [P][n_lines][n_q] after the last
 * formal solve of the last nlte_run_ali with
 * scattering (host copy); E_STATE if there is none.  nlte_formal_solve_scat (host) works
 * in the same buffers: read the field before calling it. */
nlte_status nlte_scattering_field(nlte_ctx *ctx, double *jnu);

/* ---------------------------------------------------------------- ALI */

/*
 * Accelerated Lambda iteration (Sec. 2.2.1, 3.4) from pops_init (NULL = LTE): repeat
 * formal solve + statistical equilibrium until the maximum relative change
 * |n_new - n_old| / n_new over levels with n_i / (abundance n_h2) > 1e-10 drops below
 * tol, or max_iter iterations ran.  Each model stops on its own: once its change is below
 * tol its points are no longer solved and keep their populations.  pops_out [P][n_lev];
 * rep (nullable) gets the report.  Returns NLTE_W_NOT_CONVERGED if some model did not
 * reach tol.  The _dev form orders its work after the caller's stream and returns when
 * pops_out is written.
 */
nlte_status nlte_run_ali(nlte_ctx *ctx, const double *pops_init, double *pops_out,
                         nlte_ali_report *rep);
nlte_status nlte_run_ali_dev(nlte_ctx *ctx, const double *d_pops_init, double *d_pops_out,
                             nlte_ali_report *rep, void *stream);

/* Per model after the last nlte_run_ali: iterations it took, whether it converged and its
 * last maximum relative change ([n_models] each; any pointer may be NULL). */
nlte_status nlte_get_model_status(nlte_ctx *ctx, int32_t *iterations, uint8_t *converged,
                                  double *last_change);

/* The formal-solve launch the current parameters resolve to (after the rules for the
 * choices left at 0 or -1): lines per lane, waves per SIMD of the register budget, long
 * segments (0/1), ray nodes staged per round, persistent (0/1), work items per workgroup
 * grab; any pointer may be NULL.  Needs nlte_trace (the collapse rule reads the trace). */
nlte_status nlte_get_launch(nlte_ctx *ctx, int *lines_per_lane, int *waves_per_simd, int *long_segments,
                            int *stage_nodes, int *persistent, int *tile_points);

/*
 * Time formal-solve launch choices on the current model with LTE populations and keep the
 * fastest in the context's parameters: starting from the rule's choice, one dimension at
 * a time (lines per lane, register budget of 1, 2 or 3 waves per SIMD, long or short
 * segments, nodes staged per round, grid or persistent work queue), each candidate timed
 * over `trials` launches after one warm-up (median), the best of each dimension kept
 * before the next.
 * cache_path (nullable): text file of earlier choices keyed by device, library build,
 * model size, ray, line and frequency counts, step count and precision; a hit skips the
 * timing, a miss appends the new choice.  choice (nullable, cap bytes) receives a
 * description.
 */
nlte_status nlte_autotune(nlte_ctx *ctx, const char *cache_path, int trials, char *choice, int cap);

/* ---------------------------------------------------------------- imaging */

/*
 * Image of the model (Sec. 3.5) along direction `ray` (the direction of propagation,
 * toward the observer) in line `line` at n_ch (1..1024) observer-frame channel velocities
 * v_ch [cm/s] (host array; channel frequency nu_l (1 + v/c), profile offset
 * x = (v - n.v_k)/v_w,k at node k): I [P][n_ch] is the intensity leaving the model at the
 * far end of the ray pair through each point, 2 u_E - I_in from the pair's second-order
 * solution with CMB intensity (line centre, t_cmb) entering at both ends; xy [P][2]
 * (nullable) the point's image-plane coordinates (x . e1, x . e2), e1 = (z x n)/|z x n|
 * (the x axis in place of z when |n_z| > 0.9), e2 = n x e1.  Populations pops [P][n_lev]
 * give the line coefficients (FP64 whatever the precision setting).  Needs nlte_trace.
 */
nlte_status nlte_image(nlte_ctx *ctx, const double *pops, int ray, int line, int n_ch, const double *v_ch,
                       double *I, double *xy);
nlte_status nlte_image_dev(nlte_ctx *ctx, const double *d_pops, int ray, int line, int n_ch,
                           const double *v_ch, double *d_I, double *d_xy, void *stream);

/* ---------------------------------------------------------------- warm start */

/*
 * Learned starting populations for the ALI.  The paper's iteration (Sec. 2.2.1, 3.4)
 * needs initial populations and is otherwise started in LTE; this surrogate predicts
 * them from local conditions instead.  It is not part of the paper's method: the ALI
 * run from the prediction is still what decides the result, and nlte_run_ali_warm falls
 * back to an LTE start when it does not converge.
 *
 * Features, per point (nlte_features, FP64 [P][8], needs nlte_trace):
 *   0 log10 n_H2; 1 log10 T; 2 log10 of the mean over the point's neighbours of
 *   |v_m - v_p| / |x_m - x_p| (floored at 1e-30 s^-1); 3..7 log10 of the minimum, lower
 *   quartile, median, upper quartile and maximum over all rays of the H2 column from the
 *   point to the end of its cached walk (Sec. 3.2; trapezoid in the projected distance,
 *   at least half a cell's column n_H2 d/2, d the mean distance to the point's
 *   neighbours, which a walk without cells at the model's edge takes, and at least
 *   1 cm^-2; quantiles interpolate linearly between order statistics at position
 *   q (n_rays - 1)).
 * Network: 8 standardised inputs -> 128 -> 128 -> 128 -> n_out, erf GELU after each
 * hidden layer; output i is the departure of level i from LTE, log10 (f_i / f_i^LTE),
 * with f_i = n_i / (abundance n_H2) and f_i^LTE the Boltzmann fraction at the point's
 * temperature (both floored at 1e-300); an output of zero is the LTE start.
 * Parameters: one FP32 vector [nlte_mlp_param_count(n_out)], matrices row-major
 * [out][in], order W1 [128][8], b1, W2 [128][128], b2, W3 [128][128], b3, W4 [n_out][128],
 * b4.  Products use bfloat16 operands (inputs, weights, hidden activations and output
 * gradients rounded to nearest even) with FP32 accumulation; biases, master weights and
 * Adam moments are FP32.  Loss: mean squared error over rows and outputs.
 */
#define NLTE_MLP_INPUTS 8
#define NLTE_MLP_HIDDEN 128

typedef struct {
    int64_t steps;   /* optimiser steps */
    int batch;       /* rows per step (1..65536); step t (counted since init/set_weights) takes rows
                        (t-1)*batch ... t*batch-1 modulo the row count */
    double lr, beta1, beta2, eps;  /* Adam (Kingma & Ba 2015) */
} nlte_train_params;

/* steps 1000, batch 4096, lr 1e-3, beta1 0.9, beta2 0.999, eps 1e-8. */
void nlte_default_train_params(nlte_train_params *p);

/* Parameter count for n_out outputs (35,466 for 10); -1 if n_out is outside 1..16. */
int64_t nlte_mlp_param_count(int n_out);

/* Raw (unstandardised) features of every point, F [P][8]. */
nlte_status nlte_features(nlte_ctx *ctx, double *F);
nlte_status nlte_features_dev(nlte_ctx *ctx, double *d_F, void *stream);

/* Fresh network with n_out (1..16) outputs: weights uniform in +-sqrt(6/(in+out)) from a
 * SplitMix64 stream seeded with `seed` (layer by layer, row-major), zero biases; resets
 * the optimiser and keeps the current standardisation (initially mean 0, std 1). */
nlte_status nlte_mlp_init(nlte_ctx *ctx, int n_out, uint64_t seed);
/* Replace the parameters (host FP32 vector as above; must be finite); resets the optimiser. */
nlte_status nlte_mlp_set_weights(nlte_ctx *ctx, int n_out, const float *theta);
nlte_status nlte_mlp_get_weights(nlte_ctx *ctx, float *theta);
/* Feature standardisation used by predict: x = (F - mean) / std ([8] each, std > 0). */
nlte_status nlte_mlp_set_norm(nlte_ctx *ctx, const double *mean, const double *std);

/* Training rows of the current model from populations d_pops [P][n_lev] (device):
 * standardised features d_X [P][8] (with the current standardisation, so it need not
 * have weights yet) and targets d_T [P][n_lev], the departures log10 (f_i / f_i^LTE). */
nlte_status nlte_mlp_rows_dev(nlte_ctx *ctx, const double *d_pops, float *d_X, float *d_T, void *stream);

/* Network outputs Y [n][n_out] for standardised inputs X [n][8] (host FP32). */
nlte_status nlte_mlp_forward(nlte_ctx *ctx, const float *X, int64_t n, float *Y);
/* Loss and gradient over all n rows (1..65536) as one batch, without an update;
 * grad [n_params] (nullable), loss (nullable). */
nlte_status nlte_mlp_loss_grad(nlte_ctx *ctx, const float *X, const float *T, int64_t n, float *grad,
                               double *loss);
/* Adam on rows X [n][8] (standardised), targets T [n][n_out]; loss_curve [steps]
 * (nullable) receives each step's batch loss before its update. */
nlte_status nlte_mlp_train(nlte_ctx *ctx, const float *X, const float *T, int64_t n,
                           const nlte_train_params *tp, float *loss_curve);
nlte_status nlte_mlp_train_dev(nlte_ctx *ctx, const float *d_X, const float *d_T, int64_t n,
                               const nlte_train_params *tp, float *d_loss_curve, void *stream);

/* Starting populations pops [P][n_lev] for the current model (n_out must equal n_lev):
 * abundance * n_H2 * w_i / sum_j w_j, w_i = f_i^LTE 10^y_i, from the network outputs y.  Points whose
 * prediction is not finite get LTE populations; *n_fallback (nullable) counts them. */
nlte_status nlte_mlp_predict(nlte_ctx *ctx, double *pops, int64_t *n_fallback);
nlte_status nlte_mlp_predict_dev(nlte_ctx *ctx, double *d_pops, int64_t *n_fallback, void *stream);

/* ALI from the predicted populations; if that stops at max_iter above tol it is run
 * again from LTE.  *used_network (nullable) tells which start the result came from. */
nlte_status nlte_run_ali_warm(nlte_ctx *ctx, double *pops_out, nlte_ali_report *rep, int *used_network);
nlte_status nlte_run_ali_warm_dev(nlte_ctx *ctx, double *d_pops_out, nlte_ali_report *rep,
                                  int *used_network, void *stream);

/* ---------------------------------------------------------------- profiling */

/* With params.profile = 1: accumulated HIP-event time [ms] and launch count of kernel
 * `name` since the last reset: "line_coef", "formal_solve", "stateq", "lte", "trace",
 * "features", "mlp_forward", "mlp_train" (forward, loss and backward of one batch),
 * "mlp_update" (gradient reduction, Adam and operand packing of one step) and "image"
 * (the emergent-intensity elimination of nlte_image, without the image-plane positions). */
nlte_status nlte_kernel_stats(nlte_ctx *ctx, const char *name, double *ms, int64_t *launches);
/* With params.profile = 1: the node-frequency elimination steps (one step of one line at one
 * frequency) that the line formal-solve kernels executed since the last
 * nlte_reset_kernel_stats.  A velocity sub-step segment whose nodes all lie beyond the
 * range of the line profile for every frequency of a wave has zero opacity throughout
 * and is eliminated in one step, which counts as one; the method's own count of steps is
 * the third output of nlte_trace_stats times n_lines times n_q. */
nlte_status nlte_executed_steps(nlte_ctx *ctx, int64_t *node_freq);
nlte_status nlte_reset_kernel_stats(nlte_ctx *ctx);

#ifdef __cplusplus
}
#endif
#endif /* NLTE_H */
