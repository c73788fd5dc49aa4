/* Plain FP64 CPU oracle: declarations.  Test infrastructure only (see nlte_oracle.c). */
#ifndef NLTE_ORACLE_H
#define NLTE_ORACLE_H
#include <stdint.h>

typedef struct or_ctx or_ctx;

or_ctx *or_create(void);
void or_destroy(or_ctx *c);
int or_set_species(or_ctx *c, int n_lev, const double *E, const double *g, double mass,
                   int n_lines, const int32_t *up, const int32_t *lo, const double *A,
                   int n_coll, const int32_t *cup, const int32_t *clo, int n_T,
                   const double *Ttab, const double *Ktab);
int or_set_model(or_ctx *c, int64_t P, const double *pos, const double *vel, const double *nh2,
                 const double *T, const double *vturb, const double *X, int k, const int32_t *nbr,
                 const uint8_t *bnd);
int or_set_rays(or_ctx *c, int n_rays, const double *dir);
int or_set_quadrature(or_ctx *c, int nq, const double *x, const double *w);
void or_set_params(or_ctx *c, double t_cmb, double f_sub, double tau_floor, int use_alo);
int or_n_pairs(const or_ctx *c);
void or_line_width_speed(const or_ctx *c, double *vw);
double or_planck(double nu, double T);
void or_coll_rates(const or_ctx *c, int64_t p, double *Cul, double *Clu);
void or_lte(const or_ctx *c, double *pops);
int or_walk(const or_ctx *c, int64_t O, int ray, int32_t *cells, double *Zs, int cap);
int or_pair_nodes(const or_ctx *c, const double *pops, int64_t O, int pair, int cap, double *z,
                  double *a, double *b, double *kap, double *S, int *io);
void or_solve_ray(int N, const double *z, const double *chi, const double *S, double I_lo,
                  double I_hi, int o, double tau_floor, double *u_o, double *lam_o,
                  double *ueff_o, double *u_all);
void or_formal_solve(const or_ctx *c, const double *pops, int64_t n_sel, const int64_t *sel,
                     double *J, double *Jeff, double *L);
void or_stateq(const or_ctx *c, const double *pops_old, const double *J, const double *Jeff,
               const double *L, double *pops_new, uint8_t *flags);
double or_rel_change(const or_ctx *c, const double *old, const double *nw, double *mean);
int or_run_ali(const or_ctx *c, const double *pops_init, double *pops_out, int max_iter, double tol,
               double *max_change);
int64_t or_walk_all(const or_ctx *c, int64_t *off, int32_t *cells);

void or_features(const or_ctx *c, double *F);
void or_formal_solve_band(const or_ctx *c, const double *pops, int64_t n_sel, const int64_t *sel,
                          double *J, double *Jeff, double *L, double *Jb, double *Ld, double *Ln);
int or_solve_ray_gen(int N, const double *z, const double *chi, const double *chim, const double *Splus,
                     const double *sigma, double I_lo, double I_hi, int o, double tau_floor,
                     double own, double *u_o, double *lam_o, double *ueff_o, double *v_o);
int or_formal_solve_scat(const or_ctx *c, const double *pops, const double *chi_sca, const double *chi_dip,
                         const double *Jnu_in, int64_t n_sel, const int64_t *sel, double *J,
                         double *Jeff, double *L, double *Jnu_out);
void or_set_threads(int n);
#endif
