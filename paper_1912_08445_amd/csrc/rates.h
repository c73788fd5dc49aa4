// Rate equations of one point (device functions shared by the local and the band
// statistical-equilibrium solves).
#pragma once

#include "nlte_internal.h"

namespace nlte {

// H2 de-excitation coefficient of collision pair ic, linear in T between table points
// and clamped at the ends; j is the table interval holding T (T inside the table).
__device__ __forceinline__ double coll_K(const SpeciesDev &sp, int ic, double T, int j, int where)
{
    const double *K = sp.Ktab + (int64_t)ic * sp.n_T;
    if (where < 0) return K[0];
    if (where > 0) return K[sp.n_T - 1];
    return K[j] + (K[j + 1] - K[j]) * (T - sp.Ttab[j]) / (sp.Ttab[j + 1] - sp.Ttab[j]);
}

// Rate matrix of one point (Eq. ourALI): u->l = A(1 - L) + B_ul Jeff + C_ul,
// l->u = B_lu Jeff + C_lu, column-sum form M[to][from]; row 0 := conservation
// sum_i n_i = ntot (rhs).  M [n][n] row-major, rhs [n].
__device__ __forceinline__ void rate_matrix(const SpeciesDev &sp, double T, double nh2, double ntot,
                                            const double *Jrow, const double *Lrow, bool with_L, double *M,
                                            double *rhs)
{
    const int n = sp.n_lev;
    for (int i = 0; i < n * n; ++i) M[i] = 0.0;
    for (int i = 0; i < n; ++i) rhs[i] = 0.0;
    // transition a -> b with rate R: gain for b, loss for a
    for (int l = 0; l < sp.n_lines; ++l) {
        const int u = sp.lu[l], lo = sp.ll[l];
        const double Lv = with_L ? Lrow[l] : 0.0;
        const double Rul = sp.A[l] * (1.0 - Lv) + sp.Bul[l] * Jrow[l];
        const double Rlu = sp.Blu[l] * Jrow[l];
        M[lo * n + u] += Rul;
        M[u * n + u] -= Rul;
        M[u * n + lo] += Rlu;
        M[lo * n + lo] -= Rlu;
    }
    int where = 0, j = 0;
    if (T <= sp.Ttab[0]) where = -1;
    else if (T >= sp.Ttab[sp.n_T - 1]) where = 1;
    else
        while (j + 2 < sp.n_T && !(T < sp.Ttab[j + 1])) ++j;
    const double kT = kKB * T;
    for (int ic = 0; ic < sp.n_coll; ++ic) {
        const int u = sp.cu[ic], lo = sp.cl[ic];
        const double Cul = coll_K(sp, ic, T, j, where) * nh2;
        // detailed balance with the Boltzmann sign
        const double Clu = Cul * (sp.g[u] / sp.g[lo]) * exp(-(sp.E[u] - sp.E[lo]) / kT);
        M[lo * n + u] += Cul;
        M[u * n + u] -= Cul;
        M[u * n + lo] += Clu;
        M[lo * n + lo] -= Clu;
    }
    for (int c = 0; c < n; ++c) M[c] = 1.0;
    rhs[0] = ntot;
}

}  // namespace nlte
