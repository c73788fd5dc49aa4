"""Statistical equilibrium with the band ALO, and the ALI that uses it (plain numpy/scipy).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke entry point and the benchmark's
CPU-baseline leg are its only users.  The HIP library never imports or links it.

With a band ALO (Sec. 3.4) the rate equations of a point contain the new upper-level
populations of the points the band reaches.  For line l = (u -> lo) at point O the net
downward rate is
    F = n_u,O [A (1 - Ld) + B_ul Jb] - n_lo,O B_lu Jb - A sum_c (k_O / k_c) Ln_c n_u,c
(Ld, Ln, Jb from the band formal solve; k = h nu/4pi (n_lo B_lu - n_u B_ul) the
profile-free opacity with the previous populations; c the first cell of the walk along
each ray).  Level u loses F, level lo gains it; collisions as in the local solve; the
first level's equation of each point is replaced by sum_i n_i = X n_H2.  The system of all
points and levels is solved at once (scipy's sparse LU).  When a population comes out
non-positive or non-finite the band is dropped (Sec. 6.1): the iteration takes the local
(diagonal ALO) solution instead.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

H = 6.62607015e-27
C_LIGHT = 2.99792458e10


def _einstein(species):
    nu = (species.energy[species.line_up] - species.energy[species.line_lo]) / H
    Bul = species.line_A * C_LIGHT ** 2 / (2.0 * H * nu ** 3)
    Blu = species.weight[species.line_up] / species.weight[species.line_lo] * Bul
    return nu, Bul, Blu


def first_cells(o):
    """First cell of the walk from every point along every ray (-1 without one)."""
    fc = np.full((o.P, o.n_rays), -1, dtype=np.int64)
    for p in range(o.P):
        for r in range(o.n_rays):
            cells, _ = o.walk(p, r)
            if cells.size:
                fc[p, r] = cells[0]
    return fc


def assemble(o, pops_old, Jb, Ld, Ln, fc, band=True):
    """Sparse matrix and right-hand side of the coupled rate equations."""
    sp_ = o.species
    P, nlev, nl, R = o.P, sp_.n_lev, sp_.n_lines, o.n_rays
    nu, Bul, Blu = _einstein(sp_)
    ntot = o.model.abundance * o.model.n_h2
    kchi = np.zeros((P, nl))
    for l in range(nl):
        u, lo = sp_.line_up[l], sp_.line_lo[l]
        kchi[:, l] = H * nu[l] / (4 * np.pi) * (pops_old[:, lo] * Blu[l] - pops_old[:, u] * Bul[l])
    rows, cols, vals = [], [], []
    rhs = np.zeros(P * nlev)

    def add(r, c, v):
        rows.append(r)
        cols.append(c)
        vals.append(v)

    cu, cl = sp_.coll_up, sp_.coll_lo
    for p in range(P):
        Rm = np.zeros((nlev, nlev))        # Rm[i, j]: rate i -> j at point p
        for l in range(nl):
            u, lo = sp_.line_up[l], sp_.line_lo[l]
            Rm[u, lo] += sp_.line_A[l] * (1.0 - Ld[p, l]) + Bul[l] * Jb[p, l]
            Rm[lo, u] += Blu[l] * Jb[p, l]
        Cul, Clu = o.coll_rates(p)
        for k in range(cu.shape[0]):
            Rm[cu[k], cl[k]] += Cul[k]
            Rm[cl[k], cu[k]] += Clu[k]
        base = p * nlev
        for i in range(1, nlev):
            for j in range(nlev):
                if j != i:
                    add(base + i, base + j, Rm[j, i])
            add(base + i, base + i, -Rm[i].sum() + Rm[i, i])
        for j in range(nlev):
            add(base, base + j, 1.0)
        rhs[base] = ntot[p]
        if not band:
            continue
        for l in range(nl):
            u, lo = sp_.line_up[l], sp_.line_lo[l]
            if not kchi[p, l] > 0:
                continue
            for r in range(R):
                c = fc[p, r]
                if c < 0 or not kchi[c, l] > 0 or Ln[p, l, r] == 0.0:
                    continue
                k = sp_.line_A[l] * kchi[p, l] / kchi[c, l] * Ln[p, l, r]
                if u != 0:
                    add(base + u, c * nlev + u, k)
                if lo != 0:
                    add(base + lo, c * nlev + u, -k)
    M = sp.csr_matrix((vals, (rows, cols)), shape=(P * nlev, P * nlev))
    return M, rhs


def stateq_band(o, pops_old, J, Jeff, L, Jb, Ld, Ln, fc):
    """New populations with the band ALO, or the local solution when the band's are not
    all positive and finite.  Returns (populations, band_used)."""
    M, rhs = assemble(o, pops_old, Jb, Ld, Ln, fc)
    x = spla.spsolve(M.tocsc(), rhs).reshape(o.P, -1)
    if np.all(np.isfinite(x)) and np.all(x > 0):
        return x, True
    local, _ = o.stateq(pops_old, J, Jeff, L)
    return local, False


def run_ali_band(o, pops_init=None, max_iter=50, tol=1e-4):
    """ALI with the band ALO (Sec. 2.2.1, 3.4); returns (populations, changes, band used
    per iteration)."""
    fc = first_cells(o)
    pops = o.lte() if pops_init is None else np.array(pops_init, dtype=np.float64)
    changes, used = [], []
    for _ in range(max_iter):
        J, Je, L, Jb, Ld, Ln = o.formal_solve_band(pops)
        new, ok = stateq_band(o, pops, J, Je, L, Jb, Ld, Ln, fc)
        ch, _ = o.rel_change(pops, new)
        changes.append(ch)
        used.append(ok)
        pops = new
        if ch < tol:
            break
    return pops, np.array(changes), used
