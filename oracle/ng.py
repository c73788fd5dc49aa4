"""Ng acceleration of the ALI (plain numpy), and the ALI loop that applies it.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke entry point and the benchmark's
CPU-baseline leg are its only users.  The HIP library never imports or links it.

Sec. 3.4 (Ng 1974; Olson, Auer & Buchler 1986): after every M regular iterations the
populations are replaced by a linear combination of the last M - 1 iterates,
    x_new = sum_j a_j x_{n-j},  j = 0 .. M-2,  sum_j a_j = 1,
whose coefficients minimise the same combination of the one-iteration changes,
    || sum_j a_j (x_{n-j} - x_{n-j-1}) ||^2,
so M iterates x_{n-M+1} .. x_n take part.  The norm weighs every (point, level) entry of
the fractional populations x / n_tot uniformly.  A point whose combined populations are
not all positive and finite keeps x_n.
"""
from __future__ import annotations

import numpy as np


def ng_coefficients(hist):
    """Coefficients a_0..a_{M-2} (a_0 for the newest iterate) from iterates hist
    (list of M arrays, oldest first), or None when the least-squares problem is singular.

    With a_0 = 1 - sum_{j>0} a_j the objective is || r_0 + sum_{j>0} a_j (r_j - r_0) ||^2
    with r_j = x_{n-j} - x_{n-j-1}; it is solved with numpy's least squares."""
    M = len(hist)
    if M < 3:
        raise ValueError("Ng needs at least three iterates")
    x = [np.asarray(h, dtype=np.float64).ravel() for h in hist[::-1]]   # newest first
    r = [x[j] - x[j + 1] for j in range(M - 1)]
    A = np.stack([r[j] - r[0] for j in range(1, M - 1)], axis=1)
    sol, _, rank, _ = np.linalg.lstsq(A, -r[0], rcond=None)
    if rank < M - 2:
        return None
    return np.concatenate([[1.0 - sol.sum()], sol])


def ng_step(hist_pops, ntot):
    """Ng-extrapolated populations from the last M iterates (oldest first, each
    [P][n_lev]) of one model; returns (populations, coefficients or None, rejected points)."""
    f = [np.asarray(h, dtype=np.float64) / ntot[:, None] for h in hist_pops]
    a = ng_coefficients(f)
    newest = np.asarray(hist_pops[-1], dtype=np.float64)
    if a is None:
        return newest.copy(), None, 0
    comb = sum(a[j] * np.asarray(hist_pops[-1 - j], dtype=np.float64) for j in range(len(a)))
    ok = np.all(np.isfinite(comb) & (comb > 0), axis=1)
    out = np.where(ok[:, None], comb, newest)
    return out, a, int((~ok).sum())


def run_ali_ng(o, ntot, pops_init=None, max_iter=50, tol=1e-4, M=4):
    """ALI of Sec. 2.2.1 / 3.4 with an Ng step after every M regular iterations
    (oracle object `o` from oracle.from_workload).  The relative change of each regular
    iteration decides convergence, as without Ng.  Returns (populations, changes,
    coefficients of each Ng step)."""
    pops = o.lte() if pops_init is None else np.array(pops_init, dtype=np.float64)
    hist, changes, coefs = [], [], []
    for it in range(1, max_iter + 1):
        J, Je, L = o.formal_solve(pops)
        new, _ = o.stateq(pops, J, Je, L)
        ch, _ = o.rel_change(pops, new)
        changes.append(ch)
        pops = new
        if ch < tol:
            break
        hist.append(pops)
        if len(hist) == M:
            pops, a, _ = ng_step(hist, ntot)
            coefs.append(a)
            hist = []
    return pops, np.array(changes), coefs
