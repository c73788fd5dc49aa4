"""Helpers shared by the test modules (comparison metric, solver/oracle construction)."""
import numpy as np


def rel(a, b):
    """The paper's relative difference 2|a-b|/(|a|+|b|), zero where both vanish."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.abs(a) + np.abs(b)
    return np.where(den > 0, 2 * np.abs(a - b) / np.where(den > 0, den, 1), 0.0)


def solver_for(w, **params):
    from paper_1912_08445_amd.binding import Solver
    s = Solver(0)
    s.setup(w, **params)
    return s


def oracle_for(w, **kw):
    import oracle
    oracle.build(force=False)
    return oracle.from_workload(w, **kw)
