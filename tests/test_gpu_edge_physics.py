"""Degenerate physics through the GPU path against the oracle: inverted (maser) lines,
whose opacity and source function are clamped to zero and counted, and a velocity jump
so large that the sub-step count of a segment reaches its cap of 2^20."""
import numpy as np
import pytest

from synth import configs, directions, species
from synth.configs import Workload
from synth.models import chain_1d

from _common import oracle_for, rel, solver_for

pytestmark = pytest.mark.gpu


def test_maser_lines_are_clamped_and_counted():
    w = configs.outflow5(n_points=300, seed=4, nside=1)
    o = oracle_for(w)
    pops = o.lte() * np.random.default_rng(9).uniform(0.3, 3.0, (w.n_points, w.species.n_lev))
    pops *= ((w.model.abundance * w.model.n_h2) / pops.sum(1))[:, None]
    sp = w.species
    g = sp.weight
    inverted = pops[:, sp.line_up] / g[sp.line_up] >= pops[:, sp.line_lo] / g[sp.line_lo]
    assert inverted.sum() > 10
    s = solver_for(w, max_iter=1, tol=0.0)
    J, Je, L = s.formal_solve(pops)
    rJ, rJe, rL = o.formal_solve(pops)
    assert rel(J, rJ).max() <= 1e-10 and rel(Je, rJe).max() <= 1e-10 and rel(L, rL).max() <= 1e-10
    _, rep = s.run_ali(pops)
    assert rep["n_maser"] == int(inverted.sum())


def test_substep_cap():
    # three points on a line, the outer two moving at -+1e10 cm/s: each segment would need
    # about 1.6e6 sub-steps of a quarter line width and takes the cap of 2^20
    x = np.array([-1e15, 0.0, 1e15])
    m = chain_1d(x, np.array([-1e10, 0.0, 1e10]), 1e4, 10.0, 0.0, 1e-6)
    qx, qw = directions.uniform_grid(31)
    w = Workload("jump", m, species.two_level(100e9, 3.0, 1e-5, 1e-10, 28.0), directions.axis_pair(), qx, qw)
    s, o = solver_for(w), oracle_for(w)
    tot, longest, steps = s.trace_stats()
    assert steps >= 2 * (1 << 20)
    pops = o.lte()
    J, Je, L = s.formal_solve(pops)
    rJ, rJe, rL = o.formal_solve(pops)
    assert rel(J, rJ).max() <= 1e-10 and rel(Je, rJe).max() <= 1e-10 and rel(L, rL).max() <= 1e-10
