"""The formal solve's count of executed node-frequency steps (profile mode), which the
benchmark's roofline uses: every step of the method where no segment has sub-steps,
fewer where far-wing segments are eliminated in one step, and cleared by a reset."""
import pytest

from synth import configs

from _common import solver_for

pytestmark = pytest.mark.gpu


def _count(w):
    s = solver_for(w)
    s.set_params(profile=1)
    s.reset_kernel_stats()
    s.formal_solve(s.lte())
    method = s.trace_stats()[2] * w.species.n_lines * w.quad_x.shape[0]
    return s, s.executed_steps(), method


def test_static_model_executes_every_step():
    w = configs.sphere2(n_points=400, seed=3)
    _, ex, method = _count(w)
    assert ex == method > 0


def test_outflow_collapses_far_wing_segments_and_reset_clears():
    w = configs.outflow5(n_points=2000, seed=5, nside=1)
    s, ex, method = _count(w)
    assert 0 < ex < method
    s.reset_kernel_stats()
    assert s.executed_steps() == 0
    s.set_params(profile=0)
    s.formal_solve(s.lte())
    assert s.executed_steps() == 0   # counted in profile mode only
