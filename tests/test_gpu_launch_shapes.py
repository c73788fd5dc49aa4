"""Every launch shape of the formal solve computes the same thing: lines per lane 1..5,
register budgets of 1, 2 and 3 waves per SIMD, LDS staging depths down to two nodes, grid
and persistent launches, one to sixteen points per workgroup.  A line's arithmetic and the order of its sums do not depend on
any of these, so the outputs agree bit for bit.  The far-wing collapse leaves the state
of a segment unchanged but restarts the profile recurrence of the following segments at
other points, so with and without it the results agree to rounding (1e-12) and each
setting is bit-identical across the other choices; all agree with the oracle to 1e-10
(FP64)."""
import itertools

import numpy as np
import pytest

from synth import configs, species

from _common import oracle_for, rel, solver_for

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_launch_shapes_agree_bitwise(precision):
    import torch
    # a moving 10-level model (nine lines, the disc's species) with long sub-step segments
    w = configs.outflow5(n_points=700, seed=61, nside=1)
    w.species = species.linear_rotor(10)
    s = solver_for(w, precision=precision)
    o = oracle_for(w)
    pops = o.lte()
    dev = torch.device("cuda:0")
    dp = torch.tensor(pops, device=dev)
    P, nl = w.n_points, w.species.n_lines
    ref = {}
    shapes = list(itertools.product([1, 2, 3, 4, 5], [1, 2, 3], [0, 1]))
    extra = [dict(stage_nodes=2), dict(stage_nodes=7), dict(stage_nodes=33), dict(persistent=1),
             dict(persistent=1, lines_per_lane=5, waves_per_simd=1, stage_nodes=16),
             dict(tile_points=3), dict(tile_points=16), dict(persistent=1, tile_points=4),
             dict(persistent=1, tile_points=13, lines_per_lane=1)]
    configs_ = [dict(lines_per_lane=a, waves_per_simd=b, long_segments=c) for a, b, c in shapes] + extra
    for k in configs_:
        print(precision, k, flush=True)
        kw = dict(lines_per_lane=0, waves_per_simd=0, long_segments=-1, stage_nodes=0, persistent=0, tile_points=0)
        kw.update(k)
        s.set_params(precision=precision, **kw)
        J, Je, L = (torch.full((P, nl), np.nan, dtype=torch.float64, device=dev) for _ in range(3))
        s.formal_solve_dev(dp, J, Je, L)
        torch.cuda.synchronize()
        out = np.stack([J.cpu().numpy(), Je.cpu().numpy(), L.cpu().numpy()])
        assert np.isfinite(out).all(), k
        far = s.launch()["long_segments"]
        if far not in ref:
            ref[far] = out
        assert np.array_equal(out, ref[far]), k
    assert set(ref) == {0, 1}
    assert rel(ref[0], ref[1]).max() <= 1e-12
    rJ, rJe, rL = o.formal_solve(pops)
    tol = 1e-10 if precision == "fp64" else 1e-4
    for out in ref.values():
        assert rel(out[0], rJ).max() <= tol and rel(out[1], rJe).max() <= tol and rel(out[2], rL).max() <= tol


def test_tile_points_range():
    from paper_1912_08445_amd.binding import NlteError
    w = configs.sphere2(n_points=50)
    s = solver_for(w)
    for bad in (-1, 17):
        with pytest.raises(NlteError):
            s.set_params(tile_points=bad)
    s.set_params(tile_points=16)
    assert s.launch()["tile_points"] == 16
    s.set_params(tile_points=0)
    assert s.launch()["tile_points"] == 1
