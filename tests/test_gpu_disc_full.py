"""The 1,000,000-point Keplerian disc (192 rays, 9 lines x 31 frequencies) at full size,
in the launch configuration the benchmark times: 200 origins (the 100 costliest and 100
random ones) against the oracle in both precision forms, the FP32 form against the FP64 one at every point, and the FP32
lane maps against each other."""
import numpy as np
import pytest

from synth import configs, directions

from _common import oracle_for, rel, solver_for

pytestmark = pytest.mark.gpu

TOL64 = 1e-10
TOL32 = 1e-4


@pytest.mark.parametrize("lpl", [1, 2, 3])
def test_fp32_lane_maps_agree(lpl):
    w = configs.disc10(n_points=3000, seed=21)
    w.rays = directions.healpix_ring(1)
    ref = solver_for(w, precision="fp32")            # lane map by rule (3 lines per lane)
    pops = ref.lte()
    a = ref.formal_solve(pops)
    b = solver_for(w, precision="fp32", lines_per_lane=lpl).formal_solve(pops)
    # the lines of a lane share only the profile, which every lane map evaluates alike
    for x, y in zip(a, b):
        assert rel(x, y).max() <= 1e-12


def _origins(s, w):
    """100 of the costliest origins (by the trace's elimination steps) and 100 seeded
    random others."""
    cost = s.point_cost()
    top = np.argsort(-cost, kind="stable")[:100]
    rest = np.setdiff1d(np.arange(w.n_points), top)
    rnd = np.random.default_rng(3).choice(rest, 100, replace=False)
    return np.sort(np.concatenate([top, rnd])), cost


def test_disc_full_size_sampled():
    w = configs.disc10()
    print("disc generated", flush=True)
    s = solver_for(w)
    print("traced", s.launch(), flush=True)
    o = oracle_for(w)
    pops = s.lte()
    J, Je, L = s.formal_solve(pops)
    print("fp64 sweep done", flush=True)
    sel, cost = _origins(s, w)
    print("origins: cost of the sampled costliest", int(cost[sel].max()), "median over the disc",
          int(np.median(cost)), flush=True)
    # the cost the persistent queue orders by: per pair of rays, the oracle's node count
    # (origin plus the sub-step nodes of both halves) plus one
    for p in list(sel[np.argsort(-cost[sel])[:2]]) + list(sel[:2]):
        n = sum(o.pair_nodes(pops, int(p), k)["z"].shape[0] + 1 for k in range(w.rays.shape[0] // 2))
        assert n == cost[p], (p, n, cost[p])
    Jo, Jeo, Lo = o.formal_solve(pops, sel)
    print("oracle done", flush=True)
    assert rel(J[sel], Jo).max() <= TOL64
    assert rel(Je[sel], Jeo).max() <= TOL64
    assert rel(L[sel], Lo).max() <= TOL64
    assert np.isfinite(J).all() and (Je >= 0).all() and (L >= 0).all() and (L <= 1).all()
    for p in sel[:3]:
        for r in range(0, 192, 37):
            assert np.array_equal(s.get_ray(p, r), o.walk(p, r)[0])
    s.set_params(precision="fp32")
    print("fp32 launch", s.launch(), flush=True)
    J32, Je32, L32 = s.formal_solve(pops)
    print("fp32 sweep done", flush=True)
    for a, b in ((J32, Jo), (Je32, Jeo), (L32, Lo)):
        assert rel(a[sel], b).max() <= TOL32
    errs = {k: (float(rel(a, b).max()), float(np.quantile(rel(a, b), 0.99)))
            for k, a, b in (("J", J32, J), ("Jeff", Je32, Je), ("L*", L32, L))}
    print("FP32 vs FP64 over all points (max, 99th percentile):", errs, flush=True)
    assert errs["J"][0] <= TOL32
