"""Seeded random configurations through the GPU path against the oracle: model shape
and size, velocity scale, ragged neighbour lists, species, quadrature, ray set, sub-step
fraction and launch choices vary together.  Walks bit-exact on sampled rays, the formal
solve on sampled origins and the stat-eq at every point within 1e-10 (FP64), and the FP32
form within 1e-4 of FP64."""
import numpy as np
import pytest

from synth import configs, directions, species

from _common import oracle_for, rel, solver_for

pytestmark = pytest.mark.gpu


def _config(seed):
    rng = np.random.default_rng(7000 + seed)
    n = int(rng.integers(60, 400))
    if rng.random() < 0.5:
        w = configs.sphere2(n_points=n, seed=int(rng.integers(1, 1000)))
    else:
        w = configs.outflow5(n_points=n, seed=int(rng.integers(1, 1000)), nside=1)
    w.model.vel *= float(rng.choice([0.0, 0.1, 1.0, 5.0]))
    drop = rng.random(w.model.nbr.shape) < float(rng.choice([0.0, 0.2]))
    w.model.nbr[drop] = -1                       # ragged neighbour lists
    nlev = int(rng.choice([2, 3, 5, 8]))
    w.species = species.two_level() if nlev == 2 else species.linear_rotor(nlev)
    q = rng.choice(["u1", "u7", "u31", "u40", "gh24"])
    w.quad_x, w.quad_w = (directions.gauss_hermite(24) if q == "gh24" else
                          directions.uniform_grid(int(q[1:]), 4.0) if q != "u1" else
                          (np.array([0.0]), np.array([1.0])))
    w.rays = [directions.axis_pair(), directions.healpix_ring(1), directions.healpix_ring(2)][int(rng.integers(0, 3))]
    w.f_sub = float(rng.choice([0.1, 0.25, 0.5]))
    launch = dict(lines_per_lane=int(rng.choice([0, 1, 2, 3, 4, 5])), waves_per_simd=int(rng.integers(0, 4)),
                  persistent=int(rng.integers(0, 2)), long_segments=int(rng.integers(-1, 2)),
                  stage_nodes=int(rng.choice([0, 2, 9, 24, 64])), tile_points=int(rng.choice([0, 1, 2, 5, 16])))
    desc = f"seed {seed}: {w.name} n={n} lev={nlev} q={q} rays={w.rays.shape[0]} f_sub={w.f_sub} {launch}"
    return w, launch, desc, rng


@pytest.mark.parametrize("seed", range(10))
def test_random_configuration(seed):
    w, launch, desc, rng = _config(seed)
    print(desc, flush=True)
    s = solver_for(w, **launch)
    o = oracle_for(w)
    for p in rng.choice(w.n_points, 4, replace=False):
        for r in range(w.rays.shape[0]):
            assert np.array_equal(s.get_ray(p, r), o.walk(p, r)[0]), (p, r)
    pops = o.lte() * rng.uniform(0.8, 1.2, (w.n_points, w.species.n_lev))
    pops *= ((w.model.abundance * w.model.n_h2) / pops.sum(1))[:, None]
    J, Je, L = s.formal_solve(pops)
    sel = rng.choice(w.n_points, min(24, w.n_points), replace=False)
    rJ, rJe, rL = o.formal_solve(pops, sel=sel)
    assert rel(J[sel], rJ).max() <= 1e-10 and rel(Je[sel], rJe).max() <= 1e-10 and rel(L[sel], rL).max() <= 1e-10
    new, flags = s.stateq(pops, J, Je, L)
    ref, rflags = o.stateq(pops, J, Je, L)
    assert np.array_equal(flags, rflags) and rel(new, ref).max() <= 1e-10
    s.set_params(precision="fp32")
    J32 = s.formal_solve(pops)[0]
    assert rel(J32, J).max() <= 1e-4
