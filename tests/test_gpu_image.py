"""Images (Sec. 3.5) on the GPU against the oracle's."""
import numpy as np
import pytest

import oracle
from synth import configs, directions

from _common import oracle_for, rel, solver_for

pytestmark = pytest.mark.gpu

TOL = 1e-10


def _cases():
    disc = configs.disc10(n_points=1200, seed=8)
    disc.rays = directions.healpix_ring(1)
    return [
        ("sphere2", configs.sphere2(n_points=300), 0, [3, 10], np.linspace(-3e4, 3e4, 5)),
        ("outflow", configs.outflow5(n_points=1500, seed=4, nside=1), 2, [0, 7, 11],
         np.linspace(-2.5e6, 2.5e6, 70)),                                  # two channel blocks
        ("disc", disc, 4, [1, 6], np.linspace(-1.2e6, 1.2e6, 9)),
        # pairs of more than 64 nodes (several staging chunks) through the innermost points,
        # and channels so far out that the profile vanishes and is evaluated directly
        ("outflow_long", configs.outflow5(n_points=30000, seed=5, nside=1), 1, [3],
         np.concatenate([np.linspace(-2.5e6, 2.5e6, 62), [-5e8, 5e8]])),
    ]


def _anti(s, r):
    d = s.get_rays()
    return int(np.argmin(np.abs(d + d[r]).sum(axis=1)))


@pytest.mark.parametrize("name,w,line,rays,v", _cases(), ids=[c[0] for c in _cases()])
def test_image_matches_oracle(name, w, line, rays, v):
    s, o = solver_for(w), oracle_for(w)
    pops = s.lte()
    if name == "outflow":
        # non-LTE populations: one ALI step from LTE
        J, Je, L = s.formal_solve(pops)
        pops, _ = s.stateq(pops, J, Je, L)
    sel = np.random.default_rng(1).choice(w.n_points, 40, replace=False)
    if name == "outflow_long":
        inner = np.argsort(np.linalg.norm(w.model.pos, axis=1))[:24]
        sel = np.unique(np.concatenate([inner, sel[:16]]))
        assert max(len(s.get_ray(p, r)) + len(s.get_ray(p, _anti(s, r)))
                   for p in inner for r in rays) >= 64
    for r in rays:
        I, xy = s.image(pops, r, line, v)
        Io, xyo = o.image(pops, r, line, v, points=sel)
        assert rel(I[sel], Io).max() <= TOL, (name, r)
        assert np.allclose(xy, xyo, rtol=1e-13, atol=1e-13 * np.abs(xyo).max())
        assert np.all(np.isfinite(I)) and np.all(I > 0)


def test_image_thermal_equilibrium_is_planck():
    w = configs.sphere2(n_points=200, seed=4)
    w.model.temperature[:] = 2.725
    s = solver_for(w)
    I, _ = s.image(s.lte(), 5, 0, np.linspace(-3e4, 3e4, 7))
    assert np.max(np.abs(I / oracle.planck(100e9, 2.725) - 1.0)) < 1e-12


def test_image_device_call_and_errors():
    import torch
    from paper_1912_08445_amd.binding import NlteError
    w = configs.sphere2(n_points=200)
    s = solver_for(w)
    pops = s.lte()
    I, xy = s.image(pops, 2, 0, [0.0, 1e4])
    dev = torch.device("cuda:0")
    Id = torch.empty((w.n_points, 2), dtype=torch.float64, device=dev)
    xyd = torch.empty((w.n_points, 2), dtype=torch.float64, device=dev)
    s.image_dev(torch.tensor(pops, device=dev), 2, 0, [0.0, 1e4], Id, xyd)
    torch.cuda.synchronize()
    assert np.array_equal(Id.cpu().numpy(), I) and np.array_equal(xyd.cpu().numpy(), xy)
    for args in [(12, 0, [0.0]), (-1, 0, [0.0]), (0, 1, [0.0]), (0, 0, [np.nan])]:
        with pytest.raises(NlteError):
            s.image(pops, *args)
