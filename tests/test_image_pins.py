"""Pins of the imaging oracle (Sec. 3.5): emergent intensities at the ends of the ray pairs."""
import numpy as np

import oracle
from synth import configs, directions, species
from synth.configs import Workload
from synth.models import chain_1d


def _two_level():
    return species.two_level(100e9, 3.0, 1e-5, 1e-10, 28.0)


def test_thermal_equilibrium_emerges_as_the_planck_function():
    # gas at the CMB temperature in LTE: S = B everywhere, u = B is the exact discrete
    # solution, so every pixel shows B at every channel
    w = configs.sphere2(n_points=150, seed=4)
    w.model.temperature[:] = 2.725
    o = oracle.from_workload(w)
    I, _ = o.image(o.lte(), 5, 0, np.linspace(-3e4, 3e4, 7))
    B = oracle.planck(100e9, 2.725)
    assert np.max(np.abs(I / B - 1.0)) < 1e-12


def _chain(n, L=1e17, nh2=3e5):
    x = np.linspace(0.0, L, n)
    m = chain_1d(x, np.zeros(n), nh2, 30.0, 1.5e4, 1e-8)
    xq, wq = directions.uniform_grid(31, 4.0)
    return Workload("chain", m, _two_level(), directions.axis_pair(), xq, wq)


def test_homogeneous_chain_converges_to_the_closed_form():
    # static uniform chain seen along +x: I = S + (I_in - S) e^{-tau}, tau = kappa e^{-x^2} L;
    # the second-order discretisation error falls as the square of the node spacing
    errs = []
    for n in (21, 41, 81, 161):
        w = _chain(n)
        o = oracle.from_workload(w)
        pops = o.lte()
        v = np.array([0.0, 2e4])
        I, xy = o.image(pops, 0, 0, v)
        # every point of the chain lies on the same line of sight
        assert np.max(np.abs(I - I[0])) <= 1e-12 * np.max(np.abs(I))
        nd = o.pair_nodes(pops, 0, 0)
        kap, S = nd["kappa"][0, 0], nd["S"][0, 0]
        vw = o.line_width_speed()[0]
        tau = kap * np.exp(-(v / vw) ** 2) * 1e17
        I_in = oracle.planck(100e9, 2.725)
        exact = S + (I_in - S) * np.exp(-tau)
        errs.append(np.max(np.abs(I[0] - exact) / exact))
    slopes = -np.diff(np.log(errs)) / np.log(2.0)
    assert np.all(np.abs(slopes - 2.0) < 0.15), (errs, slopes)


def test_static_model_is_symmetric_in_channel_velocity():
    w = configs.sphere2(n_points=120, seed=6)
    o = oracle.from_workload(w)
    v = np.array([-2e4, -7e3, 7e3, 2e4])
    I, _ = o.image(o.lte(), 2, 0, v)
    assert np.max(np.abs(I - I[:, ::-1]) / I) < 1e-13


def test_optically_thin_model_shows_the_background():
    w = configs.sphere2(n_points=120, seed=7)
    w.model.abundance[:] = 1e-22
    o = oracle.from_workload(w)
    I, _ = o.image(o.lte(), 0, 0, np.array([0.0]))
    B = oracle.planck(100e9, 2.725)
    assert np.max(np.abs(I / B - 1.0)) < 1e-8


def test_image_plane_basis():
    rng = np.random.default_rng(1)
    for n in [np.array([0, 0, 1.0]), np.array([1.0, 0, 0])] + list(rng.normal(size=(5, 3))):
        n = n / np.linalg.norm(n)
        pts = np.vstack([np.eye(3), n, rng.normal(size=(4, 3))])
        xy = oracle.image_plane(pts, n)
        # the direction itself projects to the origin; the map preserves lengths orthogonal to n
        assert np.allclose(xy[3], 0.0, atol=1e-15)
        perp = pts[4:] - np.outer(pts[4:] @ n, n)
        assert np.allclose(np.linalg.norm(xy[4:], axis=1), np.linalg.norm(perp, axis=1), rtol=1e-14)
