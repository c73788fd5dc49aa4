"""Size limits and degenerate models through every solve: the largest quadrature the
library takes (256 frequencies: four frequency chunks per wave in the line and band
kernels, four waves per line in the scattering kernel) and a model of one point (no
walks: the boundary intensity at both ends)."""
import numpy as np
import pytest

from synth import configs, directions, species
from synth.configs import Workload
from synth.models import chain_1d

from _common import oracle_for, rel, solver_for

pytestmark = pytest.mark.gpu


def _max_quadrature_outflow():
    w = configs.outflow5(n_points=200, seed=12, nside=1)
    w.quad_x, w.quad_w = directions.uniform_grid(256, 4.0)
    return w


def test_line_and_band_solves_at_256_frequencies():
    w = _max_quadrature_outflow()
    o = oracle_for(w)
    pops = o.lte()
    s = solver_for(w)
    sel = np.arange(0, 200, 9)
    J, Je, L = s.formal_solve(pops)
    rJ, rJe, rL = o.formal_solve(pops, sel=sel)
    assert rel(J[sel], rJ).max() <= 1e-10 and rel(Je[sel], rJe).max() <= 1e-10 and rel(L[sel], rL).max() <= 1e-10
    band = s.formal_solve_band(pops)
    rb = o.formal_solve_band(pops, sel=sel)
    assert rel(band[3][sel], rb[3]).max() <= 1e-9 and rel(band[4][sel], rb[4]).max() <= 1e-10


def test_scattering_solve_at_256_frequencies():
    w = _max_quadrature_outflow()
    o = oracle_for(w)
    pops = o.lte()
    nd = o.pair_nodes(pops, 0, 0)
    chi = np.broadcast_to(np.median(nd["kappa"], axis=0), (w.n_points, w.species.n_lines)).copy()
    x = np.asarray(w.quad_x)
    Jnu = o.scattering_start() * (1.5 + np.tanh(x))[None, None, :]
    s = solver_for(w)
    s.set_scattering(chi)
    J, Je, L, Jn = s.formal_solve_scat(pops, Jnu)
    sel = np.arange(3, 200, 25)
    rJ, rJe, rL, rJn = o.formal_solve_scat(pops, chi, Jnu, sel=sel)
    assert rel(J[sel], rJ).max() <= 1e-10 and rel(L[sel], rL).max() <= 1e-10 and rel(Jn[sel], rJn).max() <= 1e-10
    assert (np.abs(Je[sel] - rJe) / rJ).max() <= 1e-10


def _single_point():
    m = chain_1d(np.array([0.0]), np.zeros(1), 1e5, 40.0, 1.5e4, 1e-6)
    qx, qw = directions.uniform_grid(31)
    return Workload("one", m, species.linear_rotor(5), directions.healpix_ring(1), qx, qw)


def test_single_point_model():
    w = _single_point()
    o = oracle_for(w)
    s = solver_for(w, max_iter=5, tol=0.0)
    pops = s.lte()
    I_in = o.scattering_start()[0, :, 0]
    # no neighbours: u is the boundary intensity on every ray, L* = 0, Jeff = J
    J, Je, L = s.formal_solve(pops)
    assert rel(J[0], I_in).max() < 1e-14 and np.all(L == 0.0) and rel(Je, J).max() < 1e-14
    rJ, rJe, rL = o.formal_solve(pops)
    assert rel(J, rJ).max() <= 1e-12
    band = s.formal_solve_band(pops)
    assert np.all(band[5] == 0.0) and rel(band[3], J).max() < 1e-14
    new, used, _ = s.stateq_band(pops, J, Je, L, *band[3:])
    ref, _ = o.stateq(pops, J, Je, L)
    assert rel(new, ref).max() <= 1e-10
    s.set_scattering(np.full((1, w.species.n_lines), 1e-15))
    Jnu0 = o.scattering_start()
    Js, _, _, Jn = s.formal_solve_scat(pops, Jnu0)
    assert rel(Js, J).max() < 1e-14 and rel(Jn, Jnu0).max() < 1e-14
    pa, ra = s.run_ali()
    s.set_scattering(None)
    # an image through a point with empty walks, at the channel limit: the background
    v = np.linspace(-1e6, 1e6, 1024)
    I, _ = s.image(pops, 0, 1, v)
    assert rel(I, I_in[1]).max() < 1e-14
    assert rel(I, o.image(pops, 0, 1, v, points=[0])[0]).max() <= 1e-12
    pb, rb = s.run_ali()
    assert ra["iterations"] == rb["iterations"] == 5
    assert rel(pa, pb).max() < 1e-13
