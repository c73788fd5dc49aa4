"""The band ALO and the scattering solve on the 50,000-point outflow (48 rays, 4 lines x
31 frequencies) at full size: sampled origins against the oracle, and properties that
hold at every point."""
import numpy as np
import pytest

from synth import configs

from _common import oracle_for, rel, solver_for

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def outflow():
    w = configs.outflow5()
    s = solver_for(w)
    print("outflow traced", flush=True)
    return w, s, oracle_for(w)


def test_band_full_size_sampled(outflow):
    w, s, o = outflow
    pops = s.lte()
    got = s.formal_solve_band(pops)
    print("band sweep done", flush=True)
    sel = np.random.default_rng(5).choice(w.n_points, 4, replace=False)
    ref = o.formal_solve_band(pops, sel=sel)
    print("oracle done", flush=True)
    J, Je, L, Jb, Ld, Ln = got
    rJ, rJe, rL, rJb, rLd, rLn = ref
    assert rel(J[sel], rJ).max() <= 1e-10 and rel(L[sel], rL).max() <= 1e-10
    assert rel(Ld[sel], rLd).max() <= 1e-10
    assert (np.abs(Jb[sel] - rJb) / rJe).max() <= 1e-10
    scale = np.abs(rLn).max(axis=2, keepdims=True)
    assert (np.abs(Ln[sel] - rLn) / scale).max() <= 1e-10
    # every point: the neighbour shares add to the diagonal and are non-negative
    assert np.all(Ld >= L * (1 - 1e-12)) and np.all(Ln >= 0) and np.all(np.isfinite(Jb))


def test_scattering_full_size_sampled(outflow):
    w, s, o = outflow
    pops = s.lte()
    nd = o.pair_nodes(pops, 0, 0)
    rng = np.random.default_rng(6)
    chi = np.median(nd["kappa"], axis=0)[None, :] * rng.uniform(0.2, 2.0, (w.n_points, w.species.n_lines))
    x = np.asarray(w.quad_x)
    Jnu = o.scattering_start() * (1.0 + rng.uniform(0.5, 1.5, (w.n_points, w.species.n_lines, 1))
                                  * (1.0 + np.tanh(x - 0.5))[None, None, :])
    s.set_scattering(chi)
    J, Je, L, Jn = s.formal_solve_scat(pops, Jnu)
    print("scattering sweep done", flush=True)
    sel = np.random.default_rng(7).choice(w.n_points, 3, replace=False)
    rJ, rJe, rL, rJn = o.formal_solve_scat(pops, chi, Jnu, sel=sel)
    print("oracle done", flush=True)
    assert rel(J[sel], rJ).max() <= 1e-10 and rel(L[sel], rL).max() <= 1e-10
    assert (np.abs(Je[sel] - rJe) / rJ).max() <= 1e-10
    assert rel(Jn[sel], rJn).max() <= 1e-10
    # every point: finite, and the quadrature of J_nu is the line's J (Sec. 3.1.3: the
    # pair sum equals the ray sum for a symmetric quadrature)
    assert np.all(np.isfinite(Jn))
    assert rel((Jn * np.asarray(w.quad_w)[None, None, :]).sum(axis=2), J).max() <= 1e-12
    s.set_scattering(None)


def test_scattering_dipole_full_size_sampled(outflow):
    """The full outflow with a scattering opacity that differs by direction (dipoles up to
    the whole opacity): sampled origins against the oracle, every point finite."""
    w, s, o = outflow
    pops = s.lte()
    nd = o.pair_nodes(pops, 0, 0)
    rng = np.random.default_rng(16)
    chi = np.median(nd["kappa"], axis=0)[None, :] * rng.uniform(0.2, 2.0, (w.n_points, w.species.n_lines))
    d = rng.normal(size=(w.n_points, w.species.n_lines, 3))
    d *= (chi * rng.uniform(0.0, 1.0, chi.shape) / np.linalg.norm(d, axis=2))[:, :, None]
    Jnu = o.scattering_start() * rng.uniform(0.5, 2.0, (w.n_points, w.species.n_lines, 1))
    s.set_scattering(chi)
    s.set_scattering_dipole(d)
    J, Je, L, Jn = s.formal_solve_scat(pops, Jnu)
    print("scattering sweep done", flush=True)
    sel = np.random.default_rng(17).choice(w.n_points, 3, replace=False)
    rJ, rJe, rL, rJn = o.formal_solve_scat(pops, chi, Jnu, sel=sel, chi_dip=d)
    print("oracle done", flush=True)
    assert rel(J[sel], rJ).max() <= 1e-9 and rel(L[sel], rL).max() <= 1e-9
    assert (np.abs(Je[sel] - rJe) / rJ).max() <= 1e-9
    assert rel(Jn[sel], rJn).max() <= 1e-9
    assert np.all(np.isfinite(Jn)) and np.all(np.isfinite(J))
    s.set_scattering(None)
