"""Scattering on the GPU against the oracle: the generalised Feautrier formal solve, the
per-frequency mean intensity it returns, and the ALI with scattering."""
import numpy as np
import pytest

from synth import configs, directions
from synth.models import concat_models

from _common import oracle_for, rel, solver_for

pytestmark = pytest.mark.gpu


def _fields(o, w, seed):
    """Perturbed LTE populations, a scattering opacity comparable to the line's and a
    previous J_nu that is not symmetric in frequency."""
    rng = np.random.default_rng(seed)
    pops = o.lte() * rng.uniform(0.7, 1.3, (w.n_points, w.species.n_lev))
    pops *= ((w.model.abundance * w.model.n_h2) / pops.sum(1))[:, None]
    nd = o.pair_nodes(pops, 0, 0)
    kap = np.median(nd["kappa"], axis=0)
    chi_sca = kap[None, :] * rng.uniform(0.1, 3.0, (w.n_points, w.species.n_lines))
    x = np.asarray(w.quad_x)
    Jnu = o.scattering_start() * (1.0 + rng.uniform(0.5, 2.0, (w.n_points, w.species.n_lines, 1))
                                  * (1.0 + np.tanh(x - 0.5))[None, None, :])
    return pops, chi_sca, Jnu


def _check(got, ref, tol=1e-10):
    J, Je, L, Jn = got
    rJ, rJe, rL, rJn = ref
    assert all(np.all(np.isfinite(a)) for a in got)
    assert rel(J, rJ).max() <= tol and rel(L, rL).max() <= tol
    assert (np.abs(Je - rJe) / np.abs(rJ)).max() <= tol
    assert rel(Jn, rJn).max() <= tol


@pytest.mark.parametrize("nq", [31, 80, 1, "gh24"])
def test_scat_formal_solve_matches_oracle(nq):
    # outflow: velocity sub-steps and four lines; 80 frequencies take two waves; one
    # frequency is the degenerate grid; Gauss-Hermite offsets are not evenly spaced
    w = configs.outflow5(n_points=300, seed=2, nside=1)
    if nq == "gh24":
        w.quad_x, w.quad_w = directions.gauss_hermite(24)
    else:
        w.quad_x, w.quad_w = directions.uniform_grid(nq, 4.0) if nq > 1 else (np.array([0.0]), np.array([1.0]))
    o = oracle_for(w)
    pops, chi_sca, Jnu = _fields(o, w, 5)
    ref = o.formal_solve_scat(pops, chi_sca, Jnu)
    s = solver_for(w)
    s.set_scattering(chi_sca)
    _check(s.formal_solve_scat(pops, Jnu), ref)


def _segment_paths(o, w):
    """Counts of the sub-step segments that the isotropic kernel steps by its linear forms:
    far-wing segments (every offset beyond |y|^2 = 750 on one side at both ends) with at
    least four sub-steps, and segments whose lookups all clamp (every offset beyond the
    quadrature on one side at both ends) but that are not far-wing, with at least three."""
    x = np.asarray(w.quad_x)
    lo, hi = x.min(), x.max()
    vw = o.line_width_speed()
    vel, rays = w.model.vel, np.asarray(w.rays)
    far4 = clamp3 = 0
    for O in range(w.n_points):
        for r in range(len(rays)):
            cells, _ = o.walk(O, r)
            if len(cells) == 0:
                continue
            nodes = np.concatenate(([O], cells))
            s_ = (vel[nodes] - vel[O]) @ rays[r]
            y = (vw[O] / vw[nodes])[:, None] * x[None, :] - (s_ / vw[nodes])[:, None]
            ds = np.abs(np.diff(s_))
            thr = 0.25 * np.minimum(vw[nodes][:-1], vw[nodes][1:])
            m = np.where(ds > thr, np.ceil(ds / thr), 1)
            a, b = y[:-1], y[1:]
            clamp = np.all(((a >= hi) & (b >= hi)) | ((a <= lo) & (b <= lo)), axis=1)
            far = clamp & np.all((np.sign(a) == np.sign(b)) & (a * a > 750.0) & (b * b > 750.0), axis=1)
            far4 += int(np.sum(far & (m >= 4)))
            clamp3 += int(np.sum(clamp & ~far & (m >= 3)))
    return far4, clamp3


def test_scat_linear_segment_forms_match_oracle():
    """The isotropic kernel's linear forms (far-wing and clamped-lookup segments) on an
    outflow that has both, with no scattering opacity in about 30% of the cells (the forms'
    zero-opacity cases: no scattering term at a node, or at one end of a segment only),
    against the oracle."""
    w = configs.outflow5(n_points=300, seed=12, nside=1)
    o = oracle_for(w)
    far4, clamp3 = _segment_paths(o, w)
    assert far4 > 100 and clamp3 > 100, (far4, clamp3)
    pops, chi_sca, Jnu = _fields(o, w, 31)
    chi_sca *= np.random.default_rng(32).uniform(size=w.n_points)[:, None] > 0.3
    ref = o.formal_solve_scat(pops, chi_sca, Jnu)
    s = solver_for(w)
    s.set_scattering(chi_sca)
    _check(s.formal_solve_scat(pops, Jnu), ref)


def test_scat_formal_solve_static_sphere_matches_oracle():
    w = configs.sphere2(n_points=400, seed=7)
    o = oracle_for(w)
    pops, chi_sca, Jnu = _fields(o, w, 8)
    s = solver_for(w)
    s.set_scattering(chi_sca)
    _check(s.formal_solve_scat(pops, Jnu), o.formal_solve_scat(pops, chi_sca, Jnu))


def test_zero_scattering_opacity_gives_the_line_formal_solve():
    w = configs.outflow5(n_points=300, seed=3, nside=1)
    o = oracle_for(w)
    pops, _, Jnu = _fields(o, w, 9)
    s = solver_for(w)
    J0, E0, L0 = s.formal_solve(pops)
    s.set_scattering(np.zeros((w.n_points, w.species.n_lines)))
    J, E, L, _ = s.formal_solve_scat(pops, Jnu)
    assert np.all(np.isfinite(J)) and np.all(np.isfinite(E)) and np.all(np.isfinite(L))
    assert rel(J, J0).max() < 1e-12 and rel(L, L0).max() < 1e-12
    assert (np.abs(E - E0) / J0).max() < 1e-12


def test_thermal_equilibrium_with_scattering():
    w = configs.outflow5(n_points=200, seed=4, nside=1)
    w.model.temperature[:] = 2.725
    s = solver_for(w, max_iter=2, tol=0.0)
    o = oracle_for(w)
    pops, chi_sca, _ = _fields(o, w, 10)
    s.set_scattering(chi_sca)
    lte = s.lte()
    out, rep = s.run_ali()
    B = o.scattering_start()
    assert rel(s.scattering_field(), B).max() < 1e-12
    assert rel(out, lte).max() < 1e-12


@pytest.mark.parametrize("iters", [1, 3])
def test_scat_ali_matches_oracle(iters):
    w = configs.outflow5(n_points=100, seed=3, nside=1)
    o = oracle_for(w)
    _, chi_sca, _ = _fields(o, w, 11)
    ref, ch, Jref = o.run_ali_scat(chi_sca, max_iter=iters, tol=0.0)
    s = solver_for(w, max_iter=iters, tol=0.0)
    s.set_scattering(chi_sca)
    pops, rep = s.run_ali()
    assert rep["iterations"] == iters
    assert rel(pops, ref).max() <= 1e-9
    assert rel(s.scattering_field(), Jref).max() <= 1e-9
    assert np.allclose(rep["max_change"], ch, rtol=1e-6, atol=1e-14)


def test_scat_ali_precision_setting_does_not_change_it():
    # the scattering solve is FP64 in every form, and so is the stat-eq
    w = configs.outflow5(n_points=150, seed=6, nside=1)
    o = oracle_for(w)
    _, chi_sca, _ = _fields(o, w, 12)
    out = []
    for prec in (0, 1):
        s = solver_for(w, max_iter=3, tol=0.0, precision=prec)
        s.set_scattering(chi_sca)
        out.append(s.run_ali()[0])
    assert np.array_equal(out[0], out[1])


def test_scat_ali_is_per_model_in_a_batch():
    ws = [configs.outflow5(n_points=n, seed=sd, nside=1) for n, sd in ((150, 21), (220, 22))]
    offs, merged = concat_models([w.model for w in ws])
    wb = configs.outflow5(n_points=10, nside=1)
    wb.model, wb.offsets = merged, offs
    chis = [_fields(oracle_for(w), w, 13 + m)[1] for m, w in enumerate(ws)]
    sb = solver_for(wb, max_iter=40, tol=1e-6)
    sb.set_scattering(np.concatenate(chis))
    pb, _ = sb.run_ali()
    its, conv, _ = sb.model_status()
    jb = sb.scattering_field()
    for m, w in enumerate(ws):
        s = solver_for(w, max_iter=40, tol=1e-6)
        s.set_scattering(chis[m])
        ps, rs = s.run_ali()
        assert its[m] == rs["iterations"]
        assert rel(pb[offs[m]:offs[m + 1]], ps).max() <= 1e-13
        assert rel(jb[offs[m]:offs[m + 1]], s.scattering_field()).max() <= 1e-13


def test_scattering_argument_checks():
    from paper_1912_08445_amd.binding import NlteError
    w = configs.sphere2(n_points=100)
    s = solver_for(w)
    with pytest.raises(NlteError):
        s.set_scattering(-np.ones((w.n_points, 1)))
    with pytest.raises(NlteError):
        s.scattering_field()
    s.set_scattering(np.ones((w.n_points, 1)) * 1e-18)
    s.set_params(alo_band=1)
    with pytest.raises(NlteError):
        s.run_ali()
    s.set_params(alo_band=0)
    s.set_scattering(None)
    with pytest.raises(NlteError):
        s.formal_solve_scat(s.lte(), np.zeros((w.n_points, 1, w.quad_x.shape[0])))


# ---------------------------------------------------------------- odd scattering opacity


def _dipole(w, chi_sca, seed, frac=(0.0, 1.0)):
    rng = np.random.default_rng(seed)
    d = rng.normal(size=(w.n_points, w.species.n_lines, 3))
    d /= np.linalg.norm(d, axis=2, keepdims=True)
    return d * (chi_sca * rng.uniform(*frac, chi_sca.shape))[:, :, None]


@pytest.mark.parametrize("nq", [31, "gh24"])
def test_dipole_formal_solve_matches_oracle(nq):
    """chi_s(n) = chi_sca + chi_dip . n with dipoles up to the full opacity: J, L*, Jeff and
    the weighted field Jw against the oracle's global integrating factor (the kernel
    re-frames its elimination at every sub-step)."""
    w = configs.outflow5(n_points=300, seed=2, nside=1)
    if nq == "gh24":
        w.quad_x, w.quad_w = directions.gauss_hermite(24)
    o = oracle_for(w)
    pops, chi_sca, Jnu = _fields(o, w, 15)
    dip = _dipole(w, chi_sca, 16)
    ref = o.formal_solve_scat(pops, chi_sca, Jnu, chi_dip=dip)
    s = solver_for(w)
    s.set_scattering(chi_sca)
    s.set_scattering_dipole(dip)
    _check(s.formal_solve_scat(pops, Jnu), ref, tol=1e-9)
    # the odd part matters at this size
    iso = o.formal_solve_scat(pops, chi_sca, Jnu)
    assert rel(ref[3], iso[3]).max() > 1e-3


def test_dipole_formal_solve_static_sphere_matches_oracle():
    w = configs.sphere2(n_points=400, seed=7)
    o = oracle_for(w)
    pops, chi_sca, Jnu = _fields(o, w, 17)
    dip = _dipole(w, chi_sca, 18)
    s = solver_for(w)
    s.set_scattering(chi_sca)
    s.set_scattering_dipole(dip)
    _check(s.formal_solve_scat(pops, Jnu), o.formal_solve_scat(pops, chi_sca, Jnu, chi_dip=dip), tol=1e-9)


def test_zero_dipole_is_the_isotropic_solve():
    """A zero dipole gives the isotropic solve.  The two kernels round differently (the
    isotropic one steps far-wing and clamped-lookup segments with their node values linear
    in the sub-node index, the other through the general step), so they agree to 1e-12 of
    each output's largest value, not bit for bit."""
    w = configs.outflow5(n_points=200, seed=5, nside=1)
    o = oracle_for(w)
    pops, chi_sca, Jnu = _fields(o, w, 19)
    s = solver_for(w)
    s.set_scattering(chi_sca)
    a = s.formal_solve_scat(pops, Jnu)
    s.set_scattering_dipole(np.zeros((w.n_points, w.species.n_lines, 3)))
    b = s.formal_solve_scat(pops, Jnu)
    for x, y in zip(a, b):
        assert np.max(np.abs(x - y)) <= 1e-12 * np.max(np.abs(x))
    # a new scattering opacity drops the dipole
    s.set_scattering_dipole(_dipole(w, chi_sca, 20))
    assert not np.array_equal(s.formal_solve_scat(pops, Jnu)[3], a[3])
    s.set_scattering(chi_sca)
    assert np.array_equal(s.formal_solve_scat(pops, Jnu)[3], a[3])


@pytest.mark.parametrize("iters", [1, 3])
def test_dipole_ali_matches_oracle(iters):
    w = configs.outflow5(n_points=100, seed=3, nside=1)
    o = oracle_for(w)
    _, chi_sca, _ = _fields(o, w, 21)
    dip = _dipole(w, chi_sca, 22)
    ref, ch, Jref = o.run_ali_scat(chi_sca, max_iter=iters, tol=0.0, chi_dip=dip)
    s = solver_for(w, max_iter=iters, tol=0.0)
    s.set_scattering(chi_sca)
    s.set_scattering_dipole(dip)
    pops, rep = s.run_ali()
    assert rep["iterations"] == iters
    assert rel(pops, ref).max() <= 1e-9
    assert rel(s.scattering_field(), Jref).max() <= 1e-9
    assert np.allclose(rep["max_change"], ch, rtol=1e-6, atol=1e-14)


def test_dipole_argument_checks():
    from paper_1912_08445_amd.binding import NlteError
    w = configs.sphere2(n_points=100)
    s = solver_for(w)
    d = np.zeros((w.n_points, 1, 3))
    with pytest.raises(NlteError):
        s.set_scattering_dipole(d)          # no scattering opacity yet
    chi = np.ones((w.n_points, 1)) * 1e-18
    s.set_scattering(chi)
    d[5, 0] = [1e-18, 1e-18, 0.0]           # |d| = 1.41 chi_sca
    with pytest.raises(NlteError):
        s.set_scattering_dipole(d)
    d[5, 0] = [np.nan, 0.0, 0.0]
    with pytest.raises(NlteError):
        s.set_scattering_dipole(d)
    d[5, 0] = [0.0, 0.0, 1e-18]             # exactly the full opacity along z
    s.set_scattering_dipole(d)
    s.set_scattering_dipole(None)


def test_dipole_ali_is_per_model_in_a_batch():
    ws = [configs.outflow5(n_points=n, seed=sd, nside=1) for n, sd in ((150, 31), (220, 32))]
    offs, merged = concat_models([w.model for w in ws])
    wb = configs.outflow5(n_points=10, nside=1)
    wb.model, wb.offsets = merged, offs
    chis = [_fields(oracle_for(w), w, 33 + m)[1] for m, w in enumerate(ws)]
    dips = [_dipole(w, c, 35 + m) for m, (w, c) in enumerate(zip(ws, chis))]
    sb = solver_for(wb, max_iter=40, tol=1e-6)
    sb.set_scattering(np.concatenate(chis))
    sb.set_scattering_dipole(np.concatenate(dips))
    pb, _ = sb.run_ali()
    its, conv, _ = sb.model_status()
    jb = sb.scattering_field()
    for m, w in enumerate(ws):
        s = solver_for(w, max_iter=40, tol=1e-6)
        s.set_scattering(chis[m])
        s.set_scattering_dipole(dips[m])
        ps, rs = s.run_ali()
        assert its[m] == rs["iterations"]
        assert rel(pb[offs[m]:offs[m + 1]], ps).max() <= 1e-13
        assert rel(jb[offs[m]:offs[m + 1]], s.scattering_field()).max() <= 1e-13
