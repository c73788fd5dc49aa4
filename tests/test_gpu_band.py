"""Band ALO on the GPU against the oracle: the band entries of the formal solve, the
coupled statistical equilibrium, and the ALI that uses them."""
import numpy as np
import pytest

from oracle import band
from synth import configs, directions, species
from synth.models import concat_models

from _common import oracle_for, rel, solver_for

pytestmark = pytest.mark.gpu


def _thick_sphere(n_points=300, seed=9):
    w = configs.sphere2(n_points=n_points, seed=seed)
    w.model.abundance[:] = 1e-6
    return w


def _perturbed(o, w, seed=4):
    rng = np.random.default_rng(seed)
    pops = o.lte() * rng.uniform(0.6, 1.4, (w.n_points, w.species.n_lev))
    return pops * ((w.model.abundance * w.model.n_h2) / pops.sum(1))[:, None]


def _check_coefficients(got, ref, tol=1e-10):
    J, Je, L, Jb, Ld, Ln = got
    rJ, rJe, rL, rJb, rLd, rLn = ref
    assert rel(J, rJ).max() <= tol and rel(Je, rJe).max() <= tol and rel(L, rL).max() <= tol
    assert rel(Ld, rLd).max() <= tol
    # Jb is Jeff less the band's share: compare on the scale of Jeff
    assert (np.abs(Jb - rJb) / np.maximum(np.abs(rJe), 1e-300)).max() <= tol
    # couplings on the scale of the point's largest one
    scale = np.maximum(np.abs(rLn).max(axis=2, keepdims=True), 1e-300)
    assert (np.abs(Ln - rLn) / scale).max() <= tol


@pytest.mark.parametrize("lpl,nq", [(1, 9), (2, 9), (2, 40), (1, 80)])
def test_band_coefficients_match_oracle(lpl, nq):
    # outflow: velocity sub-steps next to the origin, several lines; nq 40 fills one lane
    # group per wave, nq 80 needs two frequency chunks
    w = configs.outflow5(n_points=300, seed=2, nside=1)
    w.quad_x, w.quad_w = directions.uniform_grid(nq, 3.0)
    o = oracle_for(w)
    pops = _perturbed(o, w)
    s = solver_for(w, lines_per_lane=lpl)
    _check_coefficients(s.formal_solve_band(pops), o.formal_solve_band(pops))


def test_band_formal_solve_keeps_the_local_outputs():
    # J, Jeff, L* of the band kernel are those of the local formal solve
    w = configs.outflow5(n_points=300, seed=6, nside=1)
    o = oracle_for(w)
    pops = _perturbed(o, w, 7)
    s = solver_for(w)
    J, Je, L = s.formal_solve(pops)
    Jb_, Je_b, L_b = s.formal_solve_band(pops)[:3]
    assert rel(J, Jb_).max() <= 1e-13 and rel(Je, Je_b).max() <= 1e-13 and rel(L, L_b).max() <= 1e-13


def test_coupled_stateq_matches_sparse_lu():
    w = _thick_sphere()
    o = oracle_for(w)
    pops = _perturbed(o, w, 11)
    J, Je, L, Jb, Ld, Ln = o.formal_solve_band(pops)
    ref, ok = band.stateq_band(o, pops, J, Je, L, Jb, Ld, Ln, band.first_cells(o))
    s = solver_for(w)
    got, used, its = s.stateq_band(pops, J, Je, L, Jb, Ld, Ln)
    assert ok and used and its > 0
    assert rel(got, ref).max() <= 1e-9


def test_coupled_stateq_multilevel_matches_sparse_lu():
    w = configs.outflow5(n_points=300, seed=2, nside=1)
    o = oracle_for(w)
    pops = o.lte()
    J, Je, L, Jb, Ld, Ln = o.formal_solve_band(pops)
    ref, ok = band.stateq_band(o, pops, J, Je, L, Jb, Ld, Ln, band.first_cells(o))
    got, used, its = solver_for(w).stateq_band(pops, J, Je, L, Jb, Ld, Ln)
    assert used == ok
    assert rel(got, ref).max() <= 1e-9


@pytest.mark.parametrize("iters", [1, 4])
def test_band_ali_iterates_match_oracle(iters):
    w = _thick_sphere()
    o = oracle_for(w)
    ref, ch, used = band.run_ali_band(o, max_iter=iters, tol=0.0)
    s = solver_for(w, alo_band=1, max_iter=iters, tol=0.0)
    pops, rep = s.run_ali()
    assert rep["iterations"] == iters and rep["n_band"] == sum(used) == iters
    assert rel(pops, ref).max() <= 1e-9
    assert np.allclose(rep["max_change"], ch, rtol=1e-6, atol=1e-14)


def test_band_ali_reaches_the_local_fixed_point_in_fewer_iterations():
    w = _thick_sphere()
    plain, rp = solver_for(w, max_iter=300, tol=1e-10).run_ali()
    acc, ra = solver_for(w, alo_band=1, max_iter=300, tol=1e-10).run_ali()
    assert rp["converged"] and ra["converged"]
    assert ra["iterations"] < rp["iterations"]
    assert rel(acc, plain).max() < 1e-8


def test_band_ali_keeps_thermal_equilibrium():
    w = configs.sphere2(n_points=120, seed=3)
    w.model.temperature[:] = 2.725
    w.model.abundance[:] = 1e-6
    s = solver_for(w, alo_band=1, max_iter=2, tol=0.0)
    pops, rep = s.run_ali()
    assert rep["n_band"] == 2
    assert rel(pops, s.lte()).max() < 1e-12


def test_band_ali_is_per_model_in_a_batch():
    ws = [_thick_sphere(300, 11), _thick_sphere(400, 12), configs.sphere2(n_points=250, seed=13)]
    offs, merged = concat_models([w.model for w in ws])
    wb = configs.sphere2(n_points=10)
    wb.model, wb.offsets = merged, offs
    sb = solver_for(wb, alo_band=1, max_iter=80, tol=1e-8)
    pb, rb = sb.run_ali()
    its, conv, _ = sb.model_status()
    assert all(conv)
    for m, w in enumerate(ws):
        ps, rs = solver_for(w, alo_band=1, max_iter=80, tol=1e-8).run_ali()
        # the coupled solve's inner products run over the whole batch: the iterates agree
        # to the solver's tolerance, the counts up to a step at the threshold
        assert abs(its[m] - rs["iterations"]) <= 1
        assert rel(pb[offs[m]:offs[m + 1]], ps).max() <= 1e-7


def test_band_needs_the_alo():
    from paper_1912_08445_amd.binding import NlteError
    w = configs.sphere2(n_points=100)
    s = solver_for(w)
    with pytest.raises(NlteError):
        s.set_params(alo_band=1, use_alo=0)
    with pytest.raises(NlteError):
        s.set_params(alo_band=2)


def _radiative_sphere(n_points, seed):
    # no collisions: with Ld = 1 and Jb = 0 a point's band rate matrix has no transitions
    w = configs.sphere2(n_points=n_points, seed=seed)
    w.species = species.two_level(100e9, 3.0, 1e-5, 0.0, 28.0)
    return w


def _singular_band_inputs(o, pops):
    J, Je, L = o.formal_solve(pops)
    n, nl, R = pops.shape[0], J.shape[1], o.n_rays
    return J, Je, L, np.zeros((n, nl)), np.ones((n, nl)), np.zeros((n, nl, R))


def test_band_fallback_on_singular_local_matrices():
    w = _radiative_sphere(120, 21)
    o = oracle_for(w)
    pops = o.lte()
    J, Je, L, Jb, Ld, Ln = _singular_band_inputs(o, pops)
    got, used, _ = solver_for(w).stateq_band(pops, J, Je, L, Jb, Ld, Ln)
    ref, ok = band.stateq_band(o, pops, J, Je, L, Jb, Ld, Ln, band.first_cells(o))
    local, flags = o.stateq(pops, J, Je, L)
    assert used == 0 and not ok and np.all(flags == 0)
    assert rel(got, local).max() <= 1e-10 and rel(ref, local).max() == 0.0


def test_band_fallback_is_per_model():
    # model 0 has singular band matrices, model 1 a regular band solve: only model 0 drops
    # to the local solve
    ws = [_radiative_sphere(120, 22), _radiative_sphere(150, 23)]
    offs, merged = concat_models([w.model for w in ws])
    wb = _radiative_sphere(10, 24)
    wb.model, wb.offsets = merged, offs
    parts, refs = [], []
    for m, w in enumerate(ws):
        o = oracle_for(w)
        pops = o.lte() * np.random.default_rng(30 + m).uniform(0.8, 1.2, (w.n_points, 2))
        pops *= ((w.model.abundance * w.model.n_h2) / pops.sum(1))[:, None]
        if m == 0:
            inp = _singular_band_inputs(o, pops)
            ref = o.stateq(pops, *inp[:3])[0]
        else:
            inp = o.formal_solve_band(pops)
            ref, ok = band.stateq_band(o, pops, *inp, band.first_cells(o))
            assert ok
        parts.append((pops, *inp))
        refs.append(ref)
    cat = [np.concatenate([p[k] for p in parts]) for k in range(7)]
    got, used, _ = solver_for(wb).stateq_band(*cat)
    assert used == 1
    assert rel(got[offs[0]:offs[1]], refs[0]).max() <= 1e-10
    assert rel(got[offs[1]:offs[2]], refs[1]).max() <= 1e-9


def test_band_with_ng_reaches_the_fixed_point():
    # Ng extrapolation of band iterates: same fixed point, no more iterations than either
    w = _thick_sphere()
    plain, rp = solver_for(w, max_iter=300, tol=1e-10).run_ali()
    _, rb = solver_for(w, alo_band=1, max_iter=300, tol=1e-10).run_ali()
    _, rn = solver_for(w, ng_every=4, max_iter=300, tol=1e-10).run_ali()
    both, rbn = solver_for(w, alo_band=1, ng_every=4, max_iter=300, tol=1e-10).run_ali()
    assert rbn["converged"] and rbn["n_ng_steps"] > 0 and rbn["n_band"] > 0
    assert rbn["iterations"] <= min(rb["iterations"], rn["iterations"])
    assert rel(both, plain).max() < 1e-8
    print("iterations plain / band / Ng / band+Ng:", rp["iterations"], rb["iterations"], rn["iterations"],
          rbn["iterations"])
