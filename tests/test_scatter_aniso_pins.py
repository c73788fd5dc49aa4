"""Pins of the scattering oracle with a direction-dependent scattering opacity (Sec. 2.1
Eq. RTE, Sec. 3.3: chi^- != 0 in Eq. RTE2 and GFE) and of the second equation of Eq. GFE
(the flux-like v): closed forms and brute-force integration of each direction, thermal
equilibrium, reductions, and the direction weights of the re-emitted field."""
import numpy as np
import pytest

from synth import configs, directions, species
from synth.models import chain_1d

from test_oracle_pins import CL, H, make, planck, rel
from test_scatter_pins import _moving_chain_exact
from test_oracle_pins import hubble_1d


# ---------------------------------------------------------------- one ray pair


def _exact_homogeneous(chit, chim, Sp, sg, I_lo, I_hi, z_o, L):
    """Both directions of Eq. RTE2 with constant coefficients: along +z
    dI/dz = chit (Sp + sg) - (chit + chim) I, along -z the same with -chim and -sg."""
    sp_ = chit * (Sp + sg) / (chit + chim)
    sm_ = chit * (Sp - sg) / (chit - chim)
    Ip = sp_ + (I_lo - sp_) * np.exp(-(chit + chim) * z_o)
    Im = sm_ + (I_hi - sm_) * np.exp(-(chit - chim) * (L - z_o))
    return Ip, Im


@pytest.mark.parametrize("L,chim", [(1.0, 0.6), (4.0, -0.9), (12.0, 1.2)])
def test_homogeneous_ray_with_odd_opacity_closed_form(oracle_lib, L, chim):
    """u +- v at the origin against the exact intensities of the two directions, whose
    opacities chit +- chi^- differ; second order in the node spacing.  (Flipping the sign
    of chi^- in the integrating factor, or leaving the boundary intensities untransformed,
    makes the error O(1).)"""
    chit, Sp, sg, I_lo, I_hi = 2.0, 1.3, 0.2, 0.1, 0.4
    Ip, Im = _exact_homogeneous(chit, chim, Sp, sg, I_lo, I_hi, 0.35 * L, L)
    errs = []
    for n in (20, 40, 80, 160):
        z = np.linspace(0.0, L, n + 1)
        o = 7 * n // 20
        one = np.ones(n + 1)
        u, lam, ue, v = oracle_lib.solve_ray_gen(z, chit * one, Sp * one, sg * one, I_lo, I_hi, o,
                                                 chim=chim * one)
        errs.append(max(abs(u + v - Ip) / abs(Ip), abs(u - v - Im) / abs(Im)))
    slopes = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(slopes - 2) < 0.3), (errs, slopes)
    # (on the thick ray the transformed sources e^M Splus change by 9% per step at n = 160)
    assert errs[-1] < (2e-4 if L < 10 else 2e-3), errs


def _rk4_dir(z, chit, chim, Sp, sg, I0, z_end, sign, steps=400):
    """dI/ds = chit (Sp + sign sg) - (chit + sign chim) I along the photon direction sign
    (+1: increasing z from z[0], -1: decreasing z from z[-1]), every coefficient linear
    between the nodes."""
    f = lambda zz, a: np.interp(zz, z, a)
    start = z[0] if sign > 0 else z[-1]
    grid = np.linspace(start, z_end, steps * len(z) + 1)
    I = I0

    def rhs(zz, II):
        ct = f(zz, chit)
        return ct * (f(zz, Sp) + sign * f(zz, sg)) - (ct + sign * f(zz, chim)) * II

    for k in range(len(grid) - 1):
        h = abs(grid[k + 1] - grid[k])
        zz, dz = grid[k], grid[k + 1] - grid[k]
        k1 = rhs(zz, I)
        k2 = rhs(zz + dz / 2, I + h / 2 * k1)
        k3 = rhs(zz + dz / 2, I + h / 2 * k2)
        k4 = rhs(zz + dz, I + h * k3)
        I = I + h / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
    return I


@pytest.mark.parametrize("seed", range(3))
def test_odd_opacity_brute_force(oracle_lib, seed):
    """Tiny rays with every coefficient varying (chit, chi^- with |chi^-| < chit, Splus,
    sigma): u_o + v_o and u_o - v_o converge at second order in the refinement to RK4 of
    each direction, which sees its own opacity chit +- chi^-."""
    rng = np.random.default_rng(500 + seed)
    N = int(rng.integers(3, 8))
    z = np.cumsum(rng.uniform(0.2, 1.0, N))
    chit = rng.uniform(0.3, 3.0, N)
    chim = chit * rng.uniform(-0.8, 0.8, N)
    Sp = rng.uniform(0.8, 2.0, N)
    sg = rng.uniform(-0.5, 0.5, N)
    I_lo, I_hi = 0.1, 0.3
    o = int(rng.integers(1, N - 1))
    Ip = _rk4_dir(z, chit, chim, Sp, sg, I_lo, z[o], +1)
    Im = _rk4_dir(z, chit, chim, Sp, sg, I_hi, z[o], -1)
    errs = []
    for m in (8, 16, 32, 64):
        zf = np.concatenate([np.linspace(z[k], z[k + 1], m + 1)[:-1] for k in range(N - 1)] + [[z[-1]]])
        cf, mf, spf, sgf = (np.interp(zf, z, a) for a in (chit, chim, Sp, sg))
        u, _, _, v = oracle_lib.solve_ray_gen(zf, cf, spf, sgf, I_lo, I_hi, o * m, chim=mf)
        errs.append(max(abs(u + v - Ip) / Ip, abs(u - v - Im) / Im))
    slopes = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(slopes > 1.7), (errs, slopes)
    assert errs[-1] < 1e-4


def test_zero_odd_opacity_is_the_isotropic_solve(oracle_lib):
    rng = np.random.default_rng(9)
    N = 9
    z = np.cumsum(rng.uniform(0.1, 2.0, N))
    chi, Sp, sg = rng.uniform(0.1, 5.0, N), rng.uniform(0.2, 2.0, N), rng.uniform(-0.3, 0.3, N)
    a = oracle_lib.solve_ray_gen(z, chi, Sp, sg, 0.3, 0.6, 4, own=Sp[4])
    b = oracle_lib.solve_ray_gen(z, chi, Sp, sg, 0.3, 0.6, 4, own=Sp[4], chim=np.zeros(N))
    assert a == b


def test_integrating_factor_range(oracle_lib):
    z = np.linspace(0.0, 1000.0, 11)
    one = np.ones(11)
    with pytest.raises(ValueError):
        oracle_lib.solve_ray_gen(z, one, one, 0 * one, 0.0, 0.0, 0, chim=0.9 * one)
    # the same ray seen from its far end stays in range only while |M| <= 700
    oracle_lib.solve_ray_gen(z[:8], one[:8], one[:8], 0 * one[:8], 0.0, 0.0, 0, chim=0.9 * one[:8])


# ---------------------------------------------------------------- the full formal solve


def _dipole(o, chi_sca, rng, frac=(0.0, 1.0)):
    d = rng.normal(size=(o.P, o.n_lines, 3))
    d /= np.linalg.norm(d, axis=2, keepdims=True)
    return d * (chi_sca * rng.uniform(*frac, chi_sca.shape))[:, :, None]


def test_thermal_equilibrium_with_odd_opacity_chain(oracle_lib):
    """T_gas = T_CMB on a static chain with a scattering opacity that differs along +x and
    -x: the reciprocal redistribution re-emits chi_s(n) B into every direction, so I = B
    solves both directions exactly.  The discretised pair carries the integrating factor
    e^M, which is not a polynomial, so the discrete Jw and J approach B at second order in
    the node spacing (and equal it to rounding without the odd part).  Along the chain the
    line-centre optical thickness is 1.3 and the scattering one 2.6; the error of a step
    goes as (mu dtau)^4 / (12 dtau^2), mu = chi^-/(chi + chi^+), so on optically thick
    steps with a strong odd part it is no longer small (with 20 times the abundance: 63%
    at 21 nodes, 3% at 81)."""
    sp = species.two_level(100e9, 3.0, 1e-5, 1e-10, 28.0)
    errs = []
    for n in (21, 41, 81):
        x = np.linspace(0.0, 1.0, n) * 1e16
        mdl = chain_1d(x, np.zeros(n), 1e4, 2.725, 1.5e4, 2e-8)
        o = make(oracle_lib, mdl, sp)
        pops = o.lte()
        nd = o.pair_nodes(pops, n // 2, 0)
        kap = nd["kappa"][nd["o"], 0]
        chi_sca = np.full((n, 1), 2.0 * kap)
        dip = np.zeros((n, 1, 3))
        dip[:, 0, 0] = 0.6 * chi_sca[:, 0]
        B = planck(100e9, 2.725)
        J, _, _, Jw = o.formal_solve_scat(pops, chi_sca, o.scattering_start(), chi_dip=dip)
        errs.append(max(np.abs(Jw / B - 1).max(), np.abs(J / B - 1).max()))
        if n == 21:
            J0, _, _, Jw0 = o.formal_solve_scat(pops, chi_sca, o.scattering_start())
            assert np.abs(Jw0 / B - 1).max() < 1e-12 and np.abs(J0 / B - 1).max() < 1e-12
    slopes = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(slopes - 2) < 0.3), (errs, slopes)
    assert errs[-1] < 1e-3, errs


@pytest.mark.parametrize("moving", [False, True])
def test_thermal_equilibrium_with_odd_opacity_3d(oracle_lib, moving):
    """The same in 3-D (HEALPix rays, random dipoles up to the full scattering opacity):
    Jw and J stay within the discretisation error of B, and without the dipoles equal it
    to rounding."""
    w = configs.sphere2(n_points=150, seed=4)
    w.model.temperature[:] = 2.725
    if not moving:
        w.model.vel[:] = 0.0
    o = oracle_lib.from_workload(w)
    pops = o.lte()
    rng = np.random.default_rng(6)
    nd = o.pair_nodes(pops, 0, 0)
    chi_sca = nd["kappa"][nd["o"], 0] * rng.uniform(0.1, 3.0, (o.P, 1))
    dip = _dipole(o, chi_sca, rng)
    B = planck(o.line_frequencies()[0], 2.725)
    J, E, L, Jw = o.formal_solve_scat(pops, chi_sca, o.scattering_start(), chi_dip=dip)
    assert np.abs(Jw / B - 1).max() < 1e-3 and np.abs(J / B - 1).max() < 1e-3
    J, E, L, Jw = o.formal_solve_scat(pops, chi_sca, o.scattering_start(), chi_dip=0.01 * dip)
    assert np.abs(Jw / B - 1).max() < 1e-5 and np.abs(J / B - 1).max() < 1e-5


def test_zero_dipole_is_the_isotropic_formal_solve(oracle_lib):
    w = configs.outflow5(n_points=120, seed=2, nside=1)
    o = oracle_lib.from_workload(w)
    pops = o.lte()
    rng = np.random.default_rng(3)
    nd = o.pair_nodes(pops, 0, 0)
    chi_sca = np.median(nd["kappa"][:, 0]) * rng.uniform(0.1, 2.0, (o.P, o.n_lines))
    Jnu = o.scattering_start() * rng.uniform(0.5, 2.0, (o.P, o.n_lines, o.n_q))
    sel = np.arange(0, 120, 11)
    a = o.formal_solve_scat(pops, chi_sca, Jnu, sel=sel)
    b = o.formal_solve_scat(pops, chi_sca, Jnu, sel=sel, chi_dip=np.zeros((o.P, o.n_lines, 3)))
    for x, y in zip(a, b):
        assert np.array_equal(x, y)
    with pytest.raises(ValueError):
        o.formal_solve_scat(pops, chi_sca, Jnu, sel=sel, chi_dip=_dipole(o, chi_sca, rng, (1.01, 1.1)))


def test_direction_weights_of_the_reemitted_field(oracle_lib):
    """A static homogeneous chain (rays +-x) with a negligible scattering opacity and, at
    one point, a dipole chi_dip = eps chi_sca x: its re-emitted field Jw is
    ((1 + eps) I(+x) + (1 - eps) I(-x))/2, so Jw(eps) - Jw(0) = eps (I(+x) - I(-x))/2 with
    I(+-x) = S + (I_b - S) exp(-kappa phi(x) l+-) over the path lengths l+- to either end."""
    n = 401
    sp = species.two_level(100e9, 3.0, 1e-5, 1e-10, 28.0)
    x = np.linspace(0.0, 1.0, n) * 1e16
    mdl = chain_1d(x, np.zeros(n), 1e4, 25.0, 1.5e4, 4e-7)
    q = directions.uniform_grid(31, 4.0)
    o = make(oracle_lib, mdl, sp, q=q)
    pops = o.lte()
    O = 120
    nd = o.pair_nodes(pops, O, 0)
    kap, S = nd["kappa"][nd["o"], 0], nd["S"][nd["o"], 0]
    chi_sca = np.full((n, 1), 1e-20 * kap)
    eps = 0.7
    dip = np.zeros((n, 1, 3))
    dip[O, 0, 0] = eps * chi_sca[O, 0]
    Jnu = o.scattering_start()
    _, _, _, J0 = o.formal_solve_scat(pops, chi_sca, Jnu, sel=[O])
    _, _, _, J1 = o.formal_solve_scat(pops, chi_sca, Jnu, sel=[O], chi_dip=dip)
    Ib = planck(100e9, 2.725)
    phi = np.exp(-q[0] ** 2)
    Ip = S + (Ib - S) * np.exp(-kap * phi * (x[O] - x[0]))
    Im = S + (Ib - S) * np.exp(-kap * phi * (x[-1] - x[O]))
    d = (J1 - J0)[0, 0]
    exact = 0.5 * eps * (Ip - Im)
    assert np.abs(exact).max() > 0.05 * abs(Ib - S)
    assert np.abs(d - exact).max() < 1e-4 * abs(Ib - S), (d, exact)


def test_odd_opacity_in_a_moving_medium_brute_force(oracle_lib):
    """A steep Hubble flow with a scattering opacity that differs along +x and -x and a
    previous Jw that is not symmetric in frequency: the oracle's Jw converges at second
    order in the sub-step size to the brute-force integration of both directions, each
    with its own opacity chi_line + chi_sca +- chi^- and emissivity (chi_sca +- chi^-) Jw,
    combined with the origin's weights 1 +- chi^-/chi_sca."""
    sp, mdl = hubble_1d(n_cells=24, dbeta_c=0.05)
    q = directions.uniform_grid(31, 4.0)
    o0 = make(oracle_lib, mdl, sp, q=q)
    pops = o0.lte()
    P = mdl.n_points
    nu = o0.line_frequencies()[0]
    I_in = planck(nu, 2.725)
    xq = q[0]
    ramp = np.linspace(0.5, 1.5, P)[:, None]
    Jnu = I_in * (1.0 + ramp * (1.0 + np.tanh(xq - 0.7)))[:, None, :]
    vw = o0.line_width_speed()
    kap_c = (H * nu / (4 * np.pi) * (pops[:, 0] * 3 - pops[:, 1]) * sp.line_A[0] * CL ** 2 /
             (2 * H * nu ** 3)) / (np.sqrt(np.pi) * nu * vw / CL)
    chi_sca = (0.3 * kap_c * np.linspace(0.5, 2.0, P))[:, None]
    cmx = chi_sca[:, 0] * np.linspace(-0.8, 0.6, P)
    dip = np.zeros((P, 1, 3))
    dip[:, 0, 0] = cmx
    sel = [5, 12, 18]
    exact = np.array([_moving_chain_exact(o0, mdl, pops, chi_sca, Jnu, O, xq, chim_x=cmx) for O in sel])
    errs = []
    for f in (0.2, 0.1, 0.05):
        o = make(oracle_lib, mdl, sp, q=q, f_sub=f)
        _, _, _, Jn = o.formal_solve_scat(pops, chi_sca, Jnu, sel=sel, chi_dip=dip)
        errs.append(rel(Jn[:, 0, :], exact).max())
    ratios = np.array(errs[:-1]) / np.array(errs[1:])
    assert np.all(ratios > 3.5), (errs, ratios)
    assert errs[-1] < 2e-6, errs
