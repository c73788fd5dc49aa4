"""Pins of the scattering oracle (the generalised Feautrier equation of Sec. 3.3 with an
isotropic, coherent scattering term): reductions to the line-only solve, thermal
equilibrium, closed forms and brute-force integration of the first-order equations."""
import numpy as np
import pytest

from synth import configs, directions, species
from synth.models import chain_1d

from test_oracle_pins import CL, H, hubble_1d, make, planck, rel, rk4_intensity


# ---------------------------------------------------------------- reductions


@pytest.mark.parametrize("seed", range(3))
def test_generalised_solve_without_sigma_is_the_line_solve(oracle_lib, seed):
    rng = np.random.default_rng(300 + seed)
    N = int(rng.integers(2, 9))
    z = np.cumsum(rng.uniform(0.1, 2.0, N))
    chi = 10.0 ** rng.uniform(-3, 2, N)
    S = rng.uniform(0.2, 2.0, N)
    o = int(rng.integers(0, N))
    u0, l0, e0 = oracle_lib.solve_ray(z, chi, S, 0.3, 0.6, o)
    u, lam, ue, v = oracle_lib.solve_ray_gen(z, chi, S, np.zeros(N), 0.3, 0.6, o, own=S[o])
    assert rel(u, u0) < 1e-13 and rel(lam, l0) < 1e-13 and rel(ue, e0) < 1e-12


def test_zero_scattering_opacity_gives_the_line_formal_solve(oracle_lib):
    w = configs.outflow5(n_points=120, seed=2, nside=1)
    o = oracle_lib.from_workload(w)
    # strongly perturbed populations: some lines are inverted (masers, zero line opacity)
    pops = o.lte() * np.random.default_rng(4).uniform(0.3, 3.0, (w.n_points, w.species.n_lev))
    g = w.species.weight
    inverted = (pops[:, 1:] / g[1:] > pops[:, :-1] / g[:-1]).any(axis=1)
    assert inverted.any()
    sel = np.arange(0, 120, 7)
    J0, E0, L0 = o.formal_solve(pops, sel=sel)
    rng = np.random.default_rng(1)
    Jnu = o.scattering_start() * rng.uniform(0.5, 2.0, (o.P, o.n_lines, o.n_q))
    J, E, L, _ = o.formal_solve_scat(pops, np.zeros((o.P, o.n_lines)), Jnu, sel=sel)
    assert rel(J, J0).max() < 1e-12 and rel(E, E0).max() < 1e-12 and rel(L, L0).max() < 1e-12


def test_zero_scattering_opacity_per_frequency_field(oracle_lib):
    """Without scattering every node's source is the line's S, also where the line opacity
    is denormal or zero (far wings): J_nu out of the scattering solve against the same
    field assembled pair by pair and frequency by frequency from the pair nodes, with
    S+ = S and sigma = 0 at every node (the line solve's rows; the generalised ray solve
    without sigma is pinned to the line solve above), and the per-frequency output formed
    from u + v and u - v of the two directions."""
    w = configs.outflow5(n_points=120, seed=2, nside=1)
    o = oracle_lib.from_workload(w)
    pops = o.lte() * np.random.default_rng(6).uniform(0.7, 1.3, (w.n_points, w.species.n_lev))
    Jnu = o.scattering_start() * np.random.default_rng(7).uniform(0.5, 2.0, (o.P, o.n_lines, o.n_q))
    sel = np.arange(3, 120, 13)
    _, _, _, Jo = o.formal_solve_scat(pops, np.zeros((o.P, o.n_lines)), Jnu, sel=sel)
    x = np.asarray(w.quad_x)
    nu = o.line_frequencies()
    denormal = 0
    for k, O in enumerate(sel):
        Jp = np.zeros((o.n_lines, o.n_q))
        Jm = np.zeros((o.n_lines, o.n_q))
        for p in range(o.n_pairs):
            nd = o.pair_nodes(pops, O, p)
            for l in range(o.n_lines):
                Ib = oracle_lib.planck(nu[l], 2.725)
                for n in range(o.n_q):
                    y = nd["a"] * x[n] - nd["b"]
                    chi = nd["kappa"][:, l] * np.exp(-y * y)
                    denormal += int(np.sum((chi > 0) & (chi < 2.2250738585072014e-308)))
                    u, _, _, v = oracle_lib.solve_ray_gen(nd["z"], chi, nd["S"][:, l], np.zeros(len(y)), Ib, Ib, nd["o"])
                    Jp[l, n] += u + v
                    Jm[l, n] += u - v
        ref = (Jp + Jm[:, ::-1]) / o.n_rays
        assert rel(Jo[k], ref).max() < 1e-12
    assert denormal > 0


# ---------------------------------------------------------------- invariants


@pytest.mark.parametrize("moving", [False, True])
def test_thermal_equilibrium_with_scattering(oracle_lib, moving):
    """T_gas = T_CMB: u = B solves every pair at every frequency for any scattering
    opacity, so J_nu = B, J = B, and Boltzmann populations stay a fixed point."""
    w = configs.sphere2(n_points=150, seed=4)
    w.model.temperature[:] = 2.725
    if not moving:
        w.model.vel[:] = 0.0
    o = oracle_lib.from_workload(w)
    pops = o.lte()
    rng = np.random.default_rng(2)
    nd = o.pair_nodes(pops, 0, 0)
    chi_sca = nd["kappa"][nd["o"], 0] * rng.uniform(0.1, 10.0, (o.P, 1))
    nu = o.line_frequencies()
    B = planck(nu[0], 2.725)
    J, E, L, Jnu = o.formal_solve_scat(pops, chi_sca, o.scattering_start())
    assert np.abs(Jnu / B - 1).max() < 1e-12 and np.abs(J / B - 1).max() < 1e-12
    new, flags = o.stateq(pops, J, E, L)
    assert np.all(flags == 0) and rel(new, pops).max() < 1e-12


def test_thermal_equilibrium_with_scattering_in_part_of_the_points(oracle_lib):
    """T_gas = T_CMB on the outflow, whose far wings reach denormal and zero line opacities,
    with no scattering opacity in about 30% of the points: u = B still solves every pair at
    every frequency, so J_nu = J = B.  This needs S+ = S at the nodes without scattering
    whatever their line opacity: an S+ formed as chi_line S / chi_tot is 0 where
    chi_line S underflows, and so is one that is 0 at nodes without opacity."""
    w = configs.outflow5(n_points=150, seed=8, nside=1)
    w.model.temperature[:] = 2.725
    o = oracle_lib.from_workload(w)
    pops = o.lte()
    rng = np.random.default_rng(9)
    nd = o.pair_nodes(pops, 0, 0)
    chi_sca = nd["kappa"][nd["o"]][None, :] * rng.uniform(0.1, 10.0, (o.P, o.n_lines))
    chi_sca *= rng.uniform(size=(o.P, 1)) > 0.3
    nu = o.line_frequencies()
    B = np.array([planck(f, 2.725) for f in nu])
    J, E, L, Jnu = o.formal_solve_scat(pops, chi_sca, o.scattering_start())
    assert np.abs(Jnu / B[None, :, None] - 1).max() < 1e-12 and np.abs(J / B[None, :] - 1).max() < 1e-12


# ---------------------------------------------------------------- per-direction intensities


def test_per_frequency_mean_intensity_hubble_lemaitre_1d(oracle_lib):
    """Without scattering, J_nu(x) at a point from u +- v of the pairs at x and -x must
    match the closed form of Sec. 4.1.1 frequency by frequency: the two directions see
    optical depths tau(x, R + r) and tau(x, R - r) (Eq. Hubble-Lemaitre1D)."""
    from scipy.special import erf
    sp, mdl = hubble_1d()
    q = directions.gauss_hermite(100)
    o = make(oracle_lib, mdl, sp, q=q)
    pops = o.lte()
    nu = (sp.energy[1] - sp.energy[0]) / H
    n = pops[0]
    Bul = sp.line_A[0] * CL ** 2 / (2 * H * nu ** 3)
    kchi = H * nu / (4 * np.pi) * (n[0] * 3 * Bul - n[1] * Bul)
    S = n[1] * sp.line_A[0] / (n[0] * 3 * Bul - n[1] * Bul)
    vw = o.line_width_speed()[0]
    Dbeta = 0.01 / CL
    I = planck(nu, 2.725)
    xpos = mdl.pos[:, 0]
    R = xpos[-1]
    tau = lambda x, l: kchi / (2 * nu * Dbeta) * (erf(x + CL * Dbeta * l / vw) - erf(x))
    sel = np.arange(1, 99, 4)
    _, _, _, Jnu = o.formal_solve_scat(pops, np.zeros((o.P, 1)), o.scattering_start(), sel=sel)
    errs = []
    for row, O in enumerate(sel):
        exact = S + 0.5 * (I - S) * (np.exp(-tau(q[0], xpos[O] + R)) + np.exp(-tau(q[0], R - xpos[O])))
        errs.append(rel(Jnu[row, 0], exact))
    errs = np.concatenate(errs)
    assert np.quantile(errs, 0.95) < 1e-4 and np.median(errs) < 1e-5


@pytest.mark.parametrize("seed", range(3))
def test_generalised_solve_brute_force(oracle_lib, seed):
    """Tiny rays with a source that differs by direction (S+ + sigma along +z, S+ - sigma
    along -z): u_o + v_o and u_o - v_o must converge, at second order in the refinement,
    to the first-order integrations of each direction (Eq. RTE2)."""
    rng = np.random.default_rng(200 + seed)
    N = int(rng.integers(3, 8))
    z = np.cumsum(rng.uniform(0.2, 1.0, N))
    chi = rng.uniform(0.3, 3.0, N)
    Sp = rng.uniform(0.8, 2.0, N)
    sg = rng.uniform(-0.5, 0.5, N)
    I_lo, I_hi = 0.1, 0.3
    o = int(rng.integers(1, N - 1))
    Ip = rk4_intensity(z, chi, Sp + sg, I_lo, z[o])
    Im = rk4_intensity(z[::-1], chi[::-1], (Sp - sg)[::-1], I_hi, z[o])
    errs = []
    for m in (8, 16, 32, 64):
        zf = np.concatenate([np.linspace(z[k], z[k + 1], m + 1)[:-1] for k in range(N - 1)] + [[z[-1]]])
        cf, spf, sgf = np.interp(zf, z, chi), np.interp(zf, z, Sp), np.interp(zf, z, sg)
        u, _, _, v = oracle_lib.solve_ray_gen(zf, cf, spf, sgf, I_lo, I_hi, o * m)
        errs.append(max(abs(u + v - Ip) / Ip, abs(u - v - Im) / Im))
    slopes = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(slopes > 1.7), (errs, slopes)
    assert errs[-1] < 1e-4


def _moving_chain_exact(o, mdl, pops, chi_sca, Jnu, O, xq, steps=60, chim_x=None):
    """J_nu(x) at chain point O by integrating dI/ds = chi_tot (S_dir - I) along +x and
    along -x, with every profile-free quantity linear between the chain nodes (what the
    velocity sub-steps discretise): Doppler coefficients a, b, line kappa and S, chi_sca,
    and the nodes' J_nu evaluated at the local offset.  With chim_x (the odd scattering
    opacity along +x per point) each direction s = +-1 has scattering opacity
    chi_sca + s chim_x and emissivity (chi_sca + s chim_x) Jw, and the result is O's
    weighted field ((1 + e) I(+x) + (1 - e) I(-x))/2, e = chim_x/chi_sca at O."""
    sp = o.species
    nu = o.line_frequencies()[0]
    Bul = sp.line_A[0] * CL ** 2 / (2 * H * nu ** 3)
    Blu = sp.weight[1] / sp.weight[0] * Bul
    vw = o.line_width_speed()
    kchi = H * nu / (4 * np.pi) * (pops[:, 0] * Blu - pops[:, 1] * Bul)
    kap = kchi / (np.sqrt(np.pi) * nu * vw / CL)
    S = pops[:, 1] * sp.line_A[0] / (pops[:, 0] * Blu - pops[:, 1] * Bul)
    x = mdl.pos[:, 0]
    s = mdl.vel[:, 0] - mdl.vel[O, 0]
    a, b = vw[O] / vw, s / vw
    qx = np.asarray(xq)
    I_in = planck(nu, 2.725)

    def jnode(k, y):
        return np.interp(y, qx, Jnu[k, 0])

    def rates(zz, sign):
        k = min(int(np.searchsorted(x, zz, side="right")) - 1, len(x) - 2)
        t = (zz - x[k]) / (x[k + 1] - x[k])
        aa, bb = a[k] + t * (a[k + 1] - a[k]), b[k] + t * (b[k + 1] - b[k])
        y = aa * qx - sign * bb
        cl = (kap[k] + t * (kap[k + 1] - kap[k])) * np.exp(-y * y)
        cs = chi_sca[k, 0] + t * (chi_sca[k + 1, 0] - chi_sca[k, 0])
        if chim_x is not None:
            cs = cs + sign * (chim_x[k] + t * (chim_x[k + 1] - chim_x[k]))
        jj = (1 - t) * jnode(k, y) + t * jnode(k + 1, y)
        Sl = S[k] + t * (S[k + 1] - S[k])
        tot = cl + cs
        return tot, (cl * Sl + cs * jj) / tot

    def integrate(z0, z1, sign):
        I = np.full(qx.shape, I_in)
        nodes = x[(x >= min(z0, z1)) & (x <= max(z0, z1))]
        nodes = nodes if z1 > z0 else nodes[::-1]
        for za, zb in zip(nodes[:-1], nodes[1:]):
            h = (zb - za) / steps
            for j in range(steps):
                zz = za + j * h
                f = lambda zq, II: (lambda ts: ts[0] * (ts[1] - II))(rates(zq, sign))
                k1 = f(zz, I)
                k2 = f(zz + h / 2, I + abs(h) / 2 * k1)
                k3 = f(zz + h / 2, I + abs(h) / 2 * k2)
                k4 = f(zz + h, I + abs(h) * k3)
                I = I + abs(h) / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
        return I

    Ip = integrate(x[0], x[O], +1.0)
    Im = integrate(x[-1], x[O], -1.0)
    e = 0.0 if chim_x is None else chim_x[O] / chi_sca[O, 0]
    return 0.5 * ((1 + e) * Ip + (1 - e) * Im)


def test_scattering_in_a_moving_medium_brute_force(oracle_lib):
    """A steep Hubble flow with scattering and a previous J_nu that is not symmetric in
    frequency, so Psi^- does not vanish: the oracle's J_nu converges to the brute-force
    integration of both directions at second order as the velocity sub-steps refine."""
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
    sel = [5, 12, 18]
    exact = np.array([_moving_chain_exact(o0, mdl, pops, chi_sca, Jnu, O, xq) for O in sel])
    errs = []
    for f in (0.2, 0.1, 0.05):
        o = make(oracle_lib, mdl, sp, q=q, f_sub=f)
        _, _, _, Jn = o.formal_solve_scat(pops, chi_sca, Jnu, sel=sel)
        errs.append(rel(Jn[:, 0, :], exact).max())
    ratios = np.array(errs[:-1]) / np.array(errs[1:])
    assert np.all(ratios > 3.5), (errs, ratios)
    assert errs[-1] < 2e-6, errs


# ---------------------------------------------------------------- closed form of the scattering fixed point


def _eps_chain(n):
    # line-centre optical thickness about 1.9 over the chain (abundance 4e-7)
    sp = species.two_level(100e9, 3.0, 1e-5, 1e-10, 28.0)
    x = np.linspace(0.0, 1.0, n) * 1e16
    mdl = chain_1d(x, np.zeros(n), 1e4, 25.0, 1.5e4, 4e-7)
    return sp, mdl


def test_scattering_fixed_point_two_stream_closed_form(oracle_lib):
    """Homogeneous static chain, one ray pair, one frequency at line centre, fixed line
    source S and thermalisation eps = chi_line/chi_tot: the scattering iteration's limit
    solves u'' = eps (u - S) with u - u' = I at both faces, whose solution is
    u = S + (I - S) cosh(k (tau - T/2)) / (cosh(kT/2) + k sinh(kT/2)), k = sqrt(eps).
    The discrete fixed point must approach it at second order in the node spacing."""
    eps = 0.3
    errs = []
    for n in (21, 41, 81):
        sp, mdl = _eps_chain(n)
        o = make(oracle_lib, mdl, sp, q=(np.array([0.0]), np.array([1.0])))
        pops = o.lte()
        nu = o.line_frequencies()[0]
        vw = o.line_width_speed()
        Bul = sp.line_A[0] * CL ** 2 / (2 * H * nu ** 3)
        kchi = H * nu / (4 * np.pi) * (pops[:, 0] * 3 * Bul - pops[:, 1] * Bul)
        kap = kchi / (np.sqrt(np.pi) * nu * vw / CL)
        S = pops[0, 1] * sp.line_A[0] / (pops[0, 0] * 3 * Bul - pops[0, 1] * Bul)
        chi_sca = (kap * (1 - eps) / eps)[:, None]
        # scale the optical thickness: T = chi_tot * length
        length = mdl.pos[-1, 0] - mdl.pos[0, 0]
        T = kap[0] / eps * length
        Jnu = o.scattering_start()
        for _ in range(400):
            J, _, _, new = o.formal_solve_scat(pops, chi_sca, Jnu)
            done = np.abs(new - Jnu).max() <= 1e-15 * np.abs(new).max()
            Jnu = new
            if done:
                break
        assert done
        I = planck(nu, 2.725)
        k = np.sqrt(eps)
        tau = kap[0] / eps * (mdl.pos[:, 0] - mdl.pos[0, 0])
        exact = S + (I - S) * np.cosh(k * (tau - T / 2)) / (np.cosh(k * T / 2) + k * np.sinh(k * T / 2))
        # with a single pair and one frequency, J_nu and J are u at every point
        assert rel(J[:, 0], Jnu[:, 0, 0]).max() < 1e-13
        errs.append(np.abs(Jnu[:, 0, 0] - exact).max() / abs(I - S))
    slopes = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(slopes - 2) < 0.25), (errs, slopes)
    assert errs[-1] < 1e-3 and 0.5 < T < 50


def test_alo_does_not_change_the_fixed_point_with_scattering(oracle_lib):
    """Eq. ALO with the scattering opacity in the denominator: at convergence the ALO
    terms cancel, so the ALI with L* and without it reach the same populations.  A warm,
    dense outflow, where trapping of line photons by the scattering matters."""
    w = configs.outflow5(n_points=100, seed=3, nside=1)
    with_alo = oracle_lib.from_workload(w)
    without = oracle_lib.from_workload(w, use_alo=False)
    pops = with_alo.lte()
    nd = with_alo.pair_nodes(pops, 0, 0)
    chi_sca = np.median(nd["kappa"][:, 0]) * np.linspace(0.2, 2.0, w.n_points)[:, None] * np.ones((1, 4))
    a, ca, _ = with_alo.run_ali_scat(chi_sca, max_iter=200, tol=1e-10)
    b, cb, _ = without.run_ali_scat(chi_sca, max_iter=200, tol=1e-10)
    assert ca[-1] < 1e-10 and cb[-1] < 1e-10
    assert rel(a, b).max() < 1e-8
    # the scattering changes the populations (it is not a no-op)
    plain, _ = with_alo.run_ali(max_iter=200, tol=1e-10)
    assert rel(a, plain).max() > 1e-4
