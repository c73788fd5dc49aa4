"""Pins of the CPU oracle to what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: a closed form, an
invariant, a special case that reduces to a library routine, a brute-force integration,
or a number the paper prints.  None of them calls the HIP library.
"""
import math
import os

import numpy as np
import pytest
from scipy.special import erf

from synth import directions, species
from synth.models import Model, chain_1d, lattice_3d, power_law_sphere

HERE = os.path.dirname(os.path.abspath(__file__))
H = 6.62607015e-27
KB = 1.380649e-16
CL = 2.99792458e10
AMU = 1.66053906660e-24


def rel(a, b):
    """The paper's relative difference 2|a-b|/(|a|+|b|), zero where both vanish."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.abs(a) + np.abs(b)
    return np.where(den > 0, 2 * np.abs(a - b) / np.where(den > 0, den, 1), 0.0)


def planck(nu, T):
    return 2 * H * nu ** 3 / CL ** 2 / np.expm1(H * nu / (KB * T))


def make(oracle_lib, model, sp, rays=None, q=None, **kw):
    if rays is None:
        rays = directions.axis_pair()
    if q is None:
        q = directions.uniform_grid(31, 4.0)
    return oracle_lib.Oracle(model, sp, rays, q[0], q[1], **kw)


# ---------------------------------------------------------------- inputs


def test_healpix_pins():
    for nside in (1, 2, 4):
        d = directions.healpix_ring(nside)
        assert d.shape == (12 * nside * nside, 3)
        assert np.abs(np.linalg.norm(d, axis=1) - 1).max() < 1e-15
        assert np.abs(d.sum(axis=0)).max() < 1e-13
        # every direction has an antipode in the set
        s = np.abs(d[:, None, :] + d[None, :, :]).sum(-1)
        assert (s.min(axis=1) < 1e-14).all()
    z1 = np.sort(directions.healpix_ring(1)[:, 2])
    assert np.allclose(z1, np.repeat([-2 / 3, 0, 2 / 3], 4), atol=1e-15)


def test_quadrature_pins():
    # Gauss-Hermite weights as written in Sec. 3.1.2: w_n = 2^(N-1) N! / (N H_{N-1}(x_n))^2.
    # That expression already carries the 1/sqrt(pi) of the normalised profile, so the
    # weights sum to one.
    for N in (5, 24, 31):
        x, w = directions.gauss_hermite(N)
        HN = np.polynomial.hermite.hermval(x, [0] * N + [1])
        assert np.abs(HN).max() < 1e-6 * math.factorial(N) ** 0.5 * 2 ** N  # roots of H_N
        Hm = np.polynomial.hermite.hermval(x, [0] * (N - 1) + [1])
        wp = 2.0 ** (N - 1) * math.factorial(N) / (N * Hm) ** 2
        assert np.abs(w / wp - 1).max() < 1e-10
        assert abs(w.sum() - 1) < 1e-14
        assert abs((w * x * x).sum() - 0.5) < 1e-13   # second moment of the Gaussian
        assert np.array_equal(x, -x[::-1]) and np.array_equal(w, w[::-1])
    x, w = directions.uniform_grid(31, 4.0)
    assert abs(w.sum() - 1) < 1e-15 and x[0] == -4.0 and x[-1] == 4.0
    assert np.array_equal(x, -x[::-1])


# ---------------------------------------------------------------- setup


def test_line_widths_printed_in_paper(oracle_lib):
    rows = np.loadtxt(os.path.join(HERE, "golden", "paper_line_widths.txt"), usecols=range(5))
    for nu, T, vt, m_amu, dnu_paper in rows:
        sp = species.two_level(nu=nu, mass_amu=m_amu)
        mdl = chain_1d(np.array([0.0, 1.0]), np.zeros(2), 1e4, T, vt, 1e-8)
        o = make(oracle_lib, mdl, sp)
        dnu = nu * o.line_width_speed()[0] / CL
        # the paper prints 5 significant digits
        assert abs(dnu - dnu_paper) / dnu_paper < 1e-5, (dnu, dnu_paper)


def test_table1_species_fixture():
    E, gr, A, K = np.loadtxt(os.path.join(HERE, "golden", "table1_species.txt"))
    sp = species.table1_species()
    assert abs((sp.energy[1] - sp.energy[0]) / (H * CL) - E) < 1e-12
    assert sp.weight[1] / sp.weight[0] == gr and sp.line_A[0] == A
    assert np.all(sp.coll_K == K)


# ---------------------------------------------------------------- Feautrier solve


def dense_system(z, chi, S, I_lo, I_hi, tau_floor=1e-100):
    """Dense matrix of the discretised second-order equation: centred second
    differences inside, second-order (Taylor) boundary rows at both ends."""
    N = len(z)
    dt = np.maximum(0.5 * (chi[:-1] + chi[1:]) * np.diff(z), tau_floor)
    T = np.zeros((N, N))
    R = np.array(S, dtype=np.float64).copy()
    for i in range(1, N - 1):
        a = 2 / (dt[i - 1] * (dt[i - 1] + dt[i]))
        c = 2 / (dt[i] * (dt[i - 1] + dt[i]))
        T[i, i - 1], T[i, i], T[i, i + 1] = -a, 1 + a + c, -c
    T[0, 0], T[0, 1] = 1 + 2 / dt[0] + 2 / dt[0] ** 2, -2 / dt[0] ** 2
    R[0] += 2 / dt[0] * I_lo
    T[-1, -1], T[-1, -2] = 1 + 2 / dt[-1] + 2 / dt[-1] ** 2, -2 / dt[-1] ** 2
    R[-1] += 2 / dt[-1] * I_hi
    return T, R


@pytest.mark.parametrize("seed", range(6))
def test_solver_matches_dense_linear_algebra(oracle_lib, seed):
    rng = np.random.default_rng(seed)
    N = int(rng.integers(2, 40))
    z = np.cumsum(rng.uniform(0.1, 1.0, N))
    # optical-depth steps from 1e-4 to 1e4
    chi = 10.0 ** rng.uniform(-4, 4, N)
    S = rng.uniform(0.1, 2.0, N)
    I_lo, I_hi = rng.uniform(0, 1, 2)
    o = int(rng.integers(0, N))
    u, lam, ue, ua = oracle_lib.solve_ray(z, chi, S, I_lo, I_hi, o, want_all=True)
    T, R = dense_system(z, chi, S, I_lo, I_hi)
    ud = np.linalg.solve(T, R)
    Ti = np.linalg.inv(T)
    assert np.abs(rel(ua, ud)).max() < 1e-11
    assert rel(lam, Ti[o, o]) < 1e-11
    ue_d = ud[o] - Ti[o, o] * S[o]
    assert rel(ue, ue_d) < 1e-8 * max(1.0, ud[o] / max(ue_d, 1e-300))
    # invariants: 0 <= Lambda_oo <= 1, ueff >= 0
    assert 0 <= lam <= 1 and ue >= 0


def test_solver_single_node():
    import oracle
    u, lam, ue = oracle.solve_ray([0.0], [1.0], [3.0], 1.0, 2.0, 0)
    assert u == 1.5 and lam == 0.0 and ue == 1.5


def slab_exact(S, I, tau_l, tau_r):
    return S + 0.5 * (I - S) * (np.exp(-tau_l) + np.exp(-tau_r))


def test_homogeneous_slab_second_order(oracle_lib):
    """Constant chi and S: I = S(1 - e^-tau) + I_bdy e^-tau from each side, so
    u_o = S + (I - S)(e^-tau_l + e^-tau_r)/2 (Sec. 4.1.1, constant-source form).
    The discretisation error must fall as the square of the step."""
    S, I, chi = 1.0, 0.2, 1.0
    errs = []
    for n in (24, 48, 96, 192):
        z = np.linspace(0.0, 3.0, n + 1)
        o = n // 3     # z_o = 1 at every resolution
        u, lam, ue = oracle_lib.solve_ray(z, np.full(n + 1, chi), np.full(n + 1, S), I, I, o)
        errs.append(abs(u - slab_exact(S, I, chi * z[o], chi * (3.0 - z[o]))))
    slopes = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(slopes - 2) < 0.15), slopes
    assert errs[-1] < 1e-5
    # I_bdy = S is reproduced exactly at any resolution
    z = np.linspace(0, 1, 7)
    u, _, _ = oracle_lib.solve_ray(z, np.full(7, 5.0), np.full(7, 0.7), 0.7, 0.7, 3)
    assert abs(u - 0.7) < 1e-15


def rk4_intensity(zn, chin, Sn, I0, z_end, steps_per_seg=400):
    """Integrate dI/ds = chi (S - I) along the photon path from zn[0] to z_end (zn
    monotone, increasing or decreasing), chi and S piecewise linear between nodes."""
    f_chi = lambda zz: np.interp(zz, zn, chin) if zn[0] < zn[-1] else np.interp(zz, zn[::-1], chin[::-1])
    f_S = lambda zz: np.interp(zz, zn, Sn) if zn[0] < zn[-1] else np.interp(zz, zn[::-1], Sn[::-1])
    grid = []
    for k in range(len(zn) - 1):
        a, b = zn[k], zn[k + 1]
        if (b - z_end) * (a - z_end) < 0 or b == z_end:
            b = z_end
        grid.append(np.linspace(a, b, steps_per_seg + 1)[:-1])
        if b == z_end:
            break
    grid = np.concatenate(grid + [[z_end]])
    I = I0
    rhs = lambda zz, II: f_chi(zz) * (f_S(zz) - II)
    for k in range(len(grid) - 1):
        h = grid[k + 1] - grid[k]        # signed step in z
        ds = abs(h)                       # path length along the photon direction
        zz = grid[k]
        k1 = rhs(zz, I)
        k2 = rhs(zz + h / 2, I + ds / 2 * k1)
        k3 = rhs(zz + h / 2, I + ds / 2 * k2)
        k4 = rhs(zz + h, I + ds * k3)
        I = I + ds / 6 * (k1 + 2 * k2 + 2 * k3 + k4)
    return I


@pytest.mark.parametrize("seed", range(3))
def test_brute_force_first_order_integration(oracle_lib, seed):
    """Tiny rays: integrate the first-order equation each way and compare u_o with the
    Feautrier solution on m-fold refined nodes (second order in 1/m)."""
    rng = np.random.default_rng(100 + seed)
    N = int(rng.integers(3, 8))
    z = np.cumsum(rng.uniform(0.2, 1.0, N))
    chi = rng.uniform(0.3, 3.0, N)
    S = rng.uniform(0.5, 2.0, N)
    I_lo, I_hi = 0.1, 0.3
    o = int(rng.integers(0, N))
    Ip = rk4_intensity(z, chi, S, I_lo, z[o]) if o > 0 else I_lo
    Im = rk4_intensity(z[::-1], chi[::-1], S[::-1], I_hi, z[o]) if o < N - 1 else I_hi
    u_ref = 0.5 * (Ip + Im)
    errs = []
    for m in (8, 16, 32, 64):
        zf = np.concatenate([np.linspace(z[k], z[k + 1], m + 1)[:-1] for k in range(N - 1)] + [[z[-1]]])
        cf, sf = np.interp(zf, z, chi), np.interp(zf, z, S)
        u, _, _ = oracle_lib.solve_ray(zf, cf, sf, I_lo, I_hi, o * m)
        errs.append(abs(u - u_ref))
    slopes = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(np.abs(slopes - 2) < 0.3), (errs, slopes)
    assert errs[-1] / u_ref < 1e-4


# ---------------------------------------------------------------- walk


def test_walk_chain_and_lattice(oracle_lib):
    sp = species.two_level()
    x = np.sort(np.random.default_rng(0).uniform(-1, 1, 40))
    o = make(oracle_lib, chain_1d(x, np.zeros(40), 1e4, 20, 1.5e4, 1e-8), sp)
    for O in (0, 17, 39):
        c, Z = o.walk(O, 0)   # +x
        assert list(c) == list(range(O + 1, 40))
        c, Z = o.walk(O, 1)   # -x
        assert list(c) == list(range(O - 1, -1, -1))
    m = 5
    lat = lattice_3d(m, 1.0)
    rays = np.array([[1.0, 0, 0], [-1.0, 0, 0], [0, 1.0, 0], [0, -1.0, 0], [0, 0, 1.0], [0, 0, -1.0]])
    o = make(oracle_lib, lat, sp, rays=rays)
    lin = lambda i, j, k: (i * m + j) * m + k
    c, _ = o.walk(lin(1, 2, 3), 0)
    assert list(c) == [lin(2, 2, 3), lin(3, 2, 3), lin(4, 2, 3)]
    c, _ = o.walk(lin(1, 2, 3), 5)
    assert list(c) == [lin(1, 2, 2), lin(1, 2, 1), lin(1, 2, 0)]


def test_walk_invariants_random_cloud(oracle_lib):
    """On a k-NN cloud every step must go to the neighbour of the current cell that lies
    farther along the ray and closest to it, and the walk must stop only when no such
    neighbour exists (Sec. 3.2)."""
    mdl = power_law_sphere(7, 600, 1.0, 0.01, 1.0, 0.0, 20.0, 0.0, 0.0, 1e-8)
    d = directions.healpix_ring(2)
    o = make(oracle_lib, mdl, species.two_level(), rays=d)
    pos = mdl.pos
    rng = np.random.default_rng(1)
    for O in rng.integers(0, 600, 25):
        for r in range(0, 48, 5):
            n = d[r]
            cells, Z = o.walk(O, r)
            cur, zc = O, 0.0
            for cell, z in zip(cells, Z):
                nb = mdl.nbr[cur][mdl.nbr[cur] >= 0]
                dd = pos[nb] - pos[O]
                zz = dd @ n
                ok = zz > zc
                assert ok.any()
                q = ((dd - np.outer(zz, n)) ** 2).sum(1)
                qmin = q[ok].min()
                assert cell in nb[ok] and abs(q[nb == cell][0] - qmin) <= 1e-12 * max(qmin, 1e-30)
                assert z > zc
                cur, zc = cell, z
            nb = mdl.nbr[cur][mdl.nbr[cur] >= 0]
            assert not ((pos[nb] - pos[O]) @ n > zc + 1e-15 * (1 + abs(zc))).any()


# ---------------------------------------------------------------- thermal equilibrium


@pytest.mark.parametrize("moving", [False, True])
def test_thermal_equilibrium_exact(oracle_lib, moving):
    """T_gas = T_boundary = const: u = B is the exact discrete solution of every ray
    pair (interior and boundary rows), so J = B(nu, T) and Boltzmann populations are a
    fixed point of the iteration, for any density and velocity field."""
    T = 20.0
    mdl = power_law_sphere(3, 300, 1e17, 1e15, 1e6, -2.0, T, 0.0, 0.0, 1e-6)
    if moving:
        rng = np.random.default_rng(5)
        mdl.vel = rng.normal(0, 3e5, mdl.vel.shape)   # forces sub-steps
    sp = species.linear_rotor(4)
    o = make(oracle_lib, mdl, sp, rays=directions.healpix_ring(1), t_cmb=T)
    lte = o.lte()
    J, Je, L = o.formal_solve(lte)
    nu = (sp.energy[sp.line_up] - sp.energy[sp.line_lo]) / H
    assert np.abs(rel(J, planck(nu, T)[None, :])).max() < 1e-13
    assert np.abs(rel(Je, J * (1 - L))).max() < 1e-9
    pops, ch = o.run_ali(lte, max_iter=3, tol=0.0)
    assert np.abs(rel(pops, lte)).max() < 1e-12


def test_lte_limit_high_density(oracle_lib):
    sp = species.table1_species()
    mdl = chain_1d(np.linspace(-1e15, 1e15, 9), np.zeros(9), 1e16, 30.0, 1.5e4, 1e-10)
    o = make(oracle_lib, mdl, sp)
    lte = o.lte()
    J, Je, L = o.formal_solve(lte)
    pops, flags = o.stateq(lte, J, Je, L)
    # departure from LTE is of order A / (K n_H2) = 1e-4 / (2e-10 * 1e16) = 5e-11
    assert np.abs(rel(pops, lte)).max() < 1e-9
    assert flags.sum() == 0


def test_two_level_closed_form(oracle_lib):
    """Two levels: n_u/n_l = (C_lu + B_lu Jeff) / (A (1 - L) + B_ul Jeff + C_ul)."""
    sp = species.two_level(nu=230e9, A=3e-6)
    mdl = chain_1d(np.linspace(0, 1e16, 5), np.zeros(5), np.geomspace(1e2, 1e6, 5), np.linspace(10, 80, 5),
                   1.5e4, 1e-6)
    o = make(oracle_lib, mdl, sp)
    rng = np.random.default_rng(2)
    J = rng.uniform(0.5, 2.0, (5, 1)) * planck(230e9, 20.0)
    L = rng.uniform(0.0, 0.9, (5, 1))
    Je = J * rng.uniform(0.1, 1.0, (5, 1))
    pops, flags = o.stateq(o.lte(), J, Je, L)
    A = 3e-6
    Bul = A * CL ** 2 / (2 * H * 230e9 ** 3)
    Blu = 3 * Bul
    for p in range(5):
        Cul, Clu = o.coll_rates(p)
        ratio = (Clu[0] + Blu * Je[p, 0]) / (A * (1 - L[p, 0]) + Bul * Je[p, 0] + Cul[0])
        assert rel(pops[p, 1] / pops[p, 0], ratio) < 1e-13
        assert rel(pops[p].sum(), 1e-6 * mdl.n_h2[p]) < 1e-14


def test_collision_excitation_gives_boltzmann(oracle_lib):
    """With no radiation (A = 0 only through collisions dominating) the collisional
    rates alone must give Boltzmann ratios at the gas temperature."""
    sp = species.linear_rotor(5)
    sp.line_A[:] = 0.0
    mdl = chain_1d(np.linspace(0, 1, 4), np.zeros(4), 1e5, np.array([5.0, 20.0, 60.0, 150.0]), 1.5e4, 1e-6)
    o = make(oracle_lib, mdl, sp)
    z = np.zeros((4, sp.n_lines))
    pops, flags = o.stateq(o.lte(), z, z, z)
    assert np.abs(rel(pops, o.lte())).max() < 1e-12


def test_population_sum_every_iteration(oracle_lib):
    from synth import configs
    w = configs.sphere2(n_points=200)
    o = oracle_lib.from_workload(w)
    p = o.lte()
    ntot = w.model.n_h2 * w.model.abundance
    for _ in range(3):
        J, Je, L = o.formal_solve(p)
        assert (Je >= 0).all() and (L >= 0).all() and (L <= 1).all()
        p, flags = o.stateq(p, J, Je, L)
        assert np.abs(p.sum(1) / ntot - 1).max() < 1e-14


# ---------------------------------------------------------------- Hubble-Lemaitre model (Sec. 4.1.1)


def hubble_1d(n_cells=100, dx=10e5, dbeta_c=0.01):
    # density scaled with the gradient so that the line optical depth stays the same
    sp = species.table1_species()
    x = (np.arange(n_cells) - (n_cells - 1) / 2) * dx
    mdl = chain_1d(x, dbeta_c * x, 1e6 * dbeta_c / 0.01, 45.0, 0.0, 1e-4)
    return sp, mdl


def hubble_exact_u(o, sp, mdl, pops, qx, Rb):
    """Per-node, per-frequency u in the pair frame, from the erf optical depth:
    tau(x, l) = k_chi / (2 nu Dbeta) [erf(x + c Dbeta l / v_w) - erf(x)]."""
    nu = (sp.energy[1] - sp.energy[0]) / H
    n = pops[0]
    Bul = sp.line_A[0] * CL ** 2 / (2 * H * nu ** 3)
    Blu = 3 * Bul
    kchi = H * nu / (4 * np.pi) * (n[0] * Blu - n[1] * Bul)
    S = n[1] * sp.line_A[0] / (n[0] * Blu - n[1] * Bul)
    vw = o.line_width_speed()[0]
    return nu, kchi, S, vw


def hubble_errors(oracle_lib, dbeta_c, f_sub):
    """Relative error of every (node, frequency) u against the closed form of
    Sec. 4.1.1 (Eq. Hubble-Lemaitre1D with the erf optical depth), LTE populations."""
    sp, mdl = hubble_1d(dbeta_c=dbeta_c)
    q = directions.gauss_hermite(100)
    o = make(oracle_lib, mdl, sp, q=q, f_sub=f_sub)
    pops = o.lte()
    nu, kchi, S, vw = hubble_exact_u(o, sp, mdl, pops, q[0], None)
    Dbeta = dbeta_c / CL
    I = planck(nu, 2.725)
    xpos = mdl.pos[:, 0]
    R = xpos[-1]
    tau = lambda x, l: kchi / (2 * nu * Dbeta) * (erf(x + CL * Dbeta * l / vw) - erf(x))
    errs = []
    for O in range(0, 100, 3):
        lb, la = xpos[O] + R, R - xpos[O]      # distances behind / ahead along +x
        exact = S + 0.5 * (I - S) * (np.exp(-tau(q[0], lb)) + np.exp(-tau(-q[0], la)))
        nd = o.pair_nodes(pops, O, 0)
        for n, xq in enumerate(q[0]):
            chi = nd["kappa"][:, 0] * np.exp(-(nd["a"] * xq - nd["b"]) ** 2)
            u, _, _ = oracle_lib.solve_ray(nd["z"], chi, nd["S"][:, 0], I, I, nd["o"])
            errs.append(rel(u, exact[n]))
    return np.array(errs)


def test_hubble_lemaitre_1d(oracle_lib):
    """At the paper's gradient (c Dbeta = 0.01 s^-1, 100 cells of 10 km) the relative
    error is below 1e-4 almost everywhere (Sec. 4.1.1)."""
    errs = hubble_errors(oracle_lib, 0.01, 0.25)
    assert np.quantile(errs, 0.95) < 1e-4 and np.median(errs) < 1e-5


def test_hubble_lemaitre_velocity_substeps(oracle_lib):
    """A 50x steeper gradient shifts the line by several widths per cell.  Without
    sub-steps the profile is undersampled; with them (Sec. 3.2) the error stays small
    and falls as the allowed velocity step shrinks."""
    e_none = np.quantile(hubble_errors(oracle_lib, 0.5, 1e9), 0.95)
    e_25 = np.quantile(hubble_errors(oracle_lib, 0.5, 0.25), 0.95)
    e_05 = np.quantile(hubble_errors(oracle_lib, 0.5, 0.05), 0.95)
    assert e_25 < 1e-4 and e_05 < e_25 and e_none > 100 * e_25, (e_none, e_25, e_05)


def test_hubble_lemaitre_line_integrated_J(oracle_lib):
    """formal_solve's J must equal the quadrature sum of the closed-form J_nu of
    Eq. (Hubble-Lemaitre1D): the pair frame and the sum over rays agree for a
    symmetric quadrature."""
    sp, mdl = hubble_1d()
    q = directions.gauss_hermite(100)
    o = make(oracle_lib, mdl, sp, q=q)
    pops = o.lte()
    nu, kchi, S, vw = hubble_exact_u(o, sp, mdl, pops, q[0], None)
    Dbeta = 0.01 / CL
    I = planck(nu, 2.725)
    xpos = mdl.pos[:, 0]
    R = xpos[-1]
    J, Je, L = o.formal_solve(pops)
    tau = lambda x, l: kchi / (2 * nu * Dbeta) * (erf(x + CL * Dbeta * l / vw) - erf(x))
    Jx = np.array([(q[1] * (S + 0.5 * (I - S) * (np.exp(-tau(q[0], xpos[O] + R)) +
                                                  np.exp(-tau(q[0], R - xpos[O]))))).sum()
                   for O in range(100)])
    assert np.median(rel(J[:, 0], Jx)) < 1e-5 and rel(J[:, 0], Jx).max() < 1e-3


# ---------------------------------------------------------------- ALI fixed point


@pytest.mark.slow
def test_alo_does_not_change_fixed_point(oracle_lib):
    """The ALO terms cancel at convergence (Eq. ourALI with N = N_dagger): the ALI and
    plain Lambda iteration converge to the same populations."""
    from synth import configs
    w = configs.sphere2(n_points=300)
    w.model.abundance[:] = 1e-7       # moderate optical depth
    a = oracle_lib.from_workload(w, use_alo=True)
    b = oracle_lib.from_workload(w, use_alo=False)
    pa, cha = a.run_ali(max_iter=200, tol=1e-12)
    pb, chb = b.run_ali(max_iter=400, tol=1e-12)
    assert cha[-1] < 1e-12 and chb[-1] < 1e-12
    assert np.abs(rel(pa, pb)).max() < 1e-9
    assert len(cha) <= len(chb)


# ---------------------------------------------------------------- Morton order

def test_morton_order_reference():
    import oracle
    from synth.models import lattice_3d
    # 2x2x2 lattice: one bit per axis, x most significant, so index order (i, j, k)
    m = lattice_3d(2, 1e15)
    assert np.array_equal(oracle.morton_order(m.pos), np.arange(8))
    # brute force on random points: codes from the definition with Python integers
    rng = np.random.default_rng(0)
    pos = rng.uniform(-1, 1, (300, 3))
    pos[:5] = pos[5]                        # equal codes keep index order
    order = oracle.morton_order(pos)
    lo, hi = pos.min(0), pos.max(0)

    def code(p):
        q = [int(np.floor((p[d] - lo[d]) / (hi[d] - lo[d]) * 2097151.0)) for d in range(3)]
        c = 0
        for b in range(21):
            for d in range(3):
                c |= ((q[d] >> b) & 1) << (3 * b + 2 - d)
        return c

    keys = [(code(pos[i]), i) for i in range(300)]
    assert np.array_equal(order, [i for _, i in sorted(keys)])
    # models are ordered separately
    offs = [0, 100, 300]
    o2 = oracle.morton_order(pos, offs)
    assert np.array_equal(np.sort(o2[:100]), np.arange(100)) and np.array_equal(o2[:100], oracle.morton_order(pos[:100]))
