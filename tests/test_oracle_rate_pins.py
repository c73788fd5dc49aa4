"""Pins of the oracle's rate and convergence arithmetic (no GPU).

* Collision rates (Sec. 2.2.1): C_ul = K_ul(T) n_H2 with K read off a table linearly in
  T and clamped at its ends, checked against numpy's piecewise-linear interpolation (a
  library routine with the same clamping) and, at the table's own temperatures, against
  the sqrt law the synthetic tables are built from; excitation by detailed balance.
* The relative-change measure the ALI stops on (undefined in the paper; the reading is
  max over levels with n_i / n_tot > 1e-10 of |n_new - n_old| / n_new, and its mean), on
  hand-built arrays whose answer is written out.
* The validity fallback of Sec. 6.1: a point whose ALO solution is not positive is
  solved again as a plain Lambda iteration (L* = 0, Jeff = J), checked against the
  two-level closed form of that system; a point where both fail keeps its old
  populations.
"""
import numpy as np

from synth import directions, species
from synth.models import chain_1d

H = 6.62607015e-27
KB = 1.380649e-16
CL = 2.99792458e10


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    den = np.abs(a) + np.abs(b)
    return np.where(den > 0, 2 * np.abs(a - b) / np.where(den > 0, den, 1), 0.0)


def make(oracle_lib, mdl, sp, **kw):
    q = directions.uniform_grid(31, 4.0)
    return oracle_lib.Oracle(mdl, sp, directions.axis_pair(), q[0], q[1], **kw)


# ---------------------------------------------------------------- collision rates


def rotor_with_table(seed=11):
    """A 4-level rotor whose six collision pairs each get their own table: the sqrt law
    times a pair factor, then (second species) values drawn at random per temperature,
    so a wrong bracket, a wrong row or a missing clamp changes the result."""
    sp = species.linear_rotor(4)
    f = 1.0 + np.arange(sp.coll_up.shape[0])[:, None]
    sp.coll_K = sp.coll_K * f
    rnd = species.linear_rotor(4)
    rng = np.random.default_rng(seed)
    rnd.coll_K = rng.uniform(1e-12, 1e-9, rnd.coll_K.shape)
    return sp, rnd


def temperatures(Tt):
    """Table temperatures, midpoints, random interior values and values beyond both ends."""
    rng = np.random.default_rng(3)
    mids = 0.5 * (Tt[:-1] + Tt[1:])
    inner = rng.uniform(Tt[0], Tt[-1], 20)
    return np.concatenate([Tt[::5], mids[::6], inner, [0.2, 0.9 * Tt[0], 1.5 * Tt[-1], 2e4]])


def test_collision_rates_table_lookup(oracle_lib):
    for sp in rotor_with_table():
        Tt = sp.coll_T
        T = temperatures(Tt)
        n = T.shape[0]
        nh2 = np.geomspace(1e2, 1e8, n)
        X = 1e-6      # C must scale with n_H2, not with the species density X n_H2
        mdl = chain_1d(np.linspace(0, 1e16, n), np.zeros(n), nh2, T, 1.5e4, X)
        o = make(oracle_lib, mdl, sp)
        for p in range(n):
            Cul, Clu = o.coll_rates(p)
            for c in range(sp.coll_up.shape[0]):
                K = np.interp(T[p], Tt, sp.coll_K[c])     # linear in T, clamped at both ends
                assert rel(Cul[c], K * nh2[p]) < 1e-14, (p, c)
                u, lo = sp.coll_up[c], sp.coll_lo[c]
                db = sp.weight[u] / sp.weight[lo] * np.exp(-(sp.energy[u] - sp.energy[lo]) / (KB * T[p]))
                assert rel(Clu[c], Cul[c] * db) < 1e-14, (p, c)


def test_collision_rates_at_table_temperatures_follow_the_sqrt_law(oracle_lib):
    """At the table's own temperatures the lookup returns the tabulated sqrt law exactly:
    C_ul = K0 sqrt(T / 20 K) n_H2 (K0 = 1e-10 cm^3 s^-1 for every rotor pair)."""
    sp = species.linear_rotor(3)
    T = sp.coll_T[[0, 7, 19, 30, 47]]
    nh2 = np.array([1e3, 1e4, 1e5, 1e6, 1e7])
    mdl = chain_1d(np.linspace(0, 1e16, 5), np.zeros(5), nh2, T, 1.5e4, 1e-6)
    o = make(oracle_lib, mdl, sp)
    for p in range(5):
        Cul, _ = o.coll_rates(p)
        assert np.abs(rel(Cul, 1e-10 * np.sqrt(T[p] / 20.0) * nh2[p])).max() < 1e-15


# ---------------------------------------------------------------- relative change


def test_rel_change_on_hand_built_arrays(oracle_lib):
    sp = species.linear_rotor(3)
    nh2 = np.array([1e4, 2e4, 5e3])
    X = 1e-6
    ntot = X * nh2                                   # 1e-2, 2e-2, 5e-3
    mdl = chain_1d(np.array([0.0, 1e15, 2e15]), np.zeros(3), nh2, 20.0, 1.5e4, X)
    o = make(oracle_lib, mdl, sp)
    new = np.array([[5e-3, 4e-3, 1e-3],
                    [1.5e-2, 2e-10 * 2e-2, 0.5e-10 * 2e-2],    # tiny level kept, tinier one masked
                    [2.5e-3, 0.0, np.nan]])                      # zero and NaN are masked
    old = np.array([[4e-3, 4e-3, 2e-3],
                    [1.2e-2, 8e-10 * 2e-2, 50e-10 * 2e-2],
                    [5e-3, 1.0, 1.0]])
    mx, mean = o.rel_change(old, new)
    # included entries and their changes |new - old| / new
    inc = [0.2, 0.0, 1.0,            # point 0
           0.2, 3.0,                 # point 1 (the 0.5e-10 level would give 99)
           1.0]                      # point 2
    assert mx == 3.0
    assert abs(mean - sum(inc) / len(inc)) < 1e-15
    # the denominator is the new value: the same arrays swapped give other numbers
    mx2, _ = o.rel_change(new, old)
    assert mx2 != mx
    # every level at or below the mask: no entry, change 0 and mean 0
    z = np.full((3, 3), 1e-12 * 1e-3)
    assert o.rel_change(z * 2, z) == (0.0, 0.0)
    assert ntot.min() > 0


# ---------------------------------------------------------------- validity fallback


def two_level_model(oracle_lib, use_alo=True):
    sp = species.two_level(nu=230e9, A=3e-6)
    nh2 = np.array([1e1, 3e1, 1e2, 3e2])            # C_ul << A: radiation decides
    T = np.array([15.0, 25.0, 40.0, 60.0])
    mdl = chain_1d(np.linspace(0, 1e16, 4), np.zeros(4), nh2, T, 1.5e4, 1e-6)
    return make(oracle_lib, mdl, sp, use_alo=use_alo), sp, mdl


def closed_form_ratio(sp, T, nh2, A, Jeff, L):
    """n_u / n_l of the two-level rate equations, rates computed here from the table."""
    nu = (sp.energy[1] - sp.energy[0]) / H
    Bul = A * CL ** 2 / (2 * H * nu ** 3)
    Blu = sp.weight[1] / sp.weight[0] * Bul
    Cul = np.interp(T, sp.coll_T, sp.coll_K[0]) * nh2
    Clu = Cul * sp.weight[1] / sp.weight[0] * np.exp(-H * nu / (KB * T))
    return (Clu + Blu * Jeff) / (A * (1 - L) + Bul * Jeff + Cul), Bul, Blu, Cul, Clu


def test_stateq_fallback_to_plain_lambda(oracle_lib):
    """L* > 1 (not physical, so the ALO rates go negative) makes the ALO solution
    negative; the point must then take the plain Lambda solution (L = 0, Jeff = J)."""
    o, sp, mdl = two_level_model(oracle_lib)
    A = sp.line_A[0]
    nu = (sp.energy[1] - sp.energy[0]) / H
    B20 = 2 * H * nu ** 3 / CL ** 2 / np.expm1(H * nu / (KB * 20.0))
    J = np.array([[0.3], [1.0], [2.0], [0.7]]) * B20
    Je = 0.01 * J
    L = np.array([[3.0], [0.2], [5.0], [0.5]])      # points 0 and 2 invalid with the ALO
    old = o.lte()
    pops, flags = o.stateq(old, J, Je, L)
    assert list(flags) == [1, 0, 1, 0]
    ntot = 1e-6 * mdl.n_h2
    for p in range(4):
        if flags[p] == 1:
            ratio, *_ = closed_form_ratio(sp, mdl.temperature[p], mdl.n_h2[p], A, J[p, 0], 0.0)
            # the ALO system would have given a negative ratio
            r_alo, *_ = closed_form_ratio(sp, mdl.temperature[p], mdl.n_h2[p], A, Je[p, 0], L[p, 0])
            assert r_alo < 0
        else:
            ratio, *_ = closed_form_ratio(sp, mdl.temperature[p], mdl.n_h2[p], A, Je[p, 0], L[p, 0])
        assert rel(pops[p, 1] / pops[p, 0], ratio) < 1e-13, p
        assert rel(pops[p].sum(), ntot[p]) < 1e-14


def test_stateq_keeps_old_populations_when_both_solves_fail(oracle_lib):
    """A negative or non-finite radiation field fails the ALO and the plain solve alike:
    the point keeps its previous populations bit for bit (flag 2); the other points are
    unaffected."""
    o, sp, mdl = two_level_model(oracle_lib)
    A = sp.line_A[0]
    old = o.lte() * np.array([[1.0], [1.1], [0.9], [1.0]])
    old[:, 1] *= 1.3
    Cul = np.interp(mdl.temperature, sp.coll_T, sp.coll_K[0]) * mdl.n_h2
    nu = (sp.energy[1] - sp.energy[0]) / H
    Clu = Cul * 3.0 * np.exp(-H * nu / (KB * mdl.temperature))
    Bul = A * CL ** 2 / (2 * H * nu ** 3)
    Blu = 3.0 * Bul
    J = np.zeros((4, 1))
    J[0, 0] = -2.0 * Clu[0] / Blu                  # numerator C_lu + B_lu J < 0, denominator > 0
    J[1, 0] = np.nan
    J[2, 0] = 1e-15
    J[3, 0] = 1e-15
    Je = J.copy()
    L = np.zeros((4, 1))
    assert A + Cul[0] + Bul * J[0, 0] > 0
    pops, flags = o.stateq(old, J, Je, L)
    assert list(flags) == [2, 2, 0, 0]
    assert np.array_equal(pops[:2], old[:2])
    for p in (2, 3):
        ratio, *_ = closed_form_ratio(sp, mdl.temperature[p], mdl.n_h2[p], A, J[p, 0], 0.0)
        assert rel(pops[p, 1] / pops[p, 0], ratio) < 1e-13


def test_stateq_plain_lambda_ignores_alo_inputs(oracle_lib):
    """use_alo = 0: the rates use J with L = 0 whatever Jeff and L* are passed."""
    o, sp, mdl = two_level_model(oracle_lib, use_alo=False)
    A = sp.line_A[0]
    nu = (sp.energy[1] - sp.energy[0]) / H
    B20 = 2 * H * nu ** 3 / CL ** 2 / np.expm1(H * nu / (KB * 20.0))
    J = np.array([[0.3], [1.0], [2.0], [0.7]]) * B20
    pops, flags = o.stateq(o.lte(), J, 0.5 * J, np.full((4, 1), 0.9))
    assert not flags.any()
    for p in range(4):
        ratio, *_ = closed_form_ratio(sp, mdl.temperature[p], mdl.n_h2[p], A, J[p, 0], 0.0)
        assert rel(pops[p, 1] / pops[p, 0], ratio) < 1e-13
