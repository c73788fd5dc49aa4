"""Pins of the Ng-acceleration oracle: exactness on linear iterations with a low-dimensional
error, conservation, singular and non-physical cases, and the ALI fixed point."""
import numpy as np

from oracle import ng
from synth import configs

from _common import oracle_for, rel


def _linear_iterates(M, dims, seed):
    """x_k = x* + sum_d c_d lam_d^k v_d, k = 1..M: the error of a linear fixed-point
    iteration that lives in a `dims`-dimensional invariant subspace."""
    rng = np.random.default_rng(seed)
    xs = rng.uniform(1.0, 2.0, (50, 5))
    lams = rng.uniform(0.3, 0.9, dims) * rng.choice([-1.0, 1.0], dims)
    vs = rng.normal(0.0, 0.1, (dims, 50, 5))
    return xs, [xs + sum(lams[d] ** k * vs[d] for d in range(dims)) for k in range(1, M + 1)]


def test_exact_for_two_dimensional_error_with_four_iterates():
    xs, hist = _linear_iterates(4, 2, seed=1)
    out, a, bad = ng.ng_step(hist, np.ones(50))
    assert bad == 0 and abs(a.sum() - 1.0) < 1e-14
    assert np.max(np.abs(out - xs)) < 1e-12
    # the plain iterate is far from it
    assert np.max(np.abs(hist[-1] - xs)) > 1e-3


def test_exact_for_one_dimensional_error_with_three_iterates():
    xs, hist = _linear_iterates(3, 1, seed=2)
    out, a, _ = ng.ng_step(hist, np.ones(50))
    assert np.max(np.abs(out - xs)) < 1e-12


def test_weighting_by_density_does_not_change_an_exact_case():
    xs, hist = _linear_iterates(4, 2, seed=3)
    out, _, _ = ng.ng_step(hist, np.random.default_rng(4).uniform(1e-3, 1e3, 50))
    assert np.max(np.abs(out - xs)) < 1e-11


def test_reduces_error_of_a_general_contraction():
    rng = np.random.default_rng(5)
    n = 40
    Q = np.linalg.qr(rng.normal(size=(n, n)))[0]
    A = Q @ np.diag(rng.uniform(0.0, 0.95, n)) @ Q.T
    xs = rng.uniform(1.0, 2.0, n)
    b = xs - A @ xs
    x = np.ones(n)
    hist = []
    for _ in range(4):
        x = A @ x + b
        hist.append(x[:, None])
    out, _, _ = ng.ng_step(hist, np.ones(n))
    # two free coefficients cannot remove a full spectrum of modes, but they must help
    assert np.linalg.norm(out[:, 0] - xs) < 0.8 * np.linalg.norm(hist[-1][:, 0] - xs)


def test_preserves_population_sums():
    rng = np.random.default_rng(6)
    ntot = rng.uniform(1.0, 10.0, 30)
    hist = []
    for _ in range(4):
        p = rng.uniform(0.5, 1.5, (30, 4))
        hist.append(ntot[:, None] * p / p.sum(1, keepdims=True))
    out, a, bad = ng.ng_step(hist, ntot)
    ok = np.all(out > 0, axis=1)
    assert np.allclose(out[ok].sum(1), ntot[ok], rtol=1e-13)


def test_singular_history_keeps_the_newest_iterate():
    x = np.random.default_rng(7).uniform(1.0, 2.0, (10, 3))
    out, a, bad = ng.ng_step([x, x, x, x], np.ones(10))
    assert a is None and np.array_equal(out, x)


def test_non_physical_points_keep_the_newest_iterate():
    # point 0 has positive iterates heading geometrically to a negative limit, which the
    # (exact, two-mode) extrapolation reaches: that point keeps the newest iterate, the
    # others take the extrapolation
    hist = []
    for k in range(1, 5):
        x = np.ones((3, 2))
        x[0, 0] = -0.01 + 0.5 ** k
        x[1, 1] = 1.0 + 0.3 * 0.8 ** k
        hist.append(x)
    out, a, bad = ng.ng_step(hist, np.ones(3))
    assert a is not None and bad == 1
    assert np.array_equal(out[0], hist[-1][0])
    assert abs(out[1, 1] - 1.0) < 1e-12 and np.all(out > 0)


def test_ali_with_ng_reaches_the_same_fixed_point():
    # an optically thick two-level sphere converges slowly; Ng keeps the fixed point
    w = configs.sphere2(n_points=300, seed=9)
    w.model.abundance[:] = 1e-6
    o = oracle_for(w)
    ntot = w.model.abundance * w.model.n_h2
    plain, ch_plain = o.run_ali(max_iter=300, tol=1e-10)
    acc, ch_ng, coefs = ng.run_ali_ng(o, ntot, max_iter=300, tol=1e-10, M=4)
    assert ch_plain[-1] < 1e-10 and ch_ng[-1] < 1e-10
    assert rel(acc, plain).max() < 1e-8
    assert len(ch_ng) < len(ch_plain)
    assert len(coefs) >= 1
