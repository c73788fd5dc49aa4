"""The seeded input generators shared by the oracle and the GPU tests (no method
arithmetic): the counter-based SplitMix64 streams against the generator's sequential
definition (Steele, Lea and Flood 2014) and its first output for a zero seed, uniform and
normal draws, and the structure and determinism of the synthetic workloads."""
import numpy as np

from synth import configs
from synth.models import keplerian_disc, knn
from synth.rng import Stream, splitmix64

M64 = (1 << 64) - 1


def _sequential(state, n):
    """The published generator: the state advances by the golden-ratio increment and each
    output is the state after two xor-shift-multiply rounds and a final xor-shift."""
    out = []
    for _ in range(n):
        state = (state + 0x9E3779B97F4A7C15) & M64
        z = state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
        out.append(z ^ (z >> 31))
    return out


def test_splitmix64_matches_the_sequential_generator():
    assert int(splitmix64(0, 0, 1)[0]) == 0xE220A8397B1DCDAF   # first output for seed 0
    for key in (0, 1, 0x123456789ABCDEF0, M64):
        seq = _sequential(key, 40)
        assert [int(v) for v in splitmix64(key, 0, 40)] == seq
        assert [int(v) for v in splitmix64(key, 17, 23)] == seq[17:]   # random access


def test_stream_draws():
    st = Stream(5, "test")
    u = st.uniform(200000)
    assert u.min() >= 0.0 and u.max() < 1.0 and abs(u.mean() - 0.5) < 3e-3
    g = Stream(5, "test-normal").normal(200001)
    assert g.shape == (200001,) and abs(g.mean()) < 1e-2 and abs(g.std() - 1.0) < 1e-2
    assert np.array_equal(Stream(5, "test").uniform(10), u[:10])
    assert not np.array_equal(Stream(6, "test").uniform(10), u[:10])
    assert not np.array_equal(Stream(5, "other").uniform(10), u[:10])


def test_workloads_are_deterministic_and_seed_dependent():
    a, b = configs.outflow5(n_points=400, seed=3), configs.outflow5(n_points=400, seed=3)
    c = configs.outflow5(n_points=400, seed=4)
    for f in ("pos", "vel", "n_h2", "temperature", "nbr"):
        assert np.array_equal(getattr(a.model, f), getattr(b.model, f))
    assert not np.array_equal(a.model.pos, c.model.pos)
    x, w = np.asarray(a.quad_x), np.asarray(a.quad_w)
    assert x.shape == (31,) and np.allclose(x, -x[::-1]) and abs(w.sum() - 1.0) < 1e-12
    assert a.rays.shape == (48, 3) and configs.disc10.__defaults__[0] == 1_000_000


def test_disc_structure():
    m = keplerian_disc(7, 3000)
    R = np.hypot(m.pos[:, 0], m.pos[:, 1])
    vphi = (m.pos[:, 0] * m.vel[:, 1] - m.pos[:, 1] * m.vel[:, 0]) / R
    # Keplerian rotation: v R^(1/2) constant, velocity in the plane and perpendicular to R
    k = vphi * np.sqrt(R)
    assert np.ptp(k) <= 1e-12 * k.mean() and np.all(m.vel[:, 2] == 0.0)
    assert np.abs((m.pos[:, :2] * m.vel[:, :2]).sum(axis=1)).max() <= 1e-9 * (R * np.abs(vphi)).max()
    # density falls as R^-2 in the mid-plane, temperature as R^-1/2, heights within 3 H
    assert np.all(np.abs(m.pos[:, 2]) <= 3.0 * 0.1 * R * (1 + 1e-12))
    T = m.temperature * np.sqrt(R)
    assert np.ptp(T) <= 1e-12 * T.mean()


def test_knn_is_exact():
    rng = np.random.default_rng(1)
    pos = rng.uniform(size=(300, 3))
    nb = knn(pos, 12)
    d = np.linalg.norm(pos[:, None, :] - pos[None, :, :], axis=2)
    np.fill_diagonal(d, np.inf)
    ref = np.argsort(d, axis=1, kind="stable")[:, :12]
    assert np.array_equal(np.sort(d[np.arange(300)[:, None], nb], axis=1), np.sort(d[np.arange(300)[:, None], ref], axis=1))
    assert not np.any(nb == np.arange(300)[:, None])
