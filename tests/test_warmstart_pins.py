"""Pins of the warm-start oracle (features and the FP64 multilayer perceptron) against
closed forms, library routines and finite differences.  CPU only."""
import numpy as np
import pytest
import torch

import oracle
from oracle import mlp
from synth import directions, species
from synth.configs import Workload
from synth.models import chain_1d, lattice_3d
from synth.rng import Stream



def nrel(a, b):
    """Largest absolute difference relative to the largest magnitude of the reference."""
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / np.max(np.abs(b)))


def _workload(model, rays, sp=None):
    x, w = directions.uniform_grid(31, 4.0)
    return Workload("pin", model, sp or species.two_level(100e9, 3.0, 1e-5, 1e-10, 28.0), rays, x, w)


# ------------------------------------------------------------------ features

def _floor(m, p):
    """Half a cell's column at p: n_H2(p) times half the mean distance to its valid
    neighbours (at least 1 cm^-2)."""
    nb = m.nbr[p][m.nbr[p] >= 0]
    if nb.size == 0:
        return 1.0
    return max(0.5 * m.n_h2[p] * np.mean(np.linalg.norm(m.pos[nb] - m.pos[p], axis=1)), 1.0)


def test_features_chain_linear_density_and_hubble_gradient():
    # Points on a line with uneven spacing, n_H2 linear in x, Hubble flow v = H x:
    # the trapezoid column is exact for a linear density, and every neighbour has
    # |dv|/|dx| = H.
    st = Stream(71, "chain")
    x = np.sort(st.uniform(40)) * 3e16
    a, b, H = 2e3, 5e-14, 3e-12
    n = a + b * x
    T = 10.0 + 90.0 * st.uniform(40)
    m = chain_1d(x, H * x, n, T, 1.5e4, 1e-8)
    o = oracle.from_workload(_workload(m, directions.axis_pair()))
    F = o.features()
    x0, x1 = x[0], x[-1]
    col = lambda lo, hi: a * (hi - lo) + 0.5 * b * (hi * hi - lo * lo)
    for p in range(40):
        cols = np.sort(np.maximum([col(x[p], x1), col(x0, x[p])], _floor(m, p)))
        q = [cols[0], cols[0] + 0.25 * (cols[1] - cols[0]), 0.5 * (cols[0] + cols[1]),
             cols[0] + 0.75 * (cols[1] - cols[0]), cols[1]]
        expect = np.log10(q)
        assert np.allclose(F[p, 3:], expect, rtol=1e-12, atol=1e-12), p
        assert abs(F[p, 0] - np.log10(n[p])) < 1e-13
        assert abs(F[p, 1] - np.log10(T[p])) < 1e-13
        assert abs(F[p, 2] - np.log10(H)) < 1e-12
    # the end points see an empty column on their outward ray: half a cell's column
    assert abs(F[0, 3] - np.log10(0.5 * n[0] * (x[1] - x[0]))) < 1e-12
    assert abs(F[-1, 3] - np.log10(0.5 * n[-1] * (x[-1] - x[-2]))) < 1e-12


def test_features_lattice_axis_rays_match_numpy_quantiles():
    # Cubic lattice with the six axis rays: the walk follows lattice lines, so the
    # column along +x from (i, j, k) is n * spacing * (m - 1 - i), and so on.
    mm, d, nval = 5, 1e15, 3e4
    mdl = lattice_3d(mm, d, n_h2=nval)
    rays = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], float)
    o = oracle.from_workload(_workload(mdl, rays))
    F = o.features()
    idx = np.arange(mm)
    I, J, K = [a.ravel() for a in np.meshgrid(idx, idx, idx, indexing="ij")]
    for p in range(mm ** 3):
        cols = nval * d * np.array([mm - 1 - I[p], I[p], mm - 1 - J[p], J[p], mm - 1 - K[p], K[p]],
                                   float)
        cols = np.maximum(cols, 0.5 * nval * d)   # face neighbours at distance d: half a cell
        q = np.quantile(cols, [0.0, 0.25, 0.5, 0.75, 1.0])   # linear interpolation
        assert np.allclose(F[p, 3:], np.log10(q), rtol=1e-12, atol=1e-12)
    assert np.all(F[:, 2] == -30.0)   # static: gradient floored at 1e-30 s^-1


def test_features_columns_from_walks_on_sphere():
    # Independent recomputation on a random point cloud: columns summed in numpy along
    # the (separately pinned) walks, quantiles by numpy.
    from synth import configs
    w = configs.outflow5(n_points=600, seed=5, nside=1)
    o = oracle.from_workload(w)
    F = o.features()
    m = w.model
    for p in [0, 17, 123, 599]:
        cols = []
        for r in range(w.rays.shape[0]):
            cells, Z = o.walk(p, r)
            nn = np.concatenate([[m.n_h2[p]], m.n_h2[cells]])
            zz = np.concatenate([[0.0], Z])
            cols.append(np.sum(0.5 * (nn[1:] + nn[:-1]) * np.diff(zz)))
        q = np.quantile(np.maximum(cols, _floor(m, p)), [0.0, 0.25, 0.5, 0.75, 1.0])
        assert np.allclose(F[p, 3:], np.log10(q), rtol=1e-12, atol=1e-12)
        nb = m.nbr[p][m.nbr[p] >= 0]
        g = np.mean(np.linalg.norm(m.vel[nb] - m.vel[p], axis=1) / np.linalg.norm(m.pos[nb] - m.pos[p], axis=1))
        assert abs(F[p, 2] - np.log10(g)) < 1e-12


# ------------------------------------------------------------------ bfloat16 rounding

def test_bf16_rounding_known_values():
    assert mlp.bf16(1.0) == 1.0
    assert mlp.bf16(1.0 + 2.0 ** -9) == 1.0                    # below half a spacing
    assert mlp.bf16(1.0 + 2.0 ** -8) == 1.0                    # tie -> even (1.0)
    assert mlp.bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6    # tie -> even (up)
    assert mlp.bf16(1.0 + 2.0 ** -8 + 2.0 ** -20) == 1.0 + 2.0 ** -7
    assert mlp.bf16(-3.0e-3) == -mlp.bf16(3.0e-3)
    assert mlp.bf16(0.0) == 0.0


def test_bf16_rounding_matches_bit_level_rounding_of_float32():
    # For float32 inputs the FP64 definition must equal the integer round-to-nearest-even
    # on the upper 16 bits of the IEEE single.
    rng = np.random.default_rng(3)
    x = (rng.standard_normal(200000) * np.exp(rng.uniform(-30, 30, 200000))).astype(np.float32)
    u = x.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    ref = r.astype(np.uint32).view(np.float32).astype(np.float64)
    assert np.array_equal(mlp.bf16(x.astype(np.float64)), ref)


# ------------------------------------------------------------------ network

def _theta(n_out, seed=0, scale=1.0):
    rng = np.random.default_rng(seed)
    parts = []
    for o, i in mlp.layer_shapes(n_out):
        a = np.sqrt(6.0 / (o + i)) * scale
        parts.append(rng.uniform(-a, a, o * i))
        parts.append(rng.uniform(-0.1, 0.1, o))
    return np.concatenate(parts)


def _torch_net(theta, n_out):
    layers = [(torch.tensor(W), torch.tensor(b)) for W, b in mlp.unpack(theta, n_out)]
    for W, b in layers:
        W.requires_grad_(True)
        b.requires_grad_(True)
    return layers


def _torch_forward(layers, X):
    h = X
    for l, (W, b) in enumerate(layers):
        h = torch.nn.functional.linear(h, W, b)
        if l < len(layers) - 1:
            h = torch.nn.functional.gelu(h, approximate="none")
    return h


def test_parameter_count():
    assert mlp.n_params(10) == 35466


def test_forward_matches_torch_fp64():
    n_out = 10
    th = _theta(n_out)
    X = np.random.default_rng(1).standard_normal((50, 8))
    y, _ = mlp.forward(th, X, n_out, round_bf16=False)
    ref = _torch_forward(_torch_net(th, n_out), torch.tensor(X)).detach().numpy()
    assert nrel(y, ref) < 1e-13


def test_backward_matches_torch_autograd_fp64():
    n_out = 7
    th = _theta(n_out, seed=4)
    rng = np.random.default_rng(5)
    X = rng.standard_normal((33, 8))
    T = rng.standard_normal((33, n_out))
    loss, g = mlp.loss_and_grad(th, X, T, n_out, round_bf16=False)
    layers = _torch_net(th, n_out)
    y = _torch_forward(layers, torch.tensor(X))
    L = torch.mean((y - torch.tensor(T)) ** 2)
    L.backward()
    ref = np.concatenate([np.concatenate([W.grad.numpy().ravel(), b.grad.numpy().ravel()]) for W, b in layers])
    assert abs(loss - L.item()) < 1e-14 * max(1.0, abs(loss))
    assert np.max(np.abs(g - ref)) < 1e-13 * np.max(np.abs(ref))


def test_backward_finite_differences():
    n_out = 10
    th = _theta(n_out, seed=8)
    rng = np.random.default_rng(9)
    X = rng.standard_normal((16, 8))
    T = rng.standard_normal((16, n_out))
    loss0, g = mlp.loss_and_grad(th, X, T, n_out, round_bf16=False)
    gscale = np.max(np.abs(g))
    # a central difference carries a rounding floor of about eps * loss / h
    floor = 1e-9 * max(1.0, loss0)
    for i in rng.choice(th.shape[0], 300, replace=False):
        h = 1e-6 * max(1.0, abs(th[i]))
        tp, tm = th.copy(), th.copy()
        tp[i] += h
        tm[i] -= h
        lp, _ = mlp.loss_and_grad(tp, X, T, n_out, round_bf16=False)
        lm, _ = mlp.loss_and_grad(tm, X, T, n_out, round_bf16=False)
        fd = (lp - lm) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(abs(g[i]), 1e-3 * gscale) + floor, i


def test_bf16_rounded_network_is_close_to_fp64_and_idempotent_in_weights():
    n_out = 10
    th = _theta(n_out, seed=2)
    X = np.random.default_rng(2).standard_normal((64, 8))
    y64, _ = mlp.forward(th, X, n_out, round_bf16=False)
    y16, _ = mlp.forward(th, X, n_out, round_bf16=True)
    assert 1e-5 < nrel(y16, y64) < 5e-2
    # rounding already-rounded weights and inputs changes nothing
    lay = [(mlp.bf16(W), b) for W, b in mlp.unpack(th, n_out)]
    y16b, _ = mlp.forward(mlp.pack(lay), mlp.bf16(X), n_out, round_bf16=True)
    assert np.array_equal(y16, y16b)


def test_adam_matches_torch_optimizer():
    rng = np.random.default_rng(11)
    th = rng.standard_normal(50)
    m, v = np.zeros(50), np.zeros(50)
    p = torch.tensor(th.copy(), requires_grad=True)
    opt = torch.optim.Adam([p], lr=1e-3, betas=(0.9, 0.999), eps=1e-8)
    for t in range(1, 8):
        g = rng.standard_normal(50)
        th, m, v = mlp.adam_step(th, m, v, g, t, 1e-3, 0.9, 0.999, 1e-8)
        p.grad = torch.tensor(g)
        opt.step()
    assert np.max(np.abs(th - p.detach().numpy())) < 1e-15


def test_adam_constant_gradient_moves_by_lr():
    # With a constant gradient the bias-corrected moments are g and g^2, so every step
    # moves each parameter by exactly lr against the sign of its gradient (eps = 0).
    g = np.array([3.0, -0.02, 7e-5])
    th = np.zeros(3)
    m, v = np.zeros(3), np.zeros(3)
    for t in range(1, 6):
        th, m, v = mlp.adam_step(th, m, v, g, t, 0.01, 0.9, 0.999, 0.0)
        assert np.allclose(th, -0.01 * t * np.sign(g), rtol=1e-12, atol=0)


def test_training_fits_a_smooth_map():
    n_out = 4
    rng = np.random.default_rng(21)
    X = rng.standard_normal((512, 8))
    T = np.stack([np.tanh(X[:, 0]), X[:, 1] * X[:, 2] / 3, np.sin(X[:, 3]), 0.5 * X[:, 4]], axis=1)
    th = _theta(n_out, seed=22)
    _, losses = mlp.train(th, X, T, n_out, steps=150, batch=128, lr=3e-3)
    assert losses[-10:].mean() < 0.1 * losses[:5].mean()


def test_departure_targets_and_populations_invert_each_other():
    rng = np.random.default_rng(31)
    lte = rng.uniform(0.1, 1.0, (20, 5))
    lte[:, 4] = 1e-12                                # a level far up the ladder
    ntot = rng.uniform(1e-3, 1e3, 20)[:, None]
    lte = ntot * lte / lte.sum(1, keepdims=True)
    pops = lte * np.exp(rng.normal(0.0, 1.0, lte.shape))
    pops = ntot * pops / pops.sum(1, keepdims=True)
    y = mlp.targets(pops, lte)
    assert np.allclose(mlp.populations(y, lte), pops, rtol=1e-12, atol=0)
    # zero departure is the LTE start; equal departures cancel in the normalisation
    assert np.allclose(mlp.populations(np.zeros_like(y), lte), lte, rtol=1e-13, atol=0)
    assert np.allclose(mlp.populations(np.full_like(y, 3.7), lte), lte, rtol=1e-13, atol=0)
    assert np.allclose(mlp.targets(lte, lte), 0.0, atol=1e-14)
    # a departure of +1 on one level of two equal ones makes it ten times the other
    two = np.full((1, 2), 0.5)
    p2 = mlp.populations(np.array([[1.0, 0.0]]), two)
    assert abs(p2[0, 0] / p2[0, 1] - 10.0) < 1e-13 and abs(p2.sum() - 1.0) < 1e-15
