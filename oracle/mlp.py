"""Plain FP64 reference of the warm-start surrogate: a small multilayer perceptron that
predicts starting level populations for the accelerated Lambda iteration from local
conditions of each point.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke entry point and the benchmark's
CPU-baseline leg are its only users.  The HIP library never imports or links it.

The surrogate is not part of the paper's method; the paper's ALI (Sec. 2.2.1, 3.4)
only needs some initial populations, which it otherwise takes in LTE.  Network:
8 standardised features -> 128 -> 128 -> 128 -> n_out (one output per level, its
departure from LTE log10 (f_i / f_i^LTE) with f the fractional population), erf-form
GELU after each hidden layer, loss the mean squared error over rows and outputs,
optimiser Adam.

Parameters are one flat vector, in this order, every matrix row-major [out][in]:
    W1 [128][8], b1 [128], W2 [128][128], b2 [128], W3 [128][128], b3 [128],
    W4 [n_out][128], b4 [n_out].

Arithmetic: FP64 throughout.  With ``round_bf16=True`` values are rounded to bfloat16
(round to nearest, ties to even) at the points where the GPU kernels round them, so
that the two agree up to FP32-versus-FP64 accumulation:
    the inputs X and every weight matrix (biases stay as given);
    each hidden activation after GELU;
    in the backward pass, the output-side gradient dZ of every layer where it enters a
    product (the bias gradient sums the unrounded dZ).
With ``round_bf16=False`` the network is the plain FP64 function, which is what the
finite-difference and library checks pin.
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf

N_IN = 8
HIDDEN = 128


def n_params(n_out: int) -> int:
    H = HIDDEN
    return N_IN * H + H + 2 * (H * H + H) + n_out * H + n_out


def layer_shapes(n_out: int):
    H = HIDDEN
    return [(H, N_IN), (H, H), (H, H), (n_out, H)]


def unpack(theta, n_out: int):
    """Flat parameter vector -> [(W, b)] per layer (views)."""
    theta = np.asarray(theta, dtype=np.float64)
    if theta.shape != (n_params(n_out),):
        raise ValueError("parameter vector has the wrong length")
    out, k = [], 0
    for o, i in layer_shapes(n_out):
        W = theta[k:k + o * i].reshape(o, i)
        k += o * i
        b = theta[k:k + o]
        k += o
        out.append((W, b))
    return out


def pack(layers) -> np.ndarray:
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in layers])


def bf16(x):
    """Round to the nearest bfloat16 value (8 significant bits), ties to even.
    Finite inputs in the normal bfloat16 range; zero stays zero."""
    x = np.asarray(x, dtype=np.float64)
    m, e = np.frexp(x)                 # x = m 2^e, 0.5 <= |m| < 1
    q = np.ldexp(1.0, e - 8)           # spacing of bfloat16 values at that magnitude
    return np.where(x == 0.0, 0.0, np.round(x / q) * q)   # np.round: ties to even


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / np.sqrt(2.0)))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / np.sqrt(2.0))) + z * np.exp(-0.5 * z * z) / np.sqrt(2.0 * np.pi)


def forward(theta, X, n_out: int, round_bf16: bool = True):
    """Outputs [rows][n_out] and the activations the backward pass needs."""
    q = bf16 if round_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    layers = unpack(theta, n_out)
    h = q(X)
    hs, zs = [h], []
    for l, (W, b) in enumerate(layers):
        z = h @ q(W).T + b
        if l == len(layers) - 1:
            return z, (hs, zs)
        zs.append(z)
        h = q(gelu(z))
        hs.append(h)


def loss_and_grad(theta, X, T, n_out: int, round_bf16: bool = True):
    """Mean squared error over rows and outputs and its gradient (flat, like theta)."""
    q = bf16 if round_bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    layers = unpack(theta, n_out)
    y, (hs, zs) = forward(theta, X, n_out, round_bf16)
    T = np.asarray(T, dtype=np.float64)
    rows = y.shape[0]
    diff = y - T
    loss = float(np.sum(diff * diff) / (rows * n_out))
    dZ = 2.0 * diff / (rows * n_out)
    grads = [None] * len(layers)
    for l in range(len(layers) - 1, -1, -1):
        W, _ = layers[l]
        dW = q(dZ).T @ hs[l]
        db = dZ.sum(axis=0)
        grads[l] = (dW, db)
        if l > 0:
            dH = q(dZ) @ q(W)
            dZ = dH * gelu_grad(zs[l - 1])
    return loss, pack(grads)


def adam_step(theta, m, v, g, t: int, lr: float, beta1: float, beta2: float, eps: float):
    """One Adam update (Kingma & Ba 2015, Algorithm 1); returns new (theta, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    return theta - lr * mhat / (np.sqrt(vhat) + eps), m, v


def train(theta, X, T, n_out: int, steps: int, batch: int, lr: float = 1e-3, beta1: float = 0.9,
          beta2: float = 0.999, eps: float = 1e-8, round_bf16: bool = True):
    """Adam on consecutive batches: step t (1-based) takes rows (t-1)*batch ... t*batch-1,
    wrapping modulo the row count.  Returns the final parameters and the loss of each
    step (before its update)."""
    theta = np.asarray(theta, dtype=np.float64).copy()
    m = np.zeros_like(theta)
    v = np.zeros_like(theta)
    n = X.shape[0]
    losses = []
    for t in range(1, steps + 1):
        idx = (np.arange(batch) + (t - 1) * batch) % n
        loss, g = loss_and_grad(theta, X[idx], T[idx], n_out, round_bf16)
        losses.append(loss)
        theta, m, v = adam_step(theta, m, v, g, t, lr, beta1, beta2, eps)
    return theta, np.array(losses)


def standardise(F, mean, std):
    """(F - mean) / std per feature."""
    return (np.asarray(F, dtype=np.float64) - mean) / std


def targets(pops, lte_pops):
    """Training targets: departures from LTE, log10 (f_i / f_i^LTE), with fractional
    populations f = n / ntot (ntot = the sum over levels) floored at 1e-300."""
    p = np.asarray(pops, dtype=np.float64)
    q = np.asarray(lte_pops, dtype=np.float64)
    f = np.maximum(p / p.sum(axis=1, keepdims=True), 1e-300)
    fl = np.maximum(q / q.sum(axis=1, keepdims=True), 1e-300)
    return np.log10(f) - np.log10(fl)


def populations(y, lte_pops):
    """Level populations from predicted departures y: ntot w_i / sum_j w_j with
    w_i = f_i^LTE 10^y_i, ntot the sum of the LTE populations over levels."""
    q = np.asarray(lte_pops, dtype=np.float64)
    ntot = q.sum(axis=1, keepdims=True)
    a = np.log10(np.maximum(q / ntot, 1e-300)) + np.asarray(y, dtype=np.float64)
    w = 10.0 ** (a - a.max(axis=1, keepdims=True))
    return ntot * w / w.sum(axis=1, keepdims=True)
