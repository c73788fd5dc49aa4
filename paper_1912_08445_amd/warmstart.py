"""Training pipeline of the warm-start network on top of the library calls.

Rows come from models whose populations the ALI has converged: nlte_mlp_rows_dev builds
standardised features and log10 fractional-population targets on the GPU, the rows of
all models are concatenated and shuffled (device tensors), and nlte_mlp_train_dev runs
Adam with the library's MFMA kernels.  The only host arithmetic is the feature
standardisation statistics (mean and standard deviation of 8 columns).
"""
from __future__ import annotations

import numpy as np


def feature_norm(feature_arrays):
    """Mean and standard deviation per feature over the rows of all arrays; a constant
    feature gets std 1."""
    F = np.concatenate([np.asarray(f, dtype=np.float64) for f in feature_arrays], axis=0)
    mean = F.mean(axis=0)
    std = F.std(axis=0)
    std = np.where(std > 1e-12, std, 1.0)
    return mean, std


def converged_rows(solver, mean, std, tol=1e-6, max_iter=200, sample=None, seed=0):
    """ALI of the solver's model from LTE to `tol`, then its training rows.
    Returns (X [n][8], T [n][n_lev]) float32 device tensors and the ALI report;
    `sample` keeps that many rows chosen with a seeded permutation."""
    import torch
    dev = torch.device("cuda:0")
    solver.set_params(tol=tol, max_iter=max_iter)
    pops = torch.empty((solver.P, solver.n_lev), dtype=torch.float64, device=dev)
    rep = solver.run_ali_dev(None, pops)
    solver.mlp_set_norm(mean, std)
    X = torch.empty((solver.P, 8), dtype=torch.float32, device=dev)
    T = torch.empty((solver.P, solver.n_lev), dtype=torch.float32, device=dev)
    solver.mlp_rows_dev(pops, X, T)
    if sample is not None and sample < solver.P:
        g = torch.Generator(device="cpu").manual_seed(seed)
        idx = torch.randperm(solver.P, generator=g)[:sample].to(dev)
        X, T = X[idx].contiguous(), T[idx].contiguous()
    torch.cuda.synchronize()   # the rows are complete before the caller may release the solver
    return X, T, rep


# Training phases [(steps, learning rate), ...] at batch 4096: a long phase at 2e-3, then
# two annealing phases.  The last, low-rate phase trims the largest prediction errors,
# which decide the first iterations' maximum change.
SCHEDULE = ((12000, 2e-3), (8000, 2e-4), (4000, 2e-5))


def train(solver, rows, mean, std, phases=SCHEDULE, batch=4096, seed=0, init_seed=0):
    """Fresh network on `solver` with the rows' standardisation, trained on the
    concatenated, shuffled rows [(X, T), ...] in phases [(steps, lr), ...] (the Adam
    state carries over between phases); returns the per-step loss curve (host)."""
    import torch
    solver.mlp_set_norm(mean, std)
    X = torch.cat([r[0] for r in rows]).contiguous()
    T = torch.cat([r[1] for r in rows]).contiguous()
    g = torch.Generator(device="cpu").manual_seed(seed)
    perm = torch.randperm(X.shape[0], generator=g).to(X.device)
    X, T = X[perm].contiguous(), T[perm].contiguous()
    solver.mlp_init(T.shape[1], init_seed)
    curves = []
    for steps, lr in phases:
        curve = torch.zeros(max(steps, 1), dtype=torch.float32, device=X.device)
        solver.mlp_train_dev(X, T, loss_curve=curve, steps=steps, batch=batch, lr=lr)
        curves.append(curve[:steps])
    torch.cuda.synchronize()
    return torch.cat(curves).cpu().numpy()
