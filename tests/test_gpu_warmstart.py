"""Warm start on the GPU: features, MFMA network forward / gradient / Adam and
prediction against the FP64 oracle, and what a trained network gains over an LTE start."""
import numpy as np
import pytest

from oracle import mlp
from synth import configs, directions, species
from synth.configs import Workload
from synth.models import chain_1d, lattice_3d
from synth.rng import Stream

from _common import oracle_for, rel, solver_for

pytestmark = pytest.mark.gpu


def _glorot(n_out, seed, bias=0.1):
    rng = np.random.default_rng(seed)
    parts = []
    for o, i in mlp.layer_shapes(n_out):
        a = np.sqrt(6.0 / (o + i))
        parts.append(rng.uniform(-a, a, o * i))
        parts.append(rng.uniform(-bias, bias, o))
    return np.concatenate(parts).astype(np.float32)


def _feature_cases():
    st = Stream(71, "chain")
    x = np.sort(st.uniform(40)) * 3e16
    chain = chain_1d(x, 3e-12 * x, 2e3 + 5e-14 * x, 10.0 + 90.0 * st.uniform(40), 1.5e4, 1e-8)
    xq, wq = directions.uniform_grid(31, 4.0)
    two = species.two_level(100e9, 3.0, 1e-5, 1e-10, 28.0)
    axes6 = np.array([[1, 0, 0], [-1, 0, 0], [0, 1, 0], [0, -1, 0], [0, 0, 1], [0, 0, -1]], float)
    return [
        ("chain", Workload("chain", chain, two, directions.axis_pair(), xq, wq)),
        ("lattice", Workload("lattice", lattice_3d(5, 1e15, n_h2=3e4), two, axes6, xq, wq)),
        ("sphere2", configs.sphere2(n_points=400)),
        ("outflow", configs.outflow5(n_points=1500, seed=5, nside=2)),
        ("disc", configs.disc10(n_points=1200, seed=7)),
    ]


@pytest.mark.parametrize("name,w", _feature_cases(), ids=[c[0] for c in _feature_cases()])
def test_features_match_oracle(name, w):
    if name == "disc":
        w.rays = directions.healpix_ring(1)
    F = solver_for(w).features()
    R = oracle_for(w).features()
    assert F.shape == R.shape
    assert np.all(np.isfinite(F))
    # the same trapezoid terms; the GPU sums each ray's terms in a tree order, and log10 / sqrt
    # may differ in the last bit
    assert np.max(np.abs(F - R) / np.maximum(1.0, np.abs(R))) < 1e-13


def _net_solver(n_out, seed):
    from paper_1912_08445_amd.binding import Solver
    s = Solver(0)
    theta = _glorot(n_out, seed)
    s.mlp_set_weights(theta, n_out)
    return s, theta


@pytest.mark.parametrize("n_rows,n_out", [(1, 10), (37, 2), (1000, 10), (4099, 16)])
def test_mfma_forward_matches_oracle(n_rows, n_out):
    s, theta = _net_solver(n_out, seed=n_rows)
    X = np.random.default_rng(n_rows).standard_normal((n_rows, 8)).astype(np.float32)
    Y = s.mlp_forward(X)
    R, _ = mlp.forward(theta.astype(np.float64), X.astype(np.float64), n_out, round_bf16=True)
    d = np.abs(Y - R)
    scale = max(1.0, np.max(np.abs(R)))
    # FP32 versus FP64 accumulation of bfloat16 products; a rounding of a hidden
    # activation that lands on the other side of a bfloat16 boundary moves an output by
    # at most about 2^-8 of one product term
    assert np.max(d) < 1e-2 * scale
    assert np.quantile(d, 0.99) < 1e-4 * scale
    # and the bfloat16 network is not the FP64 one: the oracle's rounding is what matches
    R64, _ = mlp.forward(theta.astype(np.float64), X.astype(np.float64), n_out, round_bf16=False)
    if n_rows >= 37:
        assert np.median(np.abs(Y - R64)) > 10 * np.median(d)


# (4099 rows: a ragged last tile and chunk; 20000 rows: more tiles of 16 rows than the
# forward/backward kernel's 1024 workgroups, each taking several, and 79 row chunks)
@pytest.mark.parametrize("n_rows,n_out", [(64, 10), (300, 5), (1000, 10), (4099, 16), (20000, 7)])
def test_gradient_matches_oracle(n_rows, n_out):
    s, theta = _net_solver(n_out, seed=100 + n_rows)
    rng = np.random.default_rng(n_rows)
    X = rng.standard_normal((n_rows, 8)).astype(np.float32)
    T = (rng.standard_normal((n_rows, n_out)) - 2.0).astype(np.float32)
    loss, g = s.mlp_loss_grad(X, T)
    rl, rg = mlp.loss_and_grad(theta.astype(np.float64), X.astype(np.float64), T.astype(np.float64), n_out,
                               round_bf16=True)
    assert abs(loss - rl) < 1e-4 * rl
    k = 0
    for o, i in mlp.layer_shapes(n_out):
        for size in (o * i, o):  # weights, then biases
            a, b = g[k:k + size].astype(np.float64), rg[k:k + size]
            k += size
            assert np.linalg.norm(a - b) < 1e-2 * np.linalg.norm(b), (o, i, size)


def test_adam_steps_match_oracle():
    n_out, n_rows = 10, 300
    s, theta = _net_solver(n_out, seed=5)
    rng = np.random.default_rng(6)
    X = rng.standard_normal((n_rows, 8)).astype(np.float32)
    T = (np.tanh(X[:, :1]) - np.arange(n_out)[None, :] * 0.3).astype(np.float32)
    lr, steps = 1e-3, 6
    curve = s.mlp_train(X, T, steps=steps, batch=128, lr=lr)   # batches wrap around the rows
    th_gpu = s.mlp_get_weights().astype(np.float64)
    th_or, losses = mlp.train(theta.astype(np.float64), X.astype(np.float64), T.astype(np.float64), n_out,
                              steps=steps, batch=128, lr=lr)
    assert np.allclose(curve, losses, rtol=1e-4)
    # Adam moves each parameter by about lr per step whatever the gradient's size, so a
    # parameter whose gradient is at rounding level can move the other way; nearly all
    # must match closely
    d = np.abs(th_gpu - th_or)
    assert np.mean(d < 0.05 * lr * steps) > 0.98
    assert np.max(d) <= 2.0 * lr * steps + 1e-6


def test_training_curve_matches_oracle():
    n_out, n_rows = 4, 2000
    s, theta = _net_solver(n_out, seed=9)
    rng = np.random.default_rng(10)
    X = rng.standard_normal((n_rows, 8)).astype(np.float32)
    T = np.stack([np.tanh(X[:, 0]), X[:, 1] * X[:, 2] / 3, np.sin(X[:, 3]), 0.5 * X[:, 4]],
                 axis=1).astype(np.float32)
    curve = s.mlp_train(X, T, steps=120, batch=256, lr=3e-3)
    _, losses = mlp.train(theta.astype(np.float64), X.astype(np.float64), T.astype(np.float64), n_out,
                          steps=120, batch=256, lr=3e-3)
    assert curve[-10:].mean() < 0.2 * curve[:5].mean()
    assert np.max(np.abs(curve - losses) / losses) < 0.05


def test_predict_matches_oracle_and_normalises():
    w = configs.outflow5(n_points=2000, seed=11, nside=1)
    s = solver_for(w)
    o = oracle_for(w)
    n_out = w.species.n_lev
    theta = _glorot(n_out, seed=12)
    F = o.features()
    mean, std = F.mean(0), np.where(F.std(0) > 1e-12, F.std(0), 1.0)
    s.mlp_set_weights(theta, n_out)
    s.mlp_set_norm(mean, std)
    pops, bad = s.mlp_predict()
    assert bad == 0
    ntot = w.model.abundance * w.model.n_h2
    assert np.all(pops > 0)
    assert np.max(np.abs(pops.sum(1) / ntot - 1)) < 1e-13
    X = mlp.standardise(F, mean, std).astype(np.float32).astype(np.float64)
    y, _ = mlp.forward(theta.astype(np.float64), X, n_out, round_bf16=True)
    ref = mlp.populations(y, o.lte())
    r = np.abs(pops - ref) / ref
    assert np.quantile(r, 0.99) < 1e-3 and np.max(r) < 5e-2


def test_training_rows_match_oracle():
    import torch
    w = configs.sphere2(n_points=500)
    s = solver_for(w)
    o = oracle_for(w)
    lte = o.lte()
    # non-LTE populations with the right sum
    pops = lte * np.exp(np.random.default_rng(4).normal(0.0, 0.5, lte.shape))
    pops *= (lte.sum(1) / pops.sum(1))[:, None]
    mean, std = np.arange(8) * 0.5, np.linspace(1.0, 2.0, 8)
    s.mlp_set_norm(mean, std)
    dev = torch.device("cuda:0")
    X = torch.empty((w.n_points, 8), dtype=torch.float32, device=dev)
    T = torch.empty((w.n_points, w.species.n_lev), dtype=torch.float32, device=dev)
    s.mlp_rows_dev(torch.tensor(pops, device=dev), X, T)
    torch.cuda.synchronize()
    refX = mlp.standardise(o.features(), mean, std).astype(np.float32)
    refT = mlp.targets(pops, lte).astype(np.float32)
    assert np.max(np.abs(X.cpu().numpy() - refX)) <= 2e-6 * max(1.0, np.max(np.abs(refX)))
    assert np.max(np.abs(T.cpu().numpy() - refT)) <= 2e-6 * max(1.0, np.max(np.abs(refT)))


def test_nonfinite_prediction_falls_back_to_lte():
    # a standardisation that sends the inputs beyond the FP32 range makes every output
    # NaN: every point must keep its LTE populations and be counted
    w = configs.sphere2(n_points=300)
    s = solver_for(w)
    s.mlp_set_weights(_glorot(w.species.n_lev, 3), w.species.n_lev)
    s.mlp_set_norm(np.zeros(8), np.full(8, 1e-300))
    pops, bad = s.mlp_predict()
    assert bad == w.n_points
    assert np.array_equal(pops, s.lte())


def test_warm_start_api_errors():
    from paper_1912_08445_amd.binding import NlteError, Solver, param_count
    assert param_count(10) == 35466 and param_count(0) == -1 and param_count(17) == -1
    s = Solver(0)
    with pytest.raises(NlteError):
        s.n_out = 10
        s.mlp_forward(np.zeros((4, 8), np.float32))          # no weights yet
    with pytest.raises(NlteError):
        s.mlp_init(17)
    s.mlp_init(10, 1)
    with pytest.raises(NlteError):
        s.mlp_set_norm(np.zeros(8), np.zeros(8))             # std must be positive
    bad = np.zeros(param_count(10), np.float32)
    bad[5] = np.nan
    with pytest.raises(NlteError):
        s.mlp_set_weights(bad, 10)
    w = configs.sphere2(n_points=200)
    s2 = solver_for(w)
    s2.mlp_init(5, 0)                                        # 5 outputs, 2 levels
    with pytest.raises(NlteError):
        s2.mlp_predict()


def test_init_is_seeded_glorot():
    from paper_1912_08445_amd.binding import Solver
    a, b = Solver(0), Solver(0)
    a.mlp_init(10, 42)
    b.mlp_init(10, 42)
    ta, tb = a.mlp_get_weights(), b.mlp_get_weights()
    assert np.array_equal(ta, tb)
    for (W, bias), (o, i) in zip(mlp.unpack(ta.astype(np.float64), 10), mlp.layer_shapes(10)):
        lim = np.sqrt(6.0 / (o + i))
        assert np.all(np.abs(W) <= lim) and np.all(bias == 0)
        assert abs(W.std() - lim / np.sqrt(3)) < 0.1 * lim


def _disc(seed, n_points):
    w = configs.disc10(n_points=n_points, seed=seed)
    w.rays = directions.healpix_ring(1)
    return w


HELD_OUT = (200, 201, 202, 203, 204)


def test_warm_start_gain_on_five_held_out_discs():
    """Train on converged populations of sixteen discs of the family (seeds 100..115), then
    start the ALI of each of the five held-out seeds 200..204 from the prediction: a start
    at least ten times closer to the tightly converged populations than LTE, never more
    iterations to the same tolerance and fewer for most seeds, and a result as close to
    the converged populations as the LTE start's.  Then the combined fast form -- the five
    held-out models batched in one context, FP32 bulk, learned start -- against plain FP64
    from LTE run on each model alone: every model within 1e-4 of its FP64 populations
    converged to 1e-9.  (Reduced discs: 8,000 points and 12 rays each instead of 1 M points
    and 192 rays, so that the test runs in seconds.)"""
    import torch
    from paper_1912_08445_amd import warmstart
    from synth.models import concat_models
    n_points = 8000
    train = [solver_for(_disc(s, n_points)) for s in range(100, 116)]
    mean, std = warmstart.feature_norm([t.features() for t in train])
    rows = [warmstart.converged_rows(t, mean, std, tol=1e-6)[:2] for t in train]
    trainer = train[0]
    curve = warmstart.train(trainer, rows, mean, std, warmstart.SCHEDULE, batch=4096, seed=1)
    assert curve[-50:].mean() < 0.05 * curve[:5].mean()
    theta = trainer.mlp_get_weights()
    for t in train:
        t.close()

    dev = torch.device("cuda:0")
    refs, its_lte, its_warm = [], [], []
    for seed in HELD_OUT:
        w = _disc(seed, n_points)
        held = solver_for(w)
        held.mlp_set_weights(theta, w.species.n_lev)
        held.mlp_set_norm(mean, std)
        held.set_params(tol=1e-9, max_iter=200)
        ref = torch.empty((held.P, held.n_lev), dtype=torch.float64, device=dev)
        held.run_ali_dev(None, ref)
        ref = ref.cpu().numpy()
        refs.append(ref)
        held.set_params(tol=1e-4, max_iter=200)
        lte_pops, lte_rep = held.run_ali()
        warm_pops, warm_rep = held.run_ali_warm()
        pred, bad = held.mlp_predict()
        assert bad == 0 and warm_rep["used_network"]
        ntot = (w.model.abundance * w.model.n_h2)[:, None]
        mask = ref / ntot > 1e-10           # the levels the convergence criterion counts
        err = lambda p: np.abs(p - ref)[mask] / ref[mask]
        lte0 = held.lte()
        print(f"seed {seed}: iterations LTE {lte_rep['iterations']} warm {warm_rep['iterations']}; "
              f"start error max LTE {err(lte0).max():.3e} warm {err(pred).max():.3e}; "
              f"final error max LTE {err(lte_pops).max():.3e} warm {err(warm_pops).max():.3e}; "
              f"changes LTE {np.array(lte_rep['max_change'])} warm {np.array(warm_rep['max_change'])}",
              flush=True)
        assert err(pred).max() < 0.1 * err(lte0).max()
        assert warm_rep["iterations"] <= lte_rep["iterations"]
        assert err(warm_pops).max() <= max(err(lte_pops).max(), 1e-5)
        its_lte.append(lte_rep["iterations"])
        its_warm.append(warm_rep["iterations"])
        held.close()
    assert sum(a < b for a, b in zip(its_warm, its_lte)) >= 3, (its_warm, its_lte)

    # the combined fast form on the five held-out models in one batched context
    ws = [_disc(seed, n_points) for seed in HELD_OUT]
    offs, merged = concat_models([x.model for x in ws])
    bw = Workload("held-out discs", merged, ws[0].species, ws[0].rays, ws[0].quad_x, ws[0].quad_w,
                  offsets=offs)
    b = solver_for(bw, precision="fp32", persistent=1)
    b.mlp_set_weights(theta, bw.species.n_lev)
    b.mlp_set_norm(mean, std)
    b.set_params(tol=1e-4, max_iter=200)
    pops, rep = b.run_ali_warm()
    assert rep["used_network"] and rep["converged"]
    model_its = b.model_status()[0]
    ntot = (merged.abundance * merged.n_h2)[:, None]
    for m, ref in enumerate(refs):
        sl = slice(int(offs[m]), int(offs[m + 1]))
        mask = ref / ntot[sl] > 1e-10
        e = rel(pops[sl], ref)[mask].max()
        print(f"batched FP32 warm, model {m}: {model_its[m]} iterations, max rel diff {e:.2e}", flush=True)
        assert e <= 1e-4
        assert model_its[m] <= its_lte[m]


def test_default_stream_work_is_ordered_with_torch():
    # A *_dev call given torch's default stream (handle 0) runs on the context's stream,
    # which is ordered with the null stream: a torch op issued right after the call reads
    # complete rows.  Two models back to back, so stale rows of the first would show.
    import torch
    from paper_1912_08445_amd import warmstart
    dev = torch.device("cuda:0")
    solvers = [solver_for(configs.outflow5(n_points=3000, seed=sd, nside=1)) for sd in (31, 32)]
    mean, std = warmstart.feature_norm([s.features() for s in solvers])
    for s in solvers:
        s.mlp_set_norm(mean, std)
        pops = torch.tensor(s.lte(), device=dev)
        X = torch.empty((s.P, 8), dtype=torch.float32, device=dev)
        T = torch.empty((s.P, s.n_lev), dtype=torch.float32, device=dev)
        s.mlp_rows_dev(pops, X, T)
        picked = X[torch.arange(0, s.P, 7, device=dev)].cpu().numpy()
        ref = ((s.features() - mean) / std).astype(np.float32)[::7]
        assert np.allclose(picked, ref, rtol=1e-6, atol=1e-6)
        s.close()
