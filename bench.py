"""Benchmark of the ALI hot path on one MI355X.

A step is one accelerated-Lambda-iteration sweep over the whole model with inputs
resident in HBM: line coefficients, the ray-pair formal solve with J / L* / Jeff
accumulation, and the statistical-equilibrium update.  The ray walks are traced once
before timing (they depend only on the geometry).

Workload (default): disc10 -- a Keplerian disc of 1,000,000 points, 192 HEALPix rays,
10-level linear rotor (9 lines x 31 frequencies), FP64 (the largest single-GPU
configuration); --workload outflow5 selects the 50,000-point outflow sphere, which also
times the Ng, band-ALO and scattering ALI forms and the channel images.

Prints one JSON line.  `value` is formal-solve throughput in point*ray*frequency per
second of step time; `roofline` covers the formal-solve kernel, which is bound by VALU
issue: 17 FP64 flops per node-frequency step (profile: x, x^2, exponential, kappa g;
optical depth: add, multiply; Rybicki-Hummer step: h, T, 1 + D T, reciprocal, Q, y;
an FMA counted as 2, the exponential and the reciprocal as 1 each), counted on the steps the
kernel executes (a far-wing segment with zero opacity throughout is one step), against the
78.6 TFLOP/s FP64 vector peak; `cpu_baseline` is the FP64 CPU oracle timed on a bounded
sample of origin points on this host.  Beside the FP64 line: the FP32-bulk form's sweep,
the ALI forms (iterations and wall time to a relative change of 1e-4 against FP64
populations converged to 1e-9) and, on the disc family, the learned warm start on five
held-out seeds with the combined fast form (FP32 bulk, batched, learned start) against
plain FP64 from LTE.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# FP64 flops of one elimination step at one frequency (profile, optical depth,
# Rybicki-Hummer step; exp and the reciprocal count one each); velocity sub-step nodes
# add 6 for the linear interpolation of x, kappa and S.
FLOPS_PER_STEP = 17
PEAK_FP64_TFLOPS = 78.6
PEAK_FP32_TFLOPS = 157.3
PEAK_BF16_MFMA_TFLOPS = 2500.0   # dense


def mlp_flops_per_row(n_out):
    """Algorithmic flops of the 8-128-128-128-n_out network: forward, and one training
    pass (forward, weight gradients of every layer, input gradients of layers 2-4)."""
    fwd = 2 * (8 * 128 + 2 * 128 * 128 + 128 * n_out)
    return fwd, 3 * fwd - 2 * 8 * 128


def log(*a):
    print(*a, file=sys.stderr, flush=True)


KERNEL_SOURCES = ("formal_solve.hip", "formal_solve_kernels.h", "fs_fp64.hip", "fs_fp32.hip", "device_math.h")


def kernel_source_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, "paper_1912_08445_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def traffic_from_profile(workload_name, precision, launch_steps):
    """HBM bytes per formal-solve launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel source; else None."""
    p = os.path.join(ROOT, "profiles", f"formal_solve_{workload_name}_{precision}_traffic.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    if d.get("kernel_sha") != kernel_source_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def cpu_baseline(w, target_s=15.0):
    import numpy as np

    import oracle
    oracle.build(force=False)
    if w.offsets is not None:
        # models stored back to back: give the oracle global neighbour indices
        from synth.configs import Workload
        from synth.models import Model
        m = w.model
        nbr = m.nbr.copy()
        for i in range(w.n_models):
            o0, o1 = w.offsets[i], w.offsets[i + 1]
            blk = nbr[o0:o1]
            blk[blk >= 0] += o0
        w = Workload(w.name, Model(m.pos, m.vel, m.n_h2, m.temperature, m.v_turb, m.abundance, nbr),
                     w.species, w.rays, w.quad_x, w.quad_w)
    o = oracle.from_workload(w)
    pops = o.lte()
    rng = np.random.default_rng(12345)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    probe = rng.choice(w.n_points, max(threads, 8), replace=False)
    t0 = time.perf_counter()
    o.formal_solve(pops, probe)
    dt = time.perf_counter() - t0
    n = int(min(w.n_points, max(len(probe), len(probe) * target_s / max(dt, 1e-3))))
    sel = rng.choice(w.n_points, n, replace=False)
    t0 = time.perf_counter()
    o.formal_solve(pops, sel)
    dt = time.perf_counter() - t0
    per_point = w.rays.shape[0] * w.species.n_lines * w.quad_x.shape[0]
    units = n * per_point
    # one thread on a smaller sample of the same points (about a fifth of the time)
    n1 = max(1, n // (5 * max(threads, 1)))
    oracle.set_threads(1)
    t0 = time.perf_counter()
    o.formal_solve(pops, sel[:n1])
    dt1 = time.perf_counter() - t0
    oracle.set_threads(threads)
    cpu = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                cpu = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"value": units / dt, "unit": "point*ray*freq/s", "cores": threads, "kind": "oracle",
            "sample": f"{n} seeded random origin points of {w.n_points} (all {w.rays.shape[0]} rays, "
                      f"{w.species.n_lines} lines x {w.quad_x.shape[0]} frequencies), LTE "
                      f"populations, formal solve only, {dt:.1f} s wall; the rate is per origin, so the "
                      f"whole sweep is a linear extrapolation of the sample",
            "full_sweep_s_extrapolated": w.n_points * per_point / (units / dt),
            "cpu_model": cpu, "value_1_thread": n1 * per_point / dt1,
            "sample_1_thread": f"the first {n1} of those points, {dt1:.1f} s wall"}


def _rel_err(p, ref, ntot):
    """Largest paper-metric difference 2|a-b|/(|a|+|b|) over levels with n_i/n_tot > 1e-10."""
    import numpy as np
    mask = ref / ntot[:, None] > 1e-10
    a, b = p[mask], ref[mask]
    return float(np.max(2 * np.abs(a - b) / (np.abs(a) + np.abs(b))))


HELD_OUT_SEEDS = (200, 201, 202, 203, 204)


def held_out_discs(args, dev):
    """The learned warm start on the disc family (discs of args.disc_points points): a
    network trained on converged populations of args.train_models training seeds
    (100, 101, ...), evaluated on the five held-out seeds 200..204 -- per seed the plain
    FP64 ALI from LTE and the FP64 ALI from the learned start, each to a relative change
    of 1e-4 against FP64 populations converged to 1e-9 -- and the combined fast form: the
    five models batched in one context (persistent launch), FP32 bulk, learned start,
    against the plain FP64 ALIs run one model at a time.  Each form is timed twice, the
    faster run reported."""
    import numpy as np
    import torch

    from paper_1912_08445_amd import warmstart
    from paper_1912_08445_amd.binding import Solver
    from synth import configs
    from synth.configs import Workload
    from synth.models import concat_models
    n = args.disc_points
    t0 = time.perf_counter()
    mean = std = None
    rows = []
    for k, sd in enumerate(range(100, 100 + args.train_models)):
        st = Solver(0)
        st.setup(configs.disc10(n_points=n, seed=sd), precision="fp32")
        if mean is None:
            mean, std = warmstart.feature_norm([st.features()])
        X, T, rep = warmstart.converged_rows(st, mean, std, tol=1e-6, sample=args.train_sample)
        rows.append((X, T))
        st.close()
        log(f"held-out block: training disc {k + 1}/{args.train_models} (seed {sd}): {rep['iterations']} iterations")
    t_data = time.perf_counter() - t0
    # the five held-out discs batched in one context (persistent launch, FP32 bulk), which
    # also trains the network
    ws = [configs.disc10(n_points=n, seed=sd) for sd in HELD_OUT_SEEDS]
    offs, merged = concat_models([w.model for w in ws])
    bw = Workload("held-out discs", merged, ws[0].species, ws[0].rays, ws[0].quad_x, ws[0].quad_w, offsets=offs)
    b = Solver(0)
    b.setup(bw, precision="fp32", persistent=1)
    t0 = time.perf_counter()
    curve = warmstart.train(b, rows, mean, std, warmstart.SCHEDULE, batch=4096, seed=1)
    t_train = time.perf_counter() - t0
    theta = b.mlp_get_weights()
    n_lev = 10
    log(f"held-out block: {sum(int(r[0].shape[0]) for r in rows)} rows, data {t_data:.1f} s, training "
        f"{t_train:.1f} s, loss {curve[:5].mean():.3e} -> {curve[-50:].mean():.3e}")
    res = {"disc_points": n, "rays": 192, "train_seeds": list(range(100, 100 + args.train_models)),
           "rows": sum(int(r[0].shape[0]) for r in rows), "data_s": t_data, "train_s": t_train,
           "loss_start": float(curve[:5].mean()), "loss_end": float(curve[-50:].mean()), "seeds": {}}

    def best_of(fn):
        best = None
        for _ in range(2):   # the first run also captures the graphs
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            r = fn()
            torch.cuda.synchronize()
            wall = time.perf_counter() - t1
            if best is None or wall < best[0]:
                best = (wall, r)
        return best

    refs = []
    for sd, w in zip(HELD_OUT_SEEDS, ws):
        s = Solver(0)
        s.setup(w, precision="fp64")
        s.mlp_set_weights(theta, n_lev)
        s.mlp_set_norm(mean, std)
        out = torch.empty((w.n_points, n_lev), dtype=torch.float64, device=dev)
        s.set_params(tol=1e-9, max_iter=500)
        s.run_ali_dev(None, out)
        torch.cuda.synchronize()
        ref = out.cpu().numpy()
        refs.append(ref)
        ntot = w.model.abundance * w.model.n_h2
        s.set_params(tol=1e-4, max_iter=200)
        e = {}
        for key, fn in (("fp64_lte", lambda: s.run_ali_dev(None, out)), ("fp64_warm", lambda: s.run_ali_warm_dev(out))):
            wall, r = best_of(fn)
            e[key] = {"iterations": r["iterations"], "wall_s": wall,
                      "max_rel_diff_vs_fp64_reference": _rel_err(out.cpu().numpy(), ref, ntot),
                      "max_change": [float(c) for c in r["max_change"]]}
        s.close()
        res["seeds"][sd] = e
        log(f"held-out seed {sd}: FP64 from LTE {e['fp64_lte']['iterations']} iterations "
            f"{e['fp64_lte']['wall_s']:.3f} s; from the learned start {e['fp64_warm']['iterations']} iterations "
            f"{e['fp64_warm']['wall_s']:.3f} s")
    b.set_params(tol=1e-4, max_iter=200)
    out = torch.empty((bw.n_points, n_lev), dtype=torch.float64, device=dev)
    wall, r = best_of(lambda: b.run_ali_warm_dev(out))
    pops = out.cpu().numpy()
    its = b.model_status()[0]
    ntot = merged.abundance * merged.n_h2
    errs = [_rel_err(pops[offs[m]:offs[m + 1]], refs[m], ntot[offs[m]:offs[m + 1]]) for m in range(len(refs))]
    plain = sum(res["seeds"][sd]["fp64_lte"]["wall_s"] for sd in HELD_OUT_SEEDS)
    res["combined"] = {"form": "FP32 bulk, 5 models batched in one persistent launch per sweep, learned start",
                       "iterations": r["iterations"], "model_iterations": [int(x) for x in its], "wall_s": wall,
                       "used_network": r["used_network"], "max_rel_diff_vs_fp64_reference": max(errs),
                       "plain_fp64_lte_wall_s": plain, "wall_ratio": wall / plain,
                       "plain_fp64_lte_iterations": [res["seeds"][sd]["fp64_lte"]["iterations"] for sd in HELD_OUT_SEEDS]}
    log(f"combined fast form on the 5 held-out discs: {r['iterations']} iterations (models {list(its)}), "
        f"{wall:.3f} s against {plain:.3f} s of plain FP64 from LTE ({wall / plain:.2f}x), max rel diff "
        f"{max(errs):.2e}")
    b._bench_rows = rows
    res["mlp"] = mlp_timing(b, bw, dev)
    b.close()
    return res


def training_factory(args, make):
    """Single training models of the measured workload's family, by seed (None: no warm
    start for this workload)."""
    from synth import configs
    if args.workload == "discs":
        return (lambda sd: configs.disc_model(sd)), 100
    if args.workload in ("batch256", "disc10"):
        return None, 0   # (the disc family has its own held-out block)
    if args.points is None:
        return (lambda sd: make(seed=sd)), 101
    return (lambda sd: make(n_points=args.points, seed=sd)), 101


def train_warm_start(s, w, make, args, dev):
    """Network for the warm start, trained on converged populations of other seeds of the
    same workload family (never the measured model)."""
    import numpy as np

    from paper_1912_08445_amd import warmstart
    from paper_1912_08445_amd.binding import Solver
    t0 = time.perf_counter()
    factory, seed0 = training_factory(args, make)
    seeds = [seed0 + i for i in range(args.train_models)]

    def model(sd, precision="fp64"):
        st = Solver(0)
        st.setup(factory(sd), precision=precision)
        return st

    rows = []
    if args.workload == "disc10":
        # million-point discs, one resident at a time and each set up once: the first one's
        # features standardise every row, and the training ALIs run in the FP32 form
        mean = std = None
        for k, sd in enumerate(seeds):
            t1 = time.perf_counter()
            st = model(sd, "fp32")
            if mean is None:
                mean, std = warmstart.feature_norm([st.features()])
            X, T, rep = warmstart.converged_rows(st, mean, std, tol=1e-6, sample=args.train_sample)
            rows.append((X, T))
            st.close()
            log(f"training model {k + 1}/{len(seeds)} (seed {sd}): {rep['iterations']} iterations, "
                f"{time.perf_counter() - t1:.1f} s")
    else:
        # one training model resident at a time: features first (for the standardisation),
        # then the converged rows
        feats = []
        for sd in seeds:
            st = model(sd)
            feats.append(st.features())
            st.close()
        mean, std = warmstart.feature_norm(feats)
        for k, sd in enumerate(seeds):
            st = model(sd)
            X, T, rep = warmstart.converged_rows(st, mean, std, tol=1e-6, sample=args.train_sample)
            rows.append((X, T))
            st.close()
            log(f"training model {k + 1}/{len(seeds)} (seed {sd}): {rep['iterations']} iterations")
    t_data = time.perf_counter() - t0
    t0 = time.perf_counter()
    curve = warmstart.train(s, rows, mean, std, warmstart.SCHEDULE, batch=4096, seed=1)
    t_train = time.perf_counter() - t0
    n_rows = sum(int(r[0].shape[0]) for r in rows)
    s._bench_rows = rows   # kept for the kernel timing of training steps
    log(f"warm start: {len(seeds)} training models, {n_rows} rows, data {t_data:.1f} s, "
        f"training {t_train:.1f} s, loss {curve[:5].mean():.3e} -> {curve[-50:].mean():.3e}")
    return {"train_models": len(seeds), "train_seeds": seeds, "rows": n_rows, "data_s": t_data,
            "train_s": t_train, "steps": int(curve.shape[0]), "batch": 4096,
            "loss_start": float(curve[:5].mean()), "loss_end": float(curve[-50:].mean())}


def ali_forms(s, w, make, args, dev):
    """ALI wall time and iterations to a maximum relative change of 1e-4 from LTE and from
    the learned start, in FP64 and in the FP32 form, each against FP64 populations
    converged to 1e-9."""
    import numpy as np
    import torch
    ntot = w.model.abundance * w.model.n_h2
    out = torch.empty((w.n_points, w.species.n_lev), dtype=torch.float64, device=dev)
    s.set_params(precision="fp64", tol=1e-9, max_iter=500)
    rep = s.run_ali_dev(None, out)
    torch.cuda.synchronize()
    ref = out.cpu().numpy()
    res = {"tol": 1e-4, "reference": {"precision": "fp64", "tol": 1e-9, "iterations": rep["iterations"],
                                      "converged": rep["converged"]},
           "models": w.n_models, "graph": True}
    warm = None
    if training_factory(args, make)[0] is not None and args.train_models > 0:
        res["warm_start"] = train_warm_start(s, w, make, args, dev)
        warm = True
    forms = [("fp64", "lte"), ("fp32", "lte")] + ([("fp64", "warm"), ("fp32", "warm")] if warm else [])
    for prec, start in forms:
        s.set_params(precision=prec, tol=1e-4, max_iter=200)
        best = None
        for _ in range(max(1, args.ali_runs)):   # best of the runs: the first captures the graphs
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if start == "lte":
                r = s.run_ali_dev(None, out)
            else:
                r = s.run_ali_warm_dev(out)
            torch.cuda.synchronize()
            wall = time.perf_counter() - t0
            if best is None or wall < best[0]:
                best = (wall, r)
        wall, r = best
        err = _rel_err(out.cpu().numpy(), ref, ntot)
        key = f"{prec}_{start}"
        its = s.model_status()[0]
        res[key] = {"iterations": r["iterations"], "converged": r["converged"], "wall_s": wall,
                    "model_iterations": {int(k): int(v) for k, v in zip(*np.unique(its, return_counts=True))},
                    "max_rel_diff_vs_fp64_reference": err,
                    "models_converged": r["n_models_converged"],
                    "max_change": [float(c) for c in r["max_change"]]}
        if start == "warm":
            res[key]["used_network"] = r["used_network"]
        log(f"ALI {key}: {r['iterations']} iterations (models: {res[key]['model_iterations']}), "
            f"{wall * 1e3:.1f} ms, max rel diff vs FP64 reference {err:.2e}, "
            f"changes {['%.2e' % c for c in r['max_change']]}")
    if warm:
        # the combination the method is aimed at: FP32 bulk from the learned start against
        # plain FP64 from LTE, on the same model(s)
        a, b = res["fp32_warm"], res["fp64_lte"]
        res["fp32_warm_vs_fp64_lte"] = {"iterations": [a["iterations"], b["iterations"]],
                                        "wall_ratio": a["wall_s"] / b["wall_s"],
                                        "max_rel_diff_vs_fp64_reference": a["max_rel_diff_vs_fp64_reference"]}
        res["mlp"] = mlp_timing(s, w, dev)
    if not args.no_variants:
        res.update(ali_variants(s, w, out, ref, ntot, args.ali_runs))
    s.set_params(precision=args.precision)
    return res


def _timed_ali(s, out, runs):
    import torch
    best = None
    for _ in range(max(1, runs)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = s.run_ali_dev(None, out)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        if best is None or wall < best[0]:
            best = (wall, r)
    return best


def line_centre_opacity(s, w):
    """Median over points of each line's centre opacity with LTE populations [cm^-1]
    (an input scale for the scattering opacity)."""
    import numpy as np
    h, c, kb = 6.62607015e-27, 2.99792458e10, 1.380649e-16
    sp = w.species
    pops = s.lte()
    nu = (sp.energy[sp.line_up] - sp.energy[sp.line_lo]) / h
    bul = sp.line_A * c ** 2 / (2 * h * nu ** 3)
    blu = sp.weight[sp.line_up] / sp.weight[sp.line_lo] * bul
    vw = np.sqrt(2 * kb * w.model.temperature / (sp.mass) + w.model.v_turb ** 2)
    kchi = h * nu / (4 * np.pi) * (pops[:, sp.line_lo] * blu - pops[:, sp.line_up] * bul)
    return np.median(kchi / (np.sqrt(np.pi) * nu * vw[:, None] / c), axis=0)


def image_timing(s, w, pops, n_ch=64, runs=3):
    """Channel images (Sec. 3.5) of the line with index 0 along the first ray, from the
    populations `pops` (device), at n_ch channel velocities over +-(largest speed + 4 largest
    line widths). The work unit is the elimination step of one channel along the pair
    through a point; the steps of that pair over all points come from a solver traced with
    this direction and its antipode only (the walks depend only on the direction and the
    neighbours, so they are the same walks)."""
    import copy

    import numpy as np
    import torch
    from paper_1912_08445_amd.binding import Solver
    dirs = s.get_rays()
    rb = int(np.argmin(np.abs(dirs + dirs[0]).sum(axis=1)))
    w2 = copy.copy(w)
    w2.rays = dirs[[0, rb]].copy()
    s2 = Solver(0)
    s2.setup(w2)
    steps = s2.trace_stats()[2]
    s2.close()
    vmax = float(np.sqrt((w.model.vel ** 2).sum(axis=1)).max() + 4.0 * s.line_width_speed().max())
    v_ch = np.linspace(-vmax, vmax, n_ch)
    I = torch.empty((w.n_points, n_ch), dtype=torch.float64, device=pops.device)
    xy = torch.empty((w.n_points, 2), dtype=torch.float64, device=pops.device)
    s.image_dev(pops, 0, 0, v_ch, I, xy)
    torch.cuda.synchronize()
    s.set_params(profile=1)
    s.reset_kernel_stats()
    for _ in range(runs):
        s.image_dev(pops, 0, 0, v_ch, I, xy)
    torch.cuda.synchronize()
    s.set_params(profile=0)
    ms, n = s.kernel_stats("image")
    ms /= n
    node_ch = steps * n_ch
    tf = node_ch * FLOPS_PER_STEP / (ms * 1e-3) / 1e12
    r = {"channels": n_ch, "v_max_cm_s": vmax, "ray": 0, "line": 0, "kernel": "k_image", "kernel_ms": ms,
         "node_channel_per_launch": node_ch, "point_channel_per_s": w.n_points * n_ch / (ms * 1e-3),
         "roofline": {"bound": "alu", "achieved": tf, "peak": PEAK_FP64_TFLOPS, "unit": "TFLOP/s",
                      "frac": tf / PEAK_FP64_TFLOPS, "flops_per_node_channel": FLOPS_PER_STEP}}
    log(f"image: {n_ch} channels, k_image {ms:.3f} ms, {node_ch} node*channel steps, {tf:.1f} TFLOP/s "
        f"({100 * tf / PEAK_FP64_TFLOPS:.1f}% of FP64 peak)")
    return r


def ali_variants(s, w, out, ref, ntot, runs):
    """FP64 from LTE with Ng acceleration (M = 4) and with the band ALO, against the same
    reference; the ALI with a grey scattering opacity of half the median line-centre
    opacity (different physics: its own iterations, wall time and formal-solve time); and
    channel images of the converged reference populations."""
    import numpy as np
    import torch
    res = {}
    for key, extra in (("fp64_lte_ng4", {"ng_every": 4}), ("fp64_lte_band", {"alo_band": 1})):
        s.set_params(precision="fp64", tol=1e-4, max_iter=200, **extra)
        wall, r = _timed_ali(s, out, runs)
        err = _rel_err(out.cpu().numpy(), ref, ntot)
        res[key] = {"iterations": r["iterations"], "converged": r["converged"], "wall_s": wall,
                    "max_rel_diff_vs_fp64_reference": err, "n_ng_steps": r["n_ng_steps"],
                    "n_band": r["n_band"], "max_change": [float(c) for c in r["max_change"]]}
        log(f"ALI {key}: {r['iterations']} iterations, {wall * 1e3:.1f} ms, max rel diff vs FP64 "
            f"reference {err:.2e}")
        s.set_params(ng_every=0, alo_band=0)
    chi = np.broadcast_to(0.5 * line_centre_opacity(s, w), (w.n_points, w.species.n_lines)).copy()
    s.set_scattering(chi)
    s.set_params(precision="fp64", tol=1e-4, max_iter=200)
    wall, r = _timed_ali(s, out, runs)
    s.set_params(profile=1)
    s.reset_kernel_stats()
    s.set_params(max_iter=1, tol=0.0)
    s.run_ali_dev(None, out)
    torch.cuda.synchronize()
    f_ms, f_n = s.kernel_stats("formal_solve")
    s.set_params(profile=0, max_iter=200, tol=1e-4)
    s.set_scattering(None)
    res["fp64_lte_scattering"] = {"chi_sca": "0.5 x median line-centre opacity (LTE) of each line, grey, isotropic",
                                  "iterations": r["iterations"], "converged": r["converged"], "wall_s": wall,
                                  "formal_solve_ms": f_ms / f_n,
                                  "max_change": [float(c) for c in r["max_change"]]}
    log(f"ALI with scattering: {r['iterations']} iterations, {wall * 1e3:.1f} ms, formal solve "
        f"{f_ms / f_n:.1f} ms per sweep")
    out.copy_(torch.from_numpy(ref).to(out.device))
    res["image"] = image_timing(s, w, out)
    return res


def mlp_timing(s, w, dev, steps=50):
    """Per-kernel HIP-event times of prediction (features, network forward over every
    point) and of training steps, with algorithmic throughput against the dense BF16
    matrix-core peak."""
    import torch
    n_out = w.species.n_lev
    fwd_f, train_f = mlp_flops_per_row(n_out)
    out = torch.empty((w.n_points, n_out), dtype=torch.float64, device=dev)
    X = torch.cat([r[0] for r in s._bench_rows]).contiguous()
    T = torch.cat([r[1] for r in s._bench_rows]).contiguous()
    s.set_params(profile=1)
    s.reset_kernel_stats()
    for _ in range(3):
        s.mlp_predict_dev(out)
    s.mlp_train_dev(X, T, steps=steps, batch=4096, lr=2e-4)
    torch.cuda.synchronize()
    f_ms, f_n = s.kernel_stats("mlp_forward")
    ft_ms, _ = s.kernel_stats("features")
    t_ms, t_n = s.kernel_stats("mlp_train")
    u_ms, _ = s.kernel_stats("mlp_update")
    # the same kernels on the largest batch the library takes (65,536 rows): what they reach
    # once a step has work for the whole chip (the 4096-row steps the training uses are
    # bound by the latency of their dependent stages); lr = 0 leaves the weights unchanged
    big = min(65536, X.shape[0])
    s.reset_kernel_stats()
    s.mlp_train_dev(X, T, steps=10, batch=big, lr=0.0)
    torch.cuda.synchronize()
    s.set_params(profile=0)
    bt_ms, bt_n = s.kernel_stats("mlp_train")
    bu_ms, _ = s.kernel_stats("mlp_update")
    fwd_ms, tr_ms, up_ms = f_ms / f_n, t_ms / t_n, u_ms / t_n
    fwd_tf = fwd_f * w.n_points / (fwd_ms * 1e-3) / 1e12
    # "train": the forward/backward and weight-gradient kernels of one step; "step": with
    # the update kernel (chunk sums, Adam, operand packing) as well
    tr_tf = train_f * 4096 / (tr_ms * 1e-3) / 1e12
    st_tf = train_f * 4096 / ((tr_ms + up_ms) * 1e-3) / 1e12
    r = {"rows_forward": w.n_points, "forward_ms": fwd_ms, "features_ms": ft_ms / f_n,
         "forward_tflops": fwd_tf, "forward_mfma_frac": fwd_tf / PEAK_BF16_MFMA_TFLOPS,
         "train_batch": 4096, "train_kernel_ms": tr_ms, "update_ms": up_ms,
         "train_tflops": tr_tf, "train_mfma_frac": tr_tf / PEAK_BF16_MFMA_TFLOPS,
         "train_step_ms": tr_ms + up_ms, "train_step_mfma_frac": st_tf / PEAK_BF16_MFMA_TFLOPS,
         "large_batch": {"rows": big, "train_kernel_ms": bt_ms / bt_n, "update_ms": bu_ms / bt_n,
                         "train_tflops": train_f * big / (bt_ms / bt_n * 1e-3) / 1e12,
                         "train_mfma_frac": train_f * big / (bt_ms / bt_n * 1e-3) / 1e12 / PEAK_BF16_MFMA_TFLOPS},
         "flops_per_row": {"forward": fwd_f, "train": train_f}, "peak_tflops": PEAK_BF16_MFMA_TFLOPS}
    log(f"mlp: forward {fwd_ms:.3f} ms for {w.n_points} rows ({fwd_tf:.1f} TFLOP/s), features "
        f"{ft_ms / f_n:.3f} ms; train step {tr_ms:.3f} + {up_ms:.3f} ms ({tr_tf:.1f} TFLOP/s, "
        f"{st_tf:.1f} with the update); {big}-row step {bt_ms / bt_n:.3f} + {bu_ms / bt_n:.3f} ms "
        f"({train_f * big / (bt_ms / bt_n * 1e-3) / 1e12:.1f} TFLOP/s)")
    return r


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="disc10", choices=["disc10", "outflow5", "sphere2", "batch256", "discs"])
    ap.add_argument("--autotune", default=None, metavar="CACHE",
                    help="pick the formal-solve launch variant by timing (cache file path)")
    ap.add_argument("--points", type=int, default=None, help="override the point count")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "fp32"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ali", action="store_true")
    ap.add_argument("--ali-runs", type=int, default=None,
                    help="runs per ALI form, the fastest reported (the first also captures the graphs); "
                         "default 1 for disc10, else 3")
    ap.add_argument("--fp32-steps", type=int, default=2, help="timed sweeps of the FP32-bulk form")
    ap.add_argument("--no-held-out", action="store_true", help="skip the disc family's held-out warm-start block")
    ap.add_argument("--disc-points", type=int, default=100000,
                    help="points of each disc of the held-out warm-start block")
    ap.add_argument("--no-variants", action="store_true",
                    help="skip the Ng, band-ALO and scattering ALI forms and the image timing")
    ap.add_argument("--train-models", type=int, default=None,
                    help="other seeds of the workload (of the disc family for disc10) whose converged "
                         "populations train the warm start (0: no warm start; default 20 for disc10, "
                         "48 for discs, else 8)")
    ap.add_argument("--train-sample", type=int, default=None,
                    help="rows taken from each training model (default: every point of the disc family's "
                         "training discs for disc10, else 20000)")
    ap.add_argument("--mlp-only", action="store_true",
                    help="only the warm-start network's kernels (seeded weights, synthetic rows) on the workload")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="only run a plain device-to-device copy of this many MiB (4 launches), "
                         "the calibration kernel for HBM byte counters")
    args = ap.parse_args()
    if args.train_models is None:
        args.train_models = {"discs": 48, "disc10": 20}.get(args.workload, 8)
    if args.train_sample is None:
        args.train_sample = args.disc_points if args.workload == "disc10" else 20000
    if args.ali_runs is None:
        args.ali_runs = 1 if args.workload == "disc10" else 3
    if args.workload == "disc10":
        args.no_variants = True

    if args.copy_probe_mib > 0:
        import torch
        n = args.copy_probe_mib * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda:0")
        b = torch.empty_like(a)
        for _ in range(4):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": 8 * n, "copy_probe_bytes_written": 8 * n,
                          "launches": 4}))
        return

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the method shards by "
              "origin point across GPUs but this benchmark measures a single MI355X.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1912_08445_amd.binding import Solver
    from synth import configs

    make = {"outflow5": configs.outflow5, "sphere2": configs.sphere2, "disc10": configs.disc10,
            "batch256": configs.batch256, "discs": configs.discs}[args.workload]
    t0 = time.perf_counter()
    if args.points is None:
        w = make()
    elif args.workload == "batch256":
        w = make(n_models=args.points)
    else:
        w = make(n_points=args.points)
    log(f"workload {w.name}: {w.n_points} points, {w.rays.shape[0]} rays, {w.species.n_lines} lines x "
        f"{w.quad_x.shape[0]} freqs ({time.perf_counter() - t0:.1f} s to generate)")

    s = Solver(0)
    t0 = time.perf_counter()
    s.setup(w, precision=args.precision)
    total_cells, max_len, steps_per_freq = s.trace_stats()
    log(f"traced in {time.perf_counter() - t0:.2f} s: {total_cells} cells, longest ray {max_len}, "
        f"{steps_per_freq} elimination steps per frequency")
    tuned = None
    if args.autotune:
        t0 = time.perf_counter()
        tuned = s.autotune(args.autotune, trials=3)
        log(f"autotune: {tuned} ({time.perf_counter() - t0:.1f} s)")

    dev = torch.device("cuda:0")
    P, nlev, nl = w.n_points, w.species.n_lev, w.species.n_lines
    if args.mlp_only:
        import numpy as np
        # the network's kernels alone: seeded Glorot weights, unit standardisation, 131,072
        # seeded synthetic rows (inputs and targets standard normal); prints the mlp object
        s.mlp_init(nlev, seed=1)
        s.mlp_set_norm(np.zeros(8), np.ones(8))
        g = torch.Generator(device="cpu").manual_seed(7)
        X = torch.randn((131072, 8), generator=g, dtype=torch.float32).to(dev)
        T = torch.randn((131072, nlev), generator=g, dtype=torch.float32).to(dev)
        s._bench_rows = [(X, T)]
        print(json.dumps({"workload": w.name, "mlp": mlp_timing(s, w, dev)}), flush=True)
        return
    pops = torch.empty((P, nlev), dtype=torch.float64, device=dev)
    new = torch.empty_like(pops)
    J, Je, L = [torch.empty((P, nl), dtype=torch.float64, device=dev) for _ in range(3)]
    s.lte_dev(pops)
    torch.cuda.synchronize()

    bufs = [pops, new]

    def step():
        # one ALI iteration: populations bufs[0] -> bufs[1], then swap
        s.formal_solve_dev(bufs[0], J, Je, L)
        s.stateq_dev(bufs[0], J, Je, L, bufs[1])
        bufs.reverse()

    for i in range(args.warmup):
        step()
        if P >= 200000:
            torch.cuda.synchronize()
            log(f"  warmup step {i + 1}/{args.warmup}")
    torch.cuda.synchronize()
    log(f"warmup done ({args.warmup} steps)")

    # timed region: HIP events on torch's current (default) stream; the library calls
    # above get that stream's handle 0 and run on the context's stream, which is ordered
    # with the default stream both ways; per-kernel HIP events inside the library
    s.set_params(profile=1)
    s.reset_kernel_stats()
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for i in range(args.steps):
        step()
        if (i + 1) % 5 == 0 and i + 1 < args.steps:
            log(f"  timed step {i + 1}/{args.steps}")
    ev1.record(stream)
    torch.cuda.synchronize()
    ms_total = ev0.elapsed_time(ev1)
    s.set_params(profile=0)
    ms_step = ms_total / args.steps
    k_ms, k_n = s.kernel_stats("formal_solve")
    k_avg = k_ms / max(k_n, 1)
    exec_per_launch = s.executed_steps() / max(k_n, 1)
    lc_ms, _ = s.kernel_stats("line_coef")
    se_ms, _ = s.kernel_stats("stateq")
    log(f"step {ms_step:.3f} ms; formal_solve kernel {k_avg:.3f} ms avg over {k_n} launches; "
        f"line_coef {lc_ms / max(k_n, 1):.3f} ms; stateq {se_ms / max(k_n, 1):.3f} ms")

    units = P * w.rays.shape[0] * nl * w.quad_x.shape[0]
    value = units / (ms_step * 1e-3)
    launch = s.launch()
    node_freq = steps_per_freq * nl * w.quad_x.shape[0]
    # the kernel collapses far-wing segments (zero opacity throughout) into one step, so
    # the flops it performs are counted on the steps it executes, not the method's
    flops = exec_per_launch * FLOPS_PER_STEP
    achieved = flops / (k_avg * 1e-3) / 1e12
    peak = PEAK_FP64_TFLOPS
    roof = {"bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
            "frac": achieved / peak,
            "traffic": traffic_from_profile(w.name, args.precision, node_freq),
            "kernel": "k_formal_solve", "kernel_ms": k_avg, "node_freq_per_launch": node_freq,
            "executed_node_freq_per_launch": exec_per_launch,
            "flops_per_node_freq": FLOPS_PER_STEP}

    # the FP32-bulk form's sweep on the same model
    fp32_form = None
    if args.precision == "fp64" and args.fp32_steps > 0:
        s.set_params(precision="fp32")
        s.lte_dev(pops)
        s.formal_solve_dev(pops, J, Je, L)
        torch.cuda.synchronize()
        s.set_params(profile=1)
        s.reset_kernel_stats()
        for _ in range(args.fp32_steps):
            s.formal_solve_dev(pops, J, Je, L)
        torch.cuda.synchronize()
        f_ms, f_n = s.kernel_stats("formal_solve")
        f_exec = s.executed_steps() / max(f_n, 1)
        f_launch = s.launch()
        s.set_params(profile=0, precision="fp64")
        f_ms /= max(f_n, 1)
        f_tf = f_exec * FLOPS_PER_STEP / (f_ms * 1e-3) / 1e12
        fp32_form = {"kernel_ms": f_ms, "value": units / (f_ms * 1e-3), "unit": "point*ray*freq/s (kernel time)",
                     "executed_node_freq_per_launch": f_exec, "achieved_tflops": f_tf,
                     "frac_of_fp64_peak": f_tf / PEAK_FP64_TFLOPS, "launch": f_launch}
        log(f"FP32-bulk form: formal_solve kernel {f_ms:.3f} ms ({f_tf:.1f} TFLOP/s by the 17-flop count)")

    ali = None
    if not args.no_ali:
        ali = ali_forms(s, w, make, args, dev)

    held = None
    if args.workload == "disc10" and not (args.no_ali or args.no_held_out) and args.train_models > 0:
        s.close()   # one million-point model less in HBM while the block runs
        held = held_out_discs(args, dev)

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        cpu = cpu_baseline(w)
        log(f"cpu baseline {cpu['value']:.3e} {cpu['unit']} on {cpu['cores']} threads")

    desc = (f"{w.name}: {P} points, {w.rays.shape[0]} HEALPix rays, {nl} lines x "
            f"{w.quad_x.shape[0]} frequencies, {nlev} levels")
    line = {
        "metric": "formal-solve (point*ray*freq)/s; ALI wall time to 1e-4 convergence vs FP64",
        "value": value,
        "unit": "point*ray*freq/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": desc, "points": P, "rays": int(w.rays.shape[0]), "lines": nl,
                   "frequencies": int(w.quad_x.shape[0]), "levels": nlev,
                   "precision": args.precision, "cells_cached": total_cells,
                   "node_freq_per_sweep": node_freq, "models": w.n_models, "launch": launch,
                   "autotuned": tuned},
        "node_freq_per_s": node_freq / (ms_step * 1e-3),
        "roofline": roof,
        "cpu_baseline": cpu,
        "fp32_form": fp32_form,
        "ali": ali,
        "held_out_warm_start": held,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
