"""The device entry points on a caller's stream inside a caller's graph: a torch CUDA
graph captures the formal solve and the stat-eq, and every replay, with eager work and
new input values between replays, matches the eager calls exactly."""
import numpy as np
import pytest

from synth import configs

from _common import solver_for

pytestmark = pytest.mark.gpu


def test_caller_captured_formal_solve_and_stateq():
    import torch
    w = configs.outflow5(n_points=1500, seed=31, nside=1)
    s = solver_for(w)
    dev = torch.device("cuda:0")
    lte = torch.tensor(s.lte(), device=dev)
    P, nl, nv = w.n_points, w.species.n_lines, w.species.n_lev
    pops = lte.clone()
    J, Je, L = (torch.zeros((P, nl), dtype=torch.float64, device=dev) for _ in range(3))
    new = torch.zeros((P, nv), dtype=torch.float64, device=dev)

    def eager(p):
        a, b, c = (torch.empty_like(J) for _ in range(3))
        n = torch.empty_like(new)
        s.formal_solve_dev(p, a, b, c)
        s.stateq_dev(p, a, b, c, n)
        torch.cuda.synchronize()
        return a, b, c, n

    # warm the stream once outside the capture (torch's advice for graph capture)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        s.formal_solve_dev(pops, J, Je, L)
        s.stateq_dev(pops, J, Je, L, new)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        s.formal_solve_dev(pops, J, Je, L)
        s.stateq_dev(pops, J, Je, L, new)
    rng = np.random.default_rng(4)
    for k in range(4):
        scale = torch.tensor(rng.uniform(0.8, 1.2, (P, nv)), device=dev)
        trial = lte * scale
        ref = eager(trial)
        for t in (J, Je, L, new):
            t.fill_(-1.0)                       # eager work between replays
        pops.copy_(trial)
        g.replay()
        torch.cuda.synchronize()
        for got, want in zip((J, Je, L, new), ref):
            assert torch.equal(got, want), k
