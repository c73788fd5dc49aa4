"""The allocation-free formal solve (nlte_formal_solve_noalloc_dev) against the regular
device entry point: the same kernels on the same inputs, so the results must be
identical, over two calls in a row on one GPU (the second on a smaller model, after the
shared scratch held the first's data), in both precision forms and in the persistent
launch (whose work counter lives in the scratch), inside a captured graph, and a model
too large for the fixed scratch rejected with an error."""
import numpy as np
import pytest

from synth import configs, species
from synth.models import chain_1d

from _common import solver_for

pytestmark = pytest.mark.gpu


def run_both(s, w, pops):
    import torch
    P, nl = w.n_points, w.species.n_lines
    out = []
    for fn in (s.formal_solve_dev, s.formal_solve_noalloc_dev):
        J, Je, L = (torch.full((P, nl), np.nan, dtype=torch.float64, device="cuda:0") for _ in range(3))
        fn(pops, J, Je, L)
        torch.cuda.synchronize()
        out.append([t.cpu().numpy() for t in (J, Je, L)])
    return out


def test_noalloc_matches_formal_solve_dev_two_calls():
    import torch
    dev = torch.device("cuda:0")
    big = configs.outflow5(n_points=3000, seed=41, nside=1)
    small = configs.sphere2(n_points=400, seed=5)
    print("no-alloc: outflow5 3000 points then sphere2 400 points", flush=True)
    for w, params in ((big, {}), (big, dict(precision="fp32", persistent=1)), (small, {})):
        s = solver_for(w, **params)
        pops = torch.tensor(s.lte(), device=dev)
        ref, got = run_both(s, w, pops)
        for a, b in zip(ref, got):
            assert np.isfinite(a).all()
            assert np.array_equal(a, b)
        s.close()


def test_noalloc_in_a_captured_graph():
    import torch
    dev = torch.device("cuda:0")
    w = configs.outflow5(n_points=1500, seed=43, nside=1)
    s = solver_for(w)
    lte = torch.tensor(s.lte(), device=dev)
    P, nl = w.n_points, w.species.n_lines
    pops = lte.clone()
    J, Je, L = (torch.zeros((P, nl), dtype=torch.float64, device=dev) for _ in range(3))
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        s.formal_solve_noalloc_dev(pops, J, Je, L)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        s.formal_solve_noalloc_dev(pops, J, Je, L)
    for k in range(3):
        pops.copy_(lte * (1.0 + 0.1 * k))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        got = [t.cpu().numpy() for t in (J, Je, L)]
        a, b, c = (torch.empty_like(J) for _ in range(3))
        s.formal_solve_dev(pops, a, b, c)
        torch.cuda.synchronize()
        for x, y in zip(got, (a, b, c)):
            assert np.array_equal(x, y.cpu().numpy())


def test_noalloc_rejects_models_beyond_the_scratch():
    """300,000 points x 15 lines x 16 bytes exceed the 64 MiB staging: an error, no launch.
    Every point is flagged as boundary, so each walk stops after one cell and the trace
    stays small."""
    import torch
    from paper_1912_08445_amd.binding import NLTE_E_INVALID_ARG, NlteError
    from synth import directions
    from synth.configs import Workload
    P = 300_000
    sp = species.linear_rotor(16)
    m = chain_1d(np.arange(P, dtype=np.float64) * 1e14, np.zeros(P), 1e4, 20.0, 1.5e4, 1e-8)
    m.boundary = np.ones(P, dtype=np.uint8)
    q = directions.uniform_grid(31, 4.0)
    w = Workload("chain", m, sp, directions.axis_pair(), q[0], q[1])
    s = solver_for(w)
    dev = torch.device("cuda:0")
    pops = torch.zeros((P, sp.n_lev), dtype=torch.float64, device=dev)
    J, Je, L = (torch.zeros((P, sp.n_lines), dtype=torch.float64, device=dev) for _ in range(3))
    with pytest.raises(NlteError) as e:
        s.formal_solve_noalloc_dev(pops, J, Je, L)
    assert e.value.code == NLTE_E_INVALID_ARG and "scratch" in str(e.value)
    torch.cuda.synchronize()
    assert float(J.abs().max()) == 0.0
    s.close()
