"""Pins of the band-ALO oracle: the band entries against a dense inverse, the coupled rate
equations without couplings against the local solve, and the ALI fixed point."""
import numpy as np

import oracle
from oracle import band
from synth import configs, directions, species
from synth.configs import Workload
from synth.models import chain_1d

from _common import oracle_for, rel
from test_oracle_pins import dense_system


def _chain(n=9):
    # static chain with uneven spacing and varying density: every node is a cell (t = 1)
    rng = np.random.default_rng(3)
    x = np.cumsum(rng.uniform(0.5, 1.5, n)) * 2e15
    nh2 = 10.0 ** rng.uniform(3.5, 5.0, n)
    m = chain_1d(x, np.zeros(n), nh2, 25.0, 1.5e4, 1e-7)
    xq, wq = directions.uniform_grid(9, 3.0)
    return Workload("chain", m, species.two_level(100e9, 3.0, 1e-5, 1e-10, 28.0), directions.axis_pair(), xq, wq)


def test_band_entries_match_the_dense_inverse():
    w = _chain()
    o = oracle_for(w)
    pops = o.lte() * np.linspace(0.7, 1.3, w.n_points)[:, None]
    pops *= ((w.model.abundance * w.model.n_h2) / pops.sum(1))[:, None]
    O = 4
    J, Je, L, Jb, Ld, Ln = o.formal_solve_band(pops, sel=[O])
    nd = o.pair_nodes(pops, O, 0)
    z, a, b, kap, S, io = nd["z"], nd["a"], nd["b"], nd["kappa"][:, 0], nd["S"][:, 0], nd["o"]
    Ib = oracle.planck(100e9, 2.725)
    lm, lp, ld, jb = 0.0, 0.0, 0.0, 0.0
    for xq, wq in zip(w.quad_x, w.quad_w):
        x = a * xq - b
        T, R = dense_system(z, kap * np.exp(-x * x), S, Ib, Ib)
        Ti = np.linalg.inv(T)
        u = Ti @ R
        lm += wq * Ti[io, io - 1]
        lp += wq * Ti[io, io + 1]
        ld += wq * Ti[io, io]
        jb += wq * (u[io] - Ti[io, io] * S[io] - Ti[io, io - 1] * S[io - 1] - Ti[io, io + 1] * S[io + 1])
    # two rays, one pair: the average is the plain quadrature sum; the static chain has
    # no sub-steps, so the neighbours are cells and add nothing to the diagonal
    assert rel(Ln[0, 0, 0], lp) < 1e-11 and rel(Ln[0, 0, 1], lm) < 1e-11
    assert rel(Ld[0, 0], ld) < 1e-11 and rel(L[0, 0], ld) < 1e-11
    assert rel(Jb[0, 0], jb) < 1e-8


def test_neighbour_share_of_a_substep_node_goes_to_the_diagonal():
    # with velocity sub-steps next to the origin, the neighbour node interpolates the
    # origin's own source function: Ld exceeds L and the coupling to the cell shrinks
    w = configs.outflow5(n_points=300, seed=2, nside=1)
    o = oracle_for(w)
    J, Je, L, Jb, Ld, Ln = o.formal_solve_band(o.lte(), sel=np.arange(20))
    assert np.all(Ld >= L) and np.any(Ld > L * (1 + 1e-6))
    assert np.all(Ln >= 0) and np.all(Jb <= Je * (1 + 1e-12))


def test_rate_equations_without_couplings_equal_the_local_solve():
    w = configs.outflow5(n_points=200, seed=5, nside=1)
    o = oracle_for(w)
    pops = o.lte()
    J, Je, L = o.formal_solve(pops)
    M, rhs = band.assemble(o, pops, Je, L, np.zeros((o.P, w.species.n_lines, o.n_rays)), None, band=False)
    import scipy.sparse.linalg as spla
    x = spla.spsolve(M.tocsc(), rhs).reshape(o.P, -1)
    ref, flags = o.stateq(pops, J, Je, L)
    assert np.all(flags == 0)
    assert rel(x, ref).max() < 1e-11


def test_band_ali_keeps_thermal_equilibrium():
    w = configs.sphere2(n_points=120, seed=3)
    w.model.temperature[:] = 2.725
    w.model.abundance[:] = 1e-6
    o = oracle_for(w)
    lte = o.lte()
    pops, ch, used = band.run_ali_band(o, max_iter=2, tol=0.0)
    assert all(used) and rel(pops, lte).max() < 1e-12


def test_band_ali_reaches_the_local_fixed_point_in_fewer_iterations():
    # optically thick two-level sphere: the ALO terms cancel at convergence, so both
    # operators share the fixed point; the band converges faster
    w = configs.sphere2(n_points=300, seed=9)
    w.model.abundance[:] = 1e-6
    o = oracle_for(w)
    plain, ch_plain = o.run_ali(max_iter=300, tol=1e-10)
    acc, ch_band, used = band.run_ali_band(o, max_iter=300, tol=1e-10)
    assert ch_band[-1] < 1e-10 and all(used)
    assert rel(acc, plain).max() < 1e-8
    assert len(ch_band) < len(ch_plain)
