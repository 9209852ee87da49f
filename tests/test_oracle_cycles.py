"""Pins of the oracle's F- and W-cycle arrangements (Sec. 3.2.1,
fig:multigrid_cycles), CPU only.

The schedules are pinned by the walk over the levels that the figure draws
for four levels (V: h 2h 4h 8h 4h 2h h; F and W as the textbook recursions
give them), by visit counts that follow from the recursions in closed form,
by the two-level case where F and W must coincide exactly, and by the fixed
point: every arrangement converges to the same discrete solution, which the
V-cycle pins of test_oracle_pins already tie to Newton, FFT and exact
solutions."""
import numpy as np
import pytest

import inputs
import oracle

OM = 0.3089


def test_four_level_walks_match_the_figure():
    # levels 32, 16, 8, 4: the 4-level picture with h the finest cell
    assert oracle.cycle_trace(32, oracle.CYCLE_V) == [0, 1, 2, 3, 2, 1, 0]
    assert oracle.cycle_trace(32, oracle.CYCLE_F) == [0, 1, 2, 3, 2, 3, 2, 1, 2, 3, 2, 1, 0]
    assert oracle.cycle_trace(32, oracle.CYCLE_W) == [0, 1, 2, 3, 2, 3, 2, 1, 2, 3, 2, 3, 2, 1, 0]


@pytest.mark.parametrize("n,nlev", [(16, 3), (32, 4), (64, 5), (128, 6)])
def test_visit_counts_follow_the_recursions(n, nlev):
    # merged walks: a V-cycle goes down and up once; the W-cycle's walk has
    # 2^(levels-1) dips to the coarsest level; the F-cycle's has levels-1
    def dips(walk):
        return sum(1 for q in walk if q == nlev - 1)
    v = oracle.cycle_trace(n, oracle.CYCLE_V)
    f = oracle.cycle_trace(n, oracle.CYCLE_F)
    w = oracle.cycle_trace(n, oracle.CYCLE_W)
    assert v == list(range(nlev)) + list(range(nlev - 2, -1, -1))
    assert dips(v) == 1
    assert dips(w) == 2 ** (nlev - 2)
    assert dips(f) == nlev - 1
    for walk in (v, f, w):
        assert walk[0] == 0 and walk[-1] == 0
        assert all(abs(a - b) == 1 for a, b in zip(walk, walk[1:]))


def test_two_level_f_and_w_coincide():
    # with levels 8 and 4 both arrangements run two coarsest solves per cycle
    n = 8
    delta = inputs.lognormal_delta(n, 5)
    m = oracle.dgp_model(1.0, OM, 1.0)
    f = oracle.solve(m, delta, tol=0.0, max_cycles=3, cycle=oracle.CYCLE_F)
    w = oracle.solve(m, delta, tol=0.0, max_cycles=3, cycle=oracle.CYCLE_W)
    v = oracle.solve(m, delta, tol=0.0, max_cycles=3, cycle=oracle.CYCLE_V)
    assert np.array_equal(f.phi, w.phi)
    assert f.hist == w.hist
    assert not np.array_equal(f.phi, v.phi)


@pytest.mark.parametrize("name", ["dgp", "kmo3"])
def test_all_arrangements_reach_the_same_solution(name):
    n = 32
    delta = inputs.lognormal_delta(n, 1)
    m = (oracle.dgp_model(1.0, OM, 1.0) if name == "dgp"
         else oracle.kmo_model(n, 0.02 * n, 3, 1.0, 0.1))
    # converged far below the size of phi (|phi| ~ 1e-5 for this Kmouflage case)
    ref = oracle.solve(m, delta, tol=1e-14, max_cycles=80)
    assert ref.status == 0
    for cyc in (oracle.CYCLE_F, oracle.CYCLE_W):
        r = oracle.solve(m, delta, tol=1e-14, max_cycles=80, cycle=cyc)
        assert r.status == 0
        assert np.abs(r.phi - ref.phi).max() <= 1e-9 * np.abs(ref.phi).max()
        # more coarse work per cycle: no more cycles than the V-cycle needs
        assert r.cycles <= ref.cycles


def test_f_and_w_contract_faster_per_cycle():
    # the first cycle's mid-cycle residual: F and W solve the coarse problem
    # more accurately than V, so the second cycle starts lower
    n = 64
    delta = inputs.lognormal_delta(n, 3)
    m = oracle.dgp_model(1.0, OM, 1.0)
    h = {c: oracle.solve(m, delta, tol=0.0, max_cycles=3, cycle=c).hist
         for c in (oracle.CYCLE_V, oracle.CYCLE_F, oracle.CYCLE_W)}
    assert h[oracle.CYCLE_F][2] < h[oracle.CYCLE_V][2]
    assert h[oracle.CYCLE_W][2] < h[oracle.CYCLE_V][2]
