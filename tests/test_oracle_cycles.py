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


# ------------------------------------------- Newton-Gauss-Seidel comparator
# The nDGP equation in its quadratic form eq:dgp_eom_code, relaxed by the
# generic Newton step of eq:relaxation_iteration (the iteration the closed
# form of Sec. 3.2.3 replaces).


def test_newton_operator_is_the_printed_equation():
    # L_N = lap + [(lap)^2 - H:H] / alpha - s delta / alpha with the full
    # discrete Hessian H, evaluated independently with NumPy
    from oracle import pins
    n, h = 16, 2.0
    phi = 3.0 * inputs.gaussian_field(n, 4, lambda k: k ** -3.0)
    delta = inputs.lognormal_delta(n, 2)
    beta, alpha, s = pins.dgp_params(0.8, OM, 1.0)
    H = pins.hessian(phi, h)
    D = pins.laplacian(phi, h)
    HH = sum(H[a][b] * H[a][b] for a in range(3) for b in range(3))
    ref = D + (D * D - HH) / alpha - s * delta / alpha
    got = oracle.residual(oracle.dgp_newton_model(0.8, OM, 1.0), phi, delta, h=h)
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("amp", [None, 20.0])
def test_newton_comparator_reaches_the_exact_sine_solution(amp):
    # in 1D the traceless part vanishes and mean(L) = 0, so the quadratic form
    # and the closed form share the exact discrete solution
    from oracle import pins
    n = 32
    m = oracle.dgp_newton_model(1.0, OM, 1.0)
    phi = pins.dgp_sine_phi_discrete(n) if amp is None else pins.sine_1d(n, amp, 1, 0)
    beta = oracle.dgp_model(1.0, OM, 1.0).beta
    delta = pins.dgp_sine_delta_discrete(phi, beta)
    r = oracle.solve(m, delta, tol=1e-13, max_cycles=100)
    phi = phi - phi.mean()
    assert r.status == 0
    assert np.abs(r.phi - phi).max() <= 1e-10 * np.abs(phi).max()


def test_newton_comparator_fixed_point_matches_closed_form_to_the_border():
    # on a periodic 3D field the two forms differ only through the bordering
    # constant (the mean of L enters the quadratic form multiplied by
    # (2/(3 alpha))(D - r_minus)): the solutions agree to about mu / alpha
    n = 32
    delta = inputs.lognormal_delta(n, 1)
    rc = oracle.solve(oracle.dgp_model(1.0, OM, 1.0), delta, tol=1e-12, max_cycles=80)
    rn = oracle.solve(oracle.dgp_newton_model(1.0, OM, 1.0), delta, tol=1e-12, max_cycles=200)
    assert rc.status == 0 and rn.status == 0
    assert np.abs(rn.phi - rc.phi).max() <= 1e-3 * np.abs(rc.phi).max()
