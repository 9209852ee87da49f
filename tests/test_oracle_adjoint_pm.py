"""Pins of the oracle's adjoint solve and its particle-mesh substrate.

The adjoint's Jacobian rows are checked against complex-step derivatives of
the independent NumPy operator, the transpose against the forward
application, the full gradient against central finite differences of the
forward solve and against a dense bordered adjoint.  CIC and the kick-drift
are checked against exact conservation laws.  CPU only.
"""
import numpy as np
import pytest

import inputs
import oracle
from oracle import pins

OM = 0.3089


def _models(n):
    dm = oracle.dgp_model(1.0, OM, 1.0)
    km = oracle.kmo_model(n, 40000.0, 3, 1.0, 0.1)
    kp = pins.kmo_params(n, 40000.0, 3, 1.0, 0.1)
    return {
        "dgp": (dm, lambda p, d: pins.dgp_term_traceless(p, d, dm.alpha, dm.s)),
        "kmo": (km, lambda p, d: pins.kmo_term_traceless(p, d, kp)),
    }


def _dense_from_rows(rows, n, h=1.0):
    nb = [(1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1),
          (1, 1, 0), (-1, -1, 0), (1, -1, 0), (-1, 1, 0), (1, 0, 1), (-1, 0, -1), (1, 0, -1),
          (-1, 0, 1), (0, 1, 1), (0, -1, -1), (0, 1, -1), (0, -1, 1)]
    n3 = n ** 3
    J = np.zeros((n3, n3))
    for k in range(n):
        for j in range(n):
            for i in range(n):
                m = (k * n + j) * n + i
                J[m, m] += -6.0 / h ** 2
                for q, (a, b, c) in enumerate(nb):
                    p = (((k + c) % n) * n + (j + b) % n) * n + (i + a) % n
                    if q < 6:
                        J[m, p] += 1.0 / h ** 2
                    J[m, p] -= rows[k, j, i, q]
    return J


@pytest.mark.parametrize("model", ["dgp", "kmo"])
def test_jacobian_rows_match_complex_step(model):
    n = 8
    m, term = _models(n)[model]
    delta = inputs.lognormal_delta(n, 9) * (1.0 if model == "dgp" else 2.0)
    phi = oracle.solve(m, delta, tol=1e-12).phi + 0.01 * inputs.gaussian_field(n, 3, lambda k: k ** -2)
    J_or = _dense_from_rows(oracle.jac_rows(m, phi, delta), n)
    J_cs = pins.complex_step_jacobian(term, phi, delta)
    assert np.abs(J_or - J_cs).max() <= 1e-11 * np.abs(J_cs).max()


def test_transpose_dot_product():
    n = 16
    m, _ = _models(n)["dgp"]
    delta = inputs.lognormal_delta(n, 1)
    phi = oracle.solve(m, delta, tol=1e-10).phi
    rows = oracle.jac_rows(m, phi, delta)
    rng = np.random.default_rng(0)
    u, v = rng.standard_normal((2, n, n, n))
    lhs = np.sum(oracle.jac_apply(rows, v) * u)
    rhs = np.sum(v * oracle.jac_t_apply(rows, u))
    assert lhs == pytest.approx(rhs, rel=1e-13)
    # constants are in the null space of J (L is shift invariant)
    assert np.abs(oracle.jac_apply(rows, np.ones((n, n, n)))).max() < 1e-12


def test_linear_adjoint_is_fft_poisson():
    n = 16
    s = 1.3
    m = oracle.linear_model(s)
    delta = inputs.lognormal_delta(n, 2)
    w = inputs.gaussian_weights(n, 3)
    phi = oracle.solve(m, delta, tol=1e-13).phi
    r = oracle.adjoint(m, delta, phi, w, tol=1e-12)
    assert r.status == 0
    mu = pins.poisson_fft(w)
    assert np.abs(r.mu - mu).max() <= 1e-10 * np.abs(mu).max()
    assert np.abs(r.grad - s * mu).max() <= 1e-10 * np.abs(s * mu).max()


@pytest.mark.parametrize("model", ["dgp", "kmo"])
def test_adjoint_matches_dense_bordered_adjoint(model):
    n = 8
    m, term = _models(n)[model]
    delta = inputs.lognormal_delta(n, 4) * (1.0 if model == "dgp" else 2.0)
    w = inputs.gaussian_weights(n, 5)
    phi = oracle.solve(m, delta, tol=1e-14, max_cycles=80).phi
    r = oracle.adjoint(m, delta, phi, w, tol=1e-13, max_cycles=80)
    assert r.status == 0
    J = pins.complex_step_jacobian(term, phi, delta)
    n3 = n ** 3
    B = np.zeros((n3 + 1, n3 + 1))
    B[:n3, :n3] = J.T
    B[:n3, n3] = 1.0
    B[n3, :n3] = 1.0
    sol = np.linalg.solve(B, np.concatenate([w.reshape(-1), [0.0]]))
    mu = sol[:n3].reshape(n, n, n)
    assert sol[n3] == pytest.approx(w.mean(), abs=1e-12)
    assert np.abs(r.mu - mu).max() <= 1e-9 * np.abs(mu).max()


@pytest.mark.parametrize("model", ["dgp", "kmo"])
def test_adjoint_gradient_matches_finite_differences(model):
    n = 16
    m, _ = _models(n)[model]
    delta = inputs.lognormal_delta(n, 1) * (1.0 if model == "dgp" else 2.0)
    w = inputs.gaussian_weights(n, 3)
    base = oracle.solve(m, delta, tol=1e-14, max_cycles=80)
    r = oracle.adjoint(m, delta, base.phi, w, tol=1e-12, max_cycles=80)
    assert r.status == 0
    cells = inputs.random_cells(n, 6, 4)
    eps = 1e-4
    fd = []
    for c in cells:
        vals = []
        for sgn in (1, -1):
            d2 = delta.copy().reshape(-1)
            d2[c] += sgn * eps
            ph = oracle.solve(m, d2.reshape(delta.shape), base.phi, tol=1e-14, max_cycles=80).phi
            vals.append(np.sum(ph * w))
        fd.append((vals[0] - vals[1]) / (2 * eps))
    fd = np.array(fd)
    g = r.grad.reshape(-1)[cells]
    assert np.abs(g - fd).max() <= 1e-6 * np.abs(fd).max()


# ------------------------------------------------------------------ CIC

def test_cic_conserves_mass_and_mean():
    pos = inputs.za_particles(16, 32, 2, amplitude=30.0)
    rho, delta = oracle.cic_density(pos, 32)
    assert rho.sum() == pytest.approx(16 ** 3, rel=1e-13)
    assert abs(delta.mean()) < 1e-13
    assert rho.min() >= 0.0


@pytest.mark.parametrize("np_, nm", [(16, 16), (8, 16)])
def test_cic_of_undisplaced_lattice_is_uniform(np_, nm):
    # particles at cell centres (N_p = N) or at cell corners 2i+1 (N_p = N/2)
    pos = inputs.lattice_positions(np_, nm).astype(np.float32)
    rho, delta = oracle.cic_density(pos, nm)
    assert np.abs(delta).max() < 1e-14


def test_cic_single_particle_weights():
    pos = np.array([[3.75, 0.25, 6.5]], np.float32)  # fx = .25, wraps in y, fz = 0
    rho, _ = oracle.cic_density(pos, 8)
    # x: t = 3.25 -> cells 3 (0.75), 4 (0.25); y: t = -0.25 -> cells 7 (0.25),
    # 0 (0.75); z: t = 6 -> cell 6 only
    assert rho[6, 7, 3] == pytest.approx(0.75 * 0.25)
    assert rho[6, 0, 3] == pytest.approx(0.75 * 0.75)
    assert rho[6, 7, 4] == pytest.approx(0.25 * 0.25)
    assert rho[6, 0, 4] == pytest.approx(0.25 * 0.75)
    assert rho.sum() == pytest.approx(1.0)


def test_newtonian_kick_conserves_momentum():
    # CIC deposit + symmetric Green's function + antisymmetric 3-point
    # gradient + CIC interpolation: no net self-force
    n = 16
    pos = inputs.za_particles(8, n, 2, amplitude=30.0)
    mom = np.zeros_like(pos)
    _, delta = oracle.cic_density(pos, n)
    psi = oracle.fft_poisson(1.5 * OM * delta)
    p2, m2 = pos.copy(), mom.copy()
    oracle.lib().or_kick_drift(n, pos.shape[0], np.ascontiguousarray(psi), p2.reshape(-1),
                               m2.reshape(-1), 1.0, 0.0)
    tot = m2.astype(np.float64).sum(axis=0)
    assert np.abs(tot).max() <= 1e-5 * np.abs(m2).max() * np.sqrt(pos.shape[0])
    assert np.abs(m2).max() > 0


def test_fft_poisson_matches_independent_inverse():
    d = inputs.lognormal_delta(16, 8)
    assert np.abs(oracle.fft_poisson(d) - pins.poisson_fft(d)).max() < 1e-13


def test_pm_step_runs_and_moves_particles():
    n = 16
    pos = inputs.za_particles(8, n, 2, amplitude=30.0)
    mom = np.zeros_like(pos)
    p2, m2, phi, delta, phin = oracle.pm_step(pos, mom, n, 1.0, 0.01)
    assert np.all((p2 >= 0) & (p2 < n))
    assert np.abs(m2).max() > 0
    # the fifth force adds to gravity: phi/2 has the sign of Phi_N at large scale
    assert np.sum(phi * phin) > 0
