"""Pins of the oracle's model-specific particle-mesh pieces, CPU only.

- Linear fifth force: for a tiny single-mode density the scalar potential is
  a fixed multiple of the Newtonian one on the same mesh (both use the same
  7-point Laplacian): nDGP (1/2) phi = Phi_N / (3 beta_DGP)
  (eq:fifth-force-ratio-asymptotic), Kmouflage beta c~ phi = (2 beta^2 / K_X)
  Phi_N with K_X = 1 + gamma b^(n-1) (the paper's F5/FN in code units).
- The Kmouflage kick: total momentum changes only by the velocity-term
  factor (no self-force of CIC + 3-point gradient + CIC), and beta = 0 is the
  Newtonian step.
"""
import numpy as np
import pytest

import inputs
import oracle
from oracle import background as bg

OM = 0.3089


def sine(n, eps):
    x = (np.arange(n) + 0.5) / n
    return np.broadcast_to(eps * np.sin(2 * np.pi * x)[None, None, :], (n, n, n)).copy()


@pytest.mark.parametrize("h0rc,a", [(1.0, 1.0), (0.5, 0.6)])
def test_dgp_linear_fifth_force_ratio(h0rc, a):
    n = 16
    d = sine(n, 1e-4)
    m = oracle.dgp_model(a, OM, h0rc)
    phin = oracle.fft_poisson(1.5 * OM / a * d)
    phi = oracle.solve(m, d, tol=1e-16, max_cycles=60).phi
    ratio = (0.5 * phi).ravel() @ phin.ravel() / (phin.ravel() @ phin.ravel())
    assert ratio == pytest.approx(1.0 / (3.0 * m.beta), rel=1e-4)


@pytest.mark.parametrize("nk,k0,beta,a", [(2, 1.0, 0.2, 0.8), (3, 10.0, 0.1, 1.0)])
def test_kmouflage_linear_fifth_force_ratio(nk, k0, beta, a):
    n, box = 16, 256.0
    b = bg.solve(nk, k0, beta)
    v = oracle.kmo_background_values(b, a, 0.0)
    m = oracle.kmo_model(n, box, nk, k0, beta, v["lam"], a, OM, v["phibar"], v["dphibar_dtau"])
    d = sine(n, 1e-5)
    A = np.exp(beta * v["phibar"])
    phin = oracle.fft_poisson(1.5 * A * OM / a * d)
    phi = oracle.solve(m, d, tol=1e-18, max_cycles=80).phi
    ctil = n / box * 2997.92458
    ratio = (beta * ctil * phi).ravel() @ phin.ravel() / (phin.ravel() @ phin.ravel())
    # K_X of the background: 1 + n K0 Xbar^(n-1), Xbar = phi'^2 / (2 lambda^2 a^2)
    xbar = v["dphibar_dtau"] ** 2 / (2 * v["lam"] ** 2 * a ** 2)
    kx = 1.0 + nk * k0 * xbar ** (nk - 1)
    assert m.C0 == pytest.approx(kx, rel=1e-12)
    assert ratio == pytest.approx(2 * beta ** 2 / kx, rel=1e-4)


def test_kmouflage_kick_momentum_and_newtonian_limit():
    n, npart, box, a, da = 16, 8, 64.0, 0.7, 0.01
    pos = inputs.za_particles(npart, n, 3, amplitude=40.0)
    mom = (np.random.default_rng(1).standard_normal(pos.shape) * 0.1).astype(np.float32)
    b = bg.solve(2, 1.0, 0.2)
    v = oracle.kmo_background_values(b, a, da)
    p2, m2, phi, d, phin = oracle.pm_step_kmouflage(pos, mom, n, a, da, box, 2, 1.0, 0.2, v,
                                                    tol=1e-12)
    damp = 1.0 - 0.2 * v["dphibar_da"] * da
    assert np.abs(m2.astype(np.float64).sum(0) - damp * mom.astype(np.float64).sum(0)).max() <= 1e-4
    # beta = 0: the Newtonian step with the same background expansion
    v0 = dict(v, phibar=0.0, dphibar_da=0.0)
    p3, m3, *_ = oracle.pm_step_kmouflage(pos, mom, n, a, da, box, 2, 1.0, 0.0, v0, tol=1e-12)
    _, dd = oracle.cic_density(pos, n)
    psi = oracle.fft_poisson(1.5 * OM / a * dd)
    p4, m4 = pos.copy(), mom.copy()
    oracle.lib().or_kick_drift(n, p4.shape[0], np.ascontiguousarray(psi), p4.reshape(-1),
                               m4.reshape(-1), da / (a * v["e_a"]),
                               da / ((a + da / 2) ** 3 * v["e_half"]))
    assert np.array_equal(m3, m4) and np.array_equal(p3, p4)
