"""Pins of the Kmouflage background oracle (Sec. 3.2.5), CPU only.

- LCDM limit (K0 = 0, beta = 0): lambda^2 = 3 (1 - Om - Or) and the closed-form
  H(a).
- Consistency of the three background equations: along a solution, the
  Raychaudhuri calH' must equal half the N-derivative of the Friedmann calH^2
  (this pins the scalar terms of both, e.g. a factor 2 in either).
- Without the K0 term: the matter-era attractor dphi/dN = -2 beta, and phibar
  linear in small beta; with it, kinetic screening at early times.
- The paper's statements on its background test (n = 2, beta = 0.2): phibar < 0
  and decreasing; the expansion rate of K0 = 1 is about 2 per cent below LCDM
  (with the same Om and H0), and the deviation shrinks as K0 grows.
"""
import numpy as np
import pytest

from oracle import background as bg

OM = 0.3089


def lcdm_hubble(a, lam):
    return np.sqrt(bg.omega_radiation() / a ** 4 + OM / a ** 3 + lam ** 2 / 3.0)


def test_radiation_density():
    # photons at 2.7255 K: Omega_gamma h^2 = 2.47e-5; neutrinos add 0.69 of that
    o = bg.omega_radiation(0.7)
    assert o * 0.49 == pytest.approx(2.4728e-5 * (1 + 3.046 * 0.2271), rel=1e-3)


def test_lcdm_limit():
    b = bg.solve(2, 0.0, 0.0)
    lam = np.sqrt(3 * (1 - OM - bg.omega_radiation()))
    assert b.lam == pytest.approx(lam, rel=1e-10)
    a = np.logspace(-4, 0, 60)
    assert np.allclose(b.hubble(a), lcdm_hubble(a, lam), rtol=1e-9, atol=0)
    assert np.abs(b.phibar(a)).max() < 1e-25


@pytest.fixture(scope="module")
def k0_1():
    return bg.solve(2, 1.0, 0.2)


def test_raychaudhuri_is_consistent_with_friedmann(k0_1):
    b = k0_1
    m, lam = b.model, b.lam
    for N in np.linspace(-6.0, -0.01, 9):
        eps = 1e-4
        y = []
        for dN in (-eps, eps):
            phi, p = b.sol.sol(N + dN)
            y.append(bg.friedmann_calh2(m, lam, N + dN, phi, p))
        phi, p = b.sol.sol(N)
        y0 = bg.friedmann_calh2(m, lam, N, phi, p)
        hp = bg.raychaudhuri(m, lam, N, phi, p, y0)
        assert hp == pytest.approx(0.5 * (y[1] - y[0]) / (2 * eps), rel=1e-6, abs=1e-9)


def test_matter_era_attractor_without_k0():
    # K0 = 0 (K_X = 1): in matter domination calH^2 = Om/a, calH' = -Om/(2a) and
    # the field equation becomes phi'' + 3/2 phi' + 3 beta = 0 (N-derivatives):
    # dphi/dN -> -2 beta; phibar is then linear in small beta
    r = []
    for beta in (1e-3, 2e-3):
        b = bg.solve(2, 0.0, beta)
        phi, p = b.sol.sol(np.log(0.05))
        assert p == pytest.approx(-2 * beta, rel=2e-2)
        r.append(b.phibar(1.0) / beta)
    assert r[1] == pytest.approx(r[0], rel=1e-2)


def test_kinetic_screening_at_early_times(k0_1):
    # with K0 > 0 the K0 X^n term dominates at early times (X grows as 1/a^4
    # in the radiation era), so the field moves less than without it
    b0 = bg.solve(2, 0.0, 0.2)
    assert abs(k0_1.phibar(1e-3)) < 0.5 * abs(b0.phibar(1e-3))


def test_paper_background_statements(k0_1):
    a = np.logspace(-3, 0, 300)
    lam_lcdm = np.sqrt(3 * (1 - OM - bg.omega_radiation()))
    dev = []
    for k0 in (1.0, 10.0, 100.0):
        b = k0_1 if k0 == 1.0 else bg.solve(2, k0, 0.2)
        assert b.phibar(1.0) < 0
        assert b.dphibar_dtau_over_h0(1.0) < 0
        dev.append((b.hubble(a) / lcdm_hubble(a, lam_lcdm) - 1).min())
    assert -0.03 < dev[0] < -0.015
    assert dev[0] < dev[1] < dev[2] < 0
