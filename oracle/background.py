"""Kmouflage background cosmology (Sec. 3.2.5), plain NumPy/SciPy.

TEST INFRASTRUCTURE ONLY: the oracle of the library's background solver.

The background field phi(N), N = ln a, with K(X) = -1 + X + K0 X^n and
A = exp(beta phi) follows the paper's procedure: at each N the modified
Friedmann equation is solved for calH^2 (calH = a H, units H0 = 1), the
Raychaudhuri equation gives calH', the field equation eq:kmf_background_eom2
gives the second N-derivative of phi, and lambda is shot until H(a=1) = H0.

Readings (the printed N-forms do not follow from the printed cosmic-time
equations; the forms used are derived here from eq:kmf_background_eom,
eq:kmf_background_Friedmann and energy conservation of the scalar fluid,
rho = 2 X K_X - K, P = K in units of lambda^2 H0^2):
  Friedmann:    calH^2 (1 - p^2/6) = Or/a^2 + A Om/a + lambda^2 a^2/3
                                     + (2n-1)/3 lambda^2 a^2 K0 X^n,
  Raychaudhuri: calH' = -(A Om/a + 2 Or/a^2)/2 + lambda^2 a^2/3 - calH^2 p^2/3
                        - (n+1)/3 lambda^2 a^2 K0 X^n,
with p = dphi/dN and X = calH^2 p^2 / (2 lambda^2 a^2).  In the LCDM limit
(K = -1) they reduce to H^2 = Or/a^4 + Om/a^3 + lambda^2/3 and
calH' = -Om/(2a) - Or/a^2 + lambda^2 a^2/3; the printed Raychaudhuri
equation has twice these scalar terms, which breaks that limit.

Library primitives used as steps: numpy.roots (the Friedmann polynomial),
scipy.integrate.solve_ivp (DOP853), scipy.optimize.brentq (shooting).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
from scipy.integrate import solve_ivp
from scipy.optimize import brentq

T_CMB = 2.7255          # K (Sec. 3.2.5)
N_EFF = 3.046           # massless neutrino flavours (Sec. 3.2.5)
H_PLANCK = 0.6774       # dimensionless Hubble constant paired with Omega_m = 0.3089
Z_INIT = 1.0e5          # start of the integration (Sec. 3.2.5)
PHI_INIT = 1.0e-30      # initial phi and dphi/dN (Sec. 3.2.5)


def omega_radiation(h: float = H_PLANCK, t_cmb: float = T_CMB, n_eff: float = N_EFF) -> float:
    """Photons at t_cmb plus n_eff massless neutrinos."""
    omega_gamma = 2.4728e-5 * (t_cmb / 2.7255) ** 4 / h ** 2
    return omega_gamma * (1.0 + n_eff * (7.0 / 8.0) * (4.0 / 11.0) ** (4.0 / 3.0))


@dataclass
class Model:
    n: int
    k0: float
    beta: float
    omega_m: float
    omega_r: float


def friedmann_calh2(m: Model, lam: float, N: float, phi: float, p: float) -> float:
    """calH^2/H0^2 from the Friedmann equation: the root of
    C y^n - b y + S = 0 that continues y = S/b of C = 0 (the smallest
    positive root), found among all roots of the polynomial."""
    a = np.exp(N)
    A = np.exp(m.beta * phi)
    S = m.omega_r / a ** 2 + A * m.omega_m / a + lam ** 2 * a ** 2 / 3.0
    b = 1.0 - p * p / 6.0
    C = (2 * m.n - 1) / 3.0 * lam ** 2 * a ** 2 * m.k0 * (p * p / (2 * lam ** 2 * a ** 2)) ** m.n
    if C == 0.0 or C * (S / b) ** m.n < 1e-17 * S:
        return S / b
    coeffs = np.zeros(m.n + 1)
    coeffs[0] = C          # y^n
    coeffs[m.n - 1] = -b   # y^1
    coeffs[m.n] = S        # y^0
    r = np.roots(coeffs)
    real = sorted(x.real for x in r if abs(x.imag) < 1e-9 * max(1.0, abs(x)) and x.real > 0)
    if not real:
        raise ValueError("no physical root of the Friedmann equation")
    return real[0]


def raychaudhuri(m: Model, lam: float, N: float, phi: float, p: float, y: float) -> float:
    """calH'/H0^2 (conformal-time derivative of calH)."""
    a = np.exp(N)
    A = np.exp(m.beta * phi)
    X = y * p * p / (2 * lam ** 2 * a ** 2)
    return (-(A * m.omega_m / a + 2 * m.omega_r / a ** 2) / 2.0 + lam ** 2 * a ** 2 / 3.0
            - y * p * p / 3.0 - (m.n + 1) / 3.0 * lam ** 2 * a ** 2 * m.k0 * X ** m.n)


def rhs(m: Model, lam: float, N: float, s):
    phi, p = s
    a = np.exp(N)
    A = np.exp(m.beta * phi)
    y = friedmann_calh2(m, lam, N, phi, p)
    hp = raychaudhuri(m, lam, N, phi, p, y)
    X = y * p * p / (2 * lam ** 2 * a ** 2)
    kx = 1.0 + m.n * m.k0 * X ** (m.n - 1)
    kxx = m.n * (m.n - 1) * m.k0 * X ** (m.n - 2) if m.n >= 2 else 0.0
    # eq:kmf_background_eom2 solved for d2phi/dN2
    c2 = kx + 2 * X * kxx
    dp = -(c2 * hp * p + 2 * (kx - X * kxx) * y * p + 3 * m.beta * A * m.omega_m * np.exp(-N)) / (c2 * y)
    return [p, dp]


@dataclass
class Background:
    model: Model
    lam: float
    sol: object           # dense output of the final integration

    def state(self, a):
        N = np.log(a)
        phi, p = self.sol.sol(N)
        y = np.array([friedmann_calh2(self.model, self.lam, n_, f_, p_)
                      for n_, f_, p_ in zip(np.atleast_1d(N), np.atleast_1d(phi), np.atleast_1d(p))])
        return N, phi, p, y

    def hubble(self, a):
        """H/H0."""
        N, phi, p, y = self.state(a)
        return np.sqrt(y) / np.exp(N)

    def phibar(self, a):
        return self.state(a)[1]

    def dphibar_dtau_over_h0(self, a):
        """phi' = d phi / d tau in units of H0: calH dphi/dN."""
        N, phi, p, y = self.state(a)
        return np.sqrt(y) * p

    def hubble_dot(self, a):
        """dH/dt / H0^2 = (calH' - calH^2) / a^2."""
        N, phi, p, y = self.state(a)
        hp = np.array([raychaudhuri(self.model, self.lam, n_, f_, p_, y_)
                       for n_, f_, p_, y_ in zip(np.atleast_1d(N), np.atleast_1d(phi),
                                                 np.atleast_1d(p), y)])
        return (hp - y) / np.exp(2 * N)


def integrate(m: Model, lam: float, rtol: float = 1e-11):
    N0 = -np.log(1.0 + Z_INIT)
    return solve_ivp(lambda N, s: rhs(m, lam, N, s), (N0, 0.0), [PHI_INIT, PHI_INIT],
                     method="DOP853", rtol=rtol, atol=1e-30, dense_output=True)


def solve(n: int, k0: float, beta: float, omega_m: float = 0.3089,
          omega_r: float | None = None, htol: float = 1e-12) -> Background:
    """Shoot lambda so that H(a = 1) = H0, then return the background."""
    if omega_r is None:
        omega_r = omega_radiation()
    m = Model(n, k0, beta, omega_m, omega_r)

    def miss(lam):
        sol = integrate(m, lam)
        phi, p = sol.y[:, -1]
        return np.sqrt(friedmann_calh2(m, lam, 0.0, phi, p)) - 1.0

    lam = brentq(miss, 0.3, 5.0, xtol=htol, rtol=htol)
    return Background(m, lam, integrate(m, lam))
