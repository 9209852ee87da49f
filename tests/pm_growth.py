"""Linear-growth helpers for the particle-mesh tests (test infrastructure):
growing-mode Zel'dovich starts, the linear growth equation in the PM step's
variables, and the large-scale growth measured from two density fields."""
import numpy as np
from scipy.integrate import solve_ivp

import inputs

OM = 0.3089


def linear_growth(a0, a1, geff, dp0, e, p0=None):
    """Linear growth D(a1) with D(a0) = 1 and D'(a0) = dp0 (or initial
    momentum p0 = a0^3 E D'), from the equations of motion of the PM step:
    dx/da = p/(a^3 E), dp/da = -grad Psi/(a E) with lap Psi = (3/2) Omega_m
    G_eff delta / a give (a^3 E D')' = (3/2) Omega_m G_eff D / (a^2 E).
    Returns (D(a1), D'(a1))."""
    f = lambda a, y: [y[1] / (a ** 3 * e(a)), 1.5 * OM * geff(a) * y[0] / (a ** 2 * e(a))]
    y0 = a0 ** 3 * e(a0) * dp0 if p0 is None else p0
    r = solve_ivp(f, (a0, a1), [1.0, y0], rtol=1e-10, atol=1e-14)
    return r.y[0, -1], r.y[1, -1] / (a1 ** 3 * e(a1))


def growing_mode_ics(n_mesh, n_part, seed, a0, e, max_disp=0.03):
    """Zel'dovich positions and momenta of the LCDM growing mode at a0
    (p = a^3 E D'/D psi in the PM step's variables); also D'/D at a0."""
    d_early, dp_early = linear_growth(1e-3, a0, lambda a: 1.0, 1.0 / 1e-3, e)
    f0 = dp_early / d_early
    q = inputs.lattice_positions(n_part, n_mesh)
    disp = inputs.za_displacement(n_part, n_mesh, seed, 1.0)
    disp *= max_disp / np.abs(disp).max()
    x = np.mod(q + disp, n_mesh).astype(np.float32)
    p = (a0 ** 3 * e(a0) * f0 * disp).astype(np.float32)
    return x, p, f0


def large_scale_growth(delta0, delta1, kmax2=4):
    """Projection of delta1 on delta0 over the modes 0 < |m|^2 <= kmax2."""
    n = delta0.shape[0]
    f0, f1 = np.fft.fftn(delta0), np.fft.fftn(delta1)
    m = np.fft.fftfreq(n) * n
    m2 = m[:, None, None] ** 2 + m[None, :, None] ** 2 + m[None, None, :] ** 2
    sel = (m2 > 0) & (m2 <= kmax2)
    return float(np.real(np.sum(f1[sel] * np.conj(f0[sel]))) / np.sum(np.abs(f0[sel]) ** 2))
