"""Independent checks that pin the oracle to the paper and to mathematics.

TEST INFRASTRUCTURE ONLY (used by tests/).  Nothing here calls the oracle's C
code: every function is a separate NumPy derivation so that a mistake in the
oracle (a dropped term, a wrong sign or index, a transposed operand) shows
up as a disagreement.

* ``hessian`` / ``dgp_term_traceless`` / ``kmo_term_traceless``: the model
  terms rebuilt from the discrete Hessian through the traceless split
  (eq:operator_split) instead of the printed long forms.
* ``fft_fixed_point``: the FFT-relaxation method the paper cites in its
  footnote on FFT use (Sec. 3.2): treat the nonlinear term as a source and
  re-solve the Poisson equation until it stops changing.
* ``newton_bordered``: brute-force Newton on the bordered system
  [L(phi) + lambda = 0, sum(phi) = 0] with a dense complex-step Jacobian
  (small grids only).
* manufactured smooth solutions of the continuum equations (eq:dgp_eom_code,
  eq:kmo_eom1) for O(h^2) convergence;
* the paper's exact 1D sine solutions (Sec. 4.2.2) in their exact discrete
  form, and the spherical top-hat profiles (Sec. 4.2.3).
"""
from __future__ import annotations

import numpy as np

OMEGA_M = 0.3089


def sh(a, dx=0, dy=0, dz=0):
    """a shifted so that sh(a,1)[k,j,i] = a[k,j,i+1] (periodic)."""
    return np.roll(a, shift=(-dz, -dy, -dx), axis=(0, 1, 2))


def laplacian(phi, h=1.0):
    return (sh(phi, 1) + sh(phi, -1) + sh(phi, 0, 1) + sh(phi, 0, -1) + sh(phi, 0, 0, 1)
            + sh(phi, 0, 0, -1) - 6.0 * phi) / h ** 2


def hessian(phi, h=1.0):
    """Discrete Hessian: second differences on the diagonal, 4-point cross
    differences off the diagonal.  Returns H[a][b] arrays."""
    H = [[None] * 3 for _ in range(3)]
    unit = [(1, 0, 0), (0, 1, 0), (0, 0, 1)]
    for a in range(3):
        e = unit[a]
        H[a][a] = (sh(phi, *e) + sh(phi, *[-x for x in e]) - 2.0 * phi) / h ** 2
        for b in range(a + 1, 3):
            f = unit[b]
            pp = sh(phi, *[e[q] + f[q] for q in range(3)])
            mm = sh(phi, *[-e[q] - f[q] for q in range(3)])
            pm = sh(phi, *[e[q] - f[q] for q in range(3)])
            mp = sh(phi, *[-e[q] + f[q] for q in range(3)])
            H[a][b] = H[b][a] = (pp + mm - pm - mp) / (4.0 * h ** 2)
    return H


def gradient(phi, h=1.0):
    return [(sh(phi, 1) - sh(phi, -1)) / (2 * h), (sh(phi, 0, 1) - sh(phi, 0, -1)) / (2 * h),
            (sh(phi, 0, 0, 1) - sh(phi, 0, 0, -1)) / (2 * h)]


def traceless(H):
    tr = H[0][0] + H[1][1] + H[2][2]
    return [[H[a][b] - (tr / 3.0 if a == b else 0.0) for b in range(3)] for a in range(3)]


def dgp_params(a=1.0, omega_m=OMEGA_M, h0rc=1.0):
    """beta (eq:beta_dgp, LCDM background), alpha and the source factor s."""
    orc = 1.0 / (4.0 * h0rc ** 2)
    beta = 1.0 + (omega_m / a ** 3 + 2 * (1 - omega_m)) / (
        2.0 * np.sqrt(orc * (omega_m / a ** 3 + 1 - omega_m)))
    alpha = 3.0 * beta * a ** 2 / h0rc ** 2
    return beta, alpha, alpha / beta * omega_m / a


def dgp_sigma_traceless(phi, delta, s, h=1.0):
    """Sigma = hat(H):hat(H) + s delta from the discrete Hessian."""
    Hh = traceless(hessian(phi, h))
    return sum(Hh[a][b] * Hh[a][b] for a in range(3) for b in range(3)) + s * delta


def dgp_term_traceless(phi, delta, alpha, s, h=1.0):
    """F = 2 Sigma / (alpha + sign(alpha) sqrt(alpha^2 + 8 Sigma / 3)), the
    cancellation-free form of the root of eq:dgp_quadratic_eom."""
    sig = dgp_sigma_traceless(phi, delta, s, h)
    return 2.0 * sig / (alpha + np.sign(alpha) * np.sqrt(alpha ** 2 + 8.0 * sig / 3.0))


def kmo_params(n_mesh, box, nk=3, k0=1.0, beta=0.1, a=1.0, omega_m=OMEGA_M, phibar=0.0,
               dphibar=0.0, lam=None):
    if lam is None:
        lam = np.sqrt(3.0 * (1.0 - omega_m))
    ctil = n_mesh / box * 2997.92458
    gamma = nk * k0 * (1.0 / (2 * a * a * lam * lam)) ** (nk - 1)
    c0 = 1.0 + gamma * (dphibar ** 2) ** (nk - 1)
    src = 3.0 * beta * np.exp(beta * phibar) * omega_m / a
    return dict(ctil=ctil, gamma=gamma, C0=c0, src=src, nk=nk)


def kmo_term_traceless(phi, delta, p, h=1.0):
    """(src delta + Sigma_2) / (c~ Sigma_1) with Q = hat(H)_ij G_i G_j built
    from the discrete traceless Hessian (independent of the printed
    coefficients)."""
    G = gradient(phi, h)
    Hh = traceless(hessian(phi, h))
    g = G[0] ** 2 + G[1] ** 2 + G[2] ** 2
    q = sum(Hh[a][b] * G[a] * G[b] for a in range(3) for b in range(3))
    nk = p["nk"]
    s1 = p["C0"] + (2 * nk + 1) / 3.0 * p["gamma"] * g ** (nk - 1)
    s2 = -2.0 * p["ctil"] * (nk - 1) * p["gamma"] * g ** (nk - 2) * q
    return (p["src"] * delta + s2) / (p["ctil"] * s1)


# ------------------------------------------------------------ FFT tools

def _eig(n, h=1.0):
    m = np.fft.fftfreq(n) * n
    s2 = np.sin(np.pi * m / n) ** 2
    return -4.0 * (s2[:, None, None] + s2[None, :, None] + s2[None, None, :]) / h ** 2


def poisson_fft(rhs, h=1.0):
    """Zero-mean u with lap_h u = rhs - mean(rhs) (exact discrete inverse)."""
    n = rhs.shape[0]
    e = _eig(n, h)
    e[0, 0, 0] = 1.0
    k = np.fft.fftn(rhs) / e
    k[0, 0, 0] = 0.0
    return np.real(np.fft.ifftn(k))


def fft_fixed_point(term, delta, tol=1e-14, max_iter=500, h=1.0):
    """phi <- lap^-1 (K(phi) - mean K(phi)) until the update is below tol
    (relative); `term(phi, delta)` is the model term K.  Returns phi, iters."""
    phi = np.zeros_like(delta)
    for it in range(1, max_iter + 1):
        new = poisson_fft(term(phi, delta), h)
        ch = np.abs(new - phi).max() / max(np.abs(new).max(), 1e-300)
        phi = new
        if ch < tol:
            return phi, it
    return phi, max_iter


# ---------------------------------------------------- bordered Newton (small n)

def complex_step_jacobian(term, phi, delta, h=1.0, step=1e-30):
    """Dense d(lap(phi) - K(phi))/dphi by the complex step (exact to rounding)."""
    n3 = phi.size
    J = np.empty((n3, n3))
    base = phi.astype(np.complex128)
    for p in range(n3):
        z = base.copy().reshape(-1)
        z[p] += 1j * step
        z = z.reshape(phi.shape)
        L = laplacian(z, h) - term(z, delta.astype(np.complex128))
        J[:, p] = (L.imag / step).reshape(-1)
    return J


def newton_bordered(term, delta, iters=8, h=1.0):
    """Newton on [L(phi) + lambda = 0, sum phi = 0]; returns phi, lambda,
    residual history."""
    n3 = delta.size
    phi = np.zeros_like(delta)
    lam = 0.0
    hist = []
    for _ in range(iters):
        L = laplacian(phi, h) - term(phi, delta)
        r = np.concatenate([(L + lam).reshape(-1), [phi.sum()]])
        hist.append(np.abs(r).max())
        if hist[-1] < 1e-15:
            break
        J = complex_step_jacobian(term, phi, delta, h)
        B = np.zeros((n3 + 1, n3 + 1))
        B[:n3, :n3] = J
        B[:n3, n3] = 1.0
        B[n3, :n3] = 1.0
        dx = np.linalg.solve(B, -r)
        phi = phi + dx[:n3].reshape(delta.shape)
        lam += dx[n3]
    return phi, lam, hist


# ------------------------------------------------ manufactured solutions

class SineSum:
    """psi(x) = sum_q A_q sin(k_q . x + t_q) on a periodic box of side B,
    with analytic gradient and Hessian."""

    def __init__(self, box, modes):
        self.box = box
        self.modes = [(np.array(m, float) * 2 * np.pi / box, A, t) for m, A, t in modes]

    def grid(self, n):
        h = self.box / n
        c = (np.arange(n) + 0.5) * h
        z, y, x = np.meshgrid(c, c, c, indexing="ij")
        return x, y, z, h

    def eval(self, n):
        x, y, z, h = self.grid(n)
        psi = np.zeros_like(x)
        G = [np.zeros_like(x) for _ in range(3)]
        H = [[np.zeros_like(x) for _ in range(3)] for _ in range(3)]
        for k, A, t in self.modes:
            ph = k[0] * x + k[1] * y + k[2] * z + t
            s, c = np.sin(ph), np.cos(ph)
            psi += A * s
            for a in range(3):
                G[a] += A * k[a] * c
                for b in range(3):
                    H[a][b] += -A * k[a] * k[b] * s
        return psi, G, H, h


def dgp_manufactured_delta(G, H, beta, alpha, a=1.0, omega_m=OMEGA_M):
    """delta from the continuum eq:dgp_eom_code given the exact Hessian:
    lap + (1/alpha)[(lap)^2 - H:H] = Omega_m delta / (beta a)."""
    lap = H[0][0] + H[1][1] + H[2][2]
    hh = sum(H[a][b] ** 2 for a in range(3) for b in range(3))
    return (lap + (lap ** 2 - hh) / alpha) * beta * a / omega_m


def kmo_manufactured_delta(G, H, p):
    """delta from the continuum eq:kmo_eom1:
    c~ div[(C0 + gamma g^(n-1)) grad phi] = src delta, g = |grad phi|^2."""
    nk = p["nk"]
    g = G[0] ** 2 + G[1] ** 2 + G[2] ** 2
    lap = H[0][0] + H[1][1] + H[2][2]
    gHg = sum(G[a] * H[a][b] * G[b] for a in range(3) for b in range(3))
    div = (p["C0"] + p["gamma"] * g ** (nk - 1)) * lap \
        + p["gamma"] * (nk - 1) * g ** (nk - 2) * 2.0 * gHg
    return p["ctil"] * div / p["src"]


# -------------------------------------------------- paper's exact 1D tests

def sine_1d(n, amplitude, waves=1, axis=0):
    """A sin(2 pi K x / N) along one axis at cell centres x = i + 1/2."""
    x = np.arange(n) + 0.5
    s = amplitude * np.sin(2 * np.pi * waves * x / n)
    shape = [1, 1, 1]
    shape[2 - axis] = n
    return np.broadcast_to(s.reshape(shape), (n, n, n)).copy()


def dgp_sine_delta_paper(n, beta, a=1.0, omega_m=OMEGA_M, axis=0):
    """eq:sine_nDGP: delta = -(a beta / (Omega_m N^2)) sin(2 pi x / N)."""
    return sine_1d(n, -a * beta / (omega_m * n * n), 1, axis)


def dgp_sine_phi_discrete(n, axis=0):
    """Exact discrete solution for eq:sine_nDGP: the analytic amplitude
    1/(4 pi^2) times (pi/N)^2 / sin^2(pi/N) (the 3-point second difference
    of sin(2 pi x/N) is -4 sin^2(pi/N) times the function)."""
    amp = 1.0 / (4 * np.pi ** 2) * (np.pi / n) ** 2 / np.sin(np.pi / n) ** 2
    return sine_1d(n, amp, 1, axis)


def dgp_sine_delta_discrete(phi, beta, a=1.0, omega_m=OMEGA_M, axis=0):
    """In 1D the discrete Sigma is (2/3) D^2 + s delta with D the second
    difference, so F(Sigma) = D exactly when delta = (beta a / Omega_m) D
    (and alpha + 4D/3 > 0)."""
    e = [0, 0, 0]
    e[axis] = 1
    D = sh(phi, *e) + sh(phi, *[-x for x in e]) - 2 * phi
    return beta * a / omega_m * D


def kmo_sine_delta_discrete(phi, p, axis=0):
    """Exact discrete source for phi varying along one axis: with G the
    central difference and D the second difference,
    src delta = c~ D [C0 + (2n - 1) gamma G^(2(n-1))]."""
    e = [0, 0, 0]
    e[axis] = 1
    D = sh(phi, *e) + sh(phi, *[-x for x in e]) - 2 * phi
    G = (sh(phi, *e) - sh(phi, *[-x for x in e])) / 2.0
    nk = p["nk"]
    return p["ctil"] * D * (p["C0"] + (2 * nk - 1) * p["gamma"] * G ** (2 * (nk - 1))) / p["src"]


# ------------------------------------------------ spherical top-hat profiles

def dgp_sphere_dphidr(r, delta_in, radius, beta, h0rc, a=1.0, omega_m=OMEGA_M):
    """Radial derivative of phi for a top-hat, derived from eq:dgp_eom_code
    in spherical symmetry:  (2/(alpha r^2)) d/dr[r phi'^2] + r^-2 d/dr[r^2 phi']
    = (Omega_m/(beta a)) delta, integrated once:
    phi' = (3 beta a^2 r / (4 R_c^2)) [sqrt(1 + 8 R_c^2 Omega_m m(r) /
    (3 beta^2 a^3 r^3)) - 1],  m(r) = delta r^3/3 (inside), delta R^3/3 (out)."""
    r = np.asarray(r, float)
    m = np.where(r <= radius, delta_in * r ** 3 / 3.0, delta_in * radius ** 3 / 3.0)
    rc2 = h0rc ** 2
    x = 8.0 * rc2 * omega_m * m / (3.0 * beta ** 2 * a ** 3 * np.maximum(r, 1e-300) ** 3)
    return 3.0 * beta * a ** 2 * r / (4.0 * rc2) * (np.sqrt(1.0 + x) - 1.0)


def kmo_sphere_dphidr(r, delta_in, radius, p, beta_kmo, omega_m=OMEGA_M, a=1.0):
    """Top-hat solution of c~ (1 + C0' + gamma E^(2(n-1))) E = f(r) with
    E = phi' (the modified Kmouflage equation in spherical symmetry,
    integrated once): f = src m(r) / (c~ r^2), m(r) = delta r^3/3 inside,
    delta R^3/3 outside; the real root is found by bisection.  For n = 2 and
    C0 = 1 it equals the paper's closed-form cubic root (Sec. 4.2.3)."""
    r = np.asarray(r, float)
    m = np.where(r <= radius, delta_in * r ** 3 / 3.0, delta_in * radius ** 3 / 3.0)
    f = p["src"] * m / (p["ctil"] * np.maximum(r, 1e-300) ** 2)
    nk = p["nk"]
    lo = np.zeros_like(f)
    hi = np.maximum(f / p["C0"], 1e-300) * 1.0001
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        val = (p["C0"] + p["gamma"] * mid ** (2 * (nk - 1))) * mid - f
        lo = np.where(val < 0, mid, lo)
        hi = np.where(val < 0, hi, mid)
    return 0.5 * (lo + hi)


def kmo_sphere_cardano_paper(r, delta_in, radius, gamma, beta_kmo, ctil, omega_m=OMEGA_M):
    """The paper's printed closed form for n = 2 (Sec. 4.2.3):
    phi' = g^(1/3)/(6 gamma) - 2/g^(1/3),
    g = gamma^2 [108 f + 20.78460969 sqrt(27 f^2 + 4/gamma)],
    f = beta Omega_m r delta / c~ (inside), beta Omega_m R^3 delta/(c~ r^2)."""
    r = np.asarray(r, float)
    f = np.where(r <= radius, beta_kmo * omega_m * r * delta_in / ctil,
                 beta_kmo * omega_m * radius ** 3 * delta_in / (ctil * np.maximum(r, 1e-300) ** 2))
    g = gamma ** 2 * (108 * f + 20.78460969 * np.sqrt(27 * f ** 2 + 4.0 / gamma))
    g3 = np.cbrt(g)
    return g3 / (6 * gamma) - 2.0 / g3
