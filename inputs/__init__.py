"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and bench.py.

This module draws random numbers and shapes them into density fields and
particle sets.  It holds none of the solver's arithmetic: no stencil, no
multigrid, no CIC deposit.  Everything is FP64 NumPy driven by
``numpy.random.default_rng(seed)``, so a (function, seed) pair gives the same
bytes on every machine running this image.

Workload recipes (the paper's tests run on seeded synthetic fields only):

* ``lognormal_delta``: a Gaussian field with P(k) = k^-2 exp(-(k/k_Ny)^2),
  k in rad/cell, normalised to unit variance and mapped to
  delta = exp(g)/mean(exp(g)) - 1 (exact zero mean, delta > -1).
* ``za_particles``: Zel'dovich displacements on a particle lattice from a
  Gaussian field with P(k) = A k^-1.5 exp(-(k/k_c)^2), k_c half the Nyquist
  wavenumber of the particle lattice.  A is fixed per (n_part, n_mesh) near
  the largest CIC density contrast the displacements reach.  Positions are
  FP32 mesh units in [0, n_mesh).
* ``tophat_delta``: the spherical top-hat of the paper's 3D screening tests
  (Sec. 4.2.3): delta inside r <= R around the box centre, 0 outside.
* ``uniform_phi``: initial guesses uniform in [-0.05, 0.05] (Sec. 4.2.1).
"""
from __future__ import annotations

import numpy as np

# Gaussian cutoff of the Zel'dovich spectrum, in units of the particle
# lattice's Nyquist wavenumber.
ZA_CUTOFF = 0.5
# Amplitudes near the maximum CIC density contrast that Zel'dovich
# displacements reach before shell crossing smears the caustics: delta_rms
# ~1.7 for one particle per cell and ~2.3 for N_p = N_mesh/2 (the nominal
# delta_rms ~ 3 is out of reach of the Zel'dovich approximation at these
# resolutions).  Frozen after a scan over amplitudes.
ZA_AMPLITUDE = {
    (256, 256): 100.0,
    (256, 512): 30.0,
    (512, 1024): 30.0,
}


def _kgrid(n: int, spacing: float = 1.0):
    """Angular wavenumbers (rad per mesh cell) of an n^3 rfft grid whose
    sites are `spacing` mesh cells apart."""
    k1 = 2.0 * np.pi * np.fft.fftfreq(n, d=spacing)
    kr = 2.0 * np.pi * np.fft.rfftfreq(n, d=spacing)
    kz = k1[:, None, None]
    ky = k1[None, :, None]
    kx = kr[None, None, :]
    return kx, ky, kz


def gaussian_field(n: int, seed: int, pk, spacing: float = 1.0) -> np.ndarray:
    """Real Gaussian field on an n^3 grid, C order [z][y][x], with spectrum
    proportional to pk(k) (k in rad per mesh cell).  P(0) is set to 0."""
    rng = np.random.default_rng(seed)
    white = rng.standard_normal((n, n, n))
    wk = np.fft.rfftn(white)
    kx, ky, kz = _kgrid(n, spacing)
    k = np.sqrt(kx * kx + ky * ky + kz * kz)
    amp = np.zeros_like(k)
    nz = k > 0
    amp[nz] = np.sqrt(pk(k[nz]))
    return np.fft.irfftn(wk * amp, s=(n, n, n), axes=(0, 1, 2))


def lognormal_delta(n: int, seed: int = 1, sigma: float = 1.0) -> np.ndarray:
    """Lognormal density contrast: Gaussian g with P(k)=k^-2 exp(-(k/pi)^2),
    scaled to std `sigma`, delta = e^g / mean(e^g) - 1 (FP64, [z][y][x])."""
    g = gaussian_field(n, seed, lambda k: k ** -2.0 * np.exp(-(k / np.pi) ** 2))
    g *= sigma / g.std()
    e = np.exp(g)
    return e / e.mean() - 1.0


def lattice_positions(n_part: int, n_mesh: int) -> np.ndarray:
    """Undisplaced particle lattice q = s*(i + 1/2), s = n_mesh/n_part: cell
    centres when n_part == n_mesh, cell corners 2i+1 when n_part == n_mesh/2.
    Returns FP64 [n_part^3, 3] in (x, y, z) order, x fastest."""
    s = n_mesh / n_part
    q1 = s * (np.arange(n_part, dtype=np.float64) + 0.5)
    qz, qy, qx = np.meshgrid(q1, q1, q1, indexing="ij")
    return np.stack([qx.ravel(), qy.ravel(), qz.ravel()], axis=1)


def za_displacement(n_part: int, n_mesh: int, seed: int, amplitude: float) -> np.ndarray:
    """Zel'dovich displacement psi (mesh units, FP64 [n_part^3, 3]) with
    psi_k = i k / k^2 * delta_k, so that div psi = -delta_L."""
    s = n_mesh / n_part
    kny = ZA_CUTOFF * np.pi / s
    dl = gaussian_field(n_part, seed,
                        lambda k: amplitude * k ** -1.5 * np.exp(-(k / kny) ** 2),
                        spacing=s)
    dk = np.fft.rfftn(dl)
    kx, ky, kz = _kgrid(n_part, s)
    k2 = kx * kx + ky * ky + kz * kz
    k2[0, 0, 0] = 1.0
    # drop the Nyquist planes of the derivative (their sign is ambiguous)
    ny = n_part // 2
    out = []
    for kc, axis in ((kx, 2), (ky, 1), (kz, 0)):
        f = 1j * kc / k2 * dk
        sl = [slice(None)] * 3
        sl[axis] = ny
        f[tuple(sl)] = 0.0
        f[0, 0, 0] = 0.0
        out.append(np.fft.irfftn(f, s=(n_part,) * 3, axes=(0, 1, 2)).ravel())
    return np.stack(out, axis=1)


def za_particles(n_part: int, n_mesh: int, seed: int, amplitude: float | None = None) -> np.ndarray:
    """FP32 particle positions [n_part^3, 3] (x, y, z) in [0, n_mesh),
    x = q + psi wrapped periodically."""
    if amplitude is None:
        amplitude = ZA_AMPLITUDE[(n_part, n_mesh)]
    x = lattice_positions(n_part, n_mesh) + za_displacement(n_part, n_mesh, seed, amplitude)
    x = np.mod(x, n_mesh).astype(np.float32)
    # float32 rounding can land exactly on n_mesh
    x[x >= np.float32(n_mesh)] = 0.0
    return x


def tophat_delta(n: int, delta_in: float, radius: float) -> np.ndarray:
    """Spherical top-hat centred at (n/2, n/2, n/2); cell i has centre i+1/2."""
    c = np.arange(n, dtype=np.float64) + 0.5 - n / 2
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    r = np.sqrt(x * x + y * y + z * z)
    return np.where(r <= radius, delta_in, 0.0)


def uniform_phi(n: int, seed: int, half_width: float = 0.05) -> np.ndarray:
    """Initial guess uniform in [-half_width, half_width] (FP64 [n]^3)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-half_width, half_width, size=(n, n, n))


def gaussian_weights(n: int, seed: int) -> np.ndarray:
    """Loss weights w ~ N(0,1) on the mesh (FP64 [n]^3)."""
    return np.random.default_rng(seed).standard_normal((n, n, n))


def random_cells(n: int, count: int, seed: int) -> np.ndarray:
    """`count` distinct flat cell indices drawn uniformly without replacement."""
    return np.sort(np.random.default_rng(seed).choice(n ** 3, size=count, replace=False))
