"""FP64 CPU oracle for the MG-GLAM derivative-coupling hot path.

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py``, never by the product package.
It shares no code with the HIP path.  The arithmetic lives in
``mg_oracle.c`` (plain loops, FP64); this module loads it with ctypes and adds
the FFT Poisson solve of the particle-mesh step (Sec. 3.1: the Newtonian
potential from the discrete Green's function of the 7-point Laplacian).

Arrays are NumPy float64 in natural C order [z][y][x] (x fastest).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "mg_oracle.c")
# MGORACLE_LIB points the checks at another build of mg_oracle.c (the
# sanitizer leg of the tests builds one with AddressSanitizer and UBSan)
_LIB = os.environ.get("MGORACLE_LIB") or os.path.join(_HERE, "libmgoracle.so")


def build(force: bool = True) -> str:
    """Compile mg_oracle.c with gcc (FP64, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-ffp-contract=off", "-shared",
                               "-fPIC", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Model(C.Structure):
    _fields_ = [("model", C.c_int), ("alpha", C.c_double), ("sgn", C.c_double),
                ("s", C.c_double), ("ctil", C.c_double), ("gamma", C.c_double),
                ("C0", C.c_double), ("src", C.c_double), ("nk", C.c_int)]


class Stats(C.Structure):
    _fields_ = [("cycles", C.c_int), ("eps0", C.c_double), ("eps", C.c_double),
                ("mu", C.c_double), ("hist", C.c_double * 256), ("nclamp", C.c_longlong),
                ("status", C.c_int)]


_lib = None
_D = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
_F = np.ctypeslib.ndpointer(np.float32, flags="C_CONTIGUOUS")
_MP = C.POINTER(Model)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = C.CDLL(_LIB)
        L.or_dgp_setup.argtypes = [C.c_double, C.c_double, C.c_double, _MP, C.POINTER(C.c_double)]
        L.or_kmo_setup.argtypes = [C.c_int, C.c_double, C.c_int, C.c_double, C.c_double,
                                   C.c_double, C.c_double, C.c_double, C.c_double, C.c_double, _MP]
        L.or_linear_setup.argtypes = [C.c_double, _MP]
        L.or_dgp_newton_setup.argtypes = [C.c_double, C.c_double, C.c_double, _MP]
        L.or_op_cell.argtypes = [_MP, _D, _D, C.c_int, C.c_double, C.c_int, C.c_int, C.c_int]
        L.or_op_cell.restype = C.c_double
        L.or_residual.argtypes = [_MP, _D, _D, C.c_void_p, C.c_double, C.c_int, C.c_double, _D,
                                  C.c_void_p]
        L.or_colour_pass.argtypes = [_MP, _D, _D, C.c_void_p, C.c_double, C.c_int, C.c_double,
                                     C.c_int, _D, C.c_void_p]
        L.or_restrict.argtypes = [_D, C.c_int, _D]
        L.or_prolong_add.argtypes = [_D, C.c_int, _D, _D]
        L.or_mean.argtypes = [_D, C.c_int]
        L.or_mean.restype = C.c_double
        L.or_solve.argtypes = [_MP, C.c_int, C.c_double, _D, _D, C.c_int, C.c_double, C.c_int, C.c_int,
                               C.c_int, C.POINTER(Stats)]
        L.or_solve_cycle.argtypes = [_MP, C.c_int, C.c_double, _D, _D, C.c_int, C.c_double,
                                     C.c_int, C.c_int, C.c_int, C.c_int, C.c_void_p, C.c_int,
                                     C.POINTER(C.c_int), C.POINTER(Stats)]
        L.or_sweep.argtypes = [_MP, _D, _D, C.c_void_p, C.c_double, C.c_int, C.c_double, _D]
        L.or_jac_rows.argtypes = [_MP, _D, _D, C.c_int, C.c_double, _D]
        L.or_jac_apply.argtypes = [_D, _D, C.c_int, C.c_double, _D]
        L.or_jac_t_apply.argtypes = [_D, _D, C.c_int, C.c_double, _D]
        L.or_adjoint.argtypes = [_MP, C.c_int, _D, _D, _D, _D, _D, C.c_int, C.c_double,
                                 C.c_int, C.c_int, C.c_int, C.POINTER(Stats)]
        L.or_cic_deposit.argtypes = [C.c_int, C.c_long, _F, _D]
        L.or_kick_drift.argtypes = [C.c_int, C.c_long, _D, _F, _F, C.c_double, C.c_double]
        L.or_kick_drift_damped.argtypes = [C.c_int, C.c_long, _D, _F, _F, C.c_double,
                                           C.c_double, C.c_double]
        _lib = L
    return _lib


# ---------------------------------------------------------------- models

OMEGA_M = 0.3089          # Planck 2015 (Sec. 5)
C_OVER_H0 = 2997.92458    # c/H0 in Mpc/h


def dgp_model(a: float = 1.0, omega_m: float = OMEGA_M, h0rc: float = 1.0) -> Model:
    m = Model()
    beta = C.c_double()
    lib().or_dgp_setup(a, omega_m, h0rc, C.byref(m), C.byref(beta))
    m.beta = beta.value
    return m


def kmo_model(n_mesh: int, box: float, nk: int = 3, k0: float = 1.0, beta: float = 0.1,
              lam: float | None = None, a: float = 1.0, omega_m: float = OMEGA_M,
              phibar: float = 0.0, dphibar_over_h0: float = 0.0) -> Model:
    """Kmouflage model; lam defaults to sqrt(3 (1 - Omega_m)), the LCDM
    limit of the Friedmann equation with K ~ -1."""
    if lam is None:
        lam = float(np.sqrt(3.0 * (1.0 - omega_m)))
    m = Model()
    lib().or_kmo_setup(n_mesh, box, nk, k0, beta, lam, a, omega_m, phibar, dphibar_over_h0,
                       C.byref(m))
    return m


def dgp_newton_model(a: float = 1.0, omega_m: float = OMEGA_M, h0rc: float = 1.0) -> Model:
    """Comparator: the nDGP quadratic form relaxed by Newton-Gauss-Seidel."""
    m = Model()
    lib().or_dgp_newton_setup(a, omega_m, h0rc, C.byref(m))
    return m


def linear_model(s: float) -> Model:
    m = Model()
    lib().or_linear_setup(s, C.byref(m))
    return m


def linearised_dgp_model(a: float = 1.0, omega_m: float = OMEGA_M, h0rc: float = 1.0) -> Model:
    """Comparator: eq:dgp_linear.  At linear order the fifth-force potential
    phi/2 is Phi_N / (3 beta_DGP), and Phi_N obeys lap Phi_N = (3/2) Omega_m
    delta / a (eq:GR_poisson_codeunit), so lap phi = Omega_m delta / (a beta)."""
    beta = dgp_model(a, omega_m, h0rc).beta
    return linear_model(omega_m / (a * beta))


def linearised_kmo_model(n_mesh: int, box: float, nk: int = 3, k0: float = 1.0,
                         beta: float = 0.1, lam: float | None = None, a: float = 1.0,
                         omega_m: float = OMEGA_M, phibar: float = 0.0,
                         dphibar_over_h0: float = 0.0) -> Model:
    """Comparator: eq:linearised_Kmo in code units.  The source of
    eq:kmf_eqn_codeunit_final, 3 beta A(phibar) Omega_m delta / a, divided by
    c~ and by the background K_X = 1 + n K0 (phibar'^2 / (2 lambda^2 a^2))^(n-1)
    (the bracket of eq:linearised_Kmo)."""
    if lam is None:
        lam = float(np.sqrt(3.0 * (1.0 - omega_m)))
    ctil = n_mesh / box * 2997.92458
    kx = 1.0 + nk * k0 * (dphibar_over_h0 ** 2 / (2.0 * lam ** 2 * a ** 2)) ** (nk - 1)
    return linear_model(3.0 * beta * np.exp(beta * phibar) * omega_m / (a * ctil * kx))


def _c(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ------------------------------------------------------------- operators

def residual(m: Model, phi, delta, f=0.0, h: float = 1.0):
    """L^h(phi) - f at every cell (f an array or a scalar)."""
    phi, delta = _c(phi), _c(delta)
    n = phi.shape[0]
    out = np.empty_like(phi)
    if np.isscalar(f):
        lib().or_residual(C.byref(m), phi, delta, None, float(f), n, h, out, None)
    else:
        fa = _c(f)
        lib().or_residual(C.byref(m), phi, delta, fa.ctypes.data, 0.0, n, h, out, None)
    return out


def op_cell(m: Model, phi, delta, i: int, j: int, k: int, h: float = 1.0) -> float:
    """L^h(phi) at one cell (x index i, y index j, z index k)."""
    phi, delta = _c(phi), _c(delta)
    return lib().or_op_cell(C.byref(m), phi, delta, phi.shape[0], h, i, j, k)


def colour_pass(m: Model, phi, delta, colour: int, f=0.0, h: float = 1.0):
    phi, delta = _c(phi), _c(delta)
    out = np.empty_like(phi)
    if np.isscalar(f):
        lib().or_colour_pass(C.byref(m), phi, delta, None, float(f), phi.shape[0], h, colour,
                             out, None)
    else:
        fa = _c(f)
        lib().or_colour_pass(C.byref(m), phi, delta, fa.ctypes.data, 0.0, phi.shape[0], h,
                             colour, out, None)
    return out


def restrict(fine):
    fine = _c(fine)
    n = fine.shape[0]
    out = np.empty((n // 2,) * 3)
    lib().or_restrict(fine, n, out)
    return out


def prolong_add(fine, uc, rc):
    fine = _c(fine).copy()
    lib().or_prolong_add(fine, fine.shape[0], _c(uc), _c(rc))
    return fine


@dataclass
class SolveResult:
    phi: np.ndarray
    status: int
    cycles: int
    eps0: float
    eps: float
    mu: float
    hist: list = field(default_factory=list)
    nclamp: int = 0


CYCLE_V, CYCLE_F, CYCLE_W = 0, 1, 2


def solve(m: Model, delta, phi0=None, max_cycles: int = 50, tol: float = 1e-8,
          nu1: int = 1, nu2: int = 1, nuc: int = 32, h0: float = 1.0,
          cycle: int = CYCLE_V) -> SolveResult:
    """FAS solve with V(nu1,nu2), F or W cycles (Sec. 3.2.1) from phi0
    (default 0) on a mesh of spacing h0; returns the zero-mean phi."""
    delta = _c(delta)
    n = delta.shape[0]
    phi = np.zeros_like(delta) if phi0 is None else _c(phi0).copy()
    st = Stats()
    lib().or_solve_cycle(C.byref(m), n, h0, delta, phi, max_cycles, tol, nu1, nu2, nuc, cycle,
                         None, 0, None, C.byref(st))
    return SolveResult(phi, st.status, st.cycles, st.eps0, st.eps, st.mu,
                       list(st.hist[:min(st.cycles, 256)]), st.nclamp)


def cycle_trace(n: int, cycle: int) -> list:
    """Levels (0 = finest) of the smoothing visits of one cycle on an n^3
    mesh, consecutive visits of the same level merged: the walk drawn in
    fig:multigrid_cycles."""
    delta = np.zeros((n, n, n))
    phi = np.zeros_like(delta)
    cap = 1 << 16
    buf = (C.c_int * cap)()
    cnt = C.c_int(0)
    st = Stats()
    lib().or_solve_cycle(C.byref(linear_model(1.0)), n, 1.0, delta, phi, 1, -1.0, 1, 1, 1, cycle,
                         C.cast(buf, C.c_void_p), cap, C.byref(cnt), C.byref(st))
    walk = []
    for q in range(min(cnt.value, cap)):
        if not walk or walk[-1] != buf[q]:
            walk.append(buf[q])
    return walk


def jac_rows(m: Model, phi, delta, h: float = 1.0):
    phi = _c(phi)
    rows = np.empty(phi.shape + (18,))
    lib().or_jac_rows(C.byref(m), phi, _c(delta), phi.shape[0], h, rows)
    return rows


def jac_apply(rows, v, h: float = 1.0):
    v = _c(v)
    y = np.empty_like(v)
    lib().or_jac_apply(np.ascontiguousarray(rows), v, v.shape[0], h, y)
    return y


def jac_t_apply(rows, v, h: float = 1.0):
    v = _c(v)
    y = np.empty_like(v)
    lib().or_jac_t_apply(np.ascontiguousarray(rows), v, v.shape[0], h, y)
    return y


@dataclass
class AdjointResult:
    grad: np.ndarray
    mu: np.ndarray
    status: int
    cycles: int
    eps0: float
    eps: float
    hist: list


def adjoint(m: Model, delta, phi, w, mu0=None, max_cycles: int = 60, tol: float = 1e-10,
            nu1: int = 1, nu2: int = 1, nuc: int = 32) -> AdjointResult:
    """Gradient of sum(phi * w) w.r.t. delta at the converged forward phi."""
    delta, phi, w = _c(delta), _c(phi), _c(w)
    n = delta.shape[0]
    mu = np.zeros_like(delta) if mu0 is None else _c(mu0).copy()
    grad = np.empty_like(delta)
    st = Stats()
    lib().or_adjoint(C.byref(m), n, delta, phi, w, grad, mu, max_cycles, tol, nu1, nu2, nuc,
                     C.byref(st))
    return AdjointResult(grad, mu, st.status, st.cycles, st.eps0, st.eps,
                         list(st.hist[:min(st.cycles, 256)]))


# ----------------------------------------------------------- PM substrate

def cic_density(pos, n_mesh: int):
    """CIC counts per cell and delta = rho / rho_bar - 1 (FP64)."""
    pos = np.ascontiguousarray(pos, dtype=np.float32)
    npart = pos.shape[0]
    rho = np.empty((n_mesh,) * 3)
    lib().or_cic_deposit(n_mesh, npart, pos.reshape(-1), rho)
    return rho, rho * (n_mesh ** 3 / npart) - 1.0


def fft_poisson(rhs):
    """Zero-mean solution of the 7-point periodic Poisson equation
    lap_h(u) = rhs - mean(rhs), h = 1 (eigenvalues -4 sum sin^2(pi m/N))."""
    rhs = _c(rhs)
    n = rhs.shape[0]
    k = np.fft.fftn(rhs)
    m1 = np.fft.fftfreq(n) * n
    s2 = np.sin(np.pi * m1 / n) ** 2
    eig = -4.0 * (s2[:, None, None] + s2[None, :, None] + s2[None, None, :])
    eig[0, 0, 0] = 1.0
    k = k / eig
    k[0, 0, 0] = 0.0
    return np.real(np.fft.ifftn(k))


def expansion_rate(a: float, omega_m: float = OMEGA_M) -> float:
    """E(a) = H/H0 for flat LCDM (eq:H_lcdm)."""
    return float(np.sqrt(omega_m / a ** 3 + 1.0 - omega_m))


def pm_step(pos, mom, n_mesh: int, a: float, da: float, h0rc: float = 1.0,
            omega_m: float = OMEGA_M, phi0=None, max_cycles: int = 50, tol: float = 1e-8):
    """One nDGP particle-mesh step: CIC density, Newtonian potential by FFT
    (eq:GR_poisson_codeunit), scalar field by multigrid (eq:dgp_eom_code),
    total potential Phi_N + phi/2 (eq:poisson_nDGP), 3-point force with CIC
    interpolation, kick with dp/da = -(H0/adot) grad Phi at a and drift with
    dx/da = (H0/adot) p/a^2 at a + da/2 (leapfrog).  Returns new (pos, mom,
    phi, delta, Phi_N)."""
    pos = np.ascontiguousarray(pos, dtype=np.float32).copy()
    mom = np.ascontiguousarray(mom, dtype=np.float32).copy()
    _, delta = cic_density(pos, n_mesh)
    phin = fft_poisson(1.5 * omega_m / a * delta)
    res = solve(dgp_model(a, omega_m, h0rc), delta, phi0, max_cycles=max_cycles, tol=tol)
    psi = phin + 0.5 * res.phi
    ah = a + 0.5 * da
    kick = da / (a * expansion_rate(a, omega_m))
    drift = da / (ah ** 3 * expansion_rate(ah, omega_m))
    lib().or_kick_drift(n_mesh, pos.shape[0], _c(psi), pos.reshape(-1), mom.reshape(-1), kick,
                        drift)
    return pos, mom, res.phi, delta, phin


def pm_step_newtonian(pos, mom, n_mesh: int, a: float, da: float, omega_m: float = OMEGA_M):
    """The GLAM step of Sec. 3.1 without a fifth force (LCDM): the pm_step
    above with Phi_N alone as the potential.  Returns new (pos, mom, delta)."""
    pos = np.ascontiguousarray(pos, dtype=np.float32).copy()
    mom = np.ascontiguousarray(mom, dtype=np.float32).copy()
    _, delta = cic_density(pos, n_mesh)
    phin = fft_poisson(1.5 * omega_m / a * delta)
    ah = a + 0.5 * da
    kick = da / (a * expansion_rate(a, omega_m))
    drift = da / (ah ** 3 * expansion_rate(ah, omega_m))
    lib().or_kick_drift(n_mesh, pos.shape[0], _c(phin), pos.reshape(-1), mom.reshape(-1), kick,
                        drift)
    return pos, mom, delta


def kmo_background_values(bg, a: float, da: float) -> dict:
    """Background inputs of a Kmouflage PM step from an oracle background
    (oracle.background.solve): E at a and a + da/2, phibar, phibar' and
    d phibar/da at a."""
    ah = a + 0.5 * da
    one = lambda x: float(np.asarray(x).reshape(-1)[0])
    e_a = one(bg.hubble(a))
    dtau = one(bg.dphibar_dtau_over_h0(a))
    return dict(lam=bg.lam, e_a=e_a, e_half=one(bg.hubble(ah)), phibar=one(bg.phibar(a)),
                dphibar_dtau=dtau, dphibar_da=dtau / (a * a * e_a))


def pm_step_kmouflage(pos, mom, n_mesh: int, a: float, da: float, box: float, nk: int,
                      k0: float, beta: float, bgv: dict, omega_m: float = OMEGA_M, phi0=None,
                      max_cycles: int = 50, tol: float = 1e-8):
    """One Kmouflage particle-mesh step (Sec. 3.2.4): CIC density, Newtonian
    potential with the rescaled mass 1.5 A(phibar) Omega_m delta / a by FFT
    (eq:kmf_Poission_eqn_codeunit), the field of eq:kmf_eqn_codeunit_final by
    multigrid, total potential Phi_N + beta c~ phi, and eq:force_Kmo1/2:
    p <- (1 - beta dphibar/da da) p - da/(a E(a)) grad, then the drift with
    da/(a_h^3 E(a_h)).  bgv: kmo_background_values.  Returns new (pos, mom,
    phi, delta, Phi_N)."""
    pos = np.ascontiguousarray(pos, dtype=np.float32).copy()
    mom = np.ascontiguousarray(mom, dtype=np.float32).copy()
    _, delta = cic_density(pos, n_mesh)
    A = np.exp(beta * bgv["phibar"])
    phin = fft_poisson(1.5 * A * omega_m / a * delta)
    m = kmo_model(n_mesh, box, nk, k0, beta, bgv["lam"], a, omega_m, bgv["phibar"],
                  bgv["dphibar_dtau"])
    res = solve(m, delta, phi0, max_cycles=max_cycles, tol=tol)
    ctil = n_mesh / box * 2997.92458
    psi = phin + beta * ctil * res.phi
    ah = a + 0.5 * da
    damp = 1.0 - beta * bgv["dphibar_da"] * da
    lib().or_kick_drift_damped(n_mesh, pos.shape[0], _c(psi), pos.reshape(-1), mom.reshape(-1),
                               damp, da / (a * bgv["e_a"]), da / (ah ** 3 * bgv["e_half"]))
    return pos, mom, res.phi, delta, phin
