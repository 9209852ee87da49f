"""MI355X (gfx950) multigrid solver for derivative-coupling modified gravity.

A thin ctypes binding over ``libmgglam.so`` (C ABI in ``include/mgglam.h``).
Every step of the solve runs in the library's HIP kernels; this module only
marshals arguments.  PyTorch provides device memory (CUDA/HIP tensors) and
the current stream.  The library must be built (``python -m
paper_2110_00566_amd.build``); importing works without it, but every call
raises if it is missing.

Main entry points (tensors are float64, C order [z][y][x], on the GPU):

* ``solve_dgp(delta, phi0=None, a=1, omega_m=0.3089, h0rc=1, ...)``
* ``solve_kmouflage(delta, phi0=None, n_k=3, k0=1, beta=0.1, ...)``
* ``solve_poisson(delta, s, phi0=None, ...)``
* ``solve_adjoint(model, params, delta, phi, w, mu0=None, ...)``
* ``DGPSolve.apply(delta, h0rc, a, omega_m, tol)`` -- autograd wrapper
* ``cic_delta(pos, n_mesh)``, ``pm_step(pos, mom, phi, ...)`` and
  ``pm_step_kmouflage(pos, mom, phi, ...)``
* ``kmo_background(n_k, k0, beta, a)`` -- Kmouflage background cosmology (host)
* comparators: ``solve_dgp_newton``, ``solve_linearised``, ``precision=MG_FP32``
* ``op_*`` single operations of the solve (for parity tests).
"""
from __future__ import annotations

import ctypes as C
import os
import re

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmgglam.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "mgglam.h")

MG_OK, MG_NOT_CONVERGED, MG_WARN_CLAMPED = 0, 1, 2
MG_ERR_ARG, MG_ERR_HIP, MG_ERR_NONFINITE, MG_ERR_DIVERGED, MG_ERR_WORKSPACE = -1, -2, -3, -4, -5
MODEL_DGP, MODEL_KMOUFLAGE, MODEL_POISSON, MODEL_DGP_NEWTON = 0, 1, 2, 3
CYCLE_V, CYCLE_F, CYCLE_W = 0, 1, 2
OMEGA_M = 0.3089
HIST = 64
LEVELS = 16


class MGError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(msg)
        self.status = status


class Opts(C.Structure):
    _fields_ = [("n", C.c_int), ("max_cycles", C.c_int), ("tol", C.c_double),
                ("nu_pre", C.c_int), ("nu_post", C.c_int), ("nu_coarse", C.c_int),
                ("precision", C.c_int), ("cycle", C.c_int), ("profile", C.c_int),
                ("delta_fp32", C.c_int), ("no_sync", C.c_int)]


class Stats(C.Structure):
    _fields_ = [("cycles", C.c_int), ("status", C.c_int), ("eps0", C.c_double),
                ("eps", C.c_double), ("eps_hist", C.c_double * HIST), ("lambda_", C.c_double),
                ("cell_updates", C.c_longlong), ("n_clamped", C.c_longlong),
                ("seconds", C.c_double), ("pass_ms_avg", C.c_double), ("pass_count", C.c_int),
                ("cycles_fp32", C.c_int), ("eps_fp32", C.c_double),
                ("level_ms", C.c_double * LEVELS), ("pm_ms", C.c_double * 4),
                ("pm_newton_cycles", C.c_int)]

    def as_dict(self):
        k = min(self.cycles, HIST)
        return dict(cycles=self.cycles, status=self.status, eps0=self.eps0, eps=self.eps,
                    eps_hist=list(self.eps_hist[:k]), lam=self.lambda_,
                    cell_updates=self.cell_updates, n_clamped=self.n_clamped,
                    seconds=self.seconds, pass_ms_avg=self.pass_ms_avg,
                    pass_count=self.pass_count, cycles_fp32=self.cycles_fp32,
                    eps_fp32=self.eps_fp32, level_ms=list(self.level_ms),
                    pm_ms=list(self.pm_ms), pm_newton_cycles=self.pm_newton_cycles)


class DgpParams(C.Structure):
    _fields_ = [("a", C.c_double), ("omega_m", C.c_double), ("h0rc", C.c_double)]


class KmoParams(C.Structure):
    _fields_ = [("n_k", C.c_int), ("k0", C.c_double), ("beta", C.c_double),
                ("lambda_", C.c_double), ("a", C.c_double), ("omega_m", C.c_double),
                ("box_mpch", C.c_double), ("phibar", C.c_double),
                ("dphibar_dtau_over_h0", C.c_double)]


class KmoBgParams(C.Structure):
    _fields_ = [("n_k", C.c_int), ("k0", C.c_double), ("beta", C.c_double),
                ("omega_m", C.c_double), ("omega_r", C.c_double), ("z_init", C.c_double),
                ("htol", C.c_double)]


class KmoBgInfo(C.Structure):
    _fields_ = [("lambda_", C.c_double), ("h_miss", C.c_double), ("shots", C.c_int),
                ("steps", C.c_int)]


class PoissonParams(C.Structure):
    _fields_ = [("s", C.c_double)]


class PmParams(C.Structure):
    _fields_ = [("n_mesh", C.c_int), ("n_part", C.c_int), ("omega_m", C.c_double),
                ("h0rc", C.c_double), ("a", C.c_double), ("da", C.c_double), ("mg", Opts)]


class KmoBgTable(C.Structure):
    _fields_ = [("n", C.c_int), ("a", C.c_void_p), ("hubble", C.c_void_p),
                ("phibar", C.c_void_p), ("dphibar_dtau", C.c_void_p), ("lambda_", C.c_double)]


class PmKmoParams(C.Structure):
    _fields_ = [("n_mesh", C.c_int), ("n_part", C.c_int), ("a", C.c_double), ("da", C.c_double),
                ("box_mpch", C.c_double), ("bg", KmoBgParams), ("table", C.POINTER(KmoBgTable)),
                ("mg", Opts)]


_lib = None
_P = C.c_void_p


def lib():
    """Load libmgglam.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libmgglam.so is not built: run python -m paper_2110_00566_amd.build")
        L = C.CDLL(LIB_PATH)
        st = C.c_int
        L.mg_workspace_bytes.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int]
        L.mg_workspace_bytes.restype = C.c_size_t
        L.mg_pm_workspace_bytes.argtypes = [C.c_int]
        L.mg_pm_workspace_bytes.restype = C.c_size_t
        L.mg_op_workspace_bytes.argtypes = [C.c_int]
        L.mg_op_workspace_bytes.restype = C.c_size_t
        for name, par in (("mg_solve_dgp", DgpParams), ("mg_solve_kmouflage", KmoParams),
                          ("mg_solve_poisson", PoissonParams), ("mg_solve_dgp_newton", DgpParams)):
            f = getattr(L, name)
            f.argtypes = [C.POINTER(Opts), C.POINTER(par), _P, _P, _P, C.c_size_t, _P,
                          C.POINTER(Stats)]
            f.restype = st
        L.mg_solve_dgp_noalloc.argtypes = [C.POINTER(Opts), C.POINTER(DgpParams), _P, _P, _P,
                                           C.POINTER(Stats)]
        L.mg_solve_dgp_noalloc.restype = st
        L.mg_fft_poisson_workspace_bytes.argtypes = [C.c_int]
        L.mg_fft_poisson_workspace_bytes.restype = C.c_size_t
        L.mg_fft_poisson.argtypes = [C.c_int, C.c_double, _P, _P, _P, C.c_size_t, _P]
        L.mg_fft_poisson.restype = st
        L.mg_solve_adjoint.argtypes = [C.POINTER(Opts), C.c_int, _P, _P, _P, _P, _P, _P, _P,
                                       C.c_size_t, _P, C.POINTER(Stats)]
        L.mg_solve_adjoint.restype = st
        L.mg_pm_step.argtypes = [C.POINTER(PmParams), _P, _P, _P, _P, _P, _P, C.c_size_t, _P,
                                 C.POINTER(Stats)]
        L.mg_pm_step.restype = st
        L.mg_pm_step_kmouflage.argtypes = [C.POINTER(PmKmoParams), _P, _P, _P, _P, _P, _P,
                                           C.c_size_t, _P, C.POINTER(Stats)]
        L.mg_pm_step_kmouflage.restype = st
        for name in ("mg_cic_delta", "mg_cic_delta_f32"):
            getattr(L, name).argtypes = [C.c_int, C.c_int, _P, _P, _P, C.c_size_t, _P]
            getattr(L, name).restype = st
        L.mg_op_residual.argtypes = [C.c_int, _P, C.c_int, C.c_double, _P, _P, _P, C.c_double,
                                     _P, _P, C.c_size_t, _P]
        L.mg_op_residual.restype = st
        L.mg_op_colour_pass.argtypes = [C.c_int, _P, C.c_int, C.c_double, C.c_int, _P, _P, _P,
                                        C.c_double, _P, _P, C.c_size_t, _P]
        L.mg_op_colour_pass.restype = st
        L.mg_op_restrict.argtypes = [C.c_int, _P, _P, _P, C.c_size_t, _P]
        L.mg_op_restrict.restype = st
        L.mg_op_prolong_add.argtypes = [C.c_int, _P, _P, _P, _P, C.c_size_t, _P]
        L.mg_op_prolong_add.restype = st
        L.mg_op_jt_apply.argtypes = [C.c_int, _P, C.c_int, C.c_double, _P, _P, _P, _P, _P,
                                     C.c_size_t, _P]
        L.mg_op_jt_apply.restype = st
        L.mg_omega_radiation.argtypes = [C.c_double, C.c_double, C.c_double]
        L.mg_omega_radiation.restype = C.c_double
        L.mg_kmo_background.argtypes = [C.POINTER(KmoBgParams), C.c_int, _P, _P, _P, _P, _P,
                                        C.POINTER(KmoBgInfo)]
        L.mg_kmo_background.restype = st
        L.mg_linear_source.argtypes = [C.c_int, _P, C.c_int, C.POINTER(C.c_double)]
        L.mg_linear_source.restype = st
        L.mg_status_string.argtypes = [C.c_int]
        L.mg_status_string.restype = C.c_char_p
        L.mg_last_error.argtypes = []
        L.mg_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def header_functions() -> list[str]:
    """Names of the functions declared in include/mgglam.h."""
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(mg_[a-z_0-9]+)\s*\(", txt)))


def _raise(rc: int):
    L = lib()
    if rc < 0:
        raise MGError(rc, "%s: %s" % (L.mg_status_string(rc).decode(), L.mg_last_error().decode()))
    return rc


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _check_mesh(t, name, dtype=torch.float64):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a GPU tensor" % name)
    if t.dtype != dtype or not t.is_contiguous() or t.dim() != 3 or len(set(t.shape)) != 1:
        raise ValueError("%s must be a contiguous %s cube" % (name, dtype))
    return t


MG_FP64, MG_MIXED, MG_FP32, MG_MIXED_DC = 0, 1, 2, 3


def workspace(n: int, model: int = MODEL_DGP, adjoint: bool = False, device=None,
              precision: int = MG_FP64):
    nbytes = lib().mg_workspace_bytes(n, precision, model, int(adjoint))
    if nbytes == 0:
        raise ValueError("invalid mesh size %d" % n)
    return torch.empty(nbytes, dtype=torch.uint8, device=device)


def make_opts(n, tol=1e-8, max_cycles=50, nu_pre=1, nu_post=1, nu_coarse=32, profile=False,
              precision=MG_FP64, cycle=CYCLE_V, delta_fp32=False, no_sync=False):
    """mg_opts.  no_sync: enqueue the solve without waiting (tol = 0, FP64;
    the call can be captured in a HIP graph)."""
    return Opts(n, max_cycles, tol, nu_pre, nu_post, nu_coarse, precision, cycle, int(profile),
                int(delta_fp32), int(no_sync))


def dgp_params(a=1.0, omega_m=OMEGA_M, h0rc=1.0):
    return DgpParams(a, omega_m, h0rc)


def kmo_params(n_mesh, box_mpch, n_k=3, k0=1.0, beta=0.1, lam=None, a=1.0, omega_m=OMEGA_M,
               phibar=0.0, dphibar_dtau_over_h0=0.0):
    if lam is None:
        lam = (3.0 * (1.0 - omega_m)) ** 0.5
    return KmoParams(n_k, k0, beta, lam, a, omega_m, box_mpch, phibar, dphibar_dtau_over_h0)


H_PLANCK = 0.6774      # dimensionless Hubble constant paired with OMEGA_M


def omega_radiation(h=H_PLANCK, t_cmb=2.7255, n_eff=3.046):
    """Radiation density today: photons at t_cmb plus n_eff massless neutrinos."""
    return lib().mg_omega_radiation(h, t_cmb, n_eff)


def kmo_background(n_k, k0, beta, a, omega_m=OMEGA_M, omega_r=None, z_init=1e5, htol=1e-10):
    """Kmouflage background (Sec. 3.2.5) at the scale factors a (increasing):
    dict with lambda, hubble (H/H0), hubble_dot ((dH/dt)/H0^2), phibar and
    dphibar_dtau ((d phibar/d tau)/H0).  Host computation in the library."""
    import numpy as np
    a = np.ascontiguousarray(np.atleast_1d(np.asarray(a, dtype=np.float64)))
    if omega_r is None:
        omega_r = omega_radiation()
    par = KmoBgParams(n_k, k0, beta, omega_m, omega_r, z_init, htol)
    out = {k: np.empty_like(a) for k in ("hubble", "hubble_dot", "phibar", "dphibar_dtau")}
    info = KmoBgInfo()
    ptr = lambda x: x.ctypes.data_as(C.c_void_p)
    _raise(lib().mg_kmo_background(C.byref(par), a.size, ptr(a), ptr(out["hubble"]),
                                   ptr(out["hubble_dot"]), ptr(out["phibar"]),
                                   ptr(out["dphibar_dtau"]), C.byref(info)))
    out.update(a=a, **{"lambda": info.lambda_, "h_miss": info.h_miss, "shots": info.shots,
                       "steps": info.steps})
    return out


def kmo_params_from_background(n_mesh, box_mpch, n_k, k0, beta, a, omega_m=OMEGA_M,
                               omega_r=None):
    """mg_kmo_params at scale factor a with lambda, phibar and phibar' from the
    background solver."""
    bg = kmo_background(n_k, k0, beta, [a], omega_m, omega_r)
    return KmoParams(n_k, k0, beta, bg["lambda"], a, omega_m, box_mpch, float(bg["phibar"][0]),
                     float(bg["dphibar_dtau"][0]))


def _check_delta(delta):
    """delta may be float64 or float32 (mg_opts.delta_fp32); returns the flag."""
    if isinstance(delta, torch.Tensor) and delta.dtype == torch.float32:
        _check_mesh(delta, "delta", torch.float32)
        return True
    _check_mesh(delta, "delta")
    return False


def _zeros64(like):
    return torch.zeros(like.shape, dtype=torch.float64, device=like.device)


def _same_shape(delta, *named):
    for t, nm in named:
        if t.shape != delta.shape:
            raise ValueError("%s must have the shape of delta %s" % (nm, tuple(delta.shape)))


def _solve(fn, par, model, delta, phi0, ws, **kw):
    d32 = _check_delta(delta)
    n = delta.shape[0]
    phi = _zeros64(delta) if phi0 is None else _check_mesh(phi0, "phi0").clone()
    _same_shape(delta, (phi, "phi0"))
    if ws is None:
        ws = workspace(n, model, False, delta.device, kw.get("precision", MG_FP64))
    o = make_opts(n, delta_fp32=d32, **kw)
    st = Stats()
    rc = fn(C.byref(o), C.byref(par), _ptr(delta), _ptr(phi), _ptr(ws), ws.numel(), _stream(),
            C.byref(st))
    _raise(rc)
    return phi, st.as_dict()


def solve_dgp(delta, phi0=None, a=1.0, omega_m=OMEGA_M, h0rc=1.0, ws=None, **kw):
    """nDGP field (eq:dgp_eom_code); returns (zero-mean phi, stats).
    Keywords: tol, max_cycles, nu_pre, nu_post, nu_coarse, profile,
    precision (MG_FP64, MG_MIXED, MG_FP32 or MG_MIXED_DC), cycle (CYCLE_V, CYCLE_F or
    CYCLE_W), no_sync (tol = 0, FP64: the call only enqueues the fixed cycles on the
    current stream; the stats carry no residuals)."""
    return _solve(lib().mg_solve_dgp, dgp_params(a, omega_m, h0rc), MODEL_DGP, delta, phi0, ws, **kw)


def solve_dgp_noalloc(delta, phi0=None, a=1.0, omega_m=OMEGA_M, h0rc=1.0, **kw):
    """solve_dgp through mg_solve_dgp_noalloc: the library's static per-GPU
    workspace, no allocation inside the call (n <= 128).  Returns (phi, stats)."""
    d32 = _check_delta(delta)
    n = delta.shape[0]
    phi = _zeros64(delta) if phi0 is None else _check_mesh(phi0, "phi0").clone()
    _same_shape(delta, (phi, "phi0"))
    o = make_opts(n, delta_fp32=d32, **kw)
    st = Stats()
    _raise(lib().mg_solve_dgp_noalloc(C.byref(o), C.byref(dgp_params(a, omega_m, h0rc)),
                                      _ptr(delta), _ptr(phi), _stream(), C.byref(st)))
    return phi, st.as_dict()


def fft_poisson(delta, s=1.0, phi=None, ws=None):
    """Zero-mean solution of lap7(phi) = s (delta - mean delta) by FFT
    (mg_fft_poisson): the Newtonian potential of the particle-mesh step.
    Returns phi (n^3 float64 on the device)."""
    _check_mesh(delta, "delta")
    n = delta.shape[0]
    if phi is None:
        phi = torch.empty_like(delta)
    elif _check_mesh(phi, "phi").shape != delta.shape:
        raise ValueError("phi and delta must have the same shape")
    if ws is None:
        ws = torch.empty(max(lib().mg_fft_poisson_workspace_bytes(n), 1), dtype=torch.uint8,
                         device=delta.device)
    _raise(lib().mg_fft_poisson(n, float(s), _ptr(delta), _ptr(phi), _ptr(ws), ws.numel(),
                                _stream()))
    return phi


def solve_dgp_newton(delta, phi0=None, a=1.0, omega_m=OMEGA_M, h0rc=1.0, ws=None, **kw):
    """Comparator: the nDGP problem in its quadratic form relaxed by
    Newton-Gauss-Seidel (see mg_solve_dgp_newton); returns (phi, stats)."""
    return _solve(lib().mg_solve_dgp_newton, dgp_params(a, omega_m, h0rc), MODEL_DGP_NEWTON, delta,
                  phi0, ws, **kw)


def solve_kmouflage(delta, phi0=None, box_mpch=512.0, n_k=3, k0=1.0, beta=0.1, lam=None, a=1.0,
                    omega_m=OMEGA_M, phibar=0.0, dphibar_dtau_over_h0=0.0, ws=None, **kw):
    """Kmouflage field (eq:kmf_eqn_codeunit_final); returns (phi, stats)."""
    par = kmo_params(delta.shape[0], box_mpch, n_k, k0, beta, lam, a, omega_m, phibar,
                     dphibar_dtau_over_h0)
    return _solve(lib().mg_solve_kmouflage, par, MODEL_KMOUFLAGE, delta, phi0, ws, **kw)


def linear_source(model, par, n=1):
    """s of the linearised equation lap(phi) = s delta (eq:dgp_linear,
    eq:linearised_Kmo) for MODEL_DGP or MODEL_KMOUFLAGE; n is the mesh size
    (enters c~ of Kmouflage)."""
    s = C.c_double()
    _raise(lib().mg_linear_source(model, C.byref(par), n, C.byref(s)))
    return s.value


def solve_linearised(model, par, delta, phi0=None, ws=None, **kw):
    """Comparator: the linearised field equation of model (MODEL_DGP or
    MODEL_KMOUFLAGE) solved by the Poisson multigrid; returns (phi, stats)."""
    return solve_poisson(delta, linear_source(model, par, delta.shape[0]), phi0, ws, **kw)


def solve_poisson(delta, s, phi0=None, ws=None, **kw):
    """lap(phi) = s (delta - mean delta) by the same multigrid."""
    return _solve(lib().mg_solve_poisson, PoissonParams(s), MODEL_POISSON, delta, phi0, ws, **kw)


def _params_for(model, par):
    if isinstance(par, (DgpParams, KmoParams, PoissonParams)):
        return par
    raise TypeError("params must be DgpParams, KmoParams or PoissonParams")


def solve_adjoint(model, par, delta, phi, w, mu0=None, ws=None, tol=1e-10, max_cycles=60, **kw):
    """Gradient of sum(phi*w) w.r.t. delta at the converged phi.
    Returns (grad_delta, mu, stats)."""
    par = _params_for(model, par)
    d32 = _check_delta(delta)
    for t, nm in ((phi, "phi"), (w, "w")):
        _check_mesh(t, nm)
    n = delta.shape[0]
    mu = _zeros64(delta) if mu0 is None else _check_mesh(mu0, "mu0").clone()
    _same_shape(delta, (phi, "phi"), (w, "w"), (mu, "mu0"))
    grad = torch.empty(delta.shape, dtype=torch.float64, device=delta.device)
    if ws is None:
        ws = workspace(n, model, True, delta.device)
    o = make_opts(n, tol=tol, max_cycles=max_cycles, delta_fp32=d32, **kw)
    st = Stats()
    rc = lib().mg_solve_adjoint(C.byref(o), model, C.byref(par), _ptr(delta), _ptr(phi), _ptr(w),
                                _ptr(grad), _ptr(mu), _ptr(ws), ws.numel(), _stream(),
                                C.byref(st))
    _raise(rc)
    return grad, mu, st.as_dict()


def _require_converged(st, what):
    # an unconverged field (MG_NOT_CONVERGED) would give a silently wrong
    # gradient; a clamped discriminant (MG_WARN_CLAMPED) is converged
    if st["status"] == MG_NOT_CONVERGED:
        raise MGError(MG_NOT_CONVERGED, "%s did not converge (residual %.3g after %d cycles)"
                      % (what, st["eps"], st["cycles"]))


class DGPSolve(torch.autograd.Function):
    """phi = solve_dgp(delta); backward through the adjoint multigrid."""

    @staticmethod
    def forward(ctx, delta, h0rc=1.0, a=1.0, omega_m=OMEGA_M, tol=1e-10):
        phi, st = solve_dgp(delta.detach(), a=a, omega_m=omega_m, h0rc=h0rc, tol=tol,
                            max_cycles=100)
        _require_converged(st, "forward nDGP solve")
        ctx.save_for_backward(delta.detach(), phi)
        ctx.par = dgp_params(a, omega_m, h0rc)
        ctx.tol = tol
        return phi

    @staticmethod
    def backward(ctx, grad_phi):
        delta, phi = ctx.saved_tensors
        g, _, st = solve_adjoint(MODEL_DGP, ctx.par, delta, phi, grad_phi.contiguous(),
                                 tol=ctx.tol, max_cycles=100)
        _require_converged(st, "adjoint solve")
        return g, None, None, None, None


def cic_delta(pos, n_mesh: int, ws=None, dtype=torch.float64):
    """CIC density contrast (n_mesh^3, float64 or float32) of float32
    [n_part^3, 3] positions."""
    if dtype not in (torch.float64, torch.float32):
        raise ValueError("dtype must be torch.float64 or torch.float32")
    if not pos.is_cuda or pos.dtype != torch.float32 or pos.dim() != 2 or pos.shape[1] != 3:
        raise ValueError("pos must be a GPU float32 [n_part^3, 3] tensor")
    n_part = round(pos.shape[0] ** (1.0 / 3.0))
    if n_part ** 3 != pos.shape[0]:
        raise ValueError("number of particles must be a cube")
    delta = torch.empty((n_mesh,) * 3, dtype=dtype, device=pos.device)
    if ws is None:
        ws = torch.empty(lib().mg_pm_workspace_bytes(n_mesh), dtype=torch.uint8, device=pos.device)
    fn = lib().mg_cic_delta if dtype == torch.float64 else lib().mg_cic_delta_f32
    _raise(fn(n_mesh, n_part, _ptr(pos.contiguous()), _ptr(delta), _ptr(ws), ws.numel(),
              _stream()))
    return delta


def _check_pm(pos, mom, phi, phi_newton, n_mesh, require_gpu=True):
    """Arguments of a PM step: pos and mom float32 [n_part^3, 3] (same shape,
    contiguous, a cube number of particles), phi and phi_newton float64
    contiguous n_mesh^3 cubes, all on the GPU.  Returns n_part; raises before
    anything reaches the library."""
    for t, nm in ((pos, "pos"), (mom, "mom")):
        if not isinstance(t, torch.Tensor) or (require_gpu and not t.is_cuda):
            raise TypeError("%s must be a GPU tensor" % nm)
        if t.dtype != torch.float32 or t.dim() != 2 or t.shape[1] != 3 or not t.is_contiguous():
            raise ValueError("%s must be a contiguous float32 [n_part^3, 3] tensor" % nm)
    if mom.shape != pos.shape:
        raise ValueError("pos and mom must have the same shape")
    n_part = round(pos.shape[0] ** (1.0 / 3.0))
    if n_part < 1 or n_part ** 3 != pos.shape[0]:
        raise ValueError("number of particles must be a positive cube")
    for t, nm in ((phi, "phi"), (phi_newton, "phi_newton")):
        if not isinstance(t, torch.Tensor) or (require_gpu and not t.is_cuda):
            raise TypeError("%s must be a GPU tensor" % nm)
        if t.dtype != torch.float64 or not t.is_contiguous() or tuple(t.shape) != (n_mesh,) * 3:
            raise ValueError("%s must be a contiguous float64 tensor of shape (%d, %d, %d)"
                             % ((nm,) + (n_mesh,) * 3))
    return n_part


def pm_step(pos, mom, phi, phi_newton, n_mesh, a, da, h0rc=1.0, omega_m=OMEGA_M, ws=None, **kw):
    """One nDGP PM step in place on pos/mom (float32 [n^3,3]), phi and phi_newton
    (float64 warm starts, updated).  Returns (delta, stats)."""
    n_part = _check_pm(pos, mom, phi, phi_newton, n_mesh)
    delta = torch.empty((n_mesh,) * 3, dtype=torch.float64, device=pos.device)
    if ws is None:
        ws = torch.empty(lib().mg_pm_workspace_bytes(n_mesh), dtype=torch.uint8, device=pos.device)
    par = PmParams(n_mesh, n_part, omega_m, h0rc, a, da, make_opts(n_mesh, **kw))
    st = Stats()
    _raise(lib().mg_pm_step(C.byref(par), _ptr(pos), _ptr(mom), _ptr(phi), _ptr(phi_newton),
                            _ptr(delta), _ptr(ws), ws.numel(), _stream(), C.byref(st)))
    return delta, st.as_dict()


def kmo_bg_params(n_k, k0, beta, omega_m=OMEGA_M, omega_r=None, z_init=1e5, htol=1e-10):
    """mg_kmo_bg_params of a Kmouflage model (omega_r from omega_radiation())."""
    return KmoBgParams(n_k, k0, beta, omega_m, omega_radiation() if omega_r is None else omega_r,
                       z_init, htol)


def pm_step_kmouflage(pos, mom, phi, phi_newton, n_mesh, a, da, box_mpch, n_k=2, k0=1.0,
                      beta=0.2, omega_m=OMEGA_M, table=None, ws=None, **kw):
    """One Kmouflage PM step in place on pos/mom (float32 [n^3,3]), phi and
    phi_newton (float64 warm starts, updated).  The library derives the
    background values of the step; table (a kmo_background() result holding
    a and a + da/2) spares it the background solve.  Returns (delta, stats)."""
    import numpy as np
    n_part = _check_pm(pos, mom, phi, phi_newton, n_mesh)
    delta = torch.empty((n_mesh,) * 3, dtype=torch.float64, device=pos.device)
    if ws is None:
        ws = torch.empty(lib().mg_pm_workspace_bytes(n_mesh), dtype=torch.uint8, device=pos.device)
    tab, keep = None, None
    if table is not None:
        keep = [np.ascontiguousarray(table[k], dtype=np.float64)
                for k in ("a", "hubble", "phibar", "dphibar_dtau")]
        if len({x.size for x in keep}) != 1:
            raise ValueError("table arrays must have equal lengths")
        tab = KmoBgTable(keep[0].size, *[x.ctypes.data for x in keep], table["lambda"])
    par = PmKmoParams(n_mesh, n_part, a, da, box_mpch, kmo_bg_params(n_k, k0, beta, omega_m),
                      C.pointer(tab) if tab is not None else None, make_opts(n_mesh, **kw))
    st = Stats()
    _raise(lib().mg_pm_step_kmouflage(C.byref(par), _ptr(pos), _ptr(mom), _ptr(phi),
                                      _ptr(phi_newton), _ptr(delta), _ptr(ws), ws.numel(),
                                      _stream(), C.byref(st)))
    del keep
    return delta, st.as_dict()


# ------------------------------------------------------------ single ops

def _op_ws(n, device):
    return torch.empty(lib().mg_op_workspace_bytes(n), dtype=torch.uint8, device=device)


def _model_of(par):
    return {DgpParams: MODEL_DGP, KmoParams: MODEL_KMOUFLAGE, PoissonParams: MODEL_POISSON}[type(par)]


def op_residual(par, phi, delta, f=0.0, h=1.0, model=None):
    """L_h(phi) - f; model defaults to the one of par (MODEL_DGP_NEWTON takes
    DgpParams)."""
    model = _model_of(par) if model is None else model
    n = phi.shape[0]
    out = torch.empty_like(phi)
    ws = _op_ws(n, phi.device)
    fa = f if isinstance(f, torch.Tensor) else None
    fs = 0.0 if fa is not None else float(f)
    _raise(lib().mg_op_residual(model, C.byref(par), n, h, _ptr(phi), _ptr(delta),
                                _ptr(fa), fs, _ptr(out), _ptr(ws), ws.numel(), _stream()))
    return out


def op_colour_pass(par, phi, delta, colour, f=0.0, h=1.0, model=None):
    model = _model_of(par) if model is None else model
    n = phi.shape[0]
    out = torch.empty_like(phi)
    ws = _op_ws(n, phi.device)
    fa = f if isinstance(f, torch.Tensor) else None
    fs = 0.0 if fa is not None else float(f)
    _raise(lib().mg_op_colour_pass(model, C.byref(par), n, h, colour, _ptr(phi),
                                   _ptr(delta), _ptr(fa), fs, _ptr(out), _ptr(ws), ws.numel(),
                                   _stream()))
    return out


def op_restrict(fine):
    n = fine.shape[0]
    out = torch.empty((n // 2,) * 3, dtype=fine.dtype, device=fine.device)
    ws = _op_ws(n, fine.device)
    _raise(lib().mg_op_restrict(n, _ptr(fine), _ptr(out), _ptr(ws), ws.numel(), _stream()))
    return out


def op_prolong_add(fine, uc, rc):
    n = fine.shape[0]
    out = fine.clone()
    ws = _op_ws(n, fine.device)
    _raise(lib().mg_op_prolong_add(n, _ptr(out), _ptr(uc), _ptr(rc), _ptr(ws), ws.numel(),
                                   _stream()))
    return out


def op_jt_apply(par, phi, delta, v, h=1.0):
    n = phi.shape[0]
    out = torch.empty_like(phi)
    ws = _op_ws(n, phi.device)
    _raise(lib().mg_op_jt_apply(_model_of(par), C.byref(par), n, h, _ptr(phi), _ptr(delta),
                                _ptr(v), _ptr(out), _ptr(ws), ws.numel(), _stream()))
    return out
