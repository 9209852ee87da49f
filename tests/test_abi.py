"""The C ABI library loads, exports every function include/mgglam.h declares,
and rejects invalid arguments before touching the GPU (CPU only)."""
import ctypes as C

import pytest

import paper_2110_00566_amd as mg


@pytest.fixture(scope="module")
def L():
    return mg.lib()


def test_header_declares_the_entry_points():
    names = mg.header_functions()
    for must in ("mg_solve_dgp", "mg_solve_kmouflage", "mg_solve_adjoint", "mg_pm_step",
                 "mg_workspace_bytes", "mg_status_string", "mg_last_error", "mg_cic_delta"):
        assert must in names


def test_every_declared_symbol_is_exported(L):
    missing = [n for n in mg.header_functions() if not hasattr(L, n)]
    assert missing == []


def test_workspace_sizes(L):
    assert L.mg_workspace_bytes(7, 0, 0, 0) == 0
    assert L.mg_workspace_bytes(4096, 0, 0, 0) == 0
    assert L.mg_workspace_bytes(32, 3, 0, 0) == 0          # unknown precision
    assert L.mg_workspace_bytes(32, 1, 0, 1) == 0          # the adjoint is FP64 only
    assert L.mg_workspace_bytes(32, 2, 0, 1) == 0
    assert L.mg_workspace_bytes(32, 2, 3, 0) == 0          # Newton-GS comparator: FP64 only
    # mixed keeps an FP32 hierarchy beside the FP64 one; all-FP32 has only the FP32 one
    assert L.mg_workspace_bytes(64, 1, 0, 0) > L.mg_workspace_bytes(64, 0, 0, 0)
    f32, f64 = L.mg_workspace_bytes(64, 2, 0, 0), L.mg_workspace_bytes(64, 0, 0, 0)
    assert f32 < 0.6 * f64
    assert L.mg_workspace_bytes(64, 1, 0, 0) >= f32 + f64 - 2 * 8 * 64 ** 3
    a = L.mg_workspace_bytes(64, 0, 0, 0)
    b = L.mg_workspace_bytes(64, 0, 0, 1)
    # finest level: 5 half-arrays of FP64 = 20 bytes per cell, coarse levels add < 1/2
    assert 20 * 64 ** 3 <= a <= 40 * 64 ** 3
    assert b > a
    # adjoint: the nDGP and Poisson minus face coefficients alias the plus
    # ones, 3 FP64 arrays of both colours (24 B/cell) fewer than Kmouflage
    bk = L.mg_workspace_bytes(64, 0, 1, 1)
    assert bk - b >= 24 * 64 ** 3
    assert L.mg_workspace_bytes(64, 0, 2, 1) == b
    assert L.mg_workspace_bytes(64, 0, 0, 0) == a          # deterministic
    assert L.mg_pm_workspace_bytes(64) >= a + 8 * 64 ** 3


def _bad_solve(L, **over):
    o = mg.make_opts(32)
    for k, v in over.items():
        setattr(o, k, v)
    st = mg.Stats()
    par = mg.dgp_params()
    dummy = C.c_void_p(0x1000)
    return L.mg_solve_dgp(C.byref(o), C.byref(par), dummy, dummy, dummy, 1 << 30, None,
                          C.byref(st))


@pytest.mark.parametrize("field,value", [("n", 24), ("n", 4), ("n", 4096), ("tol", -1.0),
                                         ("tol", float("nan")), ("max_cycles", -1),
                                         ("nu_coarse", 0), ("precision", 7), ("cycle", 3),
                                         ("cycle", -1)])
def test_invalid_options_rejected_before_gpu(L, field, value):
    assert _bad_solve(L, **{field: value}) == mg.MG_ERR_ARG
    assert len(L.mg_last_error()) > 0


def test_linear_source_host_values(L):
    # host-only coefficient of the linearised equations, against the oracle's
    # independent derivation (eq:dgp_linear, eq:linearised_Kmo)
    import oracle
    for a, h0rc in ((1.0, 1.0), (0.5, 0.3)):
        s = mg.linear_source(mg.MODEL_DGP, mg.dgp_params(a, 0.3089, h0rc))
        assert s == pytest.approx(oracle.linearised_dgp_model(a, 0.3089, h0rc).s, rel=1e-14)
    args = (128, 256.0, 3, 2.0, 0.15, 1.3, 0.9, 0.3089, 0.01, 0.7)
    s = mg.linear_source(mg.MODEL_KMOUFLAGE, mg.kmo_params(*args), 128)
    assert s == pytest.approx(oracle.linearised_kmo_model(*args).s, rel=1e-14)
    with pytest.raises(mg.MGError):
        mg.linear_source(mg.MODEL_POISSON, mg.PoissonParams(1.0))
    with pytest.raises(mg.MGError):
        mg.linear_source(mg.MODEL_DGP, mg.DgpParams(1.0, 0.3089, -1.0))
    out = C.c_double()
    assert L.mg_linear_source(mg.MODEL_DGP, None, 1, C.byref(out)) == mg.MG_ERR_ARG


def test_invalid_model_parameters_rejected(L):
    o = mg.make_opts(32)
    st = mg.Stats()
    d = C.c_void_p(0x1000)
    bad = mg.DgpParams(1.0, 0.3089, -1.0)
    assert L.mg_solve_dgp(C.byref(o), C.byref(bad), d, d, d, 1 << 30, None, C.byref(st)) == mg.MG_ERR_ARG
    badk = mg.kmo_params(32, 64.0, n_k=1)
    assert L.mg_solve_kmouflage(C.byref(o), C.byref(badk), d, d, d, 1 << 30, None,
                                C.byref(st)) == mg.MG_ERR_ARG


def test_null_pointers_and_workspace(L):
    o = mg.make_opts(32)
    st = mg.Stats()
    par = mg.dgp_params()
    d = C.c_void_p(0x1000)
    assert L.mg_solve_dgp(C.byref(o), C.byref(par), None, d, d, 1 << 30, None, C.byref(st)) == mg.MG_ERR_ARG
    assert L.mg_solve_dgp(C.byref(o), C.byref(par), d, d, None, 1 << 30, None, C.byref(st)) == mg.MG_ERR_WORKSPACE
    assert L.mg_solve_dgp(C.byref(o), C.byref(par), d, d, d, 16, None, C.byref(st)) == mg.MG_ERR_WORKSPACE
    assert L.mg_solve_dgp(None, C.byref(par), d, d, d, 1 << 30, None, C.byref(st)) == mg.MG_ERR_ARG
    # workspaces start on 256-byte boundaries (the tiled kernels read 16-byte vectors)
    odd = C.c_void_p(0x1000 + 8)
    assert L.mg_solve_dgp(C.byref(o), C.byref(par), d, d, odd, 1 << 30, None, C.byref(st)) == mg.MG_ERR_WORKSPACE
    assert b"aligned" in L.mg_last_error()
    assert L.mg_cic_delta(32, 16, d, d, odd, 1 << 40, None) == mg.MG_ERR_WORKSPACE
    assert b"aligned" in L.mg_last_error()
    assert L.mg_cic_delta_f32(32, 16, d, d, odd, 1 << 40, None) == mg.MG_ERR_WORKSPACE
    assert L.mg_cic_delta_f32(24, 16, d, d, d, 1 << 40, None) == mg.MG_ERR_ARG


def test_adjoint_accepts_v_cycles_only(L):
    o = mg.make_opts(32, cycle=mg.CYCLE_W)
    st = mg.Stats()
    d = C.c_void_p(0x1000)
    par = mg.dgp_params()
    rc = L.mg_solve_adjoint(C.byref(o), mg.MODEL_DGP, C.byref(par), d, d, d, d, d, d, 1 << 30,
                            None, C.byref(st))
    assert rc == mg.MG_ERR_ARG
    assert b"V-cycles" in L.mg_last_error()


def test_status_strings(L):
    for s in (0, 1, 2, -1, -2, -3, -4, -5):
        assert L.mg_status_string(s).startswith(b"MG_")


def test_product_does_not_import_the_oracle():
    import pathlib
    pkg = pathlib.Path(mg.__file__).parent
    for f in list(pkg.rglob("*.py")) + list(pkg.rglob("*.hip")) + list(pkg.rglob("*.h")):
        txt = f.read_text()
        assert "import oracle" not in txt and "from oracle" not in txt and "mg_oracle" not in txt


def test_bench_refuses_more_than_one_gpu():
    # one GPU only: --gpus N > 1 exits with a message before touching a device
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_pm_entry_points_reject_bad_arguments_with_a_message(L):
    d = C.c_void_p(0x1000)
    assert L.mg_cic_delta(24, 16, d, d, d, 1 << 40, None) == mg.MG_ERR_ARG
    assert b"power of two" in L.mg_last_error()
    assert L.mg_cic_delta(32, 16, d, d, None, 0, None) == mg.MG_ERR_WORKSPACE
    assert len(L.mg_last_error()) > 0
    par = mg.PmParams(32, 16, 0.3089, 1.0, 1.0, 0.01, mg.make_opts(16))
    st = mg.Stats()
    assert L.mg_pm_step(C.byref(par), d, d, d, d, d, d, 1 << 40, None, C.byref(st)) == mg.MG_ERR_ARG
    assert b"mg.n" in L.mg_last_error()
    bgp = mg.kmo_bg_params(2, 1.0, 0.2)
    kp = mg.PmKmoParams(32, 16, 0.99, 0.04, 64.0, bgp, None, mg.make_opts(32))
    assert L.mg_pm_step_kmouflage(C.byref(kp), d, d, d, d, d, d, 1 << 40, None,
                                  C.byref(st)) == mg.MG_ERR_ARG
    assert b"a + da/2 <= 1" in L.mg_last_error()
    # a table must hold a and a + da/2; the lookup fails before any GPU work
    import numpy as np
    arr = [np.array([0.5, 0.6]), np.ones(2), np.zeros(2), np.zeros(2)]
    tab = mg.KmoBgTable(2, *[x.ctypes.data for x in arr], 1.2)
    kp = mg.PmKmoParams(32, 16, 0.5, 0.01, 64.0, bgp, C.pointer(tab), mg.make_opts(32))
    assert L.mg_pm_step_kmouflage(C.byref(kp), d, d, d, d, d, d, 1 << 40, None,
                                  C.byref(st)) == mg.MG_ERR_ARG
    assert b"a + da/2" in L.mg_last_error()
    bad = mg.KmoBgParams(2, 1.0, 0.2, 1.5, 0.0, 1e5, 1e-10)   # Omega_m > 1
    kp = mg.PmKmoParams(32, 16, 0.5, 0.01, 64.0, bad, None, mg.make_opts(32))
    assert L.mg_pm_step_kmouflage(C.byref(kp), d, d, d, d, d, d, 1 << 40, None,
                                  C.byref(st)) == mg.MG_ERR_ARG
    assert b"background parameters" in L.mg_last_error()


def _cpu_pm_args(n_part=4, n_mesh=8):
    import torch
    pos = torch.zeros((n_part ** 3, 3), dtype=torch.float32)
    return pos, pos.clone(), torch.zeros((n_mesh,) * 3, dtype=torch.float64), \
        torch.zeros((n_mesh,) * 3, dtype=torch.float64)


def test_pm_binding_rejects_bad_tensors_before_the_library(monkeypatch):
    # every malformed argument raises in the binding, before any library call
    import torch
    monkeypatch.setattr(mg, "lib", lambda: pytest.fail("library reached"))
    pos, mom, phi, phin = _cpu_pm_args()
    assert mg._check_pm(pos, mom, phi, phin, 8, require_gpu=False) == 4
    cases = [
        (pos.double(), mom, phi, phin),                      # pos dtype
        (pos, mom[:-1], phi, phin),                          # mom shape
        (pos[:-1], mom[:-1], phi, phin),                     # not a cube
        (pos.t().contiguous().t(), mom, phi, phin),          # non-contiguous
        (pos, mom, phi.float(), phin),                       # phi dtype
        (pos, mom, phi, torch.zeros((8, 8, 4), dtype=torch.float64)),   # phi_newton shape
        (pos, mom, torch.zeros((16,) * 3, dtype=torch.float64), phin),  # phi size != n_mesh
        (pos[:, :2].contiguous(), mom[:, :2].contiguous(), phi, phin),  # not [N, 3]
    ]
    for args in cases:
        with pytest.raises((ValueError, TypeError)):
            mg._check_pm(*args, 8, require_gpu=False)
    # the public entry points refuse host tensors outright
    for fn, extra in ((mg.pm_step, ()), (mg.pm_step_kmouflage, (64.0,))):
        with pytest.raises(TypeError):
            fn(pos, mom, phi, phin, 8, 0.5, 0.01, *extra)


def test_autograd_refuses_an_unconverged_solve():
    with pytest.raises(mg.MGError):
        mg._require_converged({"status": mg.MG_NOT_CONVERGED, "eps": 1e-3, "cycles": 5}, "x")
    mg._require_converged({"status": mg.MG_WARN_CLAMPED, "eps": 1e-12, "cycles": 5}, "x")


def test_struct_layouts_match_the_header(tmp_path):
    # sizes and field offsets of every ABI struct, compiled from
    # include/mgglam.h by the host C compiler, against the ctypes mirrors
    import os
    import subprocess
    pairs = {"mg_opts": mg.Opts, "mg_stats": mg.Stats, "mg_dgp_params": mg.DgpParams,
             "mg_kmo_params": mg.KmoParams, "mg_kmo_bg_params": mg.KmoBgParams,
             "mg_kmo_bg_info": mg.KmoBgInfo, "mg_poisson_params": mg.PoissonParams,
             "mg_pm_params": mg.PmParams, "mg_kmo_bg_table": mg.KmoBgTable,
             "mg_pm_kmo_params": mg.PmKmoParams}
    lines, expect = [], []
    for cname, py in pairs.items():
        lines.append('printf("%%zu\\n", sizeof(%s));' % cname)
        expect.append(C.sizeof(py))
        for fname, _ in py._fields_:
            cf = fname.rstrip("_")
            lines.append('printf("%%zu\\n", offsetof(%s, %s));' % (cname, cf))
            expect.append(getattr(py, fname).offset)
    src = tmp_path / "layout.c"
    src.write_text("#include <stddef.h>\n#include <stdio.h>\n#include \"mgglam.h\"\n"
                   "int main(void) {\n" + "\n".join(lines) + "\nreturn 0;\n}\n")
    exe = tmp_path / "layout"
    inc = os.path.join(os.path.dirname(mg.HEADER))
    rocm = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "include")
    subprocess.check_call(["gcc", "-D__HIP_PLATFORM_AMD__", "-I" + rocm, "-I" + inc, str(src),
                           "-o", str(exe)])
    got = [int(x) for x in subprocess.check_output([str(exe)]).split()]
    assert got == expect


def test_noalloc_entry_point_validates_before_the_gpu(L):
    d = C.c_void_p(0x1000)
    st = mg.Stats()
    par = mg.dgp_params()
    o = mg.make_opts(256)
    assert L.mg_solve_dgp_noalloc(C.byref(o), C.byref(par), d, d, None, C.byref(st)) == mg.MG_ERR_ARG
    assert b"<= 128" in L.mg_last_error()
    o = mg.make_opts(64, profile=True)
    assert L.mg_solve_dgp_noalloc(C.byref(o), C.byref(par), d, d, None, C.byref(st)) == mg.MG_ERR_ARG
    assert b"profile" in L.mg_last_error()
    o = mg.make_opts(64)
    assert L.mg_solve_dgp_noalloc(C.byref(o), None, d, d, None, C.byref(st)) == mg.MG_ERR_ARG
    assert L.mg_solve_dgp_noalloc(C.byref(o), C.byref(par), None, d, None, C.byref(st)) == mg.MG_ERR_ARG


def test_defect_correction_arguments(L):
    # MG_MIXED_DC: n >= 128, nDGP and Poisson only (checked before the GPU)
    assert L.mg_workspace_bytes(64, mg.MG_MIXED_DC, mg.MODEL_DGP, 0) == 0
    assert L.mg_workspace_bytes(128, mg.MG_MIXED_DC, mg.MODEL_DGP, 0) > \
        L.mg_workspace_bytes(128, mg.MG_MIXED, mg.MODEL_DGP, 0)
    assert L.mg_workspace_bytes(128, mg.MG_MIXED_DC, mg.MODEL_DGP, 1) == 0
    d = C.c_void_p(0x1000)
    st = mg.Stats()
    o = mg.make_opts(64, precision=mg.MG_MIXED_DC)
    assert L.mg_solve_dgp(C.byref(o), C.byref(mg.dgp_params()), d, d, d, 1 << 40, None,
                          C.byref(st)) == mg.MG_ERR_ARG
    assert b"128" in L.mg_last_error()
    o = mg.make_opts(128, precision=mg.MG_MIXED_DC)
    kp = mg.kmo_params(128, 256.0)
    assert L.mg_solve_kmouflage(C.byref(o), C.byref(kp), d, d, d, 1 << 40, None,
                                C.byref(st)) == mg.MG_ERR_ARG
    assert b"nDGP and Poisson" in L.mg_last_error()


def test_fft_poisson_validates_before_the_gpu(L):
    assert L.mg_fft_poisson_workspace_bytes(12) == 0
    assert L.mg_fft_poisson_workspace_bytes(4096) == 0
    assert L.mg_fft_poisson_workspace_bytes(64) >= 32 * 16      # n / 2 complex twiddles
    d, e, w = C.c_void_p(0x1000), C.c_void_p(0x2000), C.c_void_p(0x3000)
    big = 1 << 20
    assert L.mg_fft_poisson(48, 1.0, d, e, w, big, None) == mg.MG_ERR_ARG
    assert b"power of two" in L.mg_last_error()
    assert L.mg_fft_poisson(64, float("nan"), d, e, w, big, None) == mg.MG_ERR_ARG
    assert L.mg_fft_poisson(64, 1.0, None, e, w, big, None) == mg.MG_ERR_ARG
    assert L.mg_fft_poisson(64, 1.0, d, d, w, big, None) == mg.MG_ERR_ARG
    assert b"alias" in L.mg_last_error()
    assert L.mg_fft_poisson(64, 1.0, d, e, None, big, None) == mg.MG_ERR_WORKSPACE
    assert L.mg_fft_poisson(64, 1.0, d, e, w, 16, None) == mg.MG_ERR_WORKSPACE
    assert L.mg_fft_poisson(64, 1.0, d, e, C.c_void_p(0x3000 + 8), big, None) == mg.MG_ERR_WORKSPACE


def test_fft_poisson_requires_16_byte_alignment(L):
    d, e, w = C.c_void_p(0x1008), C.c_void_p(0x2000), C.c_void_p(0x3000)
    assert L.mg_fft_poisson(64, 1.0, d, e, w, 1 << 20, None) == mg.MG_ERR_ARG
    assert b"16-byte" in L.mg_last_error()


def test_delta_precision_flag_validated(L):
    d = C.c_void_p(0x1000)
    st = mg.Stats()
    o = mg.make_opts(32)
    o.delta_fp32 = 2
    assert L.mg_solve_dgp(C.byref(o), C.byref(mg.dgp_params()), d, d, d, 1 << 40, None,
                          C.byref(st)) == mg.MG_ERR_ARG
    assert b"delta_fp32" in L.mg_last_error()


def test_no_sync_flag_validated(L):
    # enqueue-only solves need tol = 0, profile = 0 and FP64; the adjoint and
    # the PM steps wait for their stream and refuse the flag
    d = C.c_void_p(0x1000)
    st = mg.Stats()
    par = mg.dgp_params()
    for over in (dict(no_sync=2), dict(no_sync=1), dict(no_sync=1, tol=0.0, profile=1),
                 dict(no_sync=1, tol=0.0, precision=mg.MG_MIXED),
                 dict(no_sync=1, tol=0.0, precision=mg.MG_FP32)):
        o = mg.make_opts(32)
        for k, v in over.items():
            setattr(o, k, v)
        assert L.mg_solve_dgp(C.byref(o), C.byref(par), d, d, d, 1 << 40, None,
                              C.byref(st)) == mg.MG_ERR_ARG, over
        assert b"no_sync" in L.mg_last_error()
    o = mg.make_opts(32, tol=0.0, no_sync=True)
    assert L.mg_solve_adjoint(C.byref(o), mg.MODEL_DGP, C.byref(par), d, d, d, d, d, d, 1 << 40,
                              None, C.byref(st)) == mg.MG_ERR_ARG
    assert b"no_sync" in L.mg_last_error()
    pm = mg.PmParams(32, 16, 0.3089, 1.0, 1.0, 0.01, o)
    assert L.mg_pm_step(C.byref(pm), d, d, d, d, d, d, 1 << 40, None, C.byref(st)) == mg.MG_ERR_ARG
    assert b"no_sync" in L.mg_last_error()
    kp = mg.PmKmoParams(32, 16, 0.5, 0.01, 64.0, mg.kmo_bg_params(2, 1.0, 0.2), None, o)
    assert L.mg_pm_step_kmouflage(C.byref(kp), d, d, d, d, d, d, 1 << 40, None,
                                  C.byref(st)) == mg.MG_ERR_ARG
    assert b"no_sync" in L.mg_last_error()
