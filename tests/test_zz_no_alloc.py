"""mg_solve_dgp_noalloc (static per-GPU workspace, nothing allocated in the
call) against mg_solve_dgp (caller's workspace) through the C ABI: the same
kernels on the same inputs give the same field, residual history and cycle
count.  Two calls in a row, the second on a smaller mesh, so the second runs
on whatever the first left in the shared array."""
import ctypes as C

import numpy as np
import pytest
import torch

import inputs
import paper_2110_00566_amd as mg

pytestmark = pytest.mark.gpu


def _call_with_workspace(delta, **kw):
    n = delta.shape[0]
    ws = mg.workspace(n, mg.MODEL_DGP, False, delta.device, kw.get("precision", mg.MG_FP64))
    return mg.solve_dgp(delta, ws=ws, **kw)


def _call_noalloc(delta, **kw):
    L = mg.lib()
    n = delta.shape[0]
    phi = torch.zeros_like(delta)
    o = mg.make_opts(n, **kw)
    st = mg.Stats()
    print("mg_solve_dgp_noalloc n=%d %s" % (n, kw), flush=True)
    rc = L.mg_solve_dgp_noalloc(C.byref(o), C.byref(mg.dgp_params()), mg._ptr(delta),
                                mg._ptr(phi), mg._stream(), C.byref(st))
    torch.cuda.synchronize()
    assert rc == mg.MG_OK, (rc, L.mg_last_error())
    return phi, st.as_dict()


@pytest.mark.parametrize("precision", [0, 1, 2])
def test_noalloc_matches_workspace_entry_point_twice(precision):
    kw = dict(tol=1e-8 if precision != mg.MG_FP32 else 1e-5, max_cycles=30, precision=precision)
    for n, seed in ((128, 21), (64, 22)):          # second call smaller
        delta = torch.from_numpy(inputs.lognormal_delta(n, seed)).to("cuda")
        ref, st_ref = _call_with_workspace(delta, **kw)
        got, st = _call_noalloc(delta, **kw)
        assert st["status"] == st_ref["status"] and st["status"] >= 0
        assert st["cycles"] == st_ref["cycles"]
        assert st["eps_hist"] == st_ref["eps_hist"]
        assert torch.equal(got, ref), float((got - ref).abs().max())


def test_noalloc_rejects_meshes_beyond_its_workspace():
    L = mg.lib()
    delta = torch.zeros((256,) * 3, dtype=torch.float64, device="cuda")
    phi = torch.zeros_like(delta)
    o = mg.make_opts(256)
    st = mg.Stats()
    rc = L.mg_solve_dgp_noalloc(C.byref(o), C.byref(mg.dgp_params()), mg._ptr(delta),
                                mg._ptr(phi), mg._stream(), C.byref(st))
    assert rc == mg.MG_ERR_ARG
    assert b"<= 128" in L.mg_last_error()
    assert float(phi.abs().max()) == 0.0
