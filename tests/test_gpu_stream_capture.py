"""Enqueue-only solves (mg_opts.no_sync = 1) through the C ABI.

A no_sync call enqueues the launches of a synchronous tol = 0 solve of
max_cycles cycles and returns without waiting, so its field must equal the
synchronous one bit for bit.  Because it reads nothing back, allocates
nothing and records no memset, it can be captured in a HIP graph: each
replay of the graph (with eager work, other solves and synchronisations in
between) must give the eager result of the same input bit for bit."""
import ctypes as C
import math

import pytest
import torch

import inputs
import paper_2110_00566_amd as mg

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda:0")


def _params(model, n):
    if model == mg.MODEL_KMOUFLAGE:
        return mg.kmo_params(n, 0.02 * n, 3, 1.0, 0.1)
    if model == mg.MODEL_POISSON:
        return mg.PoissonParams(1.5 * mg.OMEGA_M)
    return mg.dgp_params()


def _entry(L, model):
    return {mg.MODEL_DGP: L.mg_solve_dgp, mg.MODEL_KMOUFLAGE: L.mg_solve_kmouflage,
            mg.MODEL_POISSON: L.mg_solve_poisson, mg.MODEL_DGP_NEWTON: L.mg_solve_dgp_newton}[model]


def _call(L, model, par, opts, delta, phi, ws):
    st = mg.Stats()
    rc = _entry(L, model)(C.byref(opts), C.byref(par), mg._ptr(delta), mg._ptr(phi),
                          mg._ptr(ws), ws.numel(), mg._stream(), C.byref(st))
    return rc, st


def _delta(n, seed):
    return torch.from_numpy(inputs.lognormal_delta(n, seed)).to(DEV)


@pytest.mark.parametrize("model,n,cycle", [(mg.MODEL_DGP, 32, mg.CYCLE_V),
                                           (mg.MODEL_DGP, 128, mg.CYCLE_V),
                                           (mg.MODEL_DGP, 128, mg.CYCLE_W),
                                           (mg.MODEL_KMOUFLAGE, 128, mg.CYCLE_V),
                                           (mg.MODEL_POISSON, 64, mg.CYCLE_F),
                                           (mg.MODEL_DGP_NEWTON, 64, mg.CYCLE_V)])
def test_no_sync_equals_the_synchronous_fixed_cycle_solve(model, n, cycle):
    print("no_sync vs sync: model %d n %d cycle %d" % (model, n, cycle), flush=True)
    L = mg.lib()
    par = _params(model, n)
    delta = _delta(n, 11)
    ws = mg.workspace(n, model, False, DEV)
    ref = torch.zeros_like(delta)
    rc, st = _call(L, model, par, mg.make_opts(n, tol=0.0, max_cycles=4, cycle=cycle),
                   delta, ref, ws)
    assert rc == mg.MG_NOT_CONVERGED, (rc, L.mg_last_error())
    assert st.cycles == 4
    phi = torch.zeros_like(delta)
    rc, st = _call(L, model, par,
                   mg.make_opts(n, tol=0.0, max_cycles=4, cycle=cycle, no_sync=True),
                   delta, phi, ws)
    assert rc == mg.MG_NOT_CONVERGED, (rc, L.mg_last_error())
    torch.cuda.synchronize()
    assert st.cycles == 4 and st.status == mg.MG_NOT_CONVERGED
    assert math.isnan(st.eps) and math.isnan(st.eps0) and math.isnan(st.lambda_)
    assert st.n_clamped == -1
    assert torch.isfinite(phi).all()
    assert torch.equal(phi, ref)


def test_no_sync_zero_cycles_is_the_gauged_initial_guess():
    # max_cycles = 0: only the initial residual, the gauge and the output
    L = mg.lib()
    n = 32
    delta = _delta(n, 12)
    ws = mg.workspace(n, mg.MODEL_DGP, False, DEV)
    phi0 = torch.from_numpy(inputs.uniform_phi(n, 13)).to(DEV)
    phi = phi0.clone()
    rc, st = _call(L, mg.MODEL_DGP, mg.dgp_params(),
                   mg.make_opts(n, tol=0.0, max_cycles=0, no_sync=True), delta, phi, ws)
    torch.cuda.synchronize()
    assert rc == mg.MG_NOT_CONVERGED and st.cycles == 0
    torch.testing.assert_close(phi, phi0 - phi0.mean(), rtol=0, atol=1e-15)


def _graph_replays(L, call_captured, call_eager, static_delta, phi, deltas):
    """Capture call_captured() once, then replay it on each input of deltas
    (copied into static_delta, phi zeroed first) and compare with
    call_eager(delta) computed between the replays."""
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):   # a first solve sets the one-time kernel attributes
        assert call_captured() == mg.MG_NOT_CONVERGED, L.mg_last_error()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    phi.zero_()
    with torch.cuda.graph(g):
        rc = call_captured()
    assert rc == mg.MG_NOT_CONVERGED, L.mg_last_error()
    for rep, d in enumerate(deltas):
        print("replay %d" % rep, flush=True)
        static_delta.copy_(d)
        phi.zero_()
        g.replay()
        torch.cuda.synchronize()
        got = phi.clone()
        ref = call_eager(d)
        torch.cuda.synchronize()
        assert torch.isfinite(got).all()
        assert torch.equal(got, ref), (rep, float((got - ref).abs().max()))
    del g


def test_no_sync_solve_replays_from_a_hip_graph():
    L = mg.lib()
    n = 128
    par = mg.dgp_params()
    deltas = [_delta(n, s) for s in (21, 22, 23)] * 2
    static_delta = deltas[0].clone()
    phi = torch.zeros_like(static_delta)
    ws = mg.workspace(n, mg.MODEL_DGP, False, DEV)
    ws_ref = mg.workspace(n, mg.MODEL_DGP, False, DEV)
    o_ns = mg.make_opts(n, tol=0.0, max_cycles=3, no_sync=True)
    o_ref = mg.make_opts(n, tol=0.0, max_cycles=3)

    def captured():
        return _call(L, mg.MODEL_DGP, par, o_ns, static_delta, phi, ws)[0]

    def eager(d):
        ref = torch.zeros_like(d)
        rc, _ = _call(L, mg.MODEL_DGP, par, o_ref, d, ref, ws_ref)
        assert rc == mg.MG_NOT_CONVERGED
        return ref

    _graph_replays(L, captured, eager, static_delta, phi, deltas)


def test_noalloc_no_sync_solve_replays_from_a_hip_graph():
    # the static-workspace entry point under capture; the eager references
    # between the replays run through the same static workspace
    L = mg.lib()
    n = 64
    par = mg.dgp_params()
    deltas = [_delta(n, s) for s in (31, 32)] * 2
    static_delta = deltas[0].clone()
    phi = torch.zeros_like(static_delta)
    o_ns = mg.make_opts(n, tol=0.0, max_cycles=3, no_sync=True)
    o_ref = mg.make_opts(n, tol=0.0, max_cycles=3)

    def noalloc(o, d, out):
        st = mg.Stats()
        return L.mg_solve_dgp_noalloc(C.byref(o), C.byref(par), mg._ptr(d), mg._ptr(out),
                                      mg._stream(), C.byref(st))

    def eager(d):
        ref = torch.zeros_like(d)
        assert noalloc(o_ref, d, ref) == mg.MG_NOT_CONVERGED
        return ref

    _graph_replays(L, lambda: noalloc(o_ns, static_delta, phi), eager, static_delta, phi,
                   deltas)
