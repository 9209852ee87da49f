"""GPU parity: every kernel of the HIP path against the FP64 oracle.

Single operations are compared element by element at sizes from the 4^3
coarsest level (one partial block) to 64^3 (hundreds of blocks), on both
colours and with array and scalar right-hand sides.  Whole solves are compared
cycle for cycle.  Tolerances: the kernels and the oracle evaluate the same
FP64 expressions in different algebraic forms (rationalised root, compact
Sigma, fused multiply-adds), so single operations agree to a few ulps of the
largest term (1e-12 relative) and fixed-cycle iterates to 1e-11 relative.
"""
import numpy as np
import pytest
import torch

import inputs
import oracle
import paper_2110_00566_amd as mg

pytestmark = pytest.mark.gpu
OM = 0.3089
DEV = "cuda"


def g(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def c(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def models(n):
    return {
        "dgp": (mg.dgp_params(1.0, OM, 1.0), oracle.dgp_model(1.0, OM, 1.0)),
        "dgp_h05": (mg.dgp_params(0.7, OM, 0.5), oracle.dgp_model(0.7, OM, 0.5)),
        "kmo3": (mg.kmo_params(n, 0.02 * n, 3, 1.0, 0.1), oracle.kmo_model(n, 0.02 * n, 3, 1.0, 0.1)),
        "kmo2": (mg.kmo_params(n, 0.05 * n, 2, 5.0, 0.2), oracle.kmo_model(n, 0.05 * n, 2, 5.0, 0.2)),
        "poisson": (mg.PoissonParams(1.3), oracle.linear_model(1.3)),
    }


def field(n, seed, amp=1.0):
    return amp * inputs.gaussian_field(n, seed, lambda k: k ** -3.0)


@pytest.mark.parametrize("n", [4, 8, 32, 64])
@pytest.mark.parametrize("name", ["dgp", "dgp_h05", "kmo3", "kmo2", "poisson"])
@pytest.mark.parametrize("h", [1.0, 4.0])
def test_residual_parity(n, name, h):
    gp, om = models(n)[name]
    phi = field(n, 1, 3.0 if "kmo" not in name else 0.5)
    delta = inputs.lognormal_delta(n, 2)
    f = field(n, 3, 0.1)
    ref = oracle.residual(om, phi, delta, f, h=h)
    out = c(mg.op_residual(gp, g(phi), g(delta), g(f), h=h))
    assert rel(out, ref) <= 1e-12
    ref_s = oracle.residual(om, phi, delta, 0.25, h=h)
    out_s = c(mg.op_residual(gp, g(phi), g(delta), 0.25, h=h))
    assert rel(out_s, ref_s) <= 1e-12


@pytest.mark.parametrize("n", [4, 8, 32, 64, 128, 256])
@pytest.mark.parametrize("name", ["dgp", "kmo3", "kmo2", "poisson"])
@pytest.mark.parametrize("colour", [0, 1])
def test_colour_pass_parity(n, name, colour):
    gp, om = models(n)[name]
    phi = field(n, 4, 3.0 if "kmo" not in name else 0.5)
    delta = inputs.lognormal_delta(n, 5)
    f = field(n, 6, 0.1)
    for h in (1.0, 2.0):
        ref = oracle.colour_pass(om, phi, delta, colour, f, h=h)
        out = c(mg.op_colour_pass(gp, g(phi), g(delta), colour, g(f), h=h))
        assert rel(out, ref) <= 1e-12
        # the other colour is untouched, bit for bit
        k, j, i = np.indices(phi.shape)
        other = (i + j + k) % 2 != colour
        assert np.array_equal(out[other], phi[other])


@pytest.mark.parametrize("n", [8, 16, 64, 128, 256])
def test_restrict_and_prolong_parity(n):
    fine = field(n, 7)
    assert rel(c(mg.op_restrict(g(fine))), oracle.restrict(fine)) <= 1e-15
    uc, rc = field(n // 2, 8), field(n // 2, 9)
    assert rel(c(mg.op_prolong_add(g(fine), g(uc), g(rc))), oracle.prolong_add(fine, uc, rc)) <= 1e-14


@pytest.mark.parametrize("n", [4, 8, 32])
@pytest.mark.parametrize("name", ["dgp", "kmo3", "kmo2", "poisson"])
def test_transpose_jacobian_parity(n, name):
    gp, om = models(n)[name]
    phi = field(n, 10, 3.0 if "kmo" not in name else 0.5)
    delta = inputs.lognormal_delta(n, 11)
    v = field(n, 12)
    for h in (1.0, 2.0):
        ref = oracle.jac_t_apply(oracle.jac_rows(om, phi, delta, h), v, h)
        out = c(mg.op_jt_apply(gp, g(phi), g(delta), g(v), h=h))
        assert rel(out, ref) <= 1e-11


# ------------------------------------------------------------- whole solves

@pytest.mark.parametrize("name,n,cycles,nu1,nu2", [("dgp", 128, 2, 1, 1), ("kmo3", 128, 2, 1, 1),
                                                   ("poisson", 128, 2, 1, 1),
                                                   ("dgp_h05", 256, 1, 1, 1), ("dgp", 128, 1, 2, 2),
                                                   ("dgp", 128, 2, 1, 0)])
def test_tiled_levels_fixed_cycles_parity(name, n, cycles, nu1, nu2):
    # levels >= 128^3 run the LDS-tiled kernels (pass, residual + restriction
    # with the residual reduction, and the prolongation fused with the first
    # colour pass of the post-smoothing; nu2 = 0 takes the plain prolongation)
    gp, om = models(n)[name]
    delta = inputs.lognormal_delta(n, 3)
    r = oracle.solve(om, delta, tol=0.0, max_cycles=cycles, nu1=nu1, nu2=nu2)
    fn = {"dgp": mg.lib().mg_solve_dgp, "dgp_h05": mg.lib().mg_solve_dgp,
          "kmo3": mg.lib().mg_solve_kmouflage, "poisson": mg.lib().mg_solve_poisson}[name]
    model = {"dgp": 0, "dgp_h05": 0, "kmo3": 1, "poisson": 2}[name]
    phi, st = mg._solve(fn, gp, model, g(delta), None, None, tol=0.0, max_cycles=cycles,
                        nu_pre=nu1, nu_post=nu2)
    assert rel(c(phi), r.phi) <= 1e-11
    assert st["eps0"] == pytest.approx(r.eps0, rel=1e-10)
    assert np.allclose(st["eps_hist"], r.hist[:cycles], rtol=1e-8, atol=1e-300)


@pytest.mark.parametrize("cycle", [mg.CYCLE_F, mg.CYCLE_W])
@pytest.mark.parametrize("name,n", [("dgp", 32), ("kmo3", 32), ("dgp", 128), ("dgp_h05", 64),
                                    ("kmo3", 128)])
def test_f_and_w_cycles_fixed_cycles_parity(name, n, cycle):
    # F- and W-cycle arrangements (Sec. 3.2.1): the host recursion on the
    # per-level kernels and the recursion inside the single-workgroup tail
    gp, om = models(n)[name]
    delta = inputs.lognormal_delta(n, 3)
    r = oracle.solve(om, delta, tol=0.0, max_cycles=2, cycle=cycle)
    fn = mg.lib().mg_solve_kmouflage if name.startswith("kmo") else mg.lib().mg_solve_dgp
    phi, st = mg._solve(fn, gp, 1 if name.startswith("kmo") else 0, g(delta), None, None,
                        tol=0.0, max_cycles=2, cycle=cycle)
    assert st["cycles"] == 2
    assert rel(c(phi), r.phi) <= 1e-11
    assert np.allclose(st["eps_hist"], r.hist[:2], rtol=1e-8, atol=1e-300)


@pytest.mark.parametrize("cycle", [mg.CYCLE_F, mg.CYCLE_W])
def test_f_and_w_cycles_converge_to_the_v_solution(cycle):
    n = 64
    delta = inputs.lognormal_delta(n, 1)
    ref = oracle.solve(oracle.dgp_model(1.0, OM, 1.0), delta, tol=1e-12, max_cycles=60)
    phi, st = mg.solve_dgp(g(delta), tol=1e-12, max_cycles=60, cycle=cycle)
    assert st["status"] == 0 and st["eps"] <= 1e-12
    assert rel(c(phi), ref.phi) <= 1e-9
    rv = oracle.solve(oracle.dgp_model(1.0, OM, 1.0), delta, tol=1e-12, max_cycles=60,
                      cycle=cycle)
    assert st["cycles"] == rv.cycles


# ------------------------------------------- Newton-Gauss-Seidel comparator

@pytest.mark.parametrize("n,h", [(8, 1.0), (32, 2.0), (128, 1.0)])
def test_newton_comparator_operations_parity(n, h):
    # The Newton step divides by dL/dphi = -(6/h^2)(1 + 4D/(3 alpha)), which
    # nears zero where a rough field has large Laplacians; there a 1-ulp
    # change of phi moves the update by ~1e-10 and no fixed tolerance is
    # meaningful.  The field amplitude keeps the step well conditioned: the
    # oracle's own update moves by < 1e-14 under a 2e-16 relative change of phi.
    gp = mg.dgp_params(0.8, OM, 1.0)
    om = oracle.dgp_newton_model(0.8, OM, 1.0)
    phi = field(n, 1, 0.3)
    delta = inputs.lognormal_delta(n, 2)
    f = field(n, 3, 0.1)
    ref = oracle.residual(om, phi, delta, f, h=h)
    out = c(mg.op_residual(gp, g(phi), g(delta), g(f), h=h, model=mg.MODEL_DGP_NEWTON))
    assert rel(out, ref) <= 1e-12
    p2 = phi * (1.0 + 2e-16 * np.random.default_rng(0).standard_normal(phi.shape))
    for colour in (0, 1):
        ref = oracle.colour_pass(om, phi, delta, colour, f, h=h)
        assert rel(oracle.colour_pass(om, p2, delta, colour, f, h=h), ref) <= 1e-14
        out = c(mg.op_colour_pass(gp, g(phi), g(delta), colour, g(f), h=h,
                                  model=mg.MODEL_DGP_NEWTON))
        assert rel(out, ref) <= 1e-12


@pytest.mark.parametrize("n,cycles,cycle,sigma", [(32, 3, mg.CYCLE_V, 1.0),
                                                  (128, 2, mg.CYCLE_V, 0.5),
                                                  (32, 2, mg.CYCLE_W, 1.0),
                                                  (128, 2, mg.CYCLE_F, 0.5)])
def test_newton_comparator_fixed_cycles_parity(n, cycles, cycle, sigma):
    delta = inputs.lognormal_delta(n, 3, sigma)
    r = oracle.solve(oracle.dgp_newton_model(1.0, OM, 1.0), delta, tol=0.0, max_cycles=cycles,
                     cycle=cycle)
    phi, st = mg.solve_dgp_newton(g(delta), tol=0.0, max_cycles=cycles, cycle=cycle)
    assert rel(c(phi), r.phi) <= 1e-11
    assert np.allclose(st["eps_hist"], r.hist[:cycles], rtol=1e-8, atol=1e-300)


def test_newton_comparator_diverges_where_the_oracle_does():
    # a log-normal density with sigma = 1 on 128^3 (peaks near 90) drives
    # dL/dphi of the quadratic form through zero: Newton-GS diverges in the
    # oracle and on the GPU alike, while the closed-form update converges
    n = 128
    delta = inputs.lognormal_delta(n, 3, 1.0)
    r = oracle.solve(oracle.dgp_newton_model(1.0, OM, 1.0), delta, tol=1e-8, max_cycles=12)
    assert r.status == mg.MG_ERR_DIVERGED
    with pytest.raises(mg.MGError) as e:
        mg.solve_dgp_newton(g(delta), tol=1e-8, max_cycles=12)
    assert e.value.status == mg.MG_ERR_DIVERGED
    phi, st = mg.solve_dgp(g(delta), tol=1e-8, max_cycles=12)
    assert st["status"] == 0


def test_newton_comparator_converged_parity():
    n = 64
    delta = inputs.lognormal_delta(n, 1)
    r = oracle.solve(oracle.dgp_newton_model(1.0, OM, 1.0), delta, tol=1e-11, max_cycles=100)
    phi, st = mg.solve_dgp_newton(g(delta), tol=1e-11, max_cycles=100)
    assert st["status"] == 0 and st["cycles"] == r.cycles
    assert rel(c(phi), r.phi) <= 1e-9


# ------------------------------------------------- linearised comparators

def test_linear_source_matches_oracle():
    for a, h0rc in ((1.0, 1.0), (0.6, 0.5), (0.8, 5.0)):
        s = mg.linear_source(mg.MODEL_DGP, mg.dgp_params(a, OM, h0rc))
        assert s == pytest.approx(oracle.linearised_dgp_model(a, OM, h0rc).s, rel=1e-14)
    for args in ((64, 128.0, 3, 1.0, 0.1, 1.2, 1.0, OM, 0.0, 0.0),
                 (256, 512.0, 2, 5.0, 0.2, 1.4, 0.7, OM, 0.03, 0.4)):
        s = mg.linear_source(mg.MODEL_KMOUFLAGE, mg.kmo_params(*args), args[0])
        assert s == pytest.approx(oracle.linearised_kmo_model(*args).s, rel=1e-14)


@pytest.mark.parametrize("name,n", [("dgp", 32), ("dgp", 128), ("kmo", 128)])
def test_linearised_solve_parity(name, n):
    delta = inputs.lognormal_delta(n, 8)
    if name == "dgp":
        par, om, model = mg.dgp_params(0.7, OM, 1.0), oracle.linearised_dgp_model(0.7, OM, 1.0), \
            mg.MODEL_DGP
    else:
        args = (n, 0.05 * n, 2, 5.0, 0.2, 1.4, 0.7, OM, 0.03, 0.4)
        par, om, model = mg.kmo_params(*args), oracle.linearised_kmo_model(*args), \
            mg.MODEL_KMOUFLAGE
    r = oracle.solve(om, delta, tol=0.0, max_cycles=2)
    phi, st = mg.solve_linearised(model, par, g(delta), tol=0.0, max_cycles=2)
    assert rel(c(phi), r.phi) <= 1e-11
    # converged, against the FFT solution of the same linear equation (the
    # residual tolerance is absolute, so it scales with the source)
    phi, st = mg.solve_linearised(model, par, g(delta), tol=1e-12 * min(1.0, om.s),
                                  max_cycles=60)
    assert st["status"] == 0
    ref = oracle.fft_poisson(om.s * delta)
    assert rel(c(phi), ref) <= 1e-9


# ----------------------------------------------------- all-FP32 variant

@pytest.mark.parametrize("name,n", [("dgp", 32), ("dgp", 128), ("kmo3", 128), ("poisson", 64)])
def test_fp32_variant_tracks_oracle(name, n):
    gp, om = models(n)[name]
    delta = inputs.lognormal_delta(n, 3)
    r = oracle.solve(om, delta, tol=0.0, max_cycles=3)
    fn = {"dgp": mg.lib().mg_solve_dgp, "kmo3": mg.lib().mg_solve_kmouflage,
          "poisson": mg.lib().mg_solve_poisson}[name]
    model = {"dgp": 0, "kmo3": 1, "poisson": 2}[name]
    phi, st = mg._solve(fn, gp, model, g(delta), None, None, tol=0.0, max_cycles=3,
                        precision=mg.MG_FP32)
    assert st["cycles"] == 3 and st["cycles_fp32"] == 3
    assert rel(c(phi), r.phi) <= 2e-5
    assert np.allclose(st["eps_hist"], r.hist[:3], rtol=1e-3)


@pytest.mark.parametrize("n", [64, 256])
def test_fp32_variant_stops_at_its_floor(n):
    delta = inputs.lognormal_delta(n, 1)
    ref, st64 = mg.solve_dgp(g(delta), tol=1e-11, max_cycles=60)
    phi, st = mg.solve_dgp(g(delta), tol=1e-11, max_cycles=60, precision=mg.MG_FP32)
    # the FP32 floor stops the cycles before the FP64 tolerance
    assert st["status"] == mg.MG_NOT_CONVERGED and st["cycles"] < 60
    assert st["eps"] > 1e-11 and st["eps"] < 1e-3 * st["eps0"]
    assert float((phi - ref).abs().max() / ref.abs().max()) <= 1e-4
    # a tolerance above the floor converges
    phi2, st2 = mg.solve_dgp(g(delta), tol=10 * st["eps"], max_cycles=60, precision=mg.MG_FP32)
    assert st2["status"] == 0 and st2["eps"] <= 10 * st["eps"]


def test_level_timing_stats():
    n = 256
    delta = inputs.lognormal_delta(n, 2)
    _, st = mg.solve_dgp(g(delta), tol=0.0, max_cycles=3, profile=True)
    lv = st["level_ms"]
    nlev = 7                                    # 256 .. 4; the tail starts at 16^3 (level 4)
    assert all(x > 0 for x in lv[:5]) and all(x == 0 for x in lv[5:])
    assert lv[0] == max(lv)
    assert sum(lv) <= 1e3 * st["seconds"]
    assert lv[0] > 4 * lv[1]                    # the finest level dominates (8x the cells)
    _, st = mg.solve_dgp(g(delta), tol=0.0, max_cycles=3)
    assert all(x == 0 for x in st["level_ms"]) and nlev == 7


def test_config1_fixed_cycles_parity():
    # 32^3 lognormal (sigma = 1), nDGP H0 r_c = 1, a = 1: three V(1,1) cycles
    n = 32
    delta = inputs.lognormal_delta(n, 1)
    r = oracle.solve(oracle.dgp_model(1.0, OM, 1.0), delta, tol=0.0, max_cycles=3)
    phi, st = mg.solve_dgp(g(delta), tol=0.0, max_cycles=3)
    assert st["cycles"] == 3 and r.cycles == 3
    assert rel(c(phi), r.phi) <= 1e-11
    assert st["eps0"] == pytest.approx(r.eps0, rel=1e-11)
    assert np.allclose(st["eps_hist"], r.hist[:3], rtol=1e-9, atol=0)
    assert st["lam"] == pytest.approx(-r.mu, rel=1e-9)


def test_config1_converged_parity():
    n = 32
    delta = inputs.lognormal_delta(n, 1)
    r = oracle.solve(oracle.dgp_model(1.0, OM, 1.0), delta, tol=1e-8)
    phi, st = mg.solve_dgp(g(delta), tol=1e-8)
    assert st["status"] == 0 and st["eps"] <= 1e-8
    assert st["cycles"] == r.cycles
    assert rel(c(phi), r.phi) <= 1e-10
    # fifth force -1/2 grad phi (eq:dgp_accel), central differences
    for ax in range(3):
        f_g = -0.25 * (np.roll(c(phi), -1, ax) - np.roll(c(phi), 1, ax))
        f_o = -0.25 * (np.roll(r.phi, -1, ax) - np.roll(r.phi, 1, ax))
        assert rel(f_g, f_o) <= 1e-9


@pytest.mark.parametrize("name,n", [("kmo3", 32), ("kmo2", 32), ("dgp_h05", 64), ("poisson", 32)])
def test_other_models_fixed_cycles_parity(name, n):
    gp, om = models(n)[name]
    delta = inputs.lognormal_delta(n, 3)
    r = oracle.solve(om, delta, tol=0.0, max_cycles=4)
    fn = {"kmo3": mg.lib().mg_solve_kmouflage, "kmo2": mg.lib().mg_solve_kmouflage,
          "dgp_h05": mg.lib().mg_solve_dgp, "poisson": mg.lib().mg_solve_poisson}[name]
    model = {"kmo3": 1, "kmo2": 1, "dgp_h05": 0, "poisson": 2}[name]
    phi, st = mg._solve(fn, gp, model, g(delta), None, None, tol=0.0, max_cycles=4)
    assert rel(c(phi), r.phi) <= 1e-11
    assert np.allclose(st["eps_hist"], r.hist[:4], rtol=1e-8, atol=1e-300)


def test_kmouflage_sphere_converges_like_oracle():
    # Sec. 4.2.3 stress case: delta = 5000 top-hat, n = 2, beta = 0.2, K0 = 100
    n = 32
    d = inputs.tophat_delta(n, 5000.0, 0.1 * n)
    d -= d.mean()
    om = oracle.kmo_model(n, float(n), 2, 100.0, 0.2)
    r = oracle.solve(om, d, tol=1e-9, max_cycles=100)
    phi, st = mg.solve_kmouflage(g(d), box_mpch=float(n), n_k=2, k0=100.0, beta=0.2, tol=1e-9,
                                 max_cycles=100)
    assert st["status"] == 0 and st["cycles"] == r.cycles
    assert rel(c(phi), r.phi) <= 1e-9


def test_initial_guess_and_uniform_density():
    # Sec. 4.2.1 on the GPU: delta = 0, random phi0 -> constant (0) field
    n = 32
    phi0 = inputs.uniform_phi(n, 7)
    phi, st = mg.solve_dgp(g(np.zeros((n, n, n))), g(phi0), tol=1e-8)
    assert st["status"] == 0
    assert np.abs(c(phi)).max() <= 1e-8


def test_solve_is_deterministic():
    n = 64
    delta = g(inputs.lognormal_delta(n, 1))
    a, _ = mg.solve_dgp(delta, tol=0.0, max_cycles=2)
    b, _ = mg.solve_dgp(delta, tol=0.0, max_cycles=2)
    assert torch.equal(a, b)


def test_nonfinite_input_reported():
    n = 16
    d = inputs.lognormal_delta(n, 1)
    d[3, 4, 5] = np.nan
    with pytest.raises(mg.MGError) as e:
        mg.solve_dgp(g(d), tol=1e-8)
    assert e.value.status == mg.MG_ERR_NONFINITE


def test_cycle_cap_status():
    n = 32
    _, st = mg.solve_dgp(g(inputs.lognormal_delta(n, 1)), tol=1e-14, max_cycles=2)
    assert st["status"] == mg.MG_NOT_CONVERGED and st["cycles"] == 2
    assert st["eps"] > 1e-14


# ---------------------------------------------------------------- adjoint

@pytest.mark.parametrize("name,n", [("dgp", 16), ("dgp", 32), ("kmo3", 16), ("poisson", 16)])
def test_adjoint_parity(name, n):
    gp, om = models(n)[name]
    delta = inputs.lognormal_delta(n, 4) * (1.0 if "kmo" not in name else 2.0)
    w = inputs.gaussian_weights(n, 5)
    phi = oracle.solve(om, delta, tol=1e-13, max_cycles=80).phi
    r = oracle.adjoint(om, delta, phi, w, tol=0.0, max_cycles=4)
    model = {"dgp": 0, "kmo3": 1, "poisson": 2}[name]
    grad, mu, st = mg.solve_adjoint(model, gp, g(delta), g(phi), g(w), tol=0.0, max_cycles=4)
    assert rel(c(mu), r.mu) <= 1e-10
    assert rel(c(grad), r.grad) <= 1e-10
    r2 = oracle.adjoint(om, delta, phi, w, tol=1e-11, max_cycles=80)
    grad2, mu2, st2 = mg.solve_adjoint(model, gp, g(delta), g(phi), g(w), tol=1e-11,
                                       max_cycles=80)
    assert st2["status"] == 0 and st2["cycles"] == r2.cycles
    assert rel(c(grad2), r2.grad) <= 1e-9


@pytest.mark.parametrize("name,n,converge", [("dgp", 128, True), ("kmo3", 128, True),
                                             ("poisson", 128, False), ("dgp", 256, False),
                                             ("kmo2", 256, False)])
def test_tiled_adjoint_parity(name, n, converge):
    # levels >= 128^3 run the LDS-tiled adjoint kernels (pass, residual +
    # restriction, coarse source) and keep the mean of mu from colour sums;
    # fixed cycles and (128^3) the converged solve against the oracle adjoint
    gp, om = models(n)[name]
    delta = inputs.lognormal_delta(n, 6) * (1.0 if "kmo" not in name else 2.0)
    w = inputs.gaussian_weights(n, 7)
    print("tiled adjoint %s n=%d" % (name, n), flush=True)
    phi = oracle.solve(om, delta, tol=1e-12, max_cycles=60).phi
    model = {"dgp": 0, "kmo3": 1, "kmo2": 1, "poisson": 2}[name]
    r = oracle.adjoint(om, delta, phi, w, tol=0.0, max_cycles=3)
    grad, mu, st = mg.solve_adjoint(model, gp, g(delta), g(phi), g(w), tol=0.0, max_cycles=3)
    assert st["cycles"] == 3
    assert rel(c(mu), r.mu) <= 1e-10
    assert rel(c(grad), r.grad) <= 1e-10
    np.testing.assert_allclose(st["eps_hist"], r.hist[:3], rtol=1e-9)
    if converge:
        r2 = oracle.adjoint(om, delta, phi, w, tol=1e-10, max_cycles=60)
        grad2, mu2, st2 = mg.solve_adjoint(model, gp, g(delta), g(phi), g(w), tol=1e-10,
                                           max_cycles=60)
        assert st2["status"] == 0 and st2["cycles"] == r2.cycles
        assert rel(c(grad2), r2.grad) <= 1e-9
        assert abs(float(mu2.mean())) <= 1e-12 * float(mu2.abs().max())


def test_autograd_matches_finite_differences():
    n = 32
    delta = g(inputs.lognormal_delta(n, 1)).requires_grad_(True)
    w = g(inputs.gaussian_weights(n, 3))
    phi = mg.DGPSolve.apply(delta, 1.0, 1.0, OM, 1e-13)
    (phi * w).sum().backward()
    cells = inputs.random_cells(n, 8, 4)
    eps = 1e-4
    base = delta.detach()
    for cidx in cells:
        vals = []
        for s in (1, -1):
            d2 = base.clone().view(-1)
            d2[cidx] += s * eps
            p2, _ = mg.solve_dgp(d2.view(base.shape), phi.detach(), tol=1e-13, max_cycles=100)
            vals.append(float((p2 * w).sum()))
        fd = (vals[0] - vals[1]) / (2 * eps)
        assert float(delta.grad.view(-1)[cidx]) == pytest.approx(fd, rel=1e-5, abs=1e-9)


# -------------------------------------------------------- CIC and PM step

@pytest.mark.parametrize("np_,nm", [(16, 32), (32, 32), (8, 16), (64, 128)])
def test_cic_parity(np_, nm):
    pos = inputs.za_particles(np_, nm, 2, amplitude=30.0)
    _, ref = oracle.cic_density(pos, nm)
    out = c(mg.cic_delta(g(pos), nm))
    # fixed point: each of the <= 8 * n_part^3 contributions is rounded to
    # 2^-33, scaled by n_mesh^3 / n_part^3
    rho, _ = oracle.cic_density(pos, nm)
    bound = 8 * (rho.max() + 1) * 2.0 ** -33 * nm ** 3 / np_ ** 3 + 1e-14
    assert np.abs(out - ref).max() <= bound
    assert abs(out.mean()) <= 1e-9


@pytest.mark.parametrize("np_,nm", [(16, 32), (8, 16)])
def test_cic_fp32_output_is_the_rounded_fp64_one(np_, nm):
    pos = g(inputs.za_particles(np_, nm, 3, amplitude=30.0))
    d64 = mg.cic_delta(pos, nm)
    d32 = mg.cic_delta(pos, nm, dtype=torch.float32)
    assert d32.dtype == torch.float32 and torch.equal(d32, d64.float())


def test_cic_lattice_is_exactly_uniform():
    pos = inputs.lattice_positions(16, 32).astype(np.float32)
    assert np.abs(c(mg.cic_delta(g(pos), 32))).max() == 0.0


@pytest.mark.parametrize("nm,np_", [(32, 16), (64, 32), (16, 16), (32, 40)])
def test_pm_step_parity(nm, np_):
    # (32, 16), (64, 32): deposit from particle lists (a mesh one tile wide
    # at 32); (16, 16) (mesh below one tile) and (32, 40) (more particles
    # than cells): scatter deposit
    pos = inputs.za_particles(np_, nm, 2, amplitude=30.0)
    mom = np.zeros_like(pos)
    p_o, m_o, phi_o, delta_o, phin_o = oracle.pm_step(pos, mom, nm, 1.0, 0.0063, tol=1e-10)
    gpos, gmom = g(pos), g(mom)
    phi = torch.zeros((nm,) * 3, dtype=torch.float64, device=DEV)
    phin = torch.zeros_like(phi)
    delta, st = mg.pm_step(gpos, gmom, phi, phin, nm, 1.0, 0.0063, tol=1e-10)
    assert rel(c(delta), delta_o) <= 1e-8
    assert rel(c(phin), phin_o) <= 1e-8
    # the FFT potential of the step's own density, to FFT rounding
    assert rel(c(phin), oracle.fft_poisson(1.5 * OM * c(delta))) <= 1e-12
    assert rel(c(phi), phi_o) <= 1e-8
    assert rel(c(gmom), m_o) <= 1e-5
    dp = np.abs(c(gpos) - p_o)
    dp = np.minimum(dp, nm - dp)
    assert dp.max() <= 1e-4


# ------------------------------------------------------ FP32 density input

@pytest.mark.parametrize("name,n,precision", [("dgp", 32, mg.MG_FP64), ("dgp", 128, mg.MG_MIXED),
                                              ("kmo3", 128, mg.MG_FP64),
                                              ("dgp_h05", 128, mg.MG_MIXED_DC),
                                              ("poisson", 64, mg.MG_FP32)])
def test_fp32_density_input_equals_the_widened_fp64_input(name, n, precision):
    # delta_fp32 = 1: the levels receive the same values as from an FP64
    # array holding the FP32 numbers, so the solves agree bit for bit
    par, _ = models(n)[name]
    d32 = g(field(n, 77)).float()
    d64 = d32.double()
    solve = {"dgp": mg.lib().mg_solve_dgp, "dgp_h05": mg.lib().mg_solve_dgp,
             "kmo3": mg.lib().mg_solve_kmouflage, "poisson": mg.lib().mg_solve_poisson}[name]
    model = {"dgp": mg.MODEL_DGP, "dgp_h05": mg.MODEL_DGP, "kmo3": mg.MODEL_KMOUFLAGE,
             "poisson": mg.MODEL_POISSON}[name]
    out = []
    for d in (d64, d32):
        phi, st = mg._solve(solve, par, model, d, None, None, tol=1e-9, max_cycles=12,
                            precision=precision)
        out.append((c(phi), st))
    assert out[0][1]["cycles"] == out[1][1]["cycles"]
    assert np.array_equal(out[0][0], out[1][0])


def test_fp32_density_input_adjoint_and_noalloc():
    n = 32
    par = mg.dgp_params(1.0, OM, 1.0)
    d32 = g(field(n, 78)).float()
    d64 = d32.double()
    phi, _ = mg.solve_dgp(d64, tol=1e-12, max_cycles=40)
    w = g(inputs.gaussian_field(n, 79, lambda k: k ** -2.0))
    g64, mu64, _ = mg.solve_adjoint(mg.MODEL_DGP, par, d64, phi, w)
    g32, mu32, _ = mg.solve_adjoint(mg.MODEL_DGP, par, d32, phi, w)
    assert torch.equal(g64, g32) and torch.equal(mu64, mu32)
    p64, _ = mg.solve_dgp_noalloc(d64, tol=1e-9)
    p32, _ = mg.solve_dgp_noalloc(d32, tol=1e-9)
    assert torch.equal(p64, p32)


# ------------------------------------------------------ FFT Poisson solve

@pytest.mark.parametrize("n", [8, 16, 32, 64, 128])
def test_fft_poisson_parity(n):
    # element by element against the oracle's complex FFT solution; both
    # round like an FFT (eps log n relative to the largest value)
    d = field(n, 40 + n) + 0.3
    s = 1.5 * OM / 0.7
    ref = oracle.fft_poisson(s * d)
    out = c(mg.fft_poisson(g(d), s))
    assert rel(out, ref) <= 1e-12
    assert abs(out.mean()) <= 1e-13 * np.abs(ref).max()


def test_fft_poisson_edge_cases():
    n = 32
    ws = torch.empty(4096, dtype=torch.uint8, device=DEV)
    # a uniform source has the zero solution
    out = c(mg.fft_poisson(torch.full((n,) * 3, 2.5, dtype=torch.float64, device=DEV), 1.0, ws=ws))
    assert np.abs(out).max() <= 1e-14
    # a single spike: the lattice Green's function, symmetric under every
    # axis reflection about the spike and under axis permutations
    d = np.zeros((n,) * 3)
    d[0, 0, 0] = 1.0
    out = c(mg.fft_poisson(g(d), 1.0, ws=ws))
    assert rel(out, oracle.fft_poisson(d)) <= 1e-12
    assert np.abs(out - np.roll(out[::-1, ::-1, ::-1], 1, axis=(0, 1, 2))).max() <= 1e-15
    assert np.abs(out - out.transpose(2, 1, 0)).max() <= 1e-15
    # the output array is overwritten, whatever it held
    phi = torch.full((n,) * 3, np.nan, dtype=torch.float64, device=DEV)
    mg.fft_poisson(g(d), 1.0, phi=phi, ws=ws)
    assert np.abs(c(phi) - out).max() == 0.0


def _plane_waves(n, z0, z1, dev=DEV):
    # cos of mode (3, 5, 7) plus 0.5 sin of mode (n/2 - 1, 1, n/4) on planes
    # z0 .. z1-1 (index order z, y, x); both are eigenfunctions of the
    # 7-point Laplacian with eigenvalue -4 sum_i sin^2(pi m_i / n)
    x = torch.arange(n, dtype=torch.float64, device=dev)
    z = torch.arange(z0, z1, dtype=torch.float64, device=dev)
    t = 2 * np.pi / n
    a = torch.cos(t * (3 * x[None, None, :] + 5 * x[None, :, None] + 7 * z[:, None, None]))
    b = torch.sin(t * ((n // 2 - 1) * x[None, None, :] + x[None, :, None]
                       + (n // 4) * z[:, None, None]))
    return a, b


def _eig(n, m):
    return -4.0 * sum(np.sin(np.pi * k / n) ** 2 for k in m)


@pytest.mark.parametrize("n", [1024, 2048])
def test_fft_poisson_full_size_plane_waves(n):
    # maximum sizes (16 and 8 lines per block): the exact discrete solution of
    # a two-mode source, checked on the device plane block by plane block
    s = 1.5 * OM
    chunk = 64
    d = torch.empty((n,) * 3, dtype=torch.float64, device=DEV)
    for z0 in range(0, n, chunk):
        a, b = _plane_waves(n, z0, z0 + chunk)
        d[z0:z0 + chunk] = a + 0.5 * b
    phi = mg.fft_poisson(d, s)
    del d
    ea, eb = _eig(n, (3, 5, 7)), _eig(n, (n // 2 - 1, 1, n // 4))
    err = 0.0
    for z0 in range(0, n, chunk):
        a, b = _plane_waves(n, z0, z0 + chunk)
        exp = s * (a / ea + 0.5 * b / eb)
        err = max(err, (phi[z0:z0 + chunk] - exp).abs().max().item())
    assert err <= 1e-12 * s / abs(ea)


# --------------------------------------------------------- mixed precision

@pytest.mark.parametrize("n,h0rc", [(32, 1.0), (128, 1.0), (128, 0.5)])
def test_mixed_precision_converges_to_fp64_accuracy(n, h0rc):
    # FP32-storage cycles then FP64 cycles; the returned field meets the FP64
    # tolerance and matches the FP64 oracle within 1e-6 relative
    delta = inputs.lognormal_delta(n, 1) if n == 32 else \
        oracle.cic_density(inputs.za_particles(n // 2, n, 6, amplitude=30.0), n)[1]
    r = oracle.solve(oracle.dgp_model(1.0, OM, h0rc), delta, tol=1e-10, max_cycles=80)
    phi, st = mg.solve_dgp(g(delta), h0rc=h0rc, tol=1e-8, precision=mg.MG_MIXED)
    assert st["status"] == 0 and st["eps"] <= 1e-8
    assert st["cycles_fp32"] >= 3
    assert rel(c(phi), r.phi) <= 1e-6
    for ax in range(3):
        f_g = np.roll(c(phi), -1, ax) - np.roll(c(phi), 1, ax)
        f_o = np.roll(r.phi, -1, ax) - np.roll(r.phi, 1, ax)
        assert rel(f_g, f_o) <= 1e-5


@pytest.mark.parametrize("name,n", [("dgp", 128), ("dgp_h05", 256), ("poisson", 128)])
def test_defect_correction_converges_to_the_oracle(name, n):
    # MG_MIXED_DC: FP32 cycles to their floor, then outer steps of FP64
    # residual + one FP32 correction-form cycle + FP64 accumulation; it must
    # reach the FP64 tolerance (far below the FP32 floor) and the oracle's
    # converged field
    gp, om = models(n)[name]
    pos = inputs.za_particles(n // 2, n, 9, amplitude=30.0)
    _, delta = oracle.cic_density(pos, n)
    print("defect correction %s n=%d" % (name, n), flush=True)
    ref = oracle.solve(om, delta, tol=1e-12, max_cycles=80)
    fn = {"dgp": mg.solve_dgp, "dgp_h05": mg.solve_dgp, "poisson": None}[name]
    kw = dict(tol=1e-10, max_cycles=60, precision=mg.MG_MIXED_DC)
    if name == "poisson":
        phi, st = mg.solve_poisson(g(delta), gp.s, **kw)
    else:
        phi, st = fn(g(delta), a=gp.a, h0rc=gp.h0rc, **kw)
    assert st["status"] == 0 and st["eps"] <= 1e-10, (st["status"], st["eps"])
    assert st["cycles_fp32"] >= 1 and st["cycles"] > st["cycles_fp32"]
    assert st["eps_fp32"] > 1e-9           # the FP32 phase alone stops far above the tolerance
    dc = st["eps_hist"][st["cycles_fp32"]:st["cycles"] + 1]
    assert all(b < 0.6 * a for a, b in zip(dc, dc[1:])), dc   # contraction, no floor
    assert rel(c(phi), ref.phi) <= 1e-9
    # the residual the solver reports is the oracle's residual of the field
    r = oracle.residual(om, c(phi), delta)
    assert np.sqrt(((r - r.mean()) ** 2).mean()) == pytest.approx(st["eps"], rel=1e-3, abs=1e-13)


def test_defect_correction_matches_fp64_and_mixed():
    # same field as the FP64 and the two-phase mixed solves at the same tolerance
    n = 128
    delta = g(inputs.lognormal_delta(n, 12))
    ref, st64 = mg.solve_dgp(delta, tol=1e-11, max_cycles=60)
    for prec in (mg.MG_MIXED, mg.MG_MIXED_DC):
        phi, st = mg.solve_dgp(delta, tol=1e-11, max_cycles=60, precision=prec)
        assert st["status"] == 0 and st["eps"] <= 1e-11
        assert float((phi - ref).abs().max() / ref.abs().max()) <= 1e-9


@pytest.mark.parametrize("name,n", [("dgp", 64), ("kmo3", 32), ("poisson", 32), ("dgp", 128)])
def test_fp32_cycles_track_oracle(name, n):
    # three FP32-storage cycles (tol = 0 and the cycle cap spent in the FP32
    # phase) agree with three FP64 oracle cycles to FP32 rounding
    gp, om = models(n)[name]
    delta = inputs.lognormal_delta(n, 3)
    r = oracle.solve(om, delta, tol=0.0, max_cycles=3)
    fn = {"dgp": mg.lib().mg_solve_dgp, "kmo3": mg.lib().mg_solve_kmouflage,
          "poisson": mg.lib().mg_solve_poisson}[name]
    model = {"dgp": 0, "kmo3": 1, "poisson": 2}[name]
    phi, st = mg._solve(fn, gp, model, g(delta), None, None, tol=0.0, max_cycles=3,
                        precision=mg.MG_MIXED)
    assert st["cycles_fp32"] == 3 and st["cycles"] == 3
    assert rel(c(phi), r.phi) <= 2e-5


def test_mixed_kmouflage_sphere():
    n = 32
    d = inputs.tophat_delta(n, 5000.0, 0.1 * n)
    d -= d.mean()
    r = oracle.solve(oracle.kmo_model(n, float(n), 2, 10.0, 0.2), d, tol=1e-10, max_cycles=100)
    phi, st = mg.solve_kmouflage(g(d), box_mpch=float(n), n_k=2, k0=10.0, beta=0.2, tol=1e-9,
                                 max_cycles=100, precision=mg.MG_MIXED)
    assert st["status"] == 0 and st["eps"] <= 1e-9
    assert rel(c(phi), r.phi) <= 1e-6


@pytest.mark.parametrize("cycle,precision", [(mg.CYCLE_V, mg.MG_FP64), (mg.CYCLE_W, mg.MG_FP64),
                                             (mg.CYCLE_V, mg.MG_MIXED)])
def test_early_residual_read_changes_nothing(cycle, precision):
    # profile mode reads each cycle's stopping scalars after the whole cycle;
    # otherwise they are read as soon as the finest in-cycle residual is
    # reduced: the iterates, histories and stopping decisions are identical
    n = 128
    delta = g(inputs.lognormal_delta(n, 31))
    kw = dict(tol=1e-9, max_cycles=40, cycle=cycle, precision=precision)
    a, sa = mg.solve_dgp(delta, **kw)
    b, sb = mg.solve_dgp(delta, profile=True, **kw)
    assert torch.equal(a, b)
    assert sa["cycles"] == sb["cycles"] and sa["eps"] == sb["eps"]
    assert sa["eps_hist"][:sa["cycles"]] == sb["eps_hist"][:sb["cycles"]]


@pytest.mark.parametrize("n", [8, 16])
@pytest.mark.parametrize("name", ["dgp", "kmo3", "poisson"])
@pytest.mark.parametrize("cycle", [mg.CYCLE_V, mg.CYCLE_F])
def test_smallest_meshes_converged_parity(n, name, cycle):
    # the smallest meshes: every level below the finest runs in the
    # single-workgroup tail (8^3: only the 4^3 level)
    gp, om = models(n)[name]
    delta = inputs.lognormal_delta(n, 41)
    r = oracle.solve(om, delta, tol=1e-11, max_cycles=80, cycle=cycle)
    fn = {"dgp": mg.lib().mg_solve_dgp, "kmo3": mg.lib().mg_solve_kmouflage,
          "poisson": mg.lib().mg_solve_poisson}[name]
    model = {"dgp": 0, "kmo3": 1, "poisson": 2}[name]
    phi, st = mg._solve(fn, gp, model, g(delta), None, None, tol=1e-11, max_cycles=80,
                        cycle=cycle)
    assert st["status"] == 0 and st["cycles"] == r.cycles
    assert rel(c(phi), r.phi) <= 1e-9


@pytest.mark.parametrize("n", [16, 128])
def test_zero_source_and_zero_cycles(n):
    # delta = 0 from phi = 0: the initial residual is already 0, no cycle
    # runs and phi stays exactly 0, for every model
    z = g(np.zeros((n, n, n)))
    for name, fn, model in (("dgp", mg.lib().mg_solve_dgp, 0),
                            ("kmo3", mg.lib().mg_solve_kmouflage, 1),
                            ("poisson", mg.lib().mg_solve_poisson, 2)):
        gp, _ = models(n)[name]
        phi, st = mg._solve(fn, gp, model, z, None, None, tol=1e-8, max_cycles=10)
        assert st["status"] == 0 and st["cycles"] == 0 and st["eps"] == 0.0
        assert torch.count_nonzero(phi).item() == 0
    # max_cycles = 0 returns the initial guess in the zero-mean gauge
    phi0 = inputs.uniform_phi(n, 8)
    phi, st = mg.solve_dgp(g(inputs.lognormal_delta(n, 9)), g(phi0), tol=1e-8, max_cycles=0)
    assert st["cycles"] == 0 and st["status"] == mg.MG_NOT_CONVERGED
    assert np.abs(c(phi) - (phi0 - phi0.mean())).max() <= 1e-14 * np.abs(phi0).max()


@pytest.mark.parametrize("name,n", [("dgp", 64), ("dgp", 128), ("dgp_h05", 64)])
def test_warm_start_residual_is_free_of_cancellation(name, n):
    # a field within ~1e-11 of the solution, whose residual has a mean (the
    # Lagrange multiplier) many orders larger: the first residual of the call
    # must still equal the oracle's mean-projected RMS (the one-pass variance
    # of the reduction would otherwise cancel), and a tol = 0 call from the
    # converged field itself must run every cycle
    gp, om = models(n)[name]
    fn = mg.lib().mg_solve_dgp
    delta = inputs.lognormal_delta(n, 17)
    star, st = mg._solve(fn, gp, 0, g(delta), None, None, tol=1e-12, max_cycles=60)
    assert st["status"] == 0
    x = np.arange(n) * (2.0 * np.pi / n)
    pert = 1e-9 * np.sin(x)[None, None, :] * np.cos(2.0 * x)[None, :, None]
    phi0 = c(star) + pert
    Lr = oracle.residual(om, phi0, delta)
    eps_oracle = float(np.sqrt(np.mean((Lr - Lr.mean()) ** 2)))
    _, st0 = mg._solve(fn, gp, 0, g(delta), g(phi0), None, tol=0.0, max_cycles=0)
    print("\n%s %d^3: |lambda| %.3e, eps0 GPU %.6e, oracle %.6e"
          % (name, n, abs(st["lam"]), st0["eps0"], eps_oracle))
    assert abs(st["lam"]) > 1e6 * eps_oracle
    assert st0["eps0"] == pytest.approx(eps_oracle, rel=1e-3)
    _, st1 = mg._solve(fn, gp, 0, g(delta), star, None, tol=0.0, max_cycles=3)
    assert st1["status"] == mg.MG_NOT_CONVERGED and st1["cycles"] == 3
    assert 0.0 < st1["eps0"] < 1e-10
