"""Pins of the FP64 oracle against the paper and against mathematics.

Each test checks the oracle (C, printed long forms) against something it does
not share code with: the traceless-Hessian derivation, FFT inverses, a dense
bordered Newton solve, manufactured continuum solutions, closed forms and the
paper's own test cases (Sec. 4.2).  All CPU-only.
"""
import json
import os

import numpy as np
import pytest

import inputs
import oracle
from oracle import pins

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_tests.json")))
OM = GOLD["cosmology"]["omega_m"]


# ------------------------------------------------------------ coefficients

@pytest.mark.parametrize("h0rc", GOLD["sphere_test_dgp"]["h0rc"])
def test_beta_closed_form_at_a1(h0rc):
    # eq:beta_dgp at a = 1 with E = 1 and Omega_rc = 1/(4 R_c^2) collapses
    # to beta = 1 + (Omega_m + 2 Omega_L) R_c = 1 + (2 - Omega_m) R_c.
    m = oracle.dgp_model(1.0, OM, h0rc)
    assert m.beta == pytest.approx(1.0 + (2.0 - OM) * h0rc, rel=1e-14)
    assert m.alpha == pytest.approx(3.0 * m.beta / h0rc ** 2, rel=1e-14)
    assert m.s == pytest.approx(m.alpha * OM / m.beta, rel=1e-14)


def test_beta_scale_factor_dependence():
    # independent evaluation of eq:beta_dgp through eq:beta_dgp's first form
    # 1 + 2 H r_c (1 + Hdot/(3H^2)) with LCDM H (eq:H_lcdm), in H0 = c = 1 units
    a, h0rc = 0.5, 1.0
    E2 = OM / a ** 3 + 1 - OM
    dlnE2_dlna = -3 * OM / a ** 3 / E2
    hdot_over_h2 = 0.5 * dlnE2_dlna          # Hdot/H^2 = dlnH/dlna
    beta = 1.0 + 2.0 * np.sqrt(E2) * h0rc * (1.0 + hdot_over_h2 / 3.0)
    assert oracle.dgp_model(a, OM, h0rc).beta == pytest.approx(beta, rel=1e-13)


def test_kmouflage_coefficients():
    # gamma = n K0 (1/(2 a^2 lambda^2))^(n-1) with lambda^2 = 3(1-Omega_m),
    # c~ = N c/(H0 L)
    for nk, expect in ((3, 3 * (1 / (6 * (1 - OM))) ** 2), (2, 2 / (6 * (1 - OM)))):
        m = oracle.kmo_model(256, 512.0, nk, 1.0, 0.1)
        assert m.gamma == pytest.approx(expect, rel=1e-13)
        assert m.ctil == pytest.approx(256 / 512 * GOLD["c_over_H0_mpch"]["value"], rel=1e-15)
        assert m.src == pytest.approx(3 * 0.1 * OM, rel=1e-14)


# -------------------------------------------------- p1: operator identities

def _field(n, seed, amp):
    return amp * inputs.gaussian_field(n, seed, lambda k: k ** -3.0)


@pytest.mark.parametrize("h", [1.0, 4.0])
def test_dgp_sigma_equals_traceless_hessian_contraction(h):
    # printed long-form Sigma (oracle) == hat(H):hat(H) from eq:operator_split
    phi = _field(16, 11, 3.0)
    delta = inputs.lognormal_delta(16, 12)
    m = oracle.dgp_model(1.0, OM, 1.0)
    L_or = oracle.residual(m, phi, delta, h=h)
    L_np = pins.laplacian(phi, h) - pins.dgp_term_traceless(phi, delta, m.alpha, m.s, h)
    assert np.abs(L_or - L_np).max() <= 1e-12 * max(1.0, np.abs(L_np).max())


def test_dgp_term_has_no_centre_dependence():
    # the model term of L must not depend on phi_ijk (footnote on
    # eq:nonlinear_GS_DGP), so dL/dphi_ijk = -6/h^2 exactly
    phi = _field(8, 3, 2.0)
    delta = inputs.lognormal_delta(8, 4)
    for m in (oracle.dgp_model(1.0, OM, 1.0), oracle.kmo_model(8, 16.0, 3, 1.0, 0.1)):
        L0 = oracle.op_cell(m, phi, delta, 3, 4, 5)
        p2 = phi.copy()
        p2[5, 4, 3] += 0.25
        L1 = oracle.op_cell(m, p2, delta, 3, 4, 5)
        assert (L1 - L0) / 0.25 == pytest.approx(-6.0, abs=1e-9)


@pytest.mark.parametrize("nk", [2, 3])
def test_kmo_term_equals_traceless_form(nk):
    phi = _field(16, 21, 4.0)
    delta = inputs.lognormal_delta(16, 22)
    m = oracle.kmo_model(16, 32.0, nk, 1.0, 0.1)
    p = pins.kmo_params(16, 32.0, nk, 1.0, 0.1)
    L_or = oracle.residual(m, phi, delta)
    L_np = pins.laplacian(phi) - pins.kmo_term_traceless(phi, delta, p)
    assert np.abs(L_or - L_np).max() <= 1e-12 * np.abs(L_np).max()


# ------------------------------------------------------- p2: uniform density

@pytest.mark.parametrize("model", ["dgp", "kmo"])
def test_uniform_density_gives_constant_field(model):
    # Sec. 4.2.1: delta = 0 with random initial phi in [-0.05, 0.05] relaxes
    # to a constant (zero after the gauge), residual <= 1e-8
    n = 32
    phi0 = inputs.uniform_phi(n, 7, GOLD["uniform_test"]["phi0_half_width"])
    m = oracle.dgp_model(1.0, OM, 1.0) if model == "dgp" else oracle.kmo_model(n, 64.0, 2, 1.0, 0.1)
    r = oracle.solve(m, np.zeros((n, n, n)), phi0, tol=GOLD["uniform_test"]["residual"])
    assert r.status == 0 and r.eps <= 1e-8
    assert np.abs(r.phi).max() <= 1e-8


# ----------------------------------------------------- p3: exact 1D solutions

def test_paper_dgp_sine_has_exact_discrete_solution():
    # eq:sine_nDGP; the discrete solution is the analytic 1/(4 pi^2) amplitude
    # times (pi/N)^2 / sin^2(pi/N)
    n = 32
    m = oracle.dgp_model(1.0, OM, 1.0)
    amp = GOLD["sine_test"]["nDGP_phi_amplitude"]
    assert amp == pytest.approx(1 / (4 * np.pi ** 2), rel=1e-15)
    delta = pins.dgp_sine_delta_paper(n, m.beta)
    r = oracle.solve(m, delta, tol=1e-13, max_cycles=80)
    exact = pins.dgp_sine_phi_discrete(n)
    exact -= exact.mean()
    assert r.status == 0
    assert np.abs(r.phi - exact).max() <= 1e-10 * np.abs(exact).max()
    # and the continuum amplitude to O(h^2)
    analytic = pins.sine_1d(n, amp)
    assert np.abs(r.phi - analytic).max() <= 2 * (np.pi / n) ** 2 * amp


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_dgp_nonlinear_sine_exact(axis):
    # large amplitude: the branch sqrt(...) = alpha + 4D/3 must be taken
    n = 32
    m = oracle.dgp_model(1.0, OM, 1.0)
    phi = pins.sine_1d(n, 20.0, 1, axis)
    delta = pins.dgp_sine_delta_discrete(phi, m.beta, axis=axis)
    r = oracle.solve(m, delta, tol=1e-12, max_cycles=80)
    phi -= phi.mean()
    assert r.status == 0
    assert np.abs(r.phi - phi).max() <= 1e-10 * np.abs(phi).max()


@pytest.mark.parametrize("nk,amp", [(2, GOLD["sine_test"]["kmo_A"]), (2, 2.0), (3, 2.0)])
def test_kmo_sine_exact_discrete(nk, amp):
    # Sec. 4.2.2 with the exact discrete source (the printed eq:sine_Kmo is
    # garbled); amp = 2 makes gamma g^(n-1) reach ~0.5-0.8
    n = 32
    k0, beta, waves = GOLD["sine_test"]["kmo_K0"], GOLD["sine_test"]["kmo_beta"], GOLD["sine_test"]["kmo_K"]
    m = oracle.kmo_model(n, 64.0, nk, k0, beta)
    p = pins.kmo_params(n, 64.0, nk, k0, beta)
    phi = pins.sine_1d(n, amp, waves)
    delta = pins.kmo_sine_delta_discrete(phi, p)
    r = oracle.solve(m, delta, tol=1e-12, max_cycles=80)
    phi -= phi.mean()
    assert r.status == 0
    assert np.abs(r.phi - phi).max() <= 1e-10 * np.abs(phi).max()


# ----------------------------------------------- p4: linear limit vs FFT

def test_linear_model_equals_fft_poisson():
    n = 32
    delta = inputs.lognormal_delta(n, 1)
    m = oracle.linear_model(1.7)
    r = oracle.solve(m, delta, tol=1e-13, max_cycles=80)
    ref = pins.poisson_fft(1.7 * delta)
    assert np.abs(r.phi - ref).max() <= 1e-11 * np.abs(ref).max()


def test_dgp_weak_field_is_quadratically_close_to_linear():
    # eq:dgp_linear: for a small source the solution approaches the linear
    # one lap(phi) = Omega_m delta / beta with an O(eps^2) difference
    n = 32
    m = oracle.dgp_model(1.0, OM, 1.0)
    base = inputs.lognormal_delta(n, 1)
    errs = []
    for eps in (1e-2, 5e-3):
        d = eps * base
        r = oracle.solve(m, d, tol=1e-15 * eps, max_cycles=80)
        lin = pins.poisson_fft(OM / m.beta * d)
        errs.append(np.abs(r.phi - lin).max() / np.abs(lin).max())
    assert errs[0] / errs[1] == pytest.approx(2.0, rel=0.05)   # relative error ~ eps


# ------------------------------------------------ p5: FFT fixed point

def test_fft_fixed_point_agrees_with_multigrid_config1():
    n = 32
    delta = inputs.lognormal_delta(n, 1)
    m = oracle.dgp_model(1.0, OM, 1.0)
    r = oracle.solve(m, delta, tol=1e-13, max_cycles=80)
    ref, it = pins.fft_fixed_point(lambda p, d: pins.dgp_term_traceless(p, d, m.alpha, m.s), delta)
    assert it < 500
    assert np.abs(r.phi - ref).max() <= 1e-11 * np.abs(ref).max()
    # lambda = -mu is the mean of the model term
    F = pins.dgp_term_traceless(ref, delta, m.alpha, m.s)
    assert r.mu == pytest.approx(-F.mean(), abs=1e-12)


# -------------------------------------------- p6: dense bordered Newton (8^3)

@pytest.mark.parametrize("model", ["dgp", "kmo"])
def test_dense_newton_8cubed(model):
    n = 8
    delta = inputs.lognormal_delta(n, 5, sigma=1.0)
    if model == "dgp":
        m = oracle.dgp_model(1.0, OM, 1.0)
        term = lambda p, d: pins.dgp_term_traceless(p, d, m.alpha, m.s)
    else:
        # large box (small c~) so that the gradient term matters: Newton needs
        # several iterations from phi = 0
        m = oracle.kmo_model(n, 40000.0, 2, 1.0, 0.1)
        p = pins.kmo_params(n, 40000.0, 2, 1.0, 0.1)
        term = lambda ph, d: pins.kmo_term_traceless(ph, d, p)
        delta = delta * 2.0
    phi_n, lam, hist = pins.newton_bordered(term, delta)
    assert hist[-1] < 1e-12 and len(hist) >= 4
    r = oracle.solve(m, delta, tol=1e-14, max_cycles=80)
    assert r.status == 0
    assert np.abs(r.phi - phi_n).max() <= 1e-11 * np.abs(phi_n).max()
    assert -r.mu == pytest.approx(lam, abs=1e-11 * max(1.0, abs(lam)))


# ------------------------------------ p7: manufactured continuum solutions

MODES = [((1, 0, 0), 0.8, 0.3), ((0, 1, 1), 0.5, 1.1), ((1, 1, 0), 0.6, 2.0),
         ((1, -1, 1), 0.4, 0.7), ((0, 0, 2), 0.3, 0.2), ((2, 1, 0), 0.2, 1.5)]


KMO_MODES = [(m, 2.0 * A, t) for m, A, t in MODES]   # gamma g^2 up to ~2.7


def _conv(model, ns):
    box = 16.0
    ss = pins.SineSum(box, MODES if model == "dgp" else KMO_MODES)
    errs = []
    for n in ns:
        psi, G, H, h = ss.eval(n)
        if model == "dgp":
            m = oracle.dgp_model(1.0, OM, 1.0)
            delta = pins.dgp_manufactured_delta(G, H, m.beta, m.alpha)
        else:
            m = oracle.kmo_model(n, box / h * 0.02, 3, 1.0, 0.1)  # c~ independent of n
            p = pins.kmo_params(n, box / h * 0.02, 3, 1.0, 0.1)
            delta = pins.kmo_manufactured_delta(G, H, p)
        # delta enters the discrete equation at cell centres; remove the mean
        # the continuum source integrates to zero
        delta = delta - delta.mean()
        r = oracle.solve(m, delta, tol=1e-12, max_cycles=100, h0=h)
        assert r.status == 0
        psi = psi - psi.mean()
        errs.append(np.abs(r.phi - psi).max() / np.abs(psi).max())
    return errs


def test_dgp_manufactured_second_order():
    e = _conv("dgp", (16, 32, 64))
    assert 3.5 < e[0] / e[1] < 4.5 and 3.7 < e[1] / e[2] < 4.3
    assert e[2] < 2e-3


def test_kmo_manufactured_second_order():
    # pins every Kmouflage stencil coefficient, including the cross-term
    # coefficient 1/(8h^4) (the printed 1/(2h^4) does not converge)
    e = _conv("kmo", (16, 32, 64))
    assert 3.5 < e[0] / e[1] < 4.5 and 3.7 < e[1] / e[2] < 4.3


def test_kmo_manufactured_is_nonlinear():
    # the manufactured Kmouflage case must actually exercise gamma g^(n-1)
    box, n = 16.0, 32
    psi, G, H, h = pins.SineSum(box, KMO_MODES).eval(n)
    p = pins.kmo_params(n, box / h * 0.02, 3, 1.0, 0.1)
    g = G[0] ** 2 + G[1] ** 2 + G[2] ** 2
    assert (p["gamma"] * g ** 2).max() > 2.0


# ----------------------------------------- p8: spherical top-hats (shape)

def _radial_derivative(phi, n):
    # phi' along the +x axis through the centre (cells straddle the centre)
    row = phi[n // 2, n // 2, :]
    x = np.arange(n) + 0.5 - n / 2
    dphi = (np.roll(row, -1) - np.roll(row, 1)) / 2.0
    return x, dphi


@pytest.mark.parametrize("h0rc", [0.5, 1.0, 5.0])
def test_dgp_sphere_profile(h0rc):
    n = 64
    m = oracle.dgp_model(1.0, OM, h0rc)
    R = GOLD["sphere_test_dgp"]["radius_over_N"] * n
    d = inputs.tophat_delta(n, GOLD["sphere_test_dgp"]["delta"], R)
    r = oracle.solve(m, d - d.mean(), tol=1e-10, max_cycles=100)
    x, dphi = _radial_derivative(r.phi, n)
    sel = (x > 1.0) & (x < 1.5 * R)
    ana = pins.dgp_sphere_dphidr(x[sel], GOLD["sphere_test_dgp"]["delta"], R, m.beta, h0rc)
    # periodic images and the mean-subtracted background shift the profile;
    # shape agreement within 15% near the sphere
    assert np.abs(dphi[sel] - ana).max() <= 0.15 * np.abs(ana).max()


@pytest.mark.parametrize("k0", [1.0, 10.0, 100.0])
def test_kmo_sphere_profile(k0):
    n = 64
    box = n * GOLD["code_test_box"]["L_mpch"] / GOLD["code_test_box"]["N_g"]
    beta = GOLD["sphere_test_kmo"]["beta"]
    m = oracle.kmo_model(n, box, 2, k0, beta)
    p = pins.kmo_params(n, box, 2, k0, beta)
    R = GOLD["sphere_test_kmo"]["radius_over_N"] * n
    d = inputs.tophat_delta(n, GOLD["sphere_test_kmo"]["delta"], R)
    r = oracle.solve(m, d - d.mean(), tol=1e-9, max_cycles=100)
    assert r.status == 0
    x, dphi = _radial_derivative(r.phi, n)
    sel = (x > 1.0) & (x < 1.5 * R)
    ana = pins.kmo_sphere_dphidr(x[sel], GOLD["sphere_test_kmo"]["delta"], R, p, beta)
    card = pins.kmo_sphere_cardano_paper(x[sel], GOLD["sphere_test_kmo"]["delta"], R, p["gamma"],
                                         beta, p["ctil"])
    assert np.abs(ana - card).max() <= 1e-9 * np.abs(card).max()   # paper's closed form
    assert np.abs(dphi[sel] - ana).max() <= 0.15 * np.abs(ana).max()


# --------------------------------------------- p9: residual invariants

def test_residual_invariant_under_constant_shift_and_zero_mean():
    n = 16
    delta = inputs.lognormal_delta(n, 2)
    m = oracle.dgp_model(1.0, OM, 1.0)
    phi = _field(n, 5, 1.0)
    r1 = oracle.residual(m, phi, delta)
    r2 = oracle.residual(m, phi + 3.25, delta)
    assert np.abs(r1 - r2).max() <= 1e-12 * np.abs(r1).max()


def test_solve_reports_residual_of_returned_phi():
    n = 32
    delta = inputs.lognormal_delta(n, 1)
    m = oracle.dgp_model(1.0, OM, 1.0)
    r = oracle.solve(m, delta, tol=1e-8)
    L = oracle.residual(m, r.phi, delta)
    eps = np.sqrt(np.mean((L - L.mean()) ** 2))
    assert r.eps == pytest.approx(eps, rel=1e-8)
    assert -r.mu == pytest.approx(-L.mean(), abs=1e-12)
    assert abs(r.phi.mean()) < 1e-14
    # contraction of the FAS V(1,1) cycle on config-1 data
    h = np.array(r.hist)
    assert (h[1:] / h[:-1]).max() < 0.3
    assert r.cycles <= 14


def test_colour_pass_zeroes_linear_residual_of_its_colour():
    # linear model: after a pass of colour c the residual vanishes on colour c
    n = 16
    delta = inputs.lognormal_delta(n, 3)
    m = oracle.linear_model(0.9)
    phi = _field(n, 4, 1.0)
    for c in (0, 1):
        out = oracle.colour_pass(m, phi, delta, c, f=0.3)
        res = oracle.residual(m, out, delta, f=0.3)
        k, j, i = np.indices(res.shape)
        mask = (i + j + k) % 2 == c
        # the same-colour cells were updated from the pre-pass state and the
        # linear 7-point stencil couples only opposite colours
        assert np.abs(res[mask]).max() <= 1e-12


def test_solve_deterministic():
    n = 16
    delta = inputs.lognormal_delta(n, 1)
    m = oracle.dgp_model(1.0, OM, 1.0)
    a = oracle.solve(m, delta, tol=0.0, max_cycles=3)
    b = oracle.solve(m, delta, tol=0.0, max_cycles=3)
    assert np.array_equal(a.phi, b.phi)
