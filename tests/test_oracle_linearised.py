"""Pins of the oracle's linearised comparators (eq:dgp_linear,
eq:linearised_Kmo) against the paper's linear statements and against the full
nonlinear oracle in its small-amplitude limit.  CPU only."""
import numpy as np
import pytest

import inputs
import oracle
from oracle import background as bg
from oracle import pins

OM = 0.3089


def beta_dgp(a, h0rc):
    # eq:beta_dgp, first form, with the LCDM H of eq:H_lcdm (H0 = c = 1)
    e2 = OM / a ** 3 + 1.0 - OM
    hdot_over_h2 = -1.5 * OM / a ** 3 / e2
    return 1.0 + 2.0 * np.sqrt(e2) * h0rc * (1.0 + hdot_over_h2 / 3.0)


@pytest.mark.parametrize("a,h0rc", [(1.0, 1.0), (0.6, 0.5), (0.8, 5.0)])
def test_linearised_dgp_rescales_newton_by_eq_dgp_linear(a, h0rc):
    # total potential Phi_N + phi/2 obeys lap = 4 pi G a^2 (1 + 1/(3 beta)) drho,
    # i.e. (3/2) Omega_m / a (1 + 1/(3 beta)) delta in code units
    n = 16
    delta = inputs.lognormal_delta(n, 4)
    r = oracle.solve(oracle.linearised_dgp_model(a, OM, h0rc), delta, tol=1e-14, max_cycles=80)
    phin = pins.poisson_fft(1.5 * OM / a * delta)
    total = pins.poisson_fft(1.5 * OM / a * (1.0 + 1.0 / (3.0 * beta_dgp(a, h0rc))) * delta)
    assert np.abs(phin + 0.5 * r.phi - total).max() <= 1e-11 * np.abs(total).max()


@pytest.mark.parametrize("nk,k0,beta,a", [(2, 1.0, 0.2, 0.8), (3, 10.0, 0.1, 1.0)])
def test_linearised_kmo_fifth_force_ratio(nk, k0, beta, a):
    # eq:linearised_Kmo: the fifth-force potential beta c~ phi is 2 beta^2 / K_X
    # times Phi_N of lap Phi_N = (3/2) A Omega_m delta / a (eq:kmf_Poission_eqn_codeunit),
    # with K_X = 1 + n K0 (phibar'^2 / (2 lambda^2 a^2))^(n-1)
    n, box = 16, 200.0
    b = bg.solve(nk, k0, beta)
    v = oracle.kmo_background_values(b, a, 0.0)
    m = oracle.linearised_kmo_model(n, box, nk, k0, beta, v["lam"], a, OM, v["phibar"],
                                    v["dphibar_dtau"])
    delta = inputs.lognormal_delta(n, 5)
    phi = oracle.solve(m, delta, tol=1e-16, max_cycles=80).phi
    A = np.exp(beta * v["phibar"])
    kx = 1.0 + nk * k0 * (v["dphibar_dtau"] ** 2 / (2 * v["lam"] ** 2 * a ** 2)) ** (nk - 1)
    phin = pins.poisson_fft(1.5 * A * OM / a * delta)
    ctil = n / box * 2997.92458
    assert np.abs(beta * ctil * phi - 2 * beta ** 2 / kx * phin).max() <= 1e-10 * np.abs(phin).max() * 2 * beta ** 2 / kx


def _limit_errors(full, lin, base, epss, tol_scale):
    errs = []
    for eps in epss:
        d = eps * base
        pf = oracle.solve(full, d, tol=tol_scale * eps, max_cycles=100).phi
        pl = oracle.solve(lin, d, tol=tol_scale * eps, max_cycles=100).phi
        errs.append(np.abs(pf - pl).max() / np.abs(pl).max())
    return errs


def test_linearised_dgp_is_the_small_amplitude_limit():
    n, a, h0rc = 16, 0.7, 1.0
    base = inputs.lognormal_delta(n, 6)
    errs = _limit_errors(oracle.dgp_model(a, OM, h0rc), oracle.linearised_dgp_model(a, OM, h0rc),
                         base, (2e-3, 1e-3), 1e-15)
    assert errs[0] < 1e-2
    assert errs[0] / errs[1] == pytest.approx(2.0, rel=0.05)


def test_linearised_kmo_is_the_small_amplitude_limit():
    # K depends on grad phi through X only, so the full equation is odd under
    # (phi, delta) -> (-phi, -delta): the first correction to the linear
    # solution is cubic and the relative difference falls as eps^2 (the nDGP
    # quadratic form has no such symmetry and falls as eps)
    n, box, nk, k0, beta, a = 16, 32.0, 2, 1.0, 0.3, 0.9
    b = bg.solve(nk, k0, beta)
    v = oracle.kmo_background_values(b, a, 0.0)
    args = (n, box, nk, k0, beta, v["lam"], a, OM, v["phibar"], v["dphibar_dtau"])
    base = inputs.lognormal_delta(n, 7)
    errs = _limit_errors(oracle.kmo_model(*args), oracle.linearised_kmo_model(*args), base,
                         (2e-2, 1e-2), 1e-17)
    assert 0 < errs[0] < 1e-1
    assert errs[0] / errs[1] == pytest.approx(4.0, rel=0.05)


def test_full_dgp_field_is_screened_below_the_linear_one():
    # Vainshtein screening (eq:V_screening): inside a dense top-hat the full
    # fifth-force potential well is shallower than the linear one, and the
    # more so the denser the top-hat
    n, c = 32, 16
    ratios = []
    for delta_in in (50.0, 200.0, 1000.0):
        delta = inputs.tophat_delta(n, delta_in, 2.5)
        full = oracle.solve(oracle.dgp_model(1.0, OM, 1.0), delta, tol=1e-10, max_cycles=100).phi
        lin = oracle.solve(oracle.linearised_dgp_model(1.0, OM, 1.0), delta, tol=1e-10,
                           max_cycles=100).phi
        depth_full = full[c, c, c] - full[0, 0, 0]
        depth_lin = lin[c, c, c] - lin[0, 0, 0]
        assert depth_lin < depth_full < 0
        ratios.append(depth_full / depth_lin)
    assert ratios[0] > ratios[1] > ratios[2]
    assert ratios[2] < 0.5
