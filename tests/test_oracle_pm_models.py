"""Pins of the oracle's model-specific particle-mesh pieces, CPU only.

- Linear fifth force: for a tiny single-mode density the scalar potential is
  a fixed multiple of the Newtonian one on the same mesh (both use the same
  7-point Laplacian): nDGP (1/2) phi = Phi_N / (3 beta_DGP)
  (eq:fifth-force-ratio-asymptotic), Kmouflage beta c~ phi = (2 beta^2 / K_X)
  Phi_N with K_X = 1 + gamma b^(n-1) (the paper's F5/FN in code units).
- The Kmouflage kick: total momentum changes only by the velocity-term
  factor (no self-force of CIC + 3-point gradient + CIC), and beta = 0 is the
  Newtonian step.
"""
import numpy as np
import pytest

import inputs
import oracle
from oracle import background as bg

OM = 0.3089


def sine(n, eps):
    x = (np.arange(n) + 0.5) / n
    return np.broadcast_to(eps * np.sin(2 * np.pi * x)[None, None, :], (n, n, n)).copy()


@pytest.mark.parametrize("h0rc,a", [(1.0, 1.0), (0.5, 0.6)])
def test_dgp_linear_fifth_force_ratio(h0rc, a):
    n = 16
    d = sine(n, 1e-4)
    m = oracle.dgp_model(a, OM, h0rc)
    phin = oracle.fft_poisson(1.5 * OM / a * d)
    phi = oracle.solve(m, d, tol=1e-16, max_cycles=60).phi
    ratio = (0.5 * phi).ravel() @ phin.ravel() / (phin.ravel() @ phin.ravel())
    assert ratio == pytest.approx(1.0 / (3.0 * m.beta), rel=1e-4)


@pytest.mark.parametrize("nk,k0,beta,a", [(2, 1.0, 0.2, 0.8), (3, 10.0, 0.1, 1.0)])
def test_kmouflage_linear_fifth_force_ratio(nk, k0, beta, a):
    n, box = 16, 256.0
    b = bg.solve(nk, k0, beta)
    v = oracle.kmo_background_values(b, a, 0.0)
    m = oracle.kmo_model(n, box, nk, k0, beta, v["lam"], a, OM, v["phibar"], v["dphibar_dtau"])
    d = sine(n, 1e-5)
    A = np.exp(beta * v["phibar"])
    phin = oracle.fft_poisson(1.5 * A * OM / a * d)
    phi = oracle.solve(m, d, tol=1e-18, max_cycles=80).phi
    ctil = n / box * 2997.92458
    ratio = (beta * ctil * phi).ravel() @ phin.ravel() / (phin.ravel() @ phin.ravel())
    # K_X of the background: 1 + n K0 Xbar^(n-1), Xbar = phi'^2 / (2 lambda^2 a^2)
    xbar = v["dphibar_dtau"] ** 2 / (2 * v["lam"] ** 2 * a ** 2)
    kx = 1.0 + nk * k0 * xbar ** (nk - 1)
    assert m.C0 == pytest.approx(kx, rel=1e-12)
    assert ratio == pytest.approx(2 * beta ** 2 / kx, rel=1e-4)


def test_kmouflage_kick_momentum_and_newtonian_limit():
    n, npart, box, a, da = 16, 8, 64.0, 0.7, 0.01
    pos = inputs.za_particles(npart, n, 3, amplitude=40.0)
    mom = (np.random.default_rng(1).standard_normal(pos.shape) * 0.1).astype(np.float32)
    b = bg.solve(2, 1.0, 0.2)
    v = oracle.kmo_background_values(b, a, da)
    p2, m2, phi, d, phin = oracle.pm_step_kmouflage(pos, mom, n, a, da, box, 2, 1.0, 0.2, v,
                                                    tol=1e-12)
    damp = 1.0 - 0.2 * v["dphibar_da"] * da
    assert np.abs(m2.astype(np.float64).sum(0) - damp * mom.astype(np.float64).sum(0)).max() <= 1e-4
    # beta = 0: the Newtonian step with the same background expansion
    v0 = dict(v, phibar=0.0, dphibar_da=0.0)
    p3, m3, *_ = oracle.pm_step_kmouflage(pos, mom, n, a, da, box, 2, 1.0, 0.0, v0, tol=1e-12)
    _, dd = oracle.cic_density(pos, n)
    psi = oracle.fft_poisson(1.5 * OM / a * dd)
    p4, m4 = pos.copy(), mom.copy()
    oracle.lib().or_kick_drift(n, p4.shape[0], np.ascontiguousarray(psi), p4.reshape(-1),
                               m4.reshape(-1), da / (a * v["e_a"]),
                               da / ((a + da / 2) ** 3 * v["e_half"]))
    assert np.array_equal(m3, m4) and np.array_equal(p3, p4)


# ------------------------------------------------ linear growth of PM runs

from pm_growth import growing_mode_ics, large_scale_growth, linear_growth as _growth  # noqa: E402


def test_pm_runs_follow_linear_growth_with_the_dgp_enhancement():
    # eq:dgp_linear: on large scales nDGP rescales Newton's constant by
    # G_eff = 1 + 1/(3 beta_DGP(a)); 50 steps from a = 0.25 to 1 of a linear
    # growing mode must grow as the G_eff-modified linear growth equation,
    # and the LCDM run as the unmodified one
    n, npart, a0, a1, nst, h0rc = 32, 16, 0.25, 1.0, 50, 0.5
    da = (a1 - a0) / nst
    e = lambda a: np.sqrt(OM / a ** 3 + 1.0 - OM)
    beta = lambda a: 1.0 + 2.0 * e(a) * h0rc * (1.0 - 0.5 * OM / a ** 3 / e(a) ** 2)
    x0, p0, f0 = growing_mode_ics(n, npart, 11, a0, e)
    runs = {}
    for name, step in (("lcdm", lambda x, p, a: oracle.pm_step_newtonian(x, p, n, a, da)),
                       ("dgp", lambda x, p, a: oracle.pm_step(x, p, n, a, da, h0rc=h0rc))):
        x, p, a = x0, p0, a0
        for _ in range(nst):
            x, p = step(x, p, a)[:2]
            a += da
        runs[name] = x
    d0 = oracle.cic_density(x0, n)[1]
    g_lcdm = large_scale_growth(d0, oracle.cic_density(runs["lcdm"], n)[1])
    g_dgp = large_scale_growth(d0, oracle.cic_density(runs["dgp"], n)[1])
    ode_lcdm = _growth(a0, a1, lambda a: 1.0, f0, e)[0]
    ode_dgp = _growth(a0, a1, lambda a: 1.0 + 1.0 / (3.0 * beta(a)), f0, e)[0]
    # absolute growth within the PM discretisation (time step, 3-point force, CIC)
    assert g_lcdm == pytest.approx(ode_lcdm, rel=0.03)
    assert g_dgp == pytest.approx(ode_dgp, rel=0.03)
    # the enhancement, where those cancel, to 5% of itself (it is ~7%)
    assert ode_dgp / ode_lcdm - 1.0 > 0.05
    assert (g_dgp / g_lcdm - 1.0) == pytest.approx(ode_dgp / ode_lcdm - 1.0, rel=0.05)


def test_kmouflage_pm_runs_follow_eq_kmo_lin_growth():
    # eq:kmo_lin_growth in the PM step's variables: the friction
    # (d ln A/d phi) phi' becomes -beta (d phibar/da) p, and the source is
    # (3/2) Omega_m A(phibar) (1 + 2 beta^2/K_X) D / (a^2 E) with the
    # background E, phibar, phibar' of the solver
    from scipy.integrate import solve_ivp
    n, npart, a0, a1, nst = 32, 16, 0.25, 1.0, 50
    nk, k0, beta, box = 2, 1.0, 0.2, 64.0
    da = (a1 - a0) / nst
    b = bg.solve(nk, k0, beta)
    e_lcdm = lambda a: np.sqrt(OM / a ** 3 + 1.0 - OM)
    x0, p0, f0 = growing_mode_ics(n, npart, 11, a0, e_lcdm)

    def rhs(a, y):
        v = oracle.kmo_background_values(b, a, 0.0)
        xbar = v["dphibar_dtau"] ** 2 / (2 * v["lam"] ** 2 * a ** 2)
        geff = np.exp(beta * v["phibar"]) * (1.0 + 2 * beta ** 2 / (1.0 + nk * k0 * xbar ** (nk - 1)))
        return [y[1] / (a ** 3 * v["e_a"]),
                1.5 * OM * geff * y[0] / (a ** 2 * v["e_a"]) - beta * v["dphibar_da"] * y[1]]
    # same initial momentum as the particles
    ode_kmo = solve_ivp(rhs, (a0, a1), [1.0, a0 ** 3 * e_lcdm(a0) * f0], rtol=1e-9,
                        atol=1e-14).y[0, -1]
    ode_lcdm = _growth(a0, a1, lambda a: 1.0, f0, e_lcdm)[0]
    xk, pk, xl, pl, a = x0, p0, x0, p0, a0
    for _ in range(nst):
        xk, pk = oracle.pm_step_kmouflage(xk, pk, n, a, da, box, nk, k0, beta,
                                          oracle.kmo_background_values(b, a, da))[:2]
        xl, pl = oracle.pm_step_newtonian(xl, pl, n, a, da)[:2]
        a += da
    d0 = oracle.cic_density(x0, n)[1]
    g_kmo = large_scale_growth(d0, oracle.cic_density(xk, n)[1])
    g_lcdm = large_scale_growth(d0, oracle.cic_density(xl, n)[1])
    assert g_kmo == pytest.approx(ode_kmo, rel=0.03)
    assert ode_kmo / ode_lcdm - 1.0 > 0.02
    assert (g_kmo / g_lcdm - 1.0) == pytest.approx(ode_kmo / ode_lcdm - 1.0, rel=0.05)
