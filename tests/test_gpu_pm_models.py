"""GPU particle-mesh steps of both models against the oracle: one Kmouflage
step, the linear fifth-force ratios through the GPU solvers, and short
multi-step runs (nDGP and Kmouflage) from the same Zel'dovich start."""
import numpy as np
import pytest
import torch

import inputs
import oracle
import paper_2110_00566_amd as mg
from oracle import background as bg

pytestmark = pytest.mark.gpu
OM = 0.3089


def g(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def c(t):
    return t.detach().cpu().numpy()


def periodic_diff(p, q, n):
    d = np.abs(p.astype(np.float64) - q.astype(np.float64))
    return np.minimum(d, n - d)


def sine(n, eps):
    x = (np.arange(n) + 0.5) / n
    return np.broadcast_to(eps * np.sin(2 * np.pi * x)[None, None, :], (n, n, n)).copy()


def test_linear_fifth_force_ratios_on_gpu():
    n = 32
    d = g(sine(n, 1e-4))
    a = 0.8
    # nDGP: (1/2) phi = Phi_N / (3 beta)
    phin, _ = mg.solve_poisson(d, 1.5 * OM / a, tol=1e-15, max_cycles=80)
    phi, _ = mg.solve_dgp(d, a=a, h0rc=1.0, tol=1e-15, max_cycles=80)
    beta = oracle.dgp_model(a, OM, 1.0).beta
    pn, pf = c(phin).ravel(), c(phi).ravel()
    assert (0.5 * pf @ pn) / (pn @ pn) == pytest.approx(1 / (3 * beta), rel=1e-4)
    # Kmouflage: beta c~ phi = 2 beta^2 / K_X Phi_N, background from the library
    box, nk, k0, bk = 256.0, 2, 1.0, 0.2
    bgr = mg.kmo_background(nk, k0, bk, [a])
    v = dict(lam=bgr["lambda"], phibar=float(bgr["phibar"][0]),
             dphibar_dtau=float(bgr["dphibar_dtau"][0]))
    A = np.exp(bk * v["phibar"])
    d5 = g(sine(n, 1e-5))
    phin, _ = mg.solve_poisson(d5, 1.5 * A * OM / a, tol=1e-18, max_cycles=100)
    par = mg.KmoParams(nk, k0, bk, v["lam"], a, OM, box, v["phibar"], v["dphibar_dtau"])
    phi, _ = mg._solve(mg.lib().mg_solve_kmouflage, par, mg.MODEL_KMOUFLAGE, d5, None, None,
                       tol=1e-18, max_cycles=100)
    ctil = n / box * 2997.92458
    xbar = v["dphibar_dtau"] ** 2 / (2 * v["lam"] ** 2 * a ** 2)
    kx = 1 + nk * k0 * xbar ** (nk - 1)
    pn, pf = c(phin).ravel(), c(phi).ravel()
    assert (bk * ctil * pf @ pn) / (pn @ pn) == pytest.approx(2 * bk ** 2 / kx, rel=1e-4)


def test_kmouflage_pm_step_parity():
    n, npart, box, a, da = 64, 32, 128.0, 0.5, 0.02
    nk, k0, beta = 2, 1.0, 0.2
    pos = inputs.za_particles(npart, n, 7, amplitude=20.0)
    mom = np.zeros_like(pos)
    b = bg.solve(nk, k0, beta)
    vo = oracle.kmo_background_values(b, a, da)
    p_or, m_or, phi_or, d_or, phin_or = oracle.pm_step_kmouflage(pos, mom, n, a, da, box, nk, k0,
                                                                 beta, vo, tol=1e-11)
    gp, gm = g(pos), g(mom)
    phi = torch.zeros((n,) * 3, dtype=torch.float64, device="cuda")
    phin = torch.zeros_like(phi)
    delta, st = mg.pm_step_kmouflage(gp, gm, phi, phin, n, a, da, box, nk, k0, beta, tol=1e-11)
    assert st["status"] in (0, 2)
    # fixed-point CIC: 2^-33 per weight, scaled by n^3 / n_part^3 = 8
    assert np.abs(c(delta) - d_or).max() <= 2e-7
    assert np.abs(c(phin) - phin_or).max() <= 1e-8 * np.abs(phin_or).max()
    assert np.abs(c(phi) - phi_or).max() <= 1e-8 * np.abs(phi_or).max()
    assert np.abs(c(gm) - m_or).max() <= 2e-6 * np.abs(m_or).max()
    assert periodic_diff(c(gp), p_or, n).max() <= 1e-4


@pytest.mark.parametrize("model", ["dgp", "kmo"])
def test_multi_step_runs_track_the_oracle(model):
    n, npart, box = 32, 16, 64.0
    a, da, steps = 0.5, 0.025, 4
    pos = inputs.za_particles(npart, n, 8, amplitude=15.0)
    mom = np.zeros_like(pos)
    gp, gm = g(pos), g(mom)
    phi = torch.zeros((n,) * 3, dtype=torch.float64, device="cuda")
    phin = torch.zeros_like(phi)
    b = bg.solve(2, 1.0, 0.2) if model == "kmo" else None
    po, mo, phio = pos, mom, None
    for s in range(steps):
        if model == "dgp":
            po, mo, phio, _, _ = oracle.pm_step(po, mo, n, a, da, tol=1e-11, phi0=phio)
            _, st = mg.pm_step(gp, gm, phi, phin, n, a, da, tol=1e-11)
        else:
            vo = oracle.kmo_background_values(b, a, da)
            po, mo, phio, _, _ = oracle.pm_step_kmouflage(po, mo, n, a, da, box, 2, 1.0, 0.2, vo,
                                                          tol=1e-11, phi0=phio)
            _, st = mg.pm_step_kmouflage(gp, gm, phi, phin, n, a, da, box, 2, 1.0, 0.2, tol=1e-11)
        assert st["status"] in (0, 2)
        a += da
    assert periodic_diff(c(gp), po, n).max() <= 1e-3
    assert np.abs(c(gm) - mo).max() <= 1e-4 * np.abs(mo).max()
    assert np.abs(mo).max() > 0


def test_gpu_pm_runs_follow_linear_growth():
    # 50 GPU steps from a = 0.25 to 1 of a linear growing mode (64^3 mesh,
    # 32^3 particles): nDGP must grow as the growth equation with
    # G_eff = 1 + 1/(3 beta_DGP) (eq:dgp_linear), Kmouflage as eq:kmo_lin_growth,
    # against an LCDM run (the Kmouflage step with beta = 0)
    from scipy.interpolate import CubicSpline
    from pm_growth import growing_mode_ics, large_scale_growth, linear_growth
    n, npart, a0, a1, nst, h0rc, box = 64, 32, 0.25, 1.0, 50, 0.5, 128.0
    nk, k0, beta = 2, 1.0, 0.2
    da = (a1 - a0) / nst
    e_lcdm = lambda a: np.sqrt(OM / a ** 3 + 1.0 - OM)
    x0, p0, f0 = growing_mode_ics(n, npart, 12, a0, e_lcdm)
    ap = np.linspace(0.2, 1.0, 300)
    tab = {bt: mg.kmo_background(nk, k0, bt, ap) for bt in (0.0, beta)}
    sp = {bt: {k: CubicSpline(ap, tab[bt][k]) for k in ("hubble", "phibar", "dphibar_dtau")}
          for bt in tab}
    # the library's background table at every step's a and a + da/2 (the
    # Kmouflage steps look their background values up in it)
    steps_a, a = [], a0
    for _ in range(nst):
        steps_a += [a, a + 0.5 * da]
        a += da
    step_tab = {bt: mg.kmo_background(nk, k0, bt, sorted(set(steps_a))) for bt in (0.0, beta)}
    runs = {}
    for name in ("dgp", "kmo", "lcdm"):
        gp, gm = g(x0), g(p0)
        phi = torch.zeros((n,) * 3, dtype=torch.float64, device="cuda")
        phin = torch.zeros_like(phi)
        a = a0
        for _ in range(nst):
            if name == "dgp":
                _, st = mg.pm_step(gp, gm, phi, phin, n, a, da, h0rc=h0rc)
            else:
                bt = beta if name == "kmo" else 0.0
                _, st = mg.pm_step_kmouflage(gp, gm, phi, phin, n, a, da, box, nk, k0, bt,
                                             table=step_tab[bt])
            assert st["status"] in (0, 2)
            a += da
        runs[name] = mg.cic_delta(gp, n)
    d0 = c(mg.cic_delta(g(x0), n))
    grow = {k: large_scale_growth(d0, c(v)) for k, v in runs.items()}

    def ode_kmo(bt):
        s = sp[bt]
        lam = tab[bt]["lambda"]

        def geff(a):
            xbar = float(s["dphibar_dtau"](a)) ** 2 / (2 * lam ** 2 * a ** 2)
            return np.exp(bt * float(s["phibar"](a))) * (1.0 + 2 * bt ** 2 / (1.0 + nk * k0 * xbar ** (nk - 1)))

        def rhs(a, y):
            e = float(s["hubble"](a))
            dphida = float(s["dphibar_dtau"](a)) / (a * a * e)
            return [y[1] / (a ** 3 * e), 1.5 * OM * geff(a) * y[0] / (a ** 2 * e) - bt * dphida * y[1]]
        from scipy.integrate import solve_ivp
        return solve_ivp(rhs, (a0, a1), [1.0, a0 ** 3 * e_lcdm(a0) * f0], rtol=1e-9,
                         atol=1e-14).y[0, -1]
    beta_dgp = lambda a: 1.0 + 2.0 * e_lcdm(a) * h0rc * (1.0 - 0.5 * OM / a ** 3 / e_lcdm(a) ** 2)
    ode = {"dgp": linear_growth(a0, a1, lambda a: 1.0 + 1.0 / (3.0 * beta_dgp(a)), f0, e_lcdm)[0],
           "kmo": ode_kmo(beta), "lcdm": ode_kmo(0.0)}
    for k in ode:
        assert grow[k] == pytest.approx(ode[k], rel=0.03), k
    for k in ("dgp", "kmo"):
        assert ode[k] / ode["lcdm"] - 1.0 > 0.02
        assert grow[k] / grow["lcdm"] - 1.0 == pytest.approx(ode[k] / ode["lcdm"] - 1.0, rel=0.06), k
