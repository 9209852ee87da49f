"""Benchmark: nDGP multigrid solve at 512^3 on one MI355X.

One step = CIC density of 256^3 Zel'dovich-displaced particles on the 512^3
mesh (L = 512 Mpc/h) followed by the nDGP (H0 r_c = 1, a = 1) FAS V(1,1)
solve from phi = 0 to a mean-projected residual <= 1e-8, all in FP64.
Particles are resident on the GPU before the timed region.

Prints one JSON line: value = finest-level cell updates per second over the
whole step (n^3 * (nu_pre + nu_post) * cycles / step time), the dominant
kernel's roofline (finest colour pass, timed with HIP events on the stream
the solver launches on) and the FP64 CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

N_MESH, N_PART, BOX, SEED = 512, 256, 512.0, 6
H0RC, A, OMEGA_M, TOL = 1.0, 1.0, 0.3089, 1e-8
HBM_PEAK_GBS = 8000.0
# algorithmic bytes of one finest colour pass per mesh cell (FP64): read both
# colour halves (8 B), the colour's delta (4 B), write the colour (4 B)
PASS_BYTES_PER_CELL = 16
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "pass_dgp_512_traffic.json")
KERNEL_SOURCES = ["paper_2110_00566_amd/csrc/mg_device.h", "paper_2110_00566_amd/csrc/mg_kernels.h",
                  "paper_2110_00566_amd/csrc/mg_tiled.h"]


def kernel_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per pass launch from the committed rocprofv3 counter runs,
    if they were taken on the current kernel source."""
    try:
        t = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    if t.get("kernel_sha") != kernel_hash():
        return None
    return t.get("bytes_per_launch")


def cpu_baseline(pos_np):
    """FP64 oracle on the host: CIC + 3 V(1,1) cycles at 512^3 (bounded sample)."""
    import oracle
    oracle.build(force=False)
    t0 = time.perf_counter()
    _, delta = oracle.cic_density(pos_np, N_MESH)
    r = oracle.solve(oracle.dgp_model(A, OMEGA_M, H0RC), delta, tol=0.0, max_cycles=3)
    dt = time.perf_counter() - t0
    updates = N_MESH ** 3 * 2 * r.cycles
    return {"value": updates / dt, "unit": "cell-updates/s",
            "cores": int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1)),
            "kind": "oracle",
            "sample": "CIC of the 256^3 particles + 3 FAS V(1,1) cycles at 512^3 (tol=0), "
                      "%.1f s" % dt}


def vcycle_bytes(n: int, fused: bool = False) -> int:
    """Algorithmic HBM bytes of one FP64 V(1,1) cycle: per level 4 colour
    passes (16 B/cell), residual + restriction (18) and prolongation (18),
    plus the coarse FAS source (40 B per coarse cell).  fused: the bytes the
    executed kernels must move, where levels >= 128^3 fuse the prolongation
    with the first post-smoothing pass (22 B/cell instead of 18 + 16)."""
    total, m, lev = 0, n, 0
    while m > 4:
        per = 88 if (fused and m >= 128) else 100
        total += per * m ** 3 + (40 * m ** 3 if lev else 0)
        m //= 2
        lev += 1
    return total


def vcycle_time(mg, L, C, delta):
    """Time per FP64 V-cycle on delta's mesh: difference of 6- and 2-cycle
    solves (tol = 0), which cancels the set-up and the residual passes."""
    import torch
    n = delta.shape[0]
    ws = mg.workspace(n, mg.MODEL_DGP, False, delta.device)
    par = mg.dgp_params(A, OMEGA_M, H0RC)
    phi = torch.zeros_like(delta)
    times = {}
    for cyc in (2, 6, 2, 6):
        opts = mg.make_opts(n, tol=0.0, max_cycles=cyc)
        st = mg.Stats()
        phi.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        mg._raise(L.mg_solve_dgp(C.byref(opts), C.byref(par), mg._ptr(delta), mg._ptr(phi),
                                 mg._ptr(ws), ws.numel(), mg._stream(), C.byref(st)))
        torch.cuda.synchronize()
        times[cyc] = time.perf_counter() - t0
    ms = 1e3 * (times[6] - times[2]) / 4
    bytes_ = vcycle_bytes(n)
    fbytes = vcycle_bytes(n, fused=True)
    del ws, phi
    torch.cuda.empty_cache()
    return {"n_mesh": n, "ms_per_vcycle": ms, "algorithmic_bytes_per_vcycle": bytes_,
            "achieved_GBs": bytes_ / (ms * 1e-3) / 1e9,
            "frac_of_hbm_peak": bytes_ / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
            "executed_min_bytes_per_vcycle": fbytes,
            "executed_frac_of_hbm_peak": fbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS}


def cycle_types(mg, L, C, delta, ws, par, phi_ref):
    """Time to tol from phi = 0 with V(1,1), F(1,1) and W(1,1) cycles on the
    same density (the arrangements of Sec. 3.2.1): cycles, ms, and the largest
    relative difference from the V-cycle solution."""
    import numpy as np
    import torch
    n = delta.shape[0]
    phi = torch.zeros_like(delta)
    res = {}
    for name, cyc in (("V", mg.CYCLE_V), ("F", mg.CYCLE_F), ("W", mg.CYCLE_W)):
        opts = mg.make_opts(n, tol=TOL, max_cycles=60, cycle=cyc)
        secs, st = [], None
        for rep in range(4):
            phi.zero_()
            st = mg.Stats()
            mg._raise(L.mg_solve_dgp(C.byref(opts), C.byref(par), mg._ptr(delta), mg._ptr(phi),
                                     mg._ptr(ws), ws.numel(), mg._stream(), C.byref(st)))
            if rep:
                secs.append(st.seconds)
        assert st.status == 0 and st.eps <= TOL, (name, st.status)
        err = float((phi - phi_ref).abs().max() / phi_ref.abs().max())
        res[name] = {"cycles": int(st.cycles), "time_to_tol_ms": 1e3 * float(np.mean(secs)),
                     "eps": float(st.eps), "max_rel_diff_phi_vs_V": err}
    return res


def comparators(mg, L, C, delta, ws, par, phi_ref):
    """The baselines the closed-form FAS solve is compared with, from phi = 0:
    Newton-Gauss-Seidel on the quadratic form (on the bench density, and on a
    tenth of it beside the closed form on the same tenth), the linearised
    equation (eq:dgp_linear) by the same multigrid, and the all-FP32 variant
    (stops at its floor).  Status, cycles, ms, final residual and the largest
    and RMS relative differences from the FP64 closed-form solution."""
    import numpy as np
    import torch
    n = delta.shape[0]
    s_lin = mg.linear_source(mg.MODEL_DGP, par)
    ws32 = mg.workspace(n, mg.MODEL_DGP, False, delta.device, mg.MG_FP32)
    mild = 0.1 * delta
    phi = torch.zeros_like(delta)

    def run(fn, p, d, w, prec, ref):
        opts = mg.make_opts(n, tol=TOL, max_cycles=60, precision=prec)
        secs, st, rc = [], None, 0
        for rep in range(3):
            phi.zero_()
            st = mg.Stats()
            rc = fn(C.byref(opts), C.byref(p), mg._ptr(d), mg._ptr(phi), mg._ptr(w), w.numel(),
                    mg._stream(), C.byref(st))
            if rc < 0 and rc not in (mg.MG_ERR_DIVERGED, mg.MG_ERR_NONFINITE):
                mg._raise(rc)
            if rep:
                secs.append(st.seconds)
        out = {"status": L.mg_status_string(rc).decode(), "cycles": int(st.cycles),
               "time_ms": 1e3 * float(np.mean(secs)) if rc >= 0 else None,
               "eps": float(st.eps)}
        if rc >= 0 and ref is not None:
            diff = phi - ref
            out["max_rel_diff_phi_vs_fp64"] = float(diff.abs().max() / ref.abs().max())
            out["rms_rel_diff_phi_vs_fp64"] = float(diff.norm() / ref.norm())
        return out

    res = {"newton_gs": run(L.mg_solve_dgp_newton, par, delta, ws, mg.MG_FP64, phi_ref)}
    closed_mild = run(L.mg_solve_dgp, par, mild, ws, mg.MG_FP64, None)
    ref_mild = phi.clone()
    res["delta_x0.1"] = {"closed_form": closed_mild,
                         "newton_gs": run(L.mg_solve_dgp_newton, par, mild, ws, mg.MG_FP64,
                                          ref_mild)}
    del ref_mild
    res["linearised"] = run(L.mg_solve_poisson, mg.PoissonParams(s_lin), delta, ws, mg.MG_FP64,
                            phi_ref)
    res["linearised"]["s"] = s_lin
    res["fp32"] = run(L.mg_solve_dgp, par, delta, ws32, mg.MG_FP32, phi_ref)
    del ws32, mild
    return res


def other_solves(mg, delta, phi_dgp):
    """The other solves of the path on the bench density from a zero start:
    Kmouflage (n = 3, K0 = 1, beta = 0.1, L = 512 Mpc/h) in FP64 and mixed
    precision, and the nDGP adjoint of loss = sum(phi w) (w seeded N(0,1)) at
    the converged bench field: cycles, ms to tol, ms per cycle."""
    import numpy as np
    import torch
    import inputs
    n = delta.shape[0]
    res = {}
    for name, prec in (("kmouflage_fp64", mg.MG_FP64), ("kmouflage_mixed", mg.MG_MIXED)):
        ws = mg.workspace(n, mg.MODEL_KMOUFLAGE, False, delta.device, prec)
        secs, st = [], None
        for rep in range(3):
            _, st = mg.solve_kmouflage(delta, box_mpch=BOX, n_k=3, k0=1.0, beta=0.1, ws=ws,
                                       tol=TOL, max_cycles=60, precision=prec)
            if rep:
                secs.append(st["seconds"])
        assert st["status"] == 0 and st["eps"] <= TOL, (name, st["status"])
        ms = 1e3 * float(np.mean(secs))
        res[name] = {"cycles": st["cycles"], "time_to_tol_ms": ms, "ms_per_cycle": ms / st["cycles"]}
        del ws
        torch.cuda.empty_cache()
    w = torch.from_numpy(inputs.gaussian_weights(n, 3)).to(delta.device)
    ws = mg.workspace(n, mg.MODEL_DGP, True, delta.device)
    par = mg.dgp_params(A, OMEGA_M, H0RC)
    secs, st = [], None
    for rep in range(3):
        _, _, st = mg.solve_adjoint(mg.MODEL_DGP, par, delta, phi_dgp, w, ws=ws, tol=TOL,
                                    max_cycles=60)
        if rep:
            secs.append(st["seconds"])
    assert st["status"] == 0, st["status"]
    ms = 1e3 * float(np.mean(secs))
    res["adjoint_dgp_fp64"] = {"cycles": st["cycles"], "time_to_tol_ms": ms,
                               "ms_per_cycle": ms / st["cycles"]}
    del ws, w
    torch.cuda.empty_cache()
    return res


def pm_phases(sts):
    """Mean GPU time of a PM step's phases (HIP events in the library) and the
    cycles of its scalar-field solve (the Newtonian potential is an FFT)."""
    import numpy as np
    names = ("cic", "newtonian_fft", "scalar_solve", "potential_kick_drift")
    return {"phase_ms": {k: float(np.mean([s["pm_ms"][q] for s in sts]))
                         for q, k in enumerate(names)},
            "scalar_cycles_per_step": float(np.mean([s["cycles"] for s in sts]))}


def pm_steps(mg, pos0, dev, steps=3):
    """Particle-mesh steps of both models on the bench workload (512^3 mesh,
    256^3 particles, L = 512 Mpc/h) from a = 0.5, da = 0.01: CIC, Newtonian
    potential by FFT, scalar field to 1e-8 (warm-started), kick and drift."""
    import numpy as np
    import torch
    res = {}
    for model in ("dgp", "kmouflage"):
        pos = pos0.clone()
        mom = torch.zeros_like(pos)
        phi = torch.zeros((N_MESH,) * 3, dtype=torch.float64, device=dev)
        phin = torch.zeros_like(phi)
        ws = torch.empty(mg.lib().mg_pm_workspace_bytes(N_MESH), dtype=torch.uint8, device=dev)
        a, da, times, sts = 0.5, 0.01, [], []
        table = None
        if model == "kmouflage":   # background table of every step's a and a + da/2
            pts = [0.5 + q * da for q in range(steps + 1)]
            table = mg.kmo_background(2, 1.0, 0.2, sorted(pts + [x + 0.5 * da for x in pts]))
        for s in range(steps + 1):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if model == "dgp":
                _, st = mg.pm_step(pos, mom, phi, phin, N_MESH, a, da, h0rc=H0RC, ws=ws, tol=TOL)
            else:
                _, st = mg.pm_step_kmouflage(pos, mom, phi, phin, N_MESH, a, da, BOX, 2, 1.0, 0.2,
                                             table=table, ws=ws, tol=TOL)
            torch.cuda.synchronize()
            assert st["status"] >= 0
            if s:
                times.append(time.perf_counter() - t0)
                sts.append(st)
            a += da
        res[model] = {"ms_per_step": 1e3 * float(np.mean(times)), **pm_phases(sts)}
        del ws, phi, phin
        torch.cuda.empty_cache()
    res["config"] = "512^3 mesh, 256^3 particles, L=512 Mpc/h, a=0.5, da=0.01, tol=1e-8; " \
                    "Kmouflage n=2, K0=1, beta=0.2 with its background"
    return res


def vcycle_1024(mg, L, C, pos):
    """FP64 V-cycle on a 1024^3 mesh: CIC of 512^3 Zel'dovich particles
    (L = 1 Gpc/h)."""
    import torch
    delta = mg.cic_delta(pos, 1024)
    r = vcycle_time(mg, L, C, delta)
    del delta
    torch.cuda.empty_cache()
    return r


def pm_step_1024(mg, dev, pos, steps=2):
    """nDGP PM steps on the full-size PM configuration: 1024^3 mesh, 512^3
    Zel'dovich particles (pos, moved in place), L = 1 Gpc/h, a = 1,
    da = 0.0063, Newtonian potential by FFT, scalar field to 1e-8
    (warm-started after the first step)."""
    import numpy as np
    import torch
    n = 1024
    mom = torch.zeros_like(pos)
    phi = torch.zeros((n,) * 3, dtype=torch.float64, device=dev)
    phin = torch.zeros_like(phi)
    ws = torch.empty(mg.lib().mg_pm_workspace_bytes(n), dtype=torch.uint8, device=dev)
    a, da, times, sts = 1.0, 0.0063, [], []
    for s in range(steps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, st = mg.pm_step(pos, mom, phi, phin, n, a, da, h0rc=H0RC, ws=ws, tol=TOL)
        torch.cuda.synchronize()
        assert st["status"] >= 0
        if s:
            times.append(time.perf_counter() - t0)
            sts.append(st)
        a += da
    del pos, mom, phi, phin, ws
    torch.cuda.empty_cache()
    return {"ms_per_step": 1e3 * float(np.mean(times)), **pm_phases(sts),
            "config": "1024^3 mesh, 512^3 particles, L=1 Gpc/h, a=1, da=0.0063, tol=1e-8"}


SECTIONS = ("mixed", "cycle_types", "comparators", "other_solves", "vcycle_512", "pm_steps",
            "big", "cpu")


def note(what, t_start):
    """One progress line on stderr per finished part (the JSON line comes last)."""
    print("bench.py: %s done, %.1f s" % (what, time.perf_counter() - t_start), file=sys.stderr,
          flush=True)


def main():
    t_start = time.perf_counter()
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-big", action="store_true", help="skip the 1024^3 V-cycle timing")
    ap.add_argument("--main-only", action="store_true",
                    help="only the FP64 steps and the JSON line's core fields (for counter runs)")
    ap.add_argument("--sections", default=",".join(SECTIONS),
                    help="comma-separated sections after the FP64 steps (for profiler runs): "
                         + ", ".join(SECTIONS))
    args = ap.parse_args()
    sections = set(x for x in args.sections.split(",") if x)
    unknown = sections - set(SECTIONS)
    if unknown:
        ap.error("unknown sections: %s" % ", ".join(sorted(unknown)))
    if args.main_only:
        sections = set()
    if args.no_big:
        sections.discard("big")
    if args.no_cpu:
        sections.discard("cpu")
    if args.gpus != 1:
        print("bench.py measures one GPU only: the solver runs on a single MI355X "
              "(multi-GPU sharding is not built); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import inputs
    import paper_2110_00566_amd as mg

    dev = torch.device("cuda:0")
    pos_np = inputs.za_particles(N_PART, N_MESH, SEED)
    pos = torch.from_numpy(pos_np).to(dev)
    L = mg.lib()
    ws_pm = torch.empty(L.mg_pm_workspace_bytes(N_MESH), dtype=torch.uint8, device=dev)
    ws = mg.workspace(N_MESH, mg.MODEL_DGP, False, dev)
    delta = torch.empty((N_MESH,) * 3, dtype=torch.float64, device=dev)
    phi = torch.empty_like(delta)
    par = mg.dgp_params(A, OMEGA_M, H0RC)
    # the timed steps run the production solve; one extra untimed step with
    # profile = 1 (HIP events around every finest pass and level) gives the
    # pass duration and the per-level split
    opts = mg.make_opts(N_MESH, tol=TOL, max_cycles=60)
    opts_prof = mg.make_opts(N_MESH, tol=TOL, max_cycles=60, profile=True)
    import ctypes as C

    def step(o=opts):
        stream = mg._stream()
        mg._raise(L.mg_cic_delta(N_MESH, N_PART, mg._ptr(pos), mg._ptr(delta), mg._ptr(ws_pm),
                                 ws_pm.numel(), stream))
        phi.zero_()
        st = mg.Stats()
        mg._raise(L.mg_solve_dgp(C.byref(o), C.byref(par), mg._ptr(delta), mg._ptr(phi),
                                 mg._ptr(ws), ws.numel(), stream, C.byref(st)))
        return st

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    stats = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        stats.append(step())
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    prof = step(opts_prof)
    torch.cuda.synchronize()
    note("FP64 steps", t_start)

    cycles = [s.cycles for s in stats]
    assert all(s.status == 0 and s.eps <= TOL for s in stats), [s.status for s in stats]
    assert prof.status == 0 and prof.cycles == cycles[-1], (prof.status, prof.cycles)
    updates = sum(N_MESH ** 3 * 2 * c for c in cycles)
    ms_step = 1e3 * dt / args.steps
    solve_ms = 1e3 * float(np.mean([s.seconds for s in stats]))
    pass_ms = prof.pass_ms_avg
    achieved = PASS_BYTES_PER_CELL * N_MESH ** 3 / (pass_ms * 1e-3) / 1e9
    traffic = measured_traffic()
    out = {
        "metric": "cell-updates/s and time-to-residual 1e-8 per V-cycle at 512^3; % HBM peak",
        "value": updates / dt,
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "nDGP FAS V(1,1) solve, 512^3 mesh, CIC of 256^3 Zel'dovich "
                               "particles, L=512 Mpc/h, H0rc=1, a=1, phi0=0, tol=1e-8",
                   "n_mesh": N_MESH, "n_part": N_PART, "box_mpch": BOX, "h0rc": H0RC,
                   "tol": TOL, "precision": "fp64"},
        "cycles": int(round(float(np.mean(cycles)))),
        "time_to_tol_ms": solve_ms,
        "level_ms_per_cycle": [round(prof.level_ms[l] / prof.cycles, 4)
                               for l in range(mg.LEVELS) if prof.level_ms[l] > 0],
        "profiled_step": {"time_to_tol_ms": 1e3 * prof.seconds, "pass_count": prof.pass_count},
        "ms_per_vcycle": solve_ms / float(np.mean(cycles)),
        "roofline": {"bound": "hbm", "kernel": "k_pass_tiled<OP_DGP, double> (finest colour pass)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "pass_ms_avg": pass_ms,
                     "algorithmic_bytes_per_launch": PASS_BYTES_PER_CELL * N_MESH ** 3},
    }
    # the same step with the two mixed-precision solves, to the same FP64
    # tolerance: "mixed" (MG_MIXED: FP32 cycles to the FP32 floor, then FP64
    # cycles) and "mixed_dc" (MG_MIXED_DC: the same FP32 cycles, then defect
    # correction: FP64 residual, one FP32 correction cycle, FP64 accumulation)
    phi64 = phi.clone()
    for key, prec in (("mixed", mg.MG_MIXED), ("mixed_dc", mg.MG_MIXED_DC)):
        if "mixed" not in sections:
            break
        ws_mix = mg.workspace(N_MESH, mg.MODEL_DGP, False, dev, prec)
        opts_mix = mg.make_opts(N_MESH, tol=TOL, max_cycles=60, precision=prec)

        def step_mixed():
            stream = mg._stream()
            mg._raise(L.mg_cic_delta(N_MESH, N_PART, mg._ptr(pos), mg._ptr(delta),
                                     mg._ptr(ws_pm), ws_pm.numel(), stream))
            phi.zero_()
            st = mg.Stats()
            mg._raise(L.mg_solve_dgp(C.byref(opts_mix), C.byref(par), mg._ptr(delta),
                                     mg._ptr(phi), mg._ptr(ws_mix), ws_mix.numel(), stream,
                                     C.byref(st)))
            return st

        step_mixed()
        torch.cuda.synchronize()
        mstats = []
        t0 = time.perf_counter()
        for _ in range(args.steps):
            mstats.append(step_mixed())
        torch.cuda.synchronize()
        dtm = time.perf_counter() - t0
        assert all(s.status == 0 and s.eps <= TOL for s in mstats), [s.status for s in mstats]
        err = float((phi - phi64).abs().max() / phi64.abs().max())
        mix_solve_ms = 1e3 * float(np.mean([s.seconds for s in mstats]))
        out[key] = {"ms_per_step": 1e3 * dtm / args.steps, "time_to_tol_ms": mix_solve_ms,
                    "cycles": int(mstats[-1].cycles),
                    "cycles_fp32": int(mstats[-1].cycles_fp32),
                    "eps_fp32": float(mstats[-1].eps_fp32), "eps": float(mstats[-1].eps),
                    "speedup_time_to_tol_vs_fp64": solve_ms / mix_solve_ms,
                    "max_rel_diff_phi_vs_fp64": err}
        del ws_mix
        torch.cuda.empty_cache()
        note(key, t_start)
    if "cycle_types" in sections:
        out["cycle_types"] = cycle_types(mg, L, C, delta, ws, par, phi64)
        note("cycle_types", t_start)
    if "comparators" in sections:
        out["comparators"] = comparators(mg, L, C, delta, ws, par, phi64)
        note("comparators", t_start)
    if "other_solves" in sections:
        out["other_solves"] = other_solves(mg, delta, phi64)
        note("other_solves", t_start)
    del ws
    torch.cuda.empty_cache()
    if "vcycle_512" in sections:
        out["vcycle_512"] = vcycle_time(mg, L, C, delta)
        note("vcycle_512", t_start)
    if "pm_steps" in sections:
        out["pm_steps"] = pm_steps(mg, pos, dev)
        note("pm_steps", t_start)
    if "big" in sections:
        pos1024 = torch.from_numpy(inputs.za_particles(512, 1024, 5)).to(dev)
        out["vcycle_1024"] = vcycle_1024(mg, L, C, pos1024)
        note("vcycle_1024", t_start)
        out["pm_step_1024"] = pm_step_1024(mg, dev, pos1024)
        note("pm_step_1024", t_start)
        del pos1024
    if "cpu" in sections:
        out["cpu_baseline"] = cpu_baseline(pos_np)
        note("cpu_baseline", t_start)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
