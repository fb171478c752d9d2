#!/usr/bin/env python
"""Throughput of the convective right-hand side on one MI355X.

A step is one pass of the whole hot path over the state: the CFL time step
(reduced on the device), then one SSP-RK3 step, i.e. three times ghost fill,
primitives with the Newton temperature, the x/y/z Roe-characteristic
WENO5-LLF flux differences and the stage update.  The metric is interior
cell-RHS evaluations per second (3 per cell per step), FP64.  Beside it the
same line reports the FP32-mixed path (throughput and its state error
against FP64), the step with the positivity-preserving flux blend, the steps
with the ROE or GLF viscosity and with WENO-CU6, the
adjoint (VJP) throughput and adjoint/forward time ratios,
the roofline of the dominant kernel (timed live with HIP events on the stream
it runs on) and the CPU oracle on a bounded crop of the same state.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

WORKLOADS = {
    "nine_species_sbi_256": ("nine_species_sbi", dict(n=256)),
    "inert_sbi_128": ("inert_sbi", dict(n=128)),
    "two_bubble_sbi_512x256x256": ("two_bubble_sbi", dict()),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_case(name):
    from paper_2403_05910_amd import workloads as W
    fn, kw = WORKLOADS[name]
    return getattr(W, fn)(**kw)


def run_steps(ctx, U, dt_dev, steps, cfl):
    for _ in range(steps):
        ctx.rk3_step_cfl(U, cfl, dt_dev)


def timed_steps(torch, ctx, U, dt_dev, steps, cfl):
    ctx.timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    run_steps(ctx, U, dt_dev, steps, cfl)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.timing(False)
    return t1 - t0, ctx.timing_read()


PROFILE = os.path.join(ROOT, "profiles", "sweeps_nine_species_sbi_256.md")


def kernel_source_hash():
    """hash of the kernel sources and the ABI header (what the counters were taken on)"""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2403_05910_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hip", ".hpp")):
            with open(os.path.join(csrc, name), "rb") as f:
                h.update(name.encode() + b"\0" + f.read())
    with open(os.path.join(ROOT, "include", "xf.h"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel_class, precision):
    """HBM bytes per launch of a kernel class from the committed counter
    summary (FETCH_SIZE and WRITE_SIZE, calibrated against a device copy);
    None when the summary is missing or the kernels changed since"""
    try:
        with open(PROFILE) as f:
            text = f.read()
        blob = text.split("```json", 1)[1].split("```", 1)[0]
        data = json.loads(blob)
    except (OSError, IndexError, ValueError):
        return None
    if data.get("source_hash") != kernel_source_hash():
        return None
    row = data.get("traffic_bytes_per_launch", {}).get(precision, {}).get(kernel_class)
    return None if row is None else row["fetch"] + row["write"]


def roofline_of(kernels, case, precision):
    """dominant kernel class by total time; flops per launch from the
    algorithmic count; achieved = flops per launch / average launch time"""
    from paper_2403_05910_amd import perfmodel as pm
    ns = case.thermo.ns
    sweeps = {"sweep_x": 0, "sweep_y": 1, "sweep_z": 2}
    name = max(sweeps, key=lambda k: kernels[k][0])
    ms, launches = kernels[name]
    flops = pm.sweep_flops(ns, case.n, sweeps[name])
    avg_s = ms / launches / 1e3
    achieved = flops / avg_s / 1e12
    peak = pm.PEAK["fp32_vector_TFLOPs" if precision == "mixed" else "fp64_vector_TFLOPs"]
    return {"kernel": name, "bound": "alu", "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
            "frac": achieved / peak, "traffic": measured_traffic(name, precision), "traffic_unit": "bytes/launch",
            "avg_launch_ms": ms / launches, "launches": launches, "flops_per_launch": flops}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


def rollout_ratio(torch, xf, n=64, steps=64, every=8):
    """checkpointed RK3 rollout on the 5-species periodic mixture at n^3:
    wall time of the plain forward (steps RK3 steps), of the checkpointed
    forward and of its backward (segment recompute + RK3-step VJPs)"""
    from paper_2403_05910_amd import workloads as W
    case = W.periodic_mixture(n)
    ctx = xf.Context.from_case(case)
    U0 = ctx.state_from_numpy(case.U)
    ctx.fill_ghosts(U0)
    dt = 0.5 * ctx.cfl_dt(U0, 0.5).item()

    def plain():
        U = U0.clone()
        for _ in range(steps):
            ctx.rk3_step(U, dt)
        return U

    def clock(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return time.perf_counter() - t0, r

    plain()
    t_plain, _ = clock(plain)
    g = torch.randn(ctx.shape, dtype=torch.float64, device=U0.device)
    for rep in range(2):   # the first repetition warms up
        X = U0.clone().requires_grad_(True)
        t_fwd, Y = clock(lambda: xf.rollout(ctx, X, dt, steps, every))
        base = torch.cuda.memory_allocated()
        torch.cuda.reset_peak_memory_stats()
        t_bwd, _ = clock(lambda: Y.backward(g))
        peak = torch.cuda.max_memory_allocated() - base
        del X, Y
    formula = xf.rollout_memory_bytes(ctx, steps, every)
    ctx.close()
    return {"workload": f"periodic_mixture_{n}^3 (5 species)", "steps": steps, "ckpt_every": every,
            "ms_forward_plain": t_plain * 1e3, "ms_forward_checkpointed": t_fwd * 1e3,
            "ms_backward": t_bwd * 1e3, "backward_over_forward": t_bwd / t_plain,
            "extra_peak_bytes_during_backward": peak,
            "formula_bytes": formula}


def cpu_baseline(case, crop=96):
    """the oracle as it stands, on a crop^3 block of the same state (its
    halo taken from the neighbouring cells), straddling the shock and bubble"""
    import oracle as O
    t = case.thermo
    th = O.Thermo(t.W, t.a, t.T_lo, t.T_hi)
    nx, ny, nz = case.n
    x0 = max(0, min(nx - crop, int(0.15 * nx) - crop // 2))
    y0 = (ny - crop) // 2
    z0 = (nz - crop) // 2
    sub = case.U[:, z0:z0 + crop + 6, y0:y0 + crop + 6, x0:x0 + crop + 6]
    g = O.Grid(crop, crop, crop, *case.d, (0,) * 6)
    t0 = time.perf_counter()
    O.rhs(th, g, np.ascontiguousarray(sub))
    dt = time.perf_counter() - t0
    return {"value": crop ** 3 / dt, "unit": "cell-RHS evals/s", "cores": 1, "kind": "oracle",
            "sample": f"one FP64 RHS of a {crop}^3 crop (with its 3-cell halo) of the same state, "
                      f"x0={x0}, y0={y0}, z0={z0}; numpy, single thread, on {cpu_model()}",
            "seconds": dt}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="nine_species_sbi_256", choices=list(WORKLOADS))
    ap.add_argument("--cfl", type=float, default=0.5)
    ap.add_argument("--no-extras", action="store_true", help="FP64 step throughput only")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--calib", action="store_true",
                    help="first run a plain device copy of 1 GiB (counter calibration for rocprofv3 --pmc)")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU: the path is built and measured for one MI355X "
              f"(asked for --gpus {a.gpus}); see the design notes for how it would shard.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2403_05910_amd import perfmodel as pm
    from paper_2403_05910_amd import xf

    torch.cuda.set_device(0)
    if a.calib:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("[bench] calibration copy: 3 x 1 GiB read + 1 GiB written")
        del src, dst
    log(f"[bench] building workload {a.workload}")
    case = make_case(a.workload)
    cells = case.cells
    ns = case.thermo.ns
    log(f"[bench] {case.n} cells={cells} species={ns}")

    ctx = xf.Context.from_case(case, "fp64")
    U0 = ctx.state_from_numpy(case.U)
    U = U0.clone()
    dt_dev = torch.zeros(1, dtype=torch.float64, device=U.device)
    ctx.fill_ghosts(U)
    run_steps(ctx, U, dt_dev, a.warmup, a.cfl)
    torch.cuda.synchronize()
    log("[bench] fp64 warmup done")
    secs, kern = timed_steps(torch, ctx, U, dt_dev, a.steps, a.cfl)
    flags = ctx.status()
    value = 3 * cells * a.steps / secs
    log(f"[bench] fp64: {secs / a.steps * 1e3:.2f} ms/step, {value:.3e} cell-RHS/s, flags={flags}")
    roof = roofline_of(kern, case, "fp64")
    kernels_ms = {k: round(v[0] / max(v[1], 1), 4) for k, v in kern.items() if v[1]}

    out = {
        "metric": "cell-RHS evals/s (FP64)",
        "value": value,
        "unit": "cell-RHS evals/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": secs / a.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": a.workload, "grid": list(case.n), "species": ns, "cells": cells,
                   "step": "CFL dt on device + one SSP-RK3 step (3 RHS evaluations)"},
        "status_flags": flags,
        "kernel_avg_ms": kernels_ms,
        "roofline": roof,
        "hbm_frac_algorithmic": value / 3 * pm.rk3_step_bytes_per_cell(ns) / 1e9 / pm.PEAK["hbm_GBs"],
    }

    if not a.no_extras:
        # FP32-mixed path: same workload, same step
        ctxm = xf.Context.from_case(case, "mixed")
        Um = U0.clone()
        ctxm.fill_ghosts(Um)
        run_steps(ctxm, Um, dt_dev, a.warmup, a.cfl)
        torch.cuda.synchronize()
        secs_m, kern_m = timed_steps(torch, ctxm, Um, dt_dev, a.steps, a.cfl)
        vm = 3 * cells * a.steps / secs_m
        log(f"[bench] mixed: {secs_m / a.steps * 1e3:.2f} ms/step, {vm:.3e} cell-RHS/s")
        # accuracy of the mixed path: both paths advance the same state by
        # the same K steps at one fixed dt; then density, pressure (relative
        # to their largest value) and mass fractions (absolute) of the two
        # results, L_inf and mean over the interior.  (A residual compared
        # directly is ill-posed where a flux vanishes, e.g. a species at rest.)
        V = U0.clone()
        ctx.fill_ghosts(V)
        dt_fix = ctx.cfl_dt(V, a.cfl).item()
        Va, Vb = V.clone(), V.clone()
        for _ in range(a.steps):
            ctx.rk3_step(Va, dt_fix)
            ctxm.rk3_step(Vb, dt_fix)
        inner = ctx.interior[1:]
        pa, pb = ctx.primitives(Va)[(slice(None),) + inner], ctx.primitives(Vb)[(slice(None),) + inner]
        ra, rb_ = 1.0 / pa[3], 1.0 / pb[3]
        Ya, Yb = Va[ctx.interior][:ns] * pa[3], Vb[ctx.interior][:ns] * pb[3]

        def errs(x, y, scale):
            d = (x - y).abs()
            return {"linf": float(d.max() / scale), "mean": float(d.mean() / scale)}

        state_err = {"steps": a.steps, "dt": dt_fix, "vs": "FP64 path (itself within 1e-12 of the oracle)",
                     "rho_rel": errs(rb_, ra, ra.abs().max()), "p_rel": errs(pb[1], pa[1], pa[1].abs().max()),
                     "T_rel": errs(pb[0], pa[0], pa[0].abs().max()),
                     "Y_abs": [errs(Yb[k], Ya[k], 1.0) for k in range(ns)]}
        del Va, Vb, pa, pb, ra, rb_, Ya, Yb
        r64 = ctx.rhs(V)
        out["mixed"] = {"value": vm, "unit": "cell-RHS evals/s", "ms_per_step": secs_m / a.steps * 1e3,
                        "speedup_vs_fp64": vm / value,
                        "state_err_after_steps": state_err,
                        "roofline": roofline_of(kern_m, case, "mixed"),
                        "kernel_avg_ms": {k: round(v[0] / max(v[1], 1), 4) for k, v in kern_m.items() if v[1]},
                        "flags": ctxm.status()}
        ctxm.close()
        del Um
        # positivity-preserving blend (Sec. II.C.2): the same FP64 step with the
        # blend on; its cost and the status word it leaves
        ctxp = xf.Context.from_case(case, "fp64").set_positivity(True)
        Up = U0.clone()
        ctxp.fill_ghosts(Up)
        run_steps(ctxp, Up, dt_dev, a.warmup, a.cfl)
        torch.cuda.synchronize()
        secs_p, kern_p = timed_steps(torch, ctxp, Up, dt_dev, a.steps, a.cfl)
        out["positivity"] = {"value": 3 * cells * a.steps / secs_p, "unit": "cell-RHS evals/s",
                             "ms_per_step": secs_p / a.steps * 1e3, "overhead_vs_fp64": secs_p / secs - 1.0,
                             "status_flags": ctxp.status(), "status_flags_without": flags,
                             "kernel_avg_ms": {k: round(v[0] / max(v[1], 1), 4) for k, v in kern_p.items() if v[1]}}
        log(f"[bench] positivity: {secs_p / a.steps * 1e3:.2f} ms/step, flags {out['positivity']['status_flags']}")
        ctxp.close()
        del Up
        # the paper's other scheme options on the same FP64 step: ROE and GLF
        # artificial viscosity, WENO-CU6 and WENO7 reconstruction (WENO7 on the
        # same state laid out with four ghost layers)
        out["scheme_options"] = {}
        for label, visc, recon in (("ROE", "ROE", "WENO5"), ("GLF", "GLF", "WENO5"), ("CU6", "LLF", "CU6"),
                                   ("WENO7", "LLF", "WENO7"), ("viscous", "LLF", "WENO5"),
                                   ("reacting", "LLF", "WENO5")):
            if label == "reacting":
                # reaction source split off the step (Strang, 4 alpha-QSS
                # sub-steps per half step) with the seeded synthetic mechanism
                # and formation enthalpies; every rate is evaluated in every
                # cell whatever its temperature
                from paper_2403_05910_amd import workloads as W
                caser = W.rethermo(case, W.with_formation_enthalpies(case.thermo, 1))
                mech = W.synthetic_mechanism(list(1e3 * caser.thermo.W), caser.thermo, 0, 12)
                ctxo = xf.Context.from_case(caser, "fp64").set_reactions(mech, 4, "strang")
                Uo = ctxo.state_from_numpy(caser.U)
                del caser
            elif label == "viscous":
                # Navier-Stokes step: the viscous and diffusive fluxes of Eq. 2-6
                # with seeded gas-like transport tables, all terms
                from paper_2403_05910_amd import workloads as W
                ctxo = xf.Context.from_case(case, "fp64").set_viscous(W.sampled_transport(ns, 0))
                Uo = U0.clone()
            elif recon == "WENO7":
                case4 = case.with_ghosts(4)
                ctxo = xf.Context.from_case(case4, "fp64").set_reconstruction(recon)
                Uo = ctxo.state_from_numpy(case4.U)
                del case4
            else:
                ctxo = xf.Context.from_case(case, "fp64").set_dissipation(visc).set_reconstruction(recon)
                Uo = U0.clone()
            ctxo.fill_ghosts(Uo)
            run_steps(ctxo, Uo, dt_dev, 1, a.cfl)
            torch.cuda.synchronize()
            secs_o, kern_o = timed_steps(torch, ctxo, Uo, dt_dev, max(2, a.steps // 2), a.cfl)
            n_o = max(2, a.steps // 2)
            out["scheme_options"][label] = {
                "ms_per_step": secs_o / n_o * 1e3, "value": 3 * cells * n_o / secs_o, "status_flags": ctxo.status(),
                "kernel_avg_ms": {k: round(v[0] / max(v[1], 1), 4) for k, v in kern_o.items() if v[1]}}
            log(f"[bench] {label}: {secs_o / n_o * 1e3:.2f} ms/step")
            ctxo.close()
            del Uo
        # adjoint: one RHS VJP per evaluation, against one forward RHS
        rb = torch.randn_like(r64)
        Ub = torch.zeros_like(r64)
        for _ in range(2):
            ctx.rhs_vjp(V, rb, Ub)
            ctx.rhs(V, out=r64)
        reps = max(3, a.steps // 2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            ctx.rhs(V, out=r64)
        torch.cuda.synchronize()
        t_fwd = (time.perf_counter() - t0) / reps
        ctx.timing(True)
        t0 = time.perf_counter()
        for _ in range(reps):
            ctx.rhs_vjp(V, rb, Ub)
        torch.cuda.synchronize()
        t_vjp = (time.perf_counter() - t0) / reps
        ctx.timing(False)
        kv = ctx.timing_read()
        out["adjoint"] = {"value": cells / t_vjp, "unit": "cell adjoint-evals/s", "ms_per_vjp": t_vjp * 1e3,
                          "ms_per_rhs": t_fwd * 1e3, "adjoint_over_forward": t_vjp / t_fwd,
                          "kernel_avg_ms": {k: round(v[0] / max(v[1], 1), 4) for k, v in kv.items() if v[1]}}
        log(f"[bench] vjp {t_vjp * 1e3:.2f} ms vs rhs {t_fwd * 1e3:.2f} ms")
        # checkpointed RK3 adjoint step vs forward step
        try:
            lam = torch.randn_like(r64)
            ctx.rk3_step_vjp(V, 1e-9, lam)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(2):
                ctx.rk3_step_vjp(V, 1e-9, lam)
            torch.cuda.synchronize()
            t_rk3v = (time.perf_counter() - t0) / 2
            out["adjoint"]["ms_per_rk3_step_vjp"] = t_rk3v * 1e3
            out["adjoint"]["rk3_adjoint_over_forward_step"] = t_rk3v / (secs / a.steps)
        except Exception as e:  # workspace too large for the device
            out["adjoint"]["rk3_step_vjp_error"] = str(e)
        out["adjoint"]["rollout"] = rollout_ratio(torch, xf)
        log(f"[bench] rollout backward/forward {out['adjoint']['rollout']['backward_over_forward']:.2f}")
    if not a.no_cpu:
        log("[bench] cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(case)
        out["cpu_baseline"]["gpu_over_cpu"] = value / out["cpu_baseline"]["value"]
    ctx.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
