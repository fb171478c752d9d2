#!/usr/bin/env python
"""Throughput of the convective right-hand side on one MI355X.

A step is one pass of the whole hot path over the state: the CFL time step
(reduced on the device), then one SSP-RK3 step, i.e. three times ghost fill,
primitives with the Newton temperature, the x/y/z Roe-characteristic
WENO5-LLF flux differences and the stage update.  The metric is interior
cell-RHS evaluations per second (3 per cell per step), FP64, on the
nine-species shock-bubble at 256^3; the K timed steps run back to back with
no per-kernel events, and the per-step median comes from a second, synced
pass.  Beside it the same line reports:

* the FP32-mixed path (throughput and its state error against FP64);
* the adjoint: RHS VJP throughput, adjoint/forward time ratios, the
  checkpointed rollout of the 64^3 five-species mixture;
* the roofline of the dominant forward kernel and of the adjoint, from a
  separate pass with HIP events on the launch stream;
* the other workloads at their stated sizes: the 1D two-gas wave to t = 1
  (error against exact translation), the inert shock-bubble at 128^3
  (one RHS and 20 steps) and the two-bubble 512 x 256 x 256 case (32 FP64
  and 32 mixed steps and the checkpointed adjoint over the same 32 steps,
  with its device memory);
* the scheme options (positivity blend, ROE, GLF, WENO-CU6, WENO7,
  viscous fluxes, reactions) on the headline state;
* the CPU oracle on bounded samples of three workloads, one thread and all
  the host cores this process may use.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--quick]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "cell-RHS evals/s, FP64 vs FP32-mixed at stated error; adjoint/forward time"
PROFILE = os.path.join(ROOT, "profiles", "sweeps_nine_species_sbi_256.md")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernels_ms(kern):
    return {k: round(v[0] / max(v[1], 1), 4) for k, v in kern.items() if v[1]}


# ---------------------------------------------------------------------------
# timing helpers
# ---------------------------------------------------------------------------
def block_time(torch, fn, n):
    """wall time of n back-to-back calls, bracketed by device syncs"""
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(n):
        fn()
    torch.cuda.synchronize()
    return time.perf_counter() - t0


def per_call_times(torch, fn, n):
    """n synced calls: sorted wall times"""
    ts = []
    for _ in range(n):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
    return sorted(ts)


def median(ts):
    return float(np.median(ts))


def kernel_pass(torch, ctx, fn, n):
    """per-kernel average times from HIP events recorded around every launch
    on the launch stream (a separate pass: the events are not free)"""
    ctx.timing(True)
    torch.cuda.synchronize()
    for _ in range(n):
        fn()
    torch.cuda.synchronize()
    ctx.timing(False)
    return ctx.timing_read()


# ---------------------------------------------------------------------------
# roofline
# ---------------------------------------------------------------------------
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


def profile_data():
    try:
        with open(PROFILE) as f:
            text = f.read()
        blob = text.split("```json", 1)[1].split("```", 1)[0]
        data = json.loads(blob)
    except (OSError, IndexError, ValueError):
        return None
    return data if data.get("source_hash") == kernel_source_hash() else None


def measured_counters(kernel_class, precision, workload):
    """counters per launch of a kernel class from the committed summary
    (calibrated FETCH_SIZE + WRITE_SIZE bytes, VALU instructions, executed
    flops); None when the summary is missing, was taken on another workload,
    or the kernels changed since"""
    data = profile_data()
    if data is None or data.get("workload") != workload:
        return None
    return data.get("traffic_bytes_per_launch", {}).get(precision, {}).get(kernel_class)


def measured_traffic(kernel_class, precision, workload):
    row = measured_counters(kernel_class, precision, workload)
    return None if row is None else row["fetch"] + row["write"]


def roofline_of(kernels, case, precision, workload):
    """dominant sweep kernel by total time; flops per launch from the
    algorithmic count; achieved = flops per launch / average launch time.
    The path's arithmetic intensity (about 49 flop per algorithmic byte at
    nine species) is five times the FP64 ridge, so the vector-ALU roofline
    binds; the HBM fraction of the measured traffic goes beside it."""
    from paper_2403_05910_amd import perfmodel as pm
    ns = case.thermo.ns
    sweeps = {"sweep_x": 0, "sweep_y": 1, "sweep_z": 2}
    name = max(sweeps, key=lambda k: kernels[k][0])
    ms, launches = kernels[name]
    avg_s = ms / launches / 1e3
    # the mixed x sweep of an RK3 step (no viscous terms or blend) also
    # finishes the stage
    fused = precision == "mixed" and name == "sweep_x"
    flops = pm.sweep_flops(ns, case.n, sweeps[name]) + (pm.stage_flops(ns, case.n) if fused else 0)
    achieved = flops / avg_s / 1e12
    peak = pm.PEAK["fp32_vector_TFLOPs" if precision == "mixed" else "fp64_vector_TFLOPs"]
    traffic = measured_traffic(name, precision, workload)
    alg_bytes = pm.sweep_bytes(ns, case.n, sweeps[name], first=True, precision=precision, fused_stage=fused)
    out = {"kernel": name + (" (with the stage)" if fused else ""), "bound": "alu", "achieved": achieved,
           "peak": peak, "unit": "TFLOP/s",
           "frac": achieved / peak, "traffic": traffic, "traffic_unit": "bytes/launch",
           "avg_launch_ms": ms / launches, "launches": launches, "flops_per_launch": flops,
           "algorithmic_bytes_per_launch": alg_bytes,
           "hbm_frac_algorithmic": alg_bytes / avg_s / 1e9 / pm.PEAK["hbm_GBs"]}
    if traffic is not None:
        out["hbm_frac_measured"] = traffic / avg_s / 1e9 / pm.PEAK["hbm_GBs"]
    cnt = measured_counters(name, precision, workload)
    if cnt is not None:
        # what limits the kernel: neither roof is reached, so report the VALU
        # issue fraction (wave instructions x 4 cycles over the 1024 SIMDs'
        # cycles of the launch) beside the executed-flop rate
        out["executed_flops_per_launch"] = cnt["executed_flops"]
        out["achieved_executed"] = cnt["executed_flops"] / avg_s / 1e12
        out["valu_issue_frac"] = cnt["valu_instr"] * 4 / (pm.SIMDS * pm.CLOCK_HZ * avg_s)
        out["limiter"] = "latency (VALU issue {:.0%}, measured HBM {:.0%} of peak)".format(
            out["valu_issue_frac"], out.get("hbm_frac_measured", 0.0))
    return out


def adjoint_roofline(kv, case, precision):
    """roofline of the dominant face-VJP kernel class: FP64 (FP32) operations
    per face of the implemented adjoint (counted with rocprofv3's per-type
    VALU counters, see perfmodel.vjp_face_flops) over its launch time, and
    the HBM fraction of its algorithmic bytes"""
    from paper_2403_05910_amd import perfmodel as pm
    ns = case.thermo.ns
    dirs = {"vjp_x": 0, "vjp_y": 1, "vjp_z": 2}
    name = max(dirs, key=lambda k: kv[k][0])
    ms, launches = kv[name]
    d = dirs[name]
    per_dir_s = ms / launches / 1e3   # one 'launch' of the timing table = the direction's launch groups
    flops = pm.vjp_sweep_flops(ns, case.n, d, precision)
    peak = pm.PEAK["fp32_vector_TFLOPs" if precision == "mixed" else "fp64_vector_TFLOPs"]
    alg = pm.vjp_sweep_bytes(ns, case.n, d)
    out = {"kernel": name, "bound": "alu", "unit": "TFLOP/s", "peak": peak, "ms_per_direction": ms / launches,
           "flops_per_direction": flops, "algorithmic_bytes_per_direction": alg,
           "hbm_frac_algorithmic": alg / per_dir_s / 1e9 / pm.PEAK["hbm_GBs"]}
    if flops is not None:
        out["achieved"] = flops / per_dir_s / 1e12
        out["frac"] = out["achieved"] / peak
    return out


# ---------------------------------------------------------------------------
# CPU oracle baseline
# ---------------------------------------------------------------------------
def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.lower().startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown CPU"


def usable_cores():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    for var in ("OMP_NUM_THREADS", "MAX_JOBS"):
        v = os.environ.get(var, "")
        if v.isdigit() and int(v) > 0:
            n = min(n, int(v))
    return max(1, n)


def _oracle_block(args):
    """one RHS of the oracle on a block with its 3-cell halo; returns seconds"""
    import oracle as O
    W_, a_, T_lo, T_hi, n, d, U = args
    th = O.Thermo(W_, a_, T_lo, T_hi)
    g = O.Grid(n[0], n[1], n[2], *d, (0,) * 6)
    t0 = time.perf_counter()
    O.rhs(th, g, U)
    return time.perf_counter() - t0


def crop(case, n, x0=None):
    """an n^3 block of the case's padded state with its 3-cell halo taken
    from the neighbouring cells (straddling the shock and the bubble)"""
    nx, ny, nz = case.n
    n = min(n, nx, ny, nz)
    if x0 is None:
        x0 = max(0, min(nx - n, int(0.15 * nx) - n // 2))
    y0, z0 = (ny - n) // 2, (nz - n) // 2
    return np.ascontiguousarray(case.U[:, z0:z0 + n + 6, y0:y0 + n + 6, x0:x0 + n + 6]), n, (x0, y0, z0)


def cpu_baseline(cases, quick=False):
    """the oracle as it stands: one thread on an n^3 crop of each workload,
    and all usable host cores on a larger crop split into z-slabs (each slab
    an independent oracle RHS with its own halo, in separate processes)"""
    import multiprocessing as mp
    cores = usable_cores()
    res = {"kind": "oracle", "cpu": cpu_model(), "cores_available": cores, "workloads": {}}
    sizes = {"nine_species_sbi_256": (48 if quick else 64, 64 if quick else 128),
             "inert_sbi_128": (48 if quick else 64, 64 if quick else 128),
             "periodic_mixture_64": (48 if quick else 64, 64)}
    ctx = mp.get_context("spawn")
    with ctx.Pool(cores) as pool:
        for name, case in cases.items():
            n1, nall = sizes[name]
            t = case.thermo
            U1, n1, org = crop(case, n1)
            sec1 = _oracle_block((t.W, t.a, t.T_lo, t.T_hi, (n1, n1, n1), case.d, U1))
            Ua, na, orga = crop(case, nall)
            slabs = []
            nz_s = max(1, na // cores)
            z = 0
            while z < na:
                h = min(nz_s, na - z)
                slabs.append((t.W, t.a, t.T_lo, t.T_hi, (na, na, h), case.d,
                              np.ascontiguousarray(Ua[:, z:z + h + 6])))
                z += h
            t0 = time.perf_counter()
            pool.map(_oracle_block, slabs)
            secs = time.perf_counter() - t0
            res["workloads"][name] = {
                "single_thread": {"value": n1 ** 3 / sec1, "unit": "cell-RHS evals/s", "seconds": sec1,
                                  "sample": f"one FP64 RHS of a {n1}^3 crop at {org}"},
                "all_cores": {"value": na ** 3 / secs, "unit": "cell-RHS evals/s", "seconds": secs,
                              "cores": min(cores, len(slabs)),
                              "sample": f"one FP64 RHS of a {na}^3 crop at {orga} in {len(slabs)} z-slabs"}}
            log(f"[bench] cpu {name}: 1 thread {n1 ** 3 / sec1:.3e}, "
                f"{min(cores, len(slabs))} cores {na ** 3 / secs:.3e} cell-RHS/s")
    return res


# ---------------------------------------------------------------------------
# GPU parts
# ---------------------------------------------------------------------------
def fp64_headline(torch, xf, case, a):
    ctx = xf.Context.from_case(case, "fp64")
    U0 = ctx.state_from_numpy(case.U)
    U = U0.clone()
    dt_dev = torch.zeros(1, dtype=torch.float64, device=U.device)
    ctx.fill_ghosts(U)
    step = lambda: ctx.rk3_step_cfl(U, a.cfl, dt_dev)
    for _ in range(a.warmup):
        step()
    secs = block_time(torch, step, a.steps)
    flags = ctx.status()
    ts = per_call_times(torch, step, a.steps)
    kern = kernel_pass(torch, ctx, step, 3)
    return ctx, U0, secs, ts, flags, kern


def mixed_part(torch, xf, case, ctx64, U0, a, secs64):
    ns = case.thermo.ns
    cells = case.cells
    ctxm = xf.Context.from_case(case, "mixed")
    Um = U0.clone()
    dt_dev = torch.zeros(1, dtype=torch.float64, device=Um.device)
    ctxm.fill_ghosts(Um)
    step = lambda: ctxm.rk3_step_cfl(Um, a.cfl, dt_dev)
    for _ in range(a.warmup):
        step()
    secs = block_time(torch, step, a.steps)
    ts = per_call_times(torch, step, a.steps)
    kern = kernel_pass(torch, ctxm, step, 3)
    vm = 3 * cells * a.steps / secs
    # accuracy: both paths advance the same state by the same K steps at one
    # fixed dt; density, pressure, temperature (relative to their largest
    # value) and mass fractions (absolute), L_inf and mean over the interior
    V = U0.clone()
    ctx64.fill_ghosts(V)
    dt_fix = ctx64.cfl_dt(V, a.cfl).item()
    Va, Vb = V.clone(), V.clone()
    for _ in range(a.steps):
        ctx64.rk3_step(Va, dt_fix)
        ctxm.rk3_step(Vb, dt_fix)
    inner = ctx64.interior[1:]
    pa, pb = ctx64.primitives(Va)[(slice(None),) + inner], ctx64.primitives(Vb)[(slice(None),) + inner]
    ra, rb_ = 1.0 / pa[3], 1.0 / pb[3]
    Ya, Yb = Va[ctx64.interior][:ns] * pa[3], Vb[ctx64.interior][:ns] * pb[3]

    def errs(x, y, scale):
        d = (x - y).abs()
        return {"linf": float(d.max() / scale), "l1": float(d.mean() / scale)}

    state_err = {"steps": a.steps, "dt": dt_fix, "vs": "FP64 path (itself within 1e-12 of the oracle)",
                 "rho_rel": errs(rb_, ra, ra.abs().max()), "p_rel": errs(pb[1], pa[1], pa[1].abs().max()),
                 "T_rel": errs(pb[0], pa[0], pa[0].abs().max()),
                 "Y_abs": [errs(Yb[k], Ya[k], 1.0) for k in range(ns)]}
    out = {"value": vm, "unit": "cell-RHS evals/s", "ms_per_step": secs / a.steps * 1e3,
           "ms_per_step_median": median(ts) * 1e3, "speedup_vs_fp64": secs64 / secs,
           "state_err_after_steps": state_err, "roofline": roofline_of(kern, case, "mixed", "nine_species_sbi_256"),
           "kernel_avg_ms": kernels_ms(kern), "status_flags": ctxm.status()}
    return ctxm, out


def adjoint_part(torch, xf, case, ctx, ctxm, U0, a, secs64):
    cells = case.cells
    res = {}
    for label, c in (("fp64", ctx), ("mixed", ctxm)):
        V = U0.clone()
        c.fill_ghosts(V)
        r = c.rhs(V)
        rb = torch.randn_like(r)
        Ub = torch.zeros_like(r)
        fwd = lambda: c.rhs(V, out=r)
        bwd = lambda: c.rhs_vjp(V, rb, Ub)
        for _ in range(2):
            fwd()
            bwd()
        tf = per_call_times(torch, fwd, a.reps)
        tb = per_call_times(torch, bwd, a.reps)
        kv = kernel_pass(torch, c, bwd, 3)
        res[label] = {"value": cells / median(tb), "unit": "cell adjoint-evals/s", "ms_per_vjp": median(tb) * 1e3,
                      "ms_per_rhs": median(tf) * 1e3, "adjoint_over_forward": median(tb) / median(tf),
                      "kernel_avg_ms": kernels_ms(kv), "roofline": adjoint_roofline(kv, case, label)}
        log(f"[bench] vjp {label}: {median(tb) * 1e3:.2f} ms vs rhs {median(tf) * 1e3:.2f} ms")
        if label == "fp64":
            lam = torch.randn_like(r)
            c.rk3_step_vjp(V, 1e-9, lam)
            tr = per_call_times(torch, lambda: c.rk3_step_vjp(V, 1e-9, lam), 3)
            res[label]["ms_per_rk3_step_vjp"] = median(tr) * 1e3
            res[label]["rk3_adjoint_over_forward_step"] = median(tr) / (secs64 / a.steps)
        del V, r, rb, Ub
    return res


def rollout_part(torch, xf, case, steps, every, precisions=("fp64",)):
    """checkpointed RK3 rollout at fixed dt (CFL 0.5 of the initial state):
    wall time of the plain forward, of the checkpointed forward and of its
    backward, and the device memory the backward adds"""
    out = {"workload": case.name, "grid": list(case.n), "species": case.thermo.ns, "steps": steps,
           "ckpt_every": every}
    for prec in precisions:
        ctx = xf.Context.from_case(case, prec)
        U0 = ctx.state_from_numpy(case.U)
        ctx.fill_ghosts(U0)
        dt = ctx.cfl_dt(U0, 0.5).item()

        def plain():
            U = U0.clone()
            for _ in range(steps):
                ctx.rk3_step(U, dt)
            return U

        plain()
        t_plain = block_time(torch, plain, 1)
        g = torch.randn(ctx.shape, dtype=torch.float64, device=U0.device)
        for rep in range(2 if case.cells < 4e6 else 1):   # the first repetition warms up the small case
            X = U0.clone().requires_grad_(True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            Y = xf.rollout(ctx, X, dt, steps, every)
            torch.cuda.synchronize()
            t_fwd = time.perf_counter() - t0
            base = torch.cuda.memory_allocated()
            torch.cuda.reset_peak_memory_stats()
            t0 = time.perf_counter()
            Y.backward(g)
            torch.cuda.synchronize()
            t_bwd = time.perf_counter() - t0
            peak_total = torch.cuda.max_memory_allocated()
            peak = peak_total - base
            del X, Y
        S = int(np.prod(ctx.shape)) * 8
        C = (steps + every - 1) // every
        out[prec] = {"dt": dt, "ms_forward_plain": t_plain * 1e3, "ms_forward_checkpointed": t_fwd * 1e3,
                     "ms_backward": t_bwd * 1e3, "backward_over_forward": t_bwd / t_plain,
                     "extra_peak_bytes_during_backward": peak, "peak_device_bytes": peak_total,
                     "state_bytes_S": S, "checkpoints_C": C,
                     "formula_C_plus_k_plus_5_S_bytes": (C + every + 5) * S,
                     "formula_bytes_with_workspaces": xf.rollout_memory_bytes(ctx, steps, every),
                     "hbm_bytes": 288e9, "status_flags": ctx.status()}
        log(f"[bench] rollout {case.name} {prec}: fwd {t_plain * 1e3:.1f} ms, bwd {t_bwd * 1e3:.1f} ms, "
            f"peak {peak_total / 1e9:.1f} GB")
        ctx.close()
        del U0, g
        torch.cuda.empty_cache()
    return out


def wave_part(torch, xf):
    """1D two-gas wave, 200 cells, SSP-RK3 at CFL 0.5 to t = 1 (one period,
    the last step clipped): L1 error of density, pressure and Y1 against
    exact translation (the initial state)"""
    from paper_2403_05910_amd import workloads as W
    case = W.wave_1d(200)
    ctx = xf.Context.from_case(case, "fp64")
    U = ctx.state_from_numpy(case.U)
    ctx.fill_ghosts(U)
    U0 = U.clone()
    t, steps = 0.0, 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while t < 1.0 - 1e-14:
        dt = min(ctx.cfl_dt(U, 0.5).item(), 1.0 - t)
        ctx.rk3_step(U, dt)
        t += dt
        steps += 1
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    inner = ctx.interior[1:]
    p0, p1 = ctx.primitives(U0)[(slice(None),) + inner], ctx.primitives(U)[(slice(None),) + inner]
    r0, r1 = 1.0 / p0[3], 1.0 / p1[3]
    Y0, Y1 = U0[ctx.interior][0] * p0[3], U[ctx.interior][0] * p1[3]
    out = {"workload": "wave_1d_200", "t_end": t, "steps": steps, "seconds": secs,
           "L1_rho": float((r1 - r0).abs().mean()), "L1_p": float((p1[1] - p0[1]).abs().mean()),
           "L1_Y1": float((Y1 - Y0).abs().mean()), "status_flags": ctx.status()}
    ctx.close()
    return out


def inert_part(torch, xf, case, a):
    """inert shock-bubble 128^3: one RHS (median of 20) and 20 RK3 steps, FP64"""
    ctx = xf.Context.from_case(case, "fp64")
    U = ctx.state_from_numpy(case.U)
    ctx.fill_ghosts(U)
    r = ctx.rhs(U)
    trhs = per_call_times(torch, lambda: ctx.rhs(U, out=r), 20)
    dt_dev = torch.zeros(1, dtype=torch.float64, device=U.device)
    step = lambda: ctx.rk3_step_cfl(U, a.cfl, dt_dev)
    step()
    secs = block_time(torch, step, 20)
    kern = kernel_pass(torch, ctx, step, 3)
    out = {"workload": "inert_sbi_128", "grid": list(case.n), "species": case.thermo.ns,
           "rhs_ms_median": median(trhs) * 1e3, "rhs_value": case.cells / median(trhs),
           "steps": 20, "ms_per_step": secs / 20 * 1e3, "value": 3 * case.cells * 20 / secs,
           "unit": "cell-RHS evals/s", "roofline": roofline_of(kern, case, "fp64", "inert_sbi_128"), "status_flags": ctx.status()}
    ctx.close()
    return out


def large_part(torch, xf, case, a):
    """two-bubble 512 x 256 x 256: 32 FP64 and 32 mixed steps, and the
    checkpointed adjoint of the same 32 steps with its device memory"""
    out = {"workload": "two_bubble_sbi_512x256x256", "grid": list(case.n), "species": case.thermo.ns}
    dt_dev = torch.zeros(1, dtype=torch.float64, device="cuda")
    for prec in ("fp64", "mixed"):
        ctx = xf.Context.from_case(case, prec)
        U = ctx.state_from_numpy(case.U)
        ctx.fill_ghosts(U)
        step = lambda: ctx.rk3_step_cfl(U, a.cfl, dt_dev)
        step()
        secs = block_time(torch, step, 32)
        kern = kernel_pass(torch, ctx, step, 2)
        out[prec] = {"steps": 32, "ms_per_step": secs / 32 * 1e3, "value": 3 * case.cells * 32 / secs,
                     "unit": "cell-RHS evals/s", "roofline": roofline_of(kern, case, prec, "two_bubble_sbi_512x256x256"),
                     "status_flags": ctx.status()}
        log(f"[bench] large {prec}: {secs / 32 * 1e3:.2f} ms/step")
        ctx.close()
        del U
        torch.cuda.empty_cache()
    out["adjoint_rollout"] = rollout_part(torch, xf, case, 32, 8, ("fp64", "mixed"))
    return out


def options_part(torch, xf, case, U0, a):
    """the paper's other scheme options on the same FP64 step"""
    from paper_2403_05910_amd import workloads as W
    ns = case.thermo.ns
    cells = case.cells
    dt_dev = torch.zeros(1, dtype=torch.float64, device=U0.device)
    res = {}
    labels = ("positivity", "ROE", "GLF", "CU6", "WENO7", "viscous", "reacting")
    if a.options:
        labels = tuple(l for l in labels if l in a.options.split(","))
    for label in labels:
        if label == "reacting":
            # reaction source split off the step (Strang, 4 alpha-QSS sub-steps
            # per half step) with the seeded synthetic mechanism and formation
            # enthalpies; every rate is evaluated in every cell
            caser = W.rethermo(case, W.with_formation_enthalpies(case.thermo, 1))
            mech = W.synthetic_mechanism(list(1e3 * caser.thermo.W), caser.thermo, 0, 12)
            ctxo = xf.Context.from_case(caser, "fp64").set_reactions(mech, 4, "strang")
            Uo = ctxo.state_from_numpy(caser.U)
            del caser
        elif label == "viscous":
            ctxo = xf.Context.from_case(case, "fp64").set_viscous(W.sampled_transport(ns, 0))
            Uo = U0.clone()
        elif label == "WENO7":
            case4 = case.with_ghosts(4)
            ctxo = xf.Context.from_case(case4, "fp64").set_reconstruction("WENO7")
            Uo = ctxo.state_from_numpy(case4.U)
            del case4
        elif label == "positivity":
            ctxo = xf.Context.from_case(case, "fp64").set_positivity(True)
            Uo = U0.clone()
        elif label == "CU6":
            ctxo = xf.Context.from_case(case, "fp64").set_reconstruction("CU6")
            Uo = U0.clone()
        else:
            ctxo = xf.Context.from_case(case, "fp64").set_dissipation(label)
            Uo = U0.clone()
        ctxo.fill_ghosts(Uo)
        step = lambda: ctxo.rk3_step_cfl(Uo, a.cfl, dt_dev)
        step()
        n_o = max(2, a.steps // 4)
        secs = block_time(torch, step, n_o)
        kern = kernel_pass(torch, ctxo, step, 1)
        res[label] = {"ms_per_step": secs / n_o * 1e3, "value": 3 * cells * n_o / secs,
                      "status_flags": ctxo.status(), "kernel_avg_ms": kernels_ms(kern)}
        log(f"[bench] {label}: {secs / n_o * 1e3:.2f} ms/step")
        ctxo.close()
        del Uo
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cfl", type=float, default=0.5)
    ap.add_argument("--no-extras", action="store_true", help="FP64 headline only")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-large", action="store_true", help="skip the 512 x 256 x 256 workload")
    ap.add_argument("--no-options", action="store_true", help="skip the scheme options")
    ap.add_argument("--options", default="", help="comma-separated subset of the scheme options to run "
                    "(positivity, ROE, GLF, CU6, WENO7, viscous, reacting); default all")
    ap.add_argument("--no-configs", action="store_true", help="skip the other workloads and the rollouts")
    ap.add_argument("--reps", type=int, default=20, help="repetitions of the RHS and VJP timings")
    ap.add_argument("--quick", action="store_true", help="smaller CPU samples")
    ap.add_argument("--calib", action="store_true",
                    help="first run a plain device copy of 1 GiB (counter calibration for rocprofv3 --pmc)")
    a = ap.parse_args()
    if a.gpus != 1:
        print(f"bench.py runs on one GPU: the path is built and measured for one MI355X "
              f"(asked for --gpus {a.gpus}); see the design notes for how it would shard.", file=sys.stderr)
        sys.exit(2)
    from paper_2403_05910_amd import workloads as W

    cases = {}
    log("[bench] building workloads")
    cases["nine_species_sbi_256"] = W.nine_species_sbi(n=256)
    case = cases["nine_species_sbi_256"]
    if not a.no_extras and not (a.no_configs and a.no_cpu):
        cases["inert_sbi_128"] = W.inert_sbi(128)
        cases["periodic_mixture_64"] = W.periodic_mixture(64)
    cpu = None
    if not a.no_cpu:
        # before the GPU is touched; the workers are separate processes
        log("[bench] cpu baseline (oracle)")
        cpu = cpu_baseline({k: v for k, v in cases.items()}, a.quick)

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
    cells = case.cells
    ns = case.thermo.ns
    ctx, U0, secs, ts, flags, kern = fp64_headline(torch, xf, case, a)
    value = 3 * cells * a.steps / secs
    log(f"[bench] fp64: {secs / a.steps * 1e3:.2f} ms/step (median {median(ts) * 1e3:.2f}), "
        f"{value:.3e} cell-RHS/s, flags={flags}")
    roof = roofline_of(kern, case, "fp64", "nine_species_sbi_256")
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "cell-RHS evals/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": secs / a.steps * 1e3,
        "ms_per_step_median": median(ts) * 1e3,
        "ms_per_step_min": ts[0] * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "nine_species_sbi_256", "grid": list(case.n), "species": ns, "cells": cells,
                   "step": "CFL dt on device + one SSP-RK3 step (3 RHS evaluations)"},
        "status_flags": flags,
        "kernel_avg_ms": kernels_ms(kern),
        "roofline": roof,
        "hbm_frac_algorithmic": value / 3 * pm.rk3_step_bytes_per_cell(ns) / 1e9 / pm.PEAK["hbm_GBs"],
    }
    if not a.no_extras:
        ctxm, out["mixed"] = mixed_part(torch, xf, case, ctx, U0, a, secs)
        log(f"[bench] mixed: {out['mixed']['ms_per_step']:.2f} ms/step")
        out["adjoint"] = adjoint_part(torch, xf, case, ctx, ctxm, U0, a, secs)
        ctxm.close()
        if not a.no_configs:
            out["adjoint"]["rollout"] = rollout_part(torch, xf, cases["periodic_mixture_64"], 64, 8,
                                                     ("fp64", "mixed"))
        if not a.no_options:
            out["scheme_options"] = options_part(torch, xf, case, U0, a)
        ctx.close()
        del U0
        torch.cuda.empty_cache()
        if not a.no_configs:
            out["configs"] = {"wave_1d_200": wave_part(torch, xf),
                              "inert_sbi_128": inert_part(torch, xf, cases["inert_sbi_128"], a)}
            log(f"[bench] wave L1(rho) {out['configs']['wave_1d_200']['L1_rho']:.3e}, "
                f"inert {out['configs']['inert_sbi_128']['ms_per_step']:.2f} ms/step")
        if not a.no_large and not a.no_configs:
            del cases
            log("[bench] building the 512 x 256 x 256 workload")
            large = W.two_bubble_sbi()
            out["configs"]["two_bubble_sbi_512x256x256"] = large_part(torch, xf, large, a)
            del large
    else:
        ctx.close()
    if cpu is not None:
        c3 = cpu["workloads"]["nine_species_sbi_256"]
        best = c3["all_cores"] if c3["all_cores"]["value"] > c3["single_thread"]["value"] else c3["single_thread"]
        out["cpu_baseline"] = {"value": best["value"], "unit": "cell-RHS evals/s",
                               "cores": best.get("cores", 1), "kind": "oracle",
                               "sample": best["sample"] + f" of the nine-species shock-bubble, on {cpu['cpu']}",
                               "gpu_over_cpu": value / best["value"], "detail": cpu}
    print(json.dumps(out))


if __name__ == "__main__":
    main()
