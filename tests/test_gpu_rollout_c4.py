"""Gradient of a checkpointed SSP-RK3 rollout on the five-species periodic
mixture (the adjoint workload): J = sum over the interior of Y1 (1 - Y1) dV
after 64 steps of fixed dt (the CFL-0.5 step of the initial state), with
checkpoints every 8 steps, differentiated with respect to the initial mass
fractions at fixed density, velocity and pressure.  The direction is
dY = N(0, 1) * 0.05 * Y (seed 7); dU/dY dY comes from the seeded state
assembly by complex step, so the check is of the rollout adjoint itself.

* 16^3 box: against the complex-step derivative of the oracle's rollout
  (stored by tests/golden/make_c4_rollout.py, which calls the oracle only);
  FP64 bar 1e-9 relative, mixed 1e-3 (declared: FP32 projections over 192
  stages).
* 64^3, the full grid: against central differences of the GPU forward
  rollout with the dissipation speeds of every stage frozen at the base
  trajectory (xf_rhs_alpha), h swept from 1e-3 to 1e-7; FP64 bar 1e-6
  relative at the best h, the mixed adjoint against the same differences at
  1e-3.
"""
import json
import os

import numpy as np
import pytest

from paper_2403_05910_amd import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")

HERE = os.path.dirname(os.path.abspath(__file__))
STEPS, EVERY = 64, 8


def _xf():
    from paper_2403_05910_amd import xf
    return xf


def _golden(n):
    with open(os.path.join(HERE, "golden", f"c4_rollout_{n}.json")) as f:
        return json.load(f)


def _setup(n, seed=7, scale=0.05):
    tab, nn, d, rho, vel, Y, p, _ = W.periodic_mixture_fields(n)
    case = W.periodic_mixture(n)
    dY = np.random.default_rng(seed).standard_normal(Y.shape) * scale * Y

    def padded(Yv):
        interior = W.state_at_fixed_rho_u_p(tab, rho, vel, p, Yv)
        U = np.zeros(case.U.shape, dtype=interior.dtype)
        U[:, 3:-3, 3:-3, 3:-3] = interior
        return U

    h = 1e-30
    dU = padded(Y + 1j * h * dY).imag / h
    return case, Y, dY, padded, dU


def _J(ctx, U):
    Ui = U[ctx.interior]
    rho = Ui[:ctx.ns].sum(dim=0)
    Y1 = Ui[0] / rho
    return (Y1 * (1 - Y1)).sum() * (ctx.d[0] * ctx.d[1] * ctx.d[2])


def _adjoint_dd(xf, ctx, U0np, dt, dU):
    """<dJ/dU0, dU> from the checkpointed rollout's backward, and J"""
    U0 = ctx.state_from_numpy(U0np).requires_grad_(True)
    out = xf.rollout(ctx, U0, dt, STEPS, EVERY)
    J = _J(ctx, out)
    J.backward()
    g = U0.grad
    assert float(g[:, :3].abs().max()) == 0.0 and float(g[:, -3:].abs().max()) == 0.0   # ghosts folded
    return float((g * torch.from_numpy(dU).to(g.device)).sum()), float(J)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_rollout_gradient_16_against_oracle_complex_step(precision):
    xf = _xf()
    gold = _golden(16)
    assert gold["steps"] == STEPS
    case, Y, dY, padded, dU = _setup(16, gold["dir_seed"], gold["dir_scale"])
    ctx = xf.Context.from_case(case, precision)
    got, J = _adjoint_dd(xf, ctx, padded(Y), gold["dt"], dU)
    rel = abs(got - gold["dJ"]) / abs(gold["dJ"])
    bar = 1e-9 if precision == "fp64" else 1e-3
    print(f"[c4] 16^3 {precision}: dJ {got:.15e} vs oracle {gold['dJ']:.15e}, rel {rel:.3e}; "
          f"J rel {abs(J - gold['J']) / abs(gold['J']):.2e}", flush=True)
    assert ctx.status() == 0
    ctx.close()
    assert rel <= bar


def _frozen_rollout(ctx, U0, dt, alphas, record=False):
    """the same SSP-RK3 steps as xf_rk3_step, at the torch level, each stage's
    residual from xf_rhs_alpha with the given (or, recording, the scheme's)
    dissipation speeds"""
    U = U0.clone()
    k = 0

    def L(V):
        nonlocal k
        ctx.fill_ghosts(V)
        if record:
            a = torch.empty(ctx.alpha_elems(), dtype=torch.float64, device=V.device)
            r = ctx.rhs_alpha(V, alpha_out=a)
            alphas.append(a)
        else:
            r = ctx.rhs_alpha(V, alpha_in=alphas[k])
        k += 1
        return r

    for _ in range(STEPS):
        ctx.fill_ghosts(U)
        U1 = U + dt * L(U)
        U2 = 0.75 * U + 0.25 * (U1 + dt * L(U1))
        U = U / 3.0 + (2.0 / 3.0) * (U2 + dt * L(U2))
    ctx.fill_ghosts(U)
    return float(_J(ctx, U))


def test_rollout_gradient_64_against_frozen_speed_differences():
    xf = _xf()
    case, Y, dY, padded, dU = _setup(64)
    ctx = xf.Context.from_case(case, "fp64")
    U0 = ctx.state_from_numpy(padded(Y))
    ctx.fill_ghosts(U0)
    dt = ctx.cfl_dt(U0, 0.5).item()
    alphas = []
    J0 = _frozen_rollout(ctx, U0, dt, alphas, record=True)
    assert len(alphas) == 3 * STEPS
    got, J = _adjoint_dd(xf, ctx, padded(Y), dt, dU)
    print(f"[c4] 64^3 J {J:.15e} (frozen-speed replay {J0:.15e}), adjoint dJ {got:.15e}", flush=True)
    assert abs(J - J0) <= 1e-12 * abs(J0)
    errs, fds = {}, {}
    for h in (1e-3, 1e-4, 1e-5, 1e-6, 1e-7):
        Jp = _frozen_rollout(ctx, ctx.state_from_numpy(padded(Y + h * dY)), dt, alphas)
        Jm = _frozen_rollout(ctx, ctx.state_from_numpy(padded(Y - h * dY)), dt, alphas)
        fd = (Jp - Jm) / (2 * h)
        fds[h] = fd
        errs[h] = abs(fd - got) / abs(got)
        print(f"[c4] 64^3 FD h={h:.0e}: {fd:.15e}, rel {errs[h]:.3e}", flush=True)
    best_h = min(errs, key=errs.get)
    assert errs[best_h] <= 1e-6, errs
    # the mixed adjoint against the same differences
    fd_best = fds[best_h]
    ctxm = xf.Context.from_case(case, "mixed")
    gm, _ = _adjoint_dd(xf, ctxm, padded(Y), dt, dU)
    relm = abs(gm - fd_best) / abs(fd_best)
    print(f"[c4] 64^3 mixed adjoint dJ {gm:.15e}, rel {relm:.3e} (differences at h={best_h:.0e})", flush=True)
    assert relm <= 1e-3
    assert ctx.status() == 0 and ctxm.status() == 0
    ctx.close()
    ctxm.close()
