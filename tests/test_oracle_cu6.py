"""Pins of the oracle's WENO-CU6 reconstruction (the six-cell REC option of
Eq. 15) against what the scheme must satisfy, not against itself:

* the smoothness-form routine reproduces the WENO5 indicators on three-cell
  stencils, and beta_6 of a known quintic equals a direct Gauss-Legendre
  quadrature of its derivatives;
* the linear weights (1, 9, 9, 1)/20 reconstruct the edge value of any
  quintic exactly (sixth-order central interpolation);
* tau_6 >= 0, and the nonlinear scheme converges at sixth order on smooth data;
* at a jump the reconstruction stays within the data range (no new extremum
  beyond round-off) and is close to the smooth side's value;
* in the residual: a uniform state stays exactly uniform, the periodic sum
  vanishes, and the advected wave converges at better than fifth order.
"""
import numpy as np
import pytest
from numpy.polynomial import polynomial as Pn

import oracle as O
from conftest import oracle_objects
from paper_2403_05910_amd import workloads as W


def _cell_averages(coef, offsets, h=1.0):
    """averages of the polynomial sum coef[k] x^k over [c-1/2, c+1/2] h"""
    I = Pn.polyint(coef)
    return np.array([(Pn.polyval((c + 0.5) * h, I) - Pn.polyval((c - 0.5) * h, I)) / h for c in offsets])


def test_form_routine_reproduces_weno5_indicators(rng):
    v = rng.standard_normal((5, 200))
    b = O.weno5_smoothness(*v)
    for k, off in enumerate(([-2, -1, 0], [-1, 0, 1], [0, 1, 2])):
        B = O.smoothness_form(off)
        got = np.einsum("i...,ij,j...->...", v[k:k + 3], B, v[k:k + 3])
        assert np.allclose(got, b[k], rtol=1e-12, atol=1e-14)


def test_beta6_equals_quadrature_of_a_known_quintic(rng):
    for _ in range(20):
        coef = rng.standard_normal(6)
        f = _cell_averages(coef, range(-2, 4)) + rng.standard_normal() * 1e3   # beta ignores an offset
        got = O.smoothness6(f)
        xg, wg = np.polynomial.legendre.leggauss(8)
        xg, wg = 0.5 * xg, 0.5 * wg                   # [-1/2, 1/2]
        ref, d = 0.0, coef
        for _ in range(5):
            d = Pn.polyder(d)
            ref += np.sum(wg * Pn.polyval(xg, d) ** 2)
        assert abs(got - ref) <= 1e-11 * max(1.0, abs(ref))


def test_linear_weights_exact_on_quintics(rng):
    for _ in range(20):
        coef = rng.standard_normal(6)
        f = _cell_averages(coef, range(-2, 4))
        q = list(O.weno5_candidates(*f[:5])) + [(11.0 * f[3] - 7.0 * f[4] + 2.0 * f[5]) / 6.0]
        lin = sum(dk * qk for dk, qk in zip(O.CU6_D, q))
        assert abs(lin - Pn.polyval(0.5, coef)) <= 1e-12 * max(1.0, np.abs(coef).sum())


def test_tau6_nonnegative(rng):
    v = rng.standard_normal((6, 5000)) * rng.choice([1e-3, 1.0, 10.0], size=5000)
    jump = rng.uniform(size=5000) < 0.3
    v[3:, jump] += 5.0
    b0, b1, b2 = O.weno5_smoothness(*v[:5])
    b6 = np.einsum("i...,ij,j...->...", v, O.CU6_B6, v)
    tau = b6 - (b0 + 4 * b1 + b2) / 6
    assert np.all(tau >= -1e-12 * b6)


def test_sixth_order_on_smooth_data():
    errs = []
    for h in (0.2, 0.1, 0.05, 0.025):
        x0 = 0.3
        f = np.array([(np.cos(x0 + (c - 0.5) * h) - np.cos(x0 + (c + 0.5) * h)) / h for c in range(-2, 4)])
        errs.append(abs(O.weno_cu6(*f) - np.sin(x0 + 0.5 * h)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates[-1] > 5.5, rates


def test_no_new_extremum_at_a_jump(rng):
    for _ in range(200):
        lo, hi = rng.standard_normal(2) * 3
        k = rng.integers(1, 5)                         # jump inside the stencil
        f = np.where(np.arange(6) < k + 1, lo, hi) + 1e-3 * rng.standard_normal(6)
        r = O.weno_cu6(*f)
        assert f.min() - 1e-2 * abs(hi - lo) <= r <= f.max() + 1e-2 * abs(hi - lo)


def test_cu6_freestream_and_conservation(rng):
    tab = W.sampled_table([2.0, 28.0, 40.0], 1)
    case = W.random_smooth_state(tab, (10, 8, 6), seed=4, jump=True)
    th, g = oracle_objects(case)
    U = O.fill_ghosts(g, case.U)
    r = O.rhs(th, g, U, recon="CU6")
    tot = r.reshape(r.shape[0], -1).sum(axis=1)
    assert np.all(np.abs(tot) <= 1e-12 * np.abs(r).reshape(r.shape[0], -1).sum(axis=1) + 1e-300)
    c = U[:, 5, 5, 5].copy()
    Uu = np.broadcast_to(c[:, None, None, None], U.shape).copy()
    assert np.all(O.rhs(th, g, Uu, recon="CU6") == 0.0)


def test_cu6_advected_wave_converges():
    errs = []
    for n in (25, 50, 100):
        case = W.wave_1d(n)
        th, g = oracle_objects(case)
        U = O.fill_ghosts(g, case.U)
        r = O.rhs(th, g, U, recon="CU6")
        rho = U[:2].sum(axis=0)[0, 0, 3:-3]
        x = (np.arange(n) + 0.5) / n
        # d(rho)/dt = -d(rho u)/dx with u = 1: exact -0.2 * 2 pi cos(2 pi x)
        exact = -0.2 * 2 * np.pi * np.cos(2 * np.pi * x)
        errs.append(np.abs(r[:2].sum(axis=0)[0, 0, 3:-3] - exact).max())
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates[-1] > 5.0, (errs, rates)
