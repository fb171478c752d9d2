"""Pins of the oracle's WENO7 reconstruction (the seventh-order REC option of
Eq. 15) and of the four-ghost-layer grid it needs, against what the scheme
must satisfy, not against itself:

* each candidate is the edge value of the cubic whose cell averages are the
  data (exact on cubics), and the linear weights (1, 12, 18, 4)/35 turn the
  four candidates into the edge value of the sextic through all seven cells
  (exact on sextics);
* the indicators equal a direct Gauss-Legendre quadrature of the derivatives
  of a known cubic, whatever constant is added to the data;
* the nonlinear scheme converges at seventh order on smooth data, and at a
  jump it stays within the data range;
* in the residual: a uniform state stays exactly uniform, the periodic sum
  vanishes, the advected wave converges at seventh order, and the wider
  layout changes nothing for the six-cell schemes;
* the sampled-cell residual matches the whole-grid one.
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


def test_candidates_exact_on_cubics(rng):
    for _ in range(20):
        coef = rng.standard_normal(4)
        f = _cell_averages(coef, range(-3, 4))
        for qk in O.weno7_candidates(*f):
            assert abs(qk - Pn.polyval(0.5, coef)) <= 1e-12 * max(1.0, np.abs(coef).sum())


def test_linear_weights_exact_on_sextics(rng):
    assert abs(sum(O.WENO7_D) - 1.0) <= 1e-15
    for _ in range(20):
        coef = rng.standard_normal(7)
        f = _cell_averages(coef, range(-3, 4))
        lin = sum(dk * qk for dk, qk in zip(O.WENO7_D, O.weno7_candidates(*f)))
        assert abs(lin - Pn.polyval(0.5, coef)) <= 1e-12 * max(1.0, np.abs(coef).sum())
    # a degree-7 term is not reproduced: the weights are not exact beyond order 7
    coef = np.zeros(8)
    coef[7] = 1.0
    f = _cell_averages(coef, range(-3, 4))
    lin = sum(dk * qk for dk, qk in zip(O.WENO7_D, O.weno7_candidates(*f)))
    assert abs(lin - Pn.polyval(0.5, coef)) > 1e-6


def test_indicators_equal_quadrature_of_a_known_cubic(rng):
    xg, wg = np.polynomial.legendre.leggauss(6)
    xg, wg = 0.5 * xg, 0.5 * wg                      # [-1/2, 1/2], cell i
    for _ in range(20):
        coef = rng.standard_normal(4)
        shift = rng.standard_normal() * 1e3          # beta ignores constants
        for k in range(4):
            f = np.zeros(7)
            f[k:k + 4] = _cell_averages(coef, range(k - 3, k + 1)) + shift
            got = O.weno7_smoothness(*f)[k]
            ref, d = 0.0, coef
            for _ in range(3):
                d = Pn.polyder(d)
                ref += np.sum(wg * Pn.polyval(xg, d) ** 2)
            assert abs(got - ref) <= 1e-10 * max(1.0, abs(ref)), (k, got, ref)


def test_seventh_order_on_smooth_data():
    errs = []
    for h in (0.2, 0.1, 0.05, 0.025):
        x0 = 0.3
        f = np.array([(np.cos(x0 + (c - 0.5) * h) - np.cos(x0 + (c + 0.5) * h)) / h for c in range(-3, 4)])
        errs.append(abs(O.weno7(*f) - np.sin(x0 + 0.5 * h)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates[-1] > 6.5, rates


def test_no_new_extremum_at_a_jump(rng):
    for _ in range(200):
        lo, hi = rng.standard_normal(2) * 3
        k = rng.integers(1, 6)                         # jump inside the stencil
        f = np.where(np.arange(7) < k + 1, lo, hi) + 1e-3 * rng.standard_normal(7)
        r = O.weno7(*f)
        assert f.min() - 1e-2 * abs(hi - lo) <= r <= f.max() + 1e-2 * abs(hi - lo)


def test_weno7_needs_four_ghost_layers():
    case = W.wave_1d(20)
    th, g = oracle_objects(case)
    with pytest.raises(AssertionError):
        O.rhs(th, g, O.fill_ghosts(g, case.U), recon="WENO7")


def test_weno7_freestream_and_conservation():
    tab = W.sampled_table([2.0, 28.0, 40.0], 1)
    case = W.random_smooth_state(tab, (10, 8, 6), seed=4, jump=True).with_ghosts(4)
    th, g = oracle_objects(case)
    assert g.ng == 4 and case.U.shape[1:] == (14, 16, 18)
    U = O.fill_ghosts(g, case.U)
    r = O.rhs(th, g, U, recon="WENO7")
    tot = r.reshape(r.shape[0], -1).sum(axis=1)
    assert np.all(np.abs(tot) <= 1e-12 * np.abs(r).reshape(r.shape[0], -1).sum(axis=1) + 1e-300)
    c = U[:, 6, 6, 6].copy()
    Uu = np.broadcast_to(c[:, None, None, None], U.shape).copy()
    assert np.all(O.rhs(th, g, Uu, recon="WENO7") == 0.0)


def test_wider_layout_changes_nothing_for_six_cell_schemes():
    tab = W.sampled_table([2.0, 28.0, 40.0], 1)
    case3 = W.random_smooth_state(tab, (9, 7, 5), seed=5, jump=True, bc=(1, 1, 0, 0, 1, 0))
    case4 = case3.with_ghosts(4)
    th, g3 = oracle_objects(case3)
    _, g4 = oracle_objects(case4)
    U3, U4 = O.fill_ghosts(g3, case3.U), O.fill_ghosts(g4, case4.U)
    for recon in ("WENO5", "CU6"):
        r3 = O.rhs(th, g3, U3, recon=recon)
        r4 = O.rhs(th, g4, U4, recon=recon)
        assert np.array_equal(r3[(slice(None),) + g3.interior()], r4[(slice(None),) + g4.interior()])


def test_weno7_advected_wave_converges():
    errs = []
    for n in (50, 100, 200):
        case = W.wave_1d(n).with_ghosts(4)
        th, g = oracle_objects(case)
        U = O.fill_ghosts(g, case.U)
        r = O.rhs(th, g, U, recon="WENO7")
        x = (np.arange(n) + 0.5) / n
        # d(rho)/dt = -d(rho u)/dx with u = 1: exact -0.2 * 2 pi cos(2 pi x)
        exact = -0.2 * 2 * np.pi * np.cos(2 * np.pi * x)
        errs.append(np.abs(r[:2].sum(axis=0)[0, 0, 4:-4] - exact).max())
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates[-1] > 6.5, (errs, rates)


def test_sampled_cells_match_whole_grid(rng):
    tab = W.sampled_table([2.0, 28.0], 3)
    case = W.random_smooth_state(tab, (8, 7, 6), seed=6, jump=True).with_ghosts(4)
    th, g = oracle_objects(case)
    U = O.fill_ghosts(g, case.U)
    r = O.rhs(th, g, U, recon="WENO7")
    cells = np.stack([rng.integers(0, n, 12) for n in case.n], axis=1)
    got = O.rhs_at(th, g, U, cells, recon="WENO7")
    gx, gy, gz = g.g(0), g.g(1), g.g(2)
    ref = r[:, cells[:, 2] + gz, cells[:, 1] + gy, cells[:, 0] + gx]
    assert np.allclose(got, ref, rtol=0, atol=1e-12 * np.abs(r).max())
