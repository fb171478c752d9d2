"""Planted mistakes: each test plants one plausible error in the oracle (on the
CPU, through monkeypatch) and checks that at least one pin of
test_oracle_pins.py then fails.  This shows the pins are sharp enough that a
dropped term, a wrong sign or index or a transposed operand cannot pass."""
import numpy as np
import pytest

import oracle as O
import test_oracle_pins as P

X = O.xf_oracle


def _patch(monkeypatch, name, value):
    """plant `value` under `name` in the oracle module and the package that
    re-exports it (the pins call through the package)"""
    monkeypatch.setattr(X, name, value)
    if hasattr(O, name):
        monkeypatch.setattr(O, name, value)


def _fails(fn, *a, **k):
    try:
        fn(*a, **k)
    except AssertionError:
        return True
    return False


def test_wrong_linear_weights_caught(monkeypatch):
    _patch(monkeypatch, "WENO_D", (0.3, 0.6, 0.1))
    assert _fails(P.test_fifth_order_convergence_smooth_wave)


def test_wrong_smoothness_coefficient_caught(monkeypatch, rng):
    orig = X.weno5_smoothness

    def bad(a, b, c, d, e):
        b0, b1, b2 = orig(a, b, c, d, e)
        return b0, b1 - 1.0 / 12.0 * (b - 2.0 * c + d) ** 2, b2
    _patch(monkeypatch, "weno5_smoothness", bad)
    assert _fails(P.test_weno_smoothness_matches_integral_definition, rng)


def test_weight_power_one_caught(monkeypatch):
    def bad(a, b, c, d, e):
        q = X.weno5_candidates(a, b, c, d, e)
        be = X.weno5_smoothness(a, b, c, d, e)
        al = [X.WENO_D[k] / (X.WENO_EPS + be[k]) for k in range(3)]
        s = sum(al)
        return sum(al[k] / s * q[k] for k in range(3))
    _patch(monkeypatch, "weno5", bad)
    assert _fails(P.test_weno_essentially_non_oscillatory)


def test_dropped_RT_in_species_energy_caught(monkeypatch, rng):
    _patch(monkeypatch, "species_e", lambda th, T: th.R * X.h_over_R(th, T))
    assert _fails(P.test_single_gas_matches_textbook_solver, rng, "LLF")


def test_swapped_roe_weights_caught(monkeypatch, rng):
    orig = X.roe_state

    def bad(th, pL, pR):
        # weight the left state with the right density's share
        sL, sR = np.sqrt(pL["rho"]), np.sqrt(pR["rho"])
        fake = dict(pL)
        fake["rho"] = pR["rho"]
        fakeR = dict(pR)
        fakeR["rho"] = pL["rho"]
        return orig(th, fake, fakeR)
    _patch(monkeypatch, "roe_state", bad)
    assert _fails(P.test_single_gas_matches_textbook_solver, rng, "LLF")


def test_tangential_row_sign_caught(monkeypatch, rng):
    orig = X.eigen_L

    def bad(th, roe, d):
        L = orig(th, roe, d)
        L[..., th.ns + 1, :th.ns] *= -1.0
        return L
    _patch(monkeypatch, "eigen_L", bad)
    assert _fails(P.test_left_right_inverse, 2, rng)


def test_transposed_left_matrix_caught(monkeypatch, rng):
    orig = X.eigen_L
    _patch(monkeypatch, "eigen_L", lambda th, roe, d: np.swapaxes(orig(th, roe, d), -1, -2))
    assert _fails(P.test_left_right_inverse, 2, rng)


def test_dropped_RT_in_chi_caught(monkeypatch, rng):
    orig = X.roe_state

    def bad(th, pL, pR):
        r = orig(th, pL, pR)
        r["chi"] = r["chi"] - th.R * r["T"][..., None]
        r["c2"] = np.sum(r["Y"] * r["chi"], axis=-1) + r["Gam"] * (r["H"] - r["q2"])
        r["c"] = np.sqrt(r["c2"])
        return r
    _patch(monkeypatch, "roe_state", bad)
    assert _fails(P.test_flux_jacobian_eigenvectors, 3, rng)


def test_flux_sign_caught(monkeypatch):
    orig = X.face_flux

    def bad(*a, **k):
        F, al, c2 = orig(*a, **k)
        return -F, al, c2
    _patch(monkeypatch, "face_flux", bad)
    assert _fails(P.test_fifth_order_convergence_smooth_wave)


def test_wrong_acoustic_eigenvalue_caught(monkeypatch, rng):
    orig = X.eigenvalues

    def bad(th, prim, d):
        lam = orig(th, prim, d)
        return np.concatenate([lam[-1:], lam[1:]], axis=0)   # u+c used for the u-c field
    _patch(monkeypatch, "eigenvalues", bad)
    assert _fails(P.test_single_gas_matches_textbook_solver, rng, "LLF")


def test_wrong_rk3_stage_weight_caught(monkeypatch):
    def bad(L, U, dt):
        U1 = U + dt * L(U)
        U2 = 0.5 * U + 0.5 * (U1 + dt * L(U1))
        return U / 3.0 + 2.0 / 3.0 * (U2 + dt * L(U2))
    _patch(monkeypatch, "ssp_rk3", bad)
    assert _fails(P.test_ssp_rk3_linear_stability_polynomial)


def test_wrong_outflow_ghost_caught(monkeypatch, rng):
    orig = X.fill_ghosts

    def bad(grid, U):
        V = orig(grid, U)
        V[:, :, 0, :] = V[:, :, 4, :]     # -y outflow copied from the second interior row
        return V
    _patch(monkeypatch, "fill_ghosts", bad)
    assert _fails(P.test_ghost_fill_matches_numpy_pad, rng)


def test_newton_with_cp_denominator_still_converges_but_energy_with_cp_caught(monkeypatch, rng):
    """A Newton step with the wrong derivative converges to the same root (so
    the round trip cannot see it), but an energy map that uses h instead of e
    changes the EOS and the textbook comparison fails."""
    _patch(monkeypatch, "mixture_e", lambda th, Y, T: np.sum(Y * th.R * X.h_over_R(th, T), axis=-1))
    assert _fails(P.test_single_gas_matches_textbook_solver, rng, "LLF")


# -- positivity-preserving blend (pins in test_oracle_positivity.py) --------
import test_oracle_positivity as PP  # noqa: E402


def test_positivity_half_step_factor_caught(monkeypatch):
    orig = X.positivity_limit
    # half-states U -+ lam F instead of U -+ 2 lam F (Eq. 18)
    _patch(monkeypatch, "positivity_limit", lambda th, d, Ust, Pst, Fh, al, lam: orig(th, d, Ust, Pst, Fh, al, 0.5 * lam))
    assert _fails(PP.test_half_states_respect_floors_with_largest_theta, 2)


def test_positivity_side_sign_caught(monkeypatch):
    def bad(th, d, Ust, Pst, Fhat, alpha, lam):
        ns = th.ns
        lf = np.maximum(alpha[0].real, alpha[-1].real)
        FLF = X.lax_friedrichs_flux(th, d, Ust, Pst, lf)
        comps = lambda V: np.concatenate([V[:ns].sum(axis=0, keepdims=True), V[:ns]], axis=0)
        qL, qR = comps(Ust[:, 2]), comps(Ust[:, 3])
        qH, qLF = comps(Fhat), comps(FLF)
        rhoL, rhoR = qL[0].real, qR[0].real
        fr = X.PP_RHO_FLOOR * np.minimum(rhoL, rhoR)
        epsL = np.concatenate([fr[None], np.broadcast_to(-X.PP_Y_FLOOR * rhoL, (ns,) + rhoL.shape)])
        epsR = np.concatenate([fr[None], np.broadcast_to(-X.PP_Y_FLOOR * rhoR, (ns,) + rhoR.shape)])
        theta = np.ones(Fhat.shape[1])
        for q0, sgn, eps in ((qL, 1.0, epsL), (qR, -1.0, epsR)):      # planted: sides swapped
            w_hi = q0 + sgn * 2.0 * lam * qH
            w_lo = q0 + sgn * 2.0 * lam * qLF
            gap = w_lo - w_hi
            with np.errstate(all="ignore"):
                t = np.where(w_hi >= eps, 1.0, np.where(gap > 0, (w_lo - eps) / gap, 0.0))
            theta = np.minimum(theta, np.clip(t, 0.0, 1.0).min(axis=0))
        return np.where(theta == 1.0, Fhat, FLF + theta * (Fhat - FLF)), theta
    _patch(monkeypatch, "positivity_limit", bad)
    assert _fails(PP.test_half_states_respect_floors_with_largest_theta, 3)
    assert _fails(PP.test_mass_fractions_stay_above_floor_over_a_run)


def test_positivity_not_applied_caught(monkeypatch):
    _patch(monkeypatch, "positivity_limit",
           lambda th, d, Ust, Pst, Fh, al, lam: (Fh, np.ones(Fh.shape[1])))
    assert _fails(PP.test_mass_fractions_stay_above_floor_over_a_run)
    assert _fails(PP.test_half_states_respect_floors_with_largest_theta, 4)


def test_roe_speed_without_abs_caught(monkeypatch, rng):
    orig = X.face_flux

    def bad(th, d, Ust, Pst, alpha=None, visc="LLF", recon="WENO5"):
        if alpha is None and visc == "ROE":
            roe = X.roe_state(th, X._take(Pst, 2), X._take(Pst, 3))
            un, c = roe["u"][d], roe["c"]
            nv = th.ns + 4
            alpha = np.stack([un - c] + [un] * (nv - 2) + [un + c], axis=0).real   # planted: no |.|
        return orig(th, d, Ust, Pst, alpha, "LLF" if alpha is not None else visc, recon)
    _patch(monkeypatch, "face_flux", bad)
    assert _fails(P.test_single_gas_matches_textbook_solver, rng, "ROE")


def test_scaled_wave_speed_caught_for_glf(monkeypatch, rng):
    orig_eig = X.eigenvalues
    # planted: cell wave speeds scaled by 0.9 (the global maximum too small)
    _patch(monkeypatch, "eigenvalues", lambda th, prim, d: orig_eig(th, prim, d).real * 0.9)
    assert _fails(P.test_single_gas_matches_textbook_solver, rng, "GLF")


# -- WENO-CU6 (pins in test_oracle_cu6.py) ------------------------------------
import test_oracle_cu6 as CU  # noqa: E402


def test_cu6_wrong_linear_weights_caught(monkeypatch, rng):
    _patch(monkeypatch, "CU6_D", (9.0 / 20.0, 1.0 / 20.0, 1.0 / 20.0, 9.0 / 20.0))
    assert _fails(CU.test_sixth_order_on_smooth_data)


def test_cu6_downwind_candidate_sign_caught(monkeypatch):
    def bad(a, b, c, d, e, f):
        q0, q1, q2 = X.weno5_candidates(a, b, c, d, e)
        q3 = (11.0 * d + 7.0 * e - 2.0 * f) / 6.0          # planted: signs of e and f flipped
        b0, b1, b2 = X.weno5_smoothness(a, b, c, d, e)
        b6 = X.smoothness6(np.stack(np.broadcast_arrays(a, b, c, d, e, f), axis=0))
        tau = b6 - (b0 + 4.0 * b1 + b2) / 6.0
        al = [X.CU6_D[k] * (X.CU6_C + tau / (bk + X.CU6_EPS)) for k, bk in enumerate((b0, b1, b2, b6))]
        s_ = al[0] + al[1] + al[2] + al[3]
        return (al[0] * q0 + al[1] * q1 + al[2] * q2 + al[3] * q3) / s_
    _patch(monkeypatch, "weno_cu6", bad)
    assert _fails(CU.test_sixth_order_on_smooth_data)
    assert _fails(CU.test_cu6_advected_wave_converges)


# -- WENO7 (pins in test_oracle_weno7.py) -------------------------------------
import test_oracle_weno7 as W7  # noqa: E402


def test_weno7_swapped_linear_weights_caught(monkeypatch, rng):
    _patch(monkeypatch, "WENO7_D", (4.0 / 35.0, 18.0 / 35.0, 12.0 / 35.0, 1.0 / 35.0))
    assert _fails(W7.test_linear_weights_exact_on_sextics, rng)
    assert _fails(W7.test_seventh_order_on_smooth_data)


def test_weno7_candidate_coefficient_caught(monkeypatch, rng):
    orig = X.weno7_candidates

    def bad(a, b, c, d, e, f, g):
        q0, q1, q2, q3 = orig(a, b, c, d, e, f, g)
        return q0, q1, q2 + (c - e) / 12.0, q3                # planted: -c + 7d + 7e - f -> 7d + 6e - f
    _patch(monkeypatch, "weno7_candidates", bad)
    assert _fails(W7.test_candidates_exact_on_cubics, rng)
    assert _fails(W7.test_weno7_advected_wave_converges)


def test_weno7_shifted_indicator_stencil_caught(monkeypatch, rng):
    # planted: the indicator forms built on sub-stencils one cell to the right
    _patch(monkeypatch, "WENO7_PARTS", [X.smoothness_parts(range(k - 2, k + 2)) for k in range(4)])
    assert _fails(W7.test_indicators_equal_quadrature_of_a_known_cubic, rng)


def test_weno7_mirrored_minus_side_caught(monkeypatch, rng):
    # planted: the minus side read in the plus side's order (not mirrored)
    orig = X.weno7

    def flux(th, d, Ust, Pst, alpha=None, visc="LLF", recon="WENO5"):
        if recon != "WENO7":
            return orig_ff(th, d, Ust, Pst, alpha, visc, recon)
        calls = []

        def w(*v):
            calls.append(1)
            return orig(*v) if len(calls) % 2 else orig(*v[::-1])
        monkeypatch.setattr(X, "weno7", w)
        try:
            return orig_ff(th, d, Ust, Pst, alpha, visc, recon)
        finally:
            monkeypatch.setattr(X, "weno7", orig)
    orig_ff = X.face_flux
    _patch(monkeypatch, "face_flux", flux)
    assert _fails(W7.test_weno7_advected_wave_converges)


# -- viscous fluxes (pins in test_oracle_viscous.py) ---------------------------
import test_oracle_viscous as VI  # noqa: E402

XV = O.xf_viscous


def test_viscous_transposed_mixing_factor_caught(monkeypatch, rng):
    orig = XV.wilke_phi
    monkeypatch.setattr(XV, "wilke_phi", lambda W_, a: np.swapaxes(orig(W_, a), -1, -2))
    assert _fails(VI.test_mixing_rule_reductions, rng)


def test_viscous_cell_derivative_coefficient_caught(monkeypatch):
    def bad(q, ax, h):
        out = np.full(q.shape, np.nan, dtype=q.dtype)
        L = q.shape[ax]

        def sl(a, b):
            s = [slice(None)] * q.ndim
            s[ax] = slice(a, b)
            return tuple(s)
        out[sl(2, L - 2)] = (q[sl(0, L - 4)] - 7.0 * q[sl(1, L - 3)] + 7.0 * q[sl(3, L - 1)] - q[sl(4, L)]) / (12.0 * h)
        return out
    monkeypatch.setattr(XV, "cell_derivative", bad)
    assert _fails(VI.test_fourth_order_stress_convergence_2d)


def test_viscous_point_flux_difference_caught(monkeypatch):
    # planted: the plain difference of point fluxes (second order)
    monkeypatch.setattr(XV, "numerical_flux", lambda Fv, ax: np.take(Fv, np.arange(1, Fv.shape[ax] - 1), axis=ax))
    assert _fails(VI.test_fourth_order_stress_convergence_2d)


def test_viscous_linear_face_interpolation_caught(monkeypatch):
    def bad(q, n, g, ax):
        s = XV._face_slices(n, g, ax, q.ndim)
        return 0.5 * (q[s[1]] + q[s[2]])
    monkeypatch.setattr(XV, "face_value", bad)
    assert _fails(VI.test_quadratic_shear_closed_form)


def test_viscous_dropped_fit_term_caught(monkeypatch):
    orig = XV.fit_eval
    monkeypatch.setattr(XV, "fit_eval", lambda c, T: orig(c[..., :3], T))
    assert _fails(VI.test_fit_form_reproduces_a_shifted_power_law)


# -- reaction source (pins in test_oracle_reaction.py) --------------------------
import test_oracle_reaction as RE  # noqa: E402

XR = O.xf_reaction


def test_reaction_constant_alpha_caught(monkeypatch):
    monkeypatch.setattr(XR, "alpha", lambda r: 0.5 + 0.0 * np.asarray(r, dtype=np.float64))
    assert _fails(RE.test_alpha_limits_and_exactness)
    assert _fails(RE.test_first_order_decay_is_exponential)


def test_reaction_inverted_equilibrium_constant_caught(monkeypatch):
    orig = XR.equilibrium_constants
    monkeypatch.setattr(XR, "equilibrium_constants", lambda th, mech, T: 1.0 / orig(th, mech, T))
    assert _fails(RE.test_reversible_pair_reaches_its_equilibrium_constant)


def test_reaction_backward_direction_dropped_caught(monkeypatch):
    orig = XR.production_loss

    def bad(th, mech, rho, Y, T):
        # planted: every reaction treated as irreversible (no backward rate)
        m = XR.Mechanism(mech.nu_f, mech.nu_b, mech.A, mech.B, mech.E, mech.third, mech.eff,
                         np.zeros_like(mech.reversible), mech.s0)
        return orig(th, m, rho, Y, T)
    monkeypatch.setattr(XR, "production_loss", bad)
    assert _fails(RE.test_reversible_pair_reaches_its_equilibrium_constant)


def test_reaction_arrhenius_sign_caught(monkeypatch):
    orig = XR.production_loss

    def bad(th, mech, rho, Y, T):
        m = XR.Mechanism(mech.nu_f, mech.nu_b, mech.A, mech.B, -mech.E, mech.third, mech.eff, mech.reversible,
                         mech.s0)
        return orig(th, m, rho, Y, T)
    monkeypatch.setattr(XR, "production_loss", bad)
    assert _fails(RE.test_forward_rate_grows_with_temperature)


def _roe_with(th, pL, pR, Y_mean=False, T_mean=False):
    """the oracle's Roe state with one weighting replaced by the arithmetic mean"""
    sL, sR = np.sqrt(pL["rho"]), np.sqrt(pR["rho"])
    wL = sL / (sL + sR)
    wR = 1.0 - wL
    u = wL * pL["u"] + wR * pR["u"]
    H = wL * pL["H"] + wR * pR["H"]
    Y = 0.5 * (pL["Y"] + pR["Y"]) if Y_mean else wL[..., None] * pL["Y"] + wR[..., None] * pR["Y"]
    T = 0.5 * (pL["T"] + pR["T"]) if T_mean else wL * pL["T"] + wR * pR["T"]
    Gam = X.mixture_R(th, Y) / X.mixture_cv(th, Y, T)
    q2 = u[0] ** 2 + u[1] ** 2 + u[2] ** 2
    chi = Gam[..., None] * (0.5 * q2[..., None] - X.species_e(th, T)) + th.R * T[..., None]
    c2 = np.sum(Y * chi, axis=-1) + Gam * (H - q2)
    return dict(u=u, H=H, Y=Y, T=T, Gam=Gam, chi=chi, c2=c2, c=np.sqrt(c2), q2=q2)


def test_roe_arithmetic_mean_mass_fractions_caught(monkeypatch, rng):
    _patch(monkeypatch, "roe_state", lambda th, pL, pR: _roe_with(th, pL, pR, Y_mean=True))
    assert _fails(P.test_roe_condition_calorically_perfect_mixture, 5, rng)


def test_roe_arithmetic_mean_temperature_caught(monkeypatch, rng):
    _patch(monkeypatch, "roe_state", lambda th, pL, pR: _roe_with(th, pL, pR, T_mean=True))
    assert _fails(P.test_roe_condition_calorically_perfect_mixture, 5, rng)


def test_rk3_first_stage_only_caught(monkeypatch):
    """an RK3 that stops after its first (forward Euler) stage keeps the
    residual's fifth order but not the one-period accuracy"""
    def euler(L, U, dt):
        return U + dt * L(U)
    _patch(monkeypatch, "ssp_rk3", euler)
    assert _fails(P.test_rk3_one_period_fifth_order)
