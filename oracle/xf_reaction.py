"""Plain CPU oracle of the reaction source and its time integration.

TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the CPU-baseline leg
of the benchmark import this module; the library's product path never does,
and it imports nothing from the library.  It shares no code with the HIP
kernels: every formula here is written out independently from the paper
(XFluids, arXiv 2403.05910).

What it computes, in the paper's order and notation:
  * mass production rates from mass-action kinetics with third-body
    efficiencies, Arrhenius forward rates and backward rates through the
    equilibrium constants                                   (Sec. II.B, Eq. 9-12)
  * the species ODE written as production minus loss, dY/dt = q - p Y, and
    its alpha-QSS predictor-corrector step                  (Sec. II.C.4, Eq. 27-28)
  * the split coupling to the flow step (Strang or Lie-Trotter) (Sec. II.C.4)

Readings of points the paper leaves open or prints garbled:
  * Eq. 11 prints exp(E / (R_u T)); the Arrhenius law is
    k_f = A T^B exp(-E / (R_u T)) (a positive activation energy slows the
    reaction).  E in J/mol, concentrations in mol/m^3, SI rate constants.
  * [X_s] in Eq. 9 is the molar concentration rho Y_s / W_s; the third-body
    factor is Gamma_r = sum_s eps_rs [X_s] for a reaction with a third body
    and 1 otherwise (it multiplies both directions).
  * Eq. 12 with p0 = 101325 Pa and, for each species, the NASA entropy
    S_s/R_s = a0 ln T + a1 T + a2 T^2/2 + a3 T^3/3 + a4 T^4/4 + a6 (the
    constant a6 comes with the mechanism; the thermo tables carry a0..a5).
    An irreversible reaction has k_b = 0.
  * The reaction step keeps rho, the momentum and the total energy E (the
    species enthalpies include the formation enthalpy a5, so the heat release
    of Eq. 8 appears as a change of T at fixed internal energy): it updates
    the partial densities only, and T follows from e by the Newton iteration
    of Eq. 21 wherever rates are evaluated.
  * Eq. 27: q_s = (W_s / rho) sum_r (nu''_rs R_f,r + nu'_rs R_b,r) and the
    loss p_s Y_s = (W_s / rho) sum_r (nu'_rs R_f,r + nu''_rs R_b,r), with
    R_f,r = Gamma_r k_f,r prod [X]^nu' and R_b,r = Gamma_r k_b,r prod [X]^nu'';
    p_s = loss / Y_s (every loss term carries [X_s]; p_s = 0 where Y_s = 0).
  * Eq. 28's alpha is garbled: read as alpha(r) = (1 - (1 - e^-r)/r) /
    (1 - e^-r) = 1/(1 - e^-r) - 1/r, which makes one step exact for constant
    p and q (alpha(0) = 1/2, alpha(inf) = 1), evaluated as the series
    1/2 + r/12 - r^3/720 below r = 1e-3.  One predictor from the rates at
    Y^0 and one corrector from the rates at the predictor (its T from
    Newton), with p_bar = (p^0 + p^p)/2, alpha_bar = alpha(p_bar dt) and
    q_l = alpha_bar q^p + (1 - alpha_bar) q^0.
  * "Multiple time steps": n_sub equal sub-steps over the reaction
    interval, no adaptive control; after each sub-step the mass fractions
    are renormalised to sum to one (the step must not change rho).
  * Splitting: Strang R(dt/2) F(dt) R(dt/2), or Lie-Trotter F(dt) R(dt),
    with F one SSP-RK3 step of the flow and R the reaction step.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .xf_oracle import RU, h_over_R, temperature_newton

P0 = 101325.0
ALPHA_SERIES_BELOW = 1e-3


@dataclass
class Mechanism:
    """nu_f, nu_b (nr, ns): reactant and product stoichiometric coefficients
    (nu' and nu'' of Eq. 9-10); A, B, E (nr,): Arrhenius factor (SI), exponent
    and activation energy (J/mol); third (nr,) bool and eff (nr, ns):
    third-body flag and efficiencies; reversible (nr,) bool; s0 (ns,): the
    entropy constant a6 of every species."""
    nu_f: np.ndarray
    nu_b: np.ndarray
    A: np.ndarray
    B: np.ndarray
    E: np.ndarray
    third: np.ndarray
    eff: np.ndarray
    reversible: np.ndarray
    s0: np.ndarray

    def __post_init__(self):
        self.nu_f = np.asarray(self.nu_f, dtype=np.int64)
        self.nu_b = np.asarray(self.nu_b, dtype=np.int64)
        for k in ("A", "B", "E", "eff", "s0"):
            setattr(self, k, np.asarray(getattr(self, k), dtype=np.float64))
        self.third = np.asarray(self.third, dtype=bool)
        self.reversible = np.asarray(self.reversible, dtype=bool)

    @property
    def nr(self):
        return self.nu_f.shape[0]


def entropy_over_R(th, s0, T):
    """S_s / R_s of every species (NASA form with the constant s0 = a6);
    T (...) -> (..., ns)"""
    a = th.a
    T = np.asarray(T)[..., None]
    return (a[:, 0] * np.log(T) + a[:, 1] * T + a[:, 2] * T ** 2 / 2 + a[:, 3] * T ** 3 / 3
            + a[:, 4] * T ** 4 / 4 + s0)


def equilibrium_constants(th, mech, T):
    """K_c,r of Eq. 12 at T (...) -> (..., nr)"""
    g = entropy_over_R(th, mech.s0, T) - h_over_R(th, T) / np.asarray(T)[..., None]     # (..., ns)
    nu = (mech.nu_b - mech.nu_f).astype(np.float64)                                   # (nr, ns)
    dn = nu.sum(axis=1)
    return (P0 / (RU * np.asarray(T)[..., None])) ** dn * np.exp(g @ nu.T)


def production_loss(th, mech, rho, Y, T):
    """q_s and the loss p_s Y_s of Eq. 27 (1/s), and p_s; rho, T (...), Y (..., ns)"""
    W = th.W
    conc = rho[..., None] * Y / W                                                    # mol/m^3
    Tn = np.asarray(T)[..., None]
    kf = mech.A * Tn ** mech.B * np.exp(-mech.E / (RU * Tn))                          # (..., nr)
    kb = np.where(mech.reversible, kf / equilibrium_constants(th, mech, T), 0.0)
    Rf = np.zeros(kf.shape)
    Rb = np.zeros(kf.shape)
    for r in range(mech.nr):
        gam = np.sum(mech.eff[r] * conc, axis=-1) if mech.third[r] else 1.0
        pf = 1.0
        pb = 1.0
        for s in range(th.ns):
            if mech.nu_f[r, s]:
                pf = pf * conc[..., s] ** mech.nu_f[r, s]
            if mech.nu_b[r, s]:
                pb = pb * conc[..., s] ** mech.nu_b[r, s]
        Rf[..., r] = gam * kf[..., r] * pf
        Rb[..., r] = gam * kb[..., r] * pb
    q = (Rf @ mech.nu_b + Rb @ mech.nu_f) * W / rho[..., None]
    loss = (Rf @ mech.nu_f + Rb @ mech.nu_b) * W / rho[..., None]
    p = np.where(Y > 0, loss / np.where(Y > 0, Y, 1.0), 0.0)
    return q, loss, p


def alpha(r):
    """alpha(r) = 1/(1 - e^-r) - 1/r (Eq. 28), series below r = 1e-3"""
    r = np.asarray(r, dtype=np.float64)
    small = r < ALPHA_SERIES_BELOW
    rs = np.where(small, 1.0, r)
    exact = 1.0 / (-np.expm1(-rs)) - 1.0 / rs
    series = 0.5 + r / 12.0 - r ** 3 / 720.0
    return np.where(small, series, exact)


def qss_step(th, mech, rho, Y0, e, dt, renormalize=True):
    """one alpha-QSS predictor-corrector step of Eq. 28 at fixed rho and e;
    returns Y (renormalised to sum to one unless renormalize is False)"""
    T0, _ = temperature_newton(th, Y0, e)
    q0, _, p0 = production_loss(th, mech, rho, Y0, T0)
    a0 = alpha(p0 * dt)
    Yp = Y0 + dt * (q0 - p0 * Y0) / (1.0 + a0 * p0 * dt)
    Tp, _ = temperature_newton(th, Yp, e)
    qp, _, pp = production_loss(th, mech, rho, Yp, Tp)
    pbar = 0.5 * (p0 + pp)
    abar = alpha(pbar * dt)
    ql = abar * qp + (1.0 - abar) * q0
    Yc = Y0 + dt * (ql - pbar * Y0) / (1.0 + abar * pbar * dt)
    if renormalize:
        Yc = Yc / np.sum(Yc, axis=-1, keepdims=True)
    return Yc


def react_cells(th, mech, rho, Y, e, dt, n_sub, renormalize=True):
    """n_sub equal alpha-QSS sub-steps over dt; rho, e (...), Y (..., ns)"""
    h = dt / n_sub
    for _ in range(n_sub):
        Y = qss_step(th, mech, rho, Y, e, h, renormalize)
    return Y


def react(th, mech, grid, U, dt, n_sub):
    """the reaction step on the interior of the padded state U (Nv, Z, Y, X):
    partial densities updated at fixed rho, momentum and E; ghosts copied
    unchanged (the caller refills them)"""
    ns = th.ns
    U = np.array(U, copy=True)
    sel = (slice(None),) + grid.interior()
    Ui = U[sel]
    rho = Ui[:ns].sum(axis=0)
    Y = np.moveaxis(Ui[:ns] / rho, 0, -1)
    u = Ui[ns:ns + 3] / rho
    e = Ui[ns + 3] / rho - 0.5 * (u[0] ** 2 + u[1] ** 2 + u[2] ** 2)
    Yn = react_cells(th, mech, rho, Y, e, dt, n_sub)
    Ui[:ns] = np.moveaxis(Yn, -1, 0) * rho
    U[sel] = Ui
    return U
