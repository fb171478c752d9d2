"""Seeded synthetic inputs for the multicomponent convective right-hand side.

This module is shared by the tests and the benchmark.  It holds no step of the
right-hand side itself: it draws thermo tables and initial conditions and
assembles conservative states from primitive fields.  Assembly needs the
forward energy map e(T) of the thermo polynomials, which is written out here
on its own (it is the inverse direction of the Newton step the method performs).

Workload shapes follow the shock-bubble interaction set-up of the paper
(Sec. V.B, Eq. 32-33: planar shock, spherical bubble with a tanh interface,
Rankine-Hugoniot post-shock state).  Everything is synthetic and seeded; the
paper's own thermo data, mechanisms and reference solutions are not used.

Conventions: padded arrays of shape (Nv, Z, Y, X) with 3 ghost layers per
active dimension (Case.with_ghosts gives another width; ghost values are left
at zero: the caller fills them), fields in
order rho Y_1..rho Y_N, rho u, rho v, rho w, rho E, SI units.
"""
from __future__ import annotations

from dataclasses import dataclass, field

from math import comb

import numpy as np

R_UNIVERSAL = 8.314462618
T_BRACKET = (200.0, 4000.0)


@dataclass
class ThermoTable:
    W: np.ndarray            # (ns,) kg/mol
    a: np.ndarray            # (ns, 6): cp/R = a0 + a1 T + .. + a4 T^4 ; a5 = h/R constant
    T_lo: float = 0.0
    T_hi: float = 0.0        # <= 0: no Newton bracket (calorically perfect tables)

    @property
    def ns(self):
        return len(self.W)


@dataclass
class Case:
    name: str
    n: tuple                 # (nx, ny, nz)
    d: tuple                 # (dx, dy, dz)
    bc: tuple                # (-x, +x, -y, +y, -z, +z): 0 periodic, 1 outflow
    thermo: ThermoTable
    U: np.ndarray            # padded (Nv, Z, Y, X), ghosts zero
    meta: dict = field(default_factory=dict)

    @property
    def cells(self):
        return int(np.prod(self.n))

    @property
    def ng(self):
        """ghost layers per active dimension of U (3 while U is unset)"""
        if self.U is None:
            return 3
        k = next(a for a in range(3) if self.n[a] > 1)
        return (self.U.shape[3 - k] - self.n[k]) // 2

    def with_ghosts(self, ng):
        """the same case in a layout with ng ghost layers per active dimension
        (interior copied, ghosts zero)"""
        g0 = self.ng
        U, g = _padded(self.n, self.U.shape[0], ng)
        nx, ny, nz = self.n
        gz, gy, gx = (g0 if nz > 1 else 0), (g0 if ny > 1 else 0), (g0 if nx > 1 else 0)
        _place(U, g, self.U[:, gz:gz + nz, gy:gy + ny, gx:gx + nx])
        return Case(self.name, self.n, self.d, self.bc, self.thermo, U, dict(self.meta))


# ---------------------------------------------------------------------------
# thermo tables
# ---------------------------------------------------------------------------
def perfect_gas_table(gammas, W_gmol):
    """Calorically perfect species: cp/R = gamma/(gamma-1), no bracket."""
    g = np.asarray(gammas, dtype=np.float64)
    a = np.zeros((len(g), 6))
    a[:, 0] = g / (g - 1.0)
    return ThermoTable(W=np.asarray(W_gmol, dtype=np.float64) * 1e-3, a=a)


def sampled_table(W_gmol, seed=0, T_lo=T_BRACKET[0], T_hi=T_BRACKET[1]):
    """Seeded thermally perfect species.  In tau = (T - 2100)/1900 (so tau in
    [-1, 1] on 200..4000 K): cp/R = c0 + sum_{k=1..4} c_k tau^k with c0 ~ U(3, 5.5)
    and raw c_k ~ U(-1, 1) rescaled so sum |c_k| = u min(c0 - 2.5, 6 - c0),
    u ~ U(0, 1); this keeps cp/R inside [2.5, 6] on the whole range.  The
    polynomial is converted exactly to monomials in T; a5 = 0.  Species are
    drawn in index order from numpy's default_rng(seed)."""
    rng = np.random.default_rng(seed)
    ns = len(W_gmol)
    a = np.zeros((ns, 6))
    mid, half = 0.5 * (T_lo + T_hi), 0.5 * (T_hi - T_lo)
    for s in range(ns):
        c0 = rng.uniform(3.0, 5.5)
        raw = rng.uniform(-1.0, 1.0, 4)
        u = rng.uniform(0.0, 1.0)
        ck = raw / np.sum(np.abs(raw)) * u * min(c0 - 2.5, 6.0 - c0)
        tau_coef = np.concatenate([[c0], ck])
        # tau = (T - mid)/half: expand sum c_k ((T - mid)/half)^k in powers of T
        lin = np.polynomial.Polynomial([-mid / half, 1.0 / half])
        poly = np.polynomial.Polynomial([0.0])
        for k, ckk in enumerate(tau_coef):
            poly = poly + ckk * lin ** k
        coef = np.zeros(5)
        coef[:len(poly.coef)] = poly.coef
        a[s, :5] = coef
    return ThermoTable(W=np.asarray(W_gmol, dtype=np.float64) * 1e-3, a=a, T_lo=T_lo, T_hi=T_hi)


# ---------------------------------------------------------------------------
# state assembly (forward direction of the EOS; input preparation only)
# ---------------------------------------------------------------------------
# ---------------------------------------------------------------------------
# transport tables: the fitted form ln eta = sum_k c_k (ln T)^k (four
# coefficients), synthetic values of the usual magnitudes for gases
# ---------------------------------------------------------------------------
@dataclass
class TransportTable:
    mu: np.ndarray           # (ns, 4): ln(mu_s / (Pa s)) = sum_k mu[s, k] (ln T)^k
    kappa: np.ndarray        # (ns, 4): ln(kappa_s / (W/(m K)))
    D: np.ndarray            # (ns, ns, 4), symmetric: ln(D_st / (m^2/s)) at p_ref
    p_ref: float = 101325.0


def _log_poly_coeffs(v0, b, c2, c3, T0=300.0):
    """powers of ln T of ln v0 + b L + c2 L^2 + c3 L^3 with L = ln(T / T0)"""
    l0 = np.log(T0)
    e = (np.log(v0), b, c2, c3)
    coef = np.zeros(4)
    for k, ek in enumerate(e):
        for n in range(k + 1):
            coef[n] += ek * comb(k, n) * (-l0) ** (k - n)
    return coef


def sampled_transport(ns, seed=0):
    """Seeded tables: at 300 K mu_s in [1e-5, 3e-5] Pa s, kappa_s in
    [0.015, 0.18] W/(m K), D_st in [1e-5, 8e-5] m^2/s at 1 atm; temperature
    exponents 0.6-0.8, 0.7-0.95 and 1.6-1.8 with small curvature."""
    rng = np.random.default_rng(seed)
    mu = np.array([_log_poly_coeffs(rng.uniform(1e-5, 3e-5), rng.uniform(0.6, 0.8), rng.uniform(-0.03, 0.03),
                                    rng.uniform(-0.005, 0.005)) for _ in range(ns)])
    kappa = np.array([_log_poly_coeffs(rng.uniform(0.015, 0.18), rng.uniform(0.7, 0.95), rng.uniform(-0.03, 0.03),
                                       rng.uniform(-0.005, 0.005)) for _ in range(ns)])
    D = np.zeros((ns, ns, 4))
    for s_ in range(ns):
        for t in range(s_, ns):
            D[s_, t] = D[t, s_] = _log_poly_coeffs(rng.uniform(1e-5, 8e-5), rng.uniform(1.6, 1.8),
                                                   rng.uniform(-0.03, 0.03), rng.uniform(-0.005, 0.005))
    return TransportTable(mu, kappa, D)


def constant_transport(ns, mu=1.8e-5, kappa=0.026, D=2e-5):
    """temperature-independent tables (every species alike), for closed forms"""
    c = lambda v: np.array([np.log(v), 0.0, 0.0, 0.0])  # noqa: E731
    return TransportTable(np.tile(c(mu), (ns, 1)), np.tile(c(kappa), (ns, 1)), np.tile(c(D), (ns, ns, 1)))


# ---------------------------------------------------------------------------
# synthetic reaction mechanism (the paper's H2-O2 mechanisms are not used)
# ---------------------------------------------------------------------------
@dataclass
class MechanismTable:
    nu_f: np.ndarray         # (nr, ns) reactant coefficients
    nu_b: np.ndarray         # (nr, ns) product coefficients
    A: np.ndarray            # (nr,) Arrhenius factor, SI units of the reaction order
    B: np.ndarray            # (nr,) temperature exponent
    E: np.ndarray            # (nr,) activation energy, J/mol
    third: np.ndarray        # (nr,) bool: a third body M takes part
    eff: np.ndarray          # (nr, ns) third-body efficiencies
    reversible: np.ndarray   # (nr,) bool
    s0: np.ndarray           # (ns,) entropy constants a6 of the species

    @property
    def nr(self):
        return self.nu_f.shape[0]


def synthetic_mechanism(W_gmol, tab, seed=0, n_reactions=12, T_ref=1500.0):
    """Seeded mass-balanced reactions among species of the given molar
    masses: exchanges A + B = C + D (W_A + W_B = W_C + W_D) and dissociations
    A + M = B + C + M (W_A = W_B + W_C), found by searching the masses;
    n_reactions of them drawn without replacement.  Rate constants are drawn
    at T_ref (10^2..10^4 in SI units for exchanges, 10^1..10^3 for the
    three-body ones), then A follows from a temperature exponent in
    [-1, 1.5] and an activation energy in [0, 1.5e5] J/mol; efficiencies in
    [0.5, 3]; every reaction reversible.  The entropy constants a6 are set so
    that every species' S/R - h/(R T) at T_ref is a draw in [-2, 2] (random
    constants would put the equilibrium constants of the table tab at
    e^+-30 and make the backward rates absurd)."""
    rng = np.random.default_rng(seed)
    W = np.asarray(W_gmol, dtype=np.float64)
    ns = len(W)
    cands = []
    for a in range(ns):
        for b in range(a, ns):
            for c in range(ns):
                for d in range(c, ns):
                    if {a, b} == {c, d} or (c, d) < (a, b):
                        continue
                    if abs(W[a] + W[b] - W[c] - W[d]) < 1e-9:
                        cands.append(("x", (a, b), (c, d)))
    for a in range(ns):
        for b in range(ns):
            for c in range(b, ns):
                if a not in (b, c) and abs(W[a] - W[b] - W[c]) < 1e-9:
                    cands.append(("d", (a,), (b, c)))
    pick = rng.choice(len(cands), size=min(n_reactions, len(cands)), replace=False)
    nr = len(pick)
    nu_f = np.zeros((nr, ns), dtype=np.int64)
    nu_b = np.zeros((nr, ns), dtype=np.int64)
    third = np.zeros(nr, dtype=bool)
    k_ref = np.zeros(nr)
    for r, i in enumerate(sorted(pick)):
        kind, lhs, rhs_ = cands[i]
        for sp in lhs:
            nu_f[r, sp] += 1
        for sp in rhs_:
            nu_b[r, sp] += 1
        third[r] = kind == "d"
        k_ref[r] = 10.0 ** rng.uniform(1.0, 3.0) if third[r] else 10.0 ** rng.uniform(2.0, 4.0)
    B = rng.uniform(-1.0, 1.5, nr)
    E = rng.uniform(0.0, 1.5e5, nr)
    A = k_ref / (T_ref ** B * np.exp(-E / (R_UNIVERSAL * T_ref)))
    eff = rng.uniform(0.5, 3.0, (nr, ns))
    a = np.asarray(tab.a)
    T = T_ref
    s_var = a[:, 0] * np.log(T) + a[:, 1] * T + a[:, 2] * T ** 2 / 2 + a[:, 3] * T ** 3 / 3 + a[:, 4] * T ** 4 / 4
    h_RT = (a[:, 0] * T + a[:, 1] * T ** 2 / 2 + a[:, 2] * T ** 3 / 3 + a[:, 3] * T ** 4 / 4 + a[:, 4] * T ** 5 / 5
            + a[:, 5]) / T
    s0 = rng.uniform(-2.0, 2.0, ns) + h_RT - s_var
    return MechanismTable(nu_f, nu_b, A, B, E, third, eff, np.ones(nr, dtype=bool), s0)


def rethermo(case, tab):
    """the same flow (rho, u, T, Y) under the table tab, which differs from
    the case's only in the enthalpy constants a5: E gains
    sum_s rho Y_s R_s (a5_new - a5_old), so every cell keeps its temperature"""
    da = (np.asarray(tab.a)[:, 5] - np.asarray(case.thermo.a)[:, 5]) * R_UNIVERSAL / np.asarray(tab.W)
    U = case.U.copy()
    ns = len(tab.W)
    U[ns + 3] += np.tensordot(da, U[:ns], axes=(0, 0))
    return Case(case.name, case.n, case.d, case.bc, tab, U, dict(case.meta))


def with_formation_enthalpies(tab, seed=0, lo=-1000.0, hi=1000.0):
    """the table with seeded enthalpy constants a5 (K, i.e. h/R at T = 0),
    so that reactions release or absorb heat"""
    rng = np.random.default_rng(seed)
    a = tab.a.copy()
    a[:, 5] = rng.uniform(lo, hi, len(tab.W))
    return ThermoTable(tab.W, a, tab.T_lo, tab.T_hi)


def _cp_R(tab, T):
    a = tab.a
    T = np.asarray(T, dtype=np.float64)[..., None]
    return (((a[:, 4] * T + a[:, 3]) * T + a[:, 2]) * T + a[:, 1]) * T + a[:, 0]


def _e_species(tab, T):
    """e_s(T) = R_s (int_0^T cp_s/R_s dT + a5 - T)"""
    a = tab.a
    Tn = np.asarray(T, dtype=np.result_type(T, np.float64))[..., None]   # complex T stays complex
    hR = ((((a[:, 4] / 5 * Tn + a[:, 3] / 4) * Tn + a[:, 2] / 3) * Tn + a[:, 1] / 2) * Tn + a[:, 0]) * Tn + a[:, 5]
    return R_UNIVERSAL / tab.W * (hR - Tn)


def assemble(tab, rho, vel, T, Y):
    """Conservative fields from rho, velocity (3, ...), T, Y (ns, ...)."""
    Yl = np.moveaxis(np.asarray(Y), 0, -1)
    e = np.sum(Yl * _e_species(tab, T), axis=-1)
    ke = 0.5 * (vel[0] ** 2 + vel[1] ** 2 + vel[2] ** 2)
    E = rho * (e + ke)
    return np.concatenate([rho * Y, rho * vel, E[None]], axis=0)


def mixture_R(tab, Y):
    return np.tensordot(R_UNIVERSAL / tab.W, np.asarray(Y), axes=(0, 0))


def frozen_sound_speed(tab, Y, T):
    """c^2 = (1 + Rbar/cv) Rbar T for a mixture of given composition Y (ns,)"""
    Y = np.asarray(Y, dtype=np.float64)
    Rs = R_UNIVERSAL / tab.W
    Rbar = float(np.dot(Y, Rs))
    cv = float(np.dot(Y, Rs * (_cp_R(tab, T) - 1.0)))
    return np.sqrt((1.0 + Rbar / cv) * Rbar * T)


def _padded(n, nv, ng=3):
    g = [ng if k > 1 else 0 for k in n]
    shape = (nv, n[2] + 2 * g[2], n[1] + 2 * g[1], n[0] + 2 * g[0])
    return np.zeros(shape), g


def _centres(n, lo, d):
    """cell-centre coordinates x_i = lo + (i + 1/2) d per axis (point values)"""
    return [lo[k] + (np.arange(n[k]) + 0.5) * d[k] for k in range(3)]


def _place(U, g, interior):
    nz, ny, nx = interior.shape[1:]
    U[:, g[2]:g[2] + nz, g[1]:g[1] + ny, g[0]:g[0] + nx] = interior
    return U


# ---------------------------------------------------------------------------
# Rankine-Hugoniot post-shock state (Eq. 33 and its thermally perfect analogue)
# ---------------------------------------------------------------------------
def post_shock_perfect(gamma, Ma, rho0, p0, c0):
    """Eq. 33: normal-shock jump for a calorically perfect gas."""
    M2 = Ma * Ma
    rho1 = rho0 * (gamma + 1.0) * M2 / (2.0 + (gamma - 1.0) * M2)
    u1 = Ma * c0 * (1.0 - rho0 / rho1)
    p1 = p0 * (1.0 + 2.0 * gamma / (gamma + 1.0) * (M2 - 1.0))
    return rho1, u1, p1


def post_shock_thermal(tab, Y, Ma, T0, p0):
    """Normal shock of speed Ma c0 (c0 = frozen sound speed of the quiescent
    gas) running into gas at rest at (T0, p0), for thermally perfect species.
    Shock frame: mass, momentum and energy fluxes equal on both sides,
    h(T) = e(T) + Rbar T.  Solved by Newton on the post-shock temperature.
    Returns (rho1, u1 (lab frame), p1, T1)."""
    Y = np.asarray(Y, dtype=np.float64)
    Rbar = float(np.dot(Y, R_UNIVERSAL / tab.W))

    def h(T):
        return float(np.dot(Y, _e_species(tab, T))) + Rbar * T

    rho0 = p0 / (Rbar * T0)
    c0 = frozen_sound_speed(tab, Y, T0)
    W = Ma * c0
    m = rho0 * W
    P = p0 + rho0 * W * W
    Hs = h(T0) + 0.5 * W * W

    def resid(T1):
        # momentum gives rho1 from T1: p1 + m^2/rho1 = P with p1 = rho1 Rbar T1
        # -> Rbar T1 rho1^2 - P rho1 + m^2 = 0 (shocked root = larger rho1)
        disc = P * P - 4.0 * Rbar * T1 * m * m
        rho1 = (P + np.sqrt(max(disc, 0.0))) / (2.0 * Rbar * T1)
        v1 = m / rho1
        return h(T1) + 0.5 * v1 * v1 - Hs, rho1, v1

    # bracket the root between T0 (weak limit) and a generous upper bound
    lo, hi = T0 * (1.0 + 1e-9), T0 * (1.0 + Ma * Ma)
    flo = resid(lo)[0]
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        fm = resid(mid)[0]
        if (fm > 0) == (flo > 0):
            lo, flo = mid, fm
        else:
            hi = mid
        if hi - lo <= 1e-13 * hi:
            break
    T1 = 0.5 * (lo + hi)
    _, rho1, v1 = resid(T1)
    return rho1, W - v1, rho1 * Rbar * T1, T1


# ---------------------------------------------------------------------------
# bubble geometry
# ---------------------------------------------------------------------------
def _real_sph_harm(theta, phi, coef, lmax):
    """S(theta, phi) = sum_{l=1..lmax} sum_{m=-l..l} a_lm Y_lm^real(theta, phi),
    theta the polar angle, phi the azimuth; coef holds the a_lm in (l, m) order."""
    from scipy.special import sph_harm_y
    S = np.zeros(np.broadcast(theta, phi).shape)
    i = 0
    for l in range(1, lmax + 1):
        for m in range(-l, l + 1):
            Y = sph_harm_y(l, abs(m), theta, phi)
            if m > 0:
                Yr = np.sqrt(2.0) * (-1) ** m * Y.real
            elif m < 0:
                Yr = np.sqrt(2.0) * (-1) ** m * Y.imag
            else:
                Yr = Y.real
            S = S + coef[i] * Yr
            i += 1
    return S


def _harmonic_radius_fn(seed, lmax=8, amp=0.01):
    """r(theta, phi)/r0 = 1 + amp S with a_lm ~ N(0, 1) drawn from
    default_rng(seed) and S normalised to max|S| = 1 on a 256 x 512
    (theta, phi) grid."""
    rng = np.random.default_rng(seed)
    coef = rng.standard_normal(sum(2 * l + 1 for l in range(1, lmax + 1)))
    th = np.linspace(0, np.pi, 256)
    ph = np.linspace(0, 2 * np.pi, 512, endpoint=False)
    TH, PH = np.meshgrid(th, ph, indexing="ij")
    scale = 1.0 / np.max(np.abs(_real_sph_harm(TH, PH, coef, lmax)))

    def fn(theta, phi):
        return 1.0 + amp * scale * _real_sph_harm(theta, phi, coef, lmax)

    return fn


def _bubble_phi(X, Y, Z, centre, r0, width, radius_fn=None):
    """phi = 1/2 (1 - tanh(dist/width)): 1 inside, 0 outside; dist = |x - x0| - r
    (the interface function of Eq. 32, with the interface about two cells wide)."""
    dx, dy, dz = X - centre[0], Y - centre[1], Z - centre[2]
    rr = np.sqrt(dx * dx + dy * dy + dz * dz)
    r = np.full(rr.shape, float(r0))
    if radius_fn is not None:
        # the perturbed radius matters only near the interface: beyond 16
        # interface widths tanh has saturated to within 2e-14
        near = np.abs(rr - r0) < 16.0 * width
        theta = np.arccos(np.clip(dz[near] / np.maximum(rr[near], 1e-300), -1.0, 1.0))
        phi = np.mod(np.arctan2(dy[near], dx[near]), 2 * np.pi)
        r[near] = r0 * radius_fn(theta, phi)
    return 0.5 * (1.0 - np.tanh((rr - r) / width))


def _shock_bubble(name, tab, n, lo, hi, bubbles, Y_amb, Y_bub, Ma, x_shock,
                  T0=300.0, p0=101325.0, radius_fn=None, perfect_gamma=None):
    nv = tab.ns + 4
    d = tuple((hi[k] - lo[k]) / n[k] for k in range(3))
    xs, ys, zs = _centres(n, lo, d)
    Z, Yc, X = np.meshgrid(zs, ys, xs, indexing="ij")
    phi = np.zeros_like(X)
    for (c, r0) in bubbles:
        phi = np.maximum(phi, _bubble_phi(X, Yc, Z, c, r0, d[0], radius_fn))
    Y_amb = np.asarray(Y_amb, dtype=np.float64)
    Y_bub = np.asarray(Y_bub, dtype=np.float64)
    Yf = phi[None] * Y_bub[:, None, None, None] + (1.0 - phi[None]) * Y_amb[:, None, None, None]
    Rbar = mixture_R(tab, Yf)
    T = np.full(X.shape, T0)
    rho = p0 / (Rbar * T)
    vel = np.zeros((3,) + X.shape)
    # post-shock region x < x_shock (pure ambient gas there)
    if perfect_gamma is not None:
        Rg = float(np.dot(Y_amb, R_UNIVERSAL / tab.W))
        rho0 = p0 / (Rg * T0)
        c0 = np.sqrt(perfect_gamma * p0 / rho0)
        rho1, u1, p1 = post_shock_perfect(perfect_gamma, Ma, rho0, p0, c0)
        T1 = p1 / (rho1 * Rg)
    else:
        rho1, u1, p1, T1 = post_shock_thermal(tab, Y_amb, Ma, T0, p0)
    post = X < x_shock
    rho = np.where(post, rho1, rho)
    T = np.where(post, T1, T)
    vel[0] = np.where(post, u1, 0.0)
    interior = assemble(tab, rho, vel, T, Yf)
    U, g = _padded(n, nv)
    _place(U, g, interior)
    bc = (1, 1, 0, 0, 0, 0)
    return Case(name, tuple(n), d, bc, tab, U,
                meta=dict(post_shock=(rho1, u1, p1, T1), Ma=Ma, T0=T0, p0=p0))


# ---------------------------------------------------------------------------
# the workloads
# ---------------------------------------------------------------------------
def wave_1d(nx=200):
    """1D advected two-species wave on [0,1], periodic: rho = 1 + 0.2 sin 2 pi x,
    u = 1, p = 1, Y1 = 0.5 + 0.4 sin 2 pi x; calorically perfect species
    (gamma, W) = (1.4, 28.96), (1.667, 4.003)."""
    tab = perfect_gas_table([1.4, 1.667], [28.96, 4.003])
    x = (np.arange(nx) + 0.5) / nx
    rho = 1.0 + 0.2 * np.sin(2 * np.pi * x)
    Y1 = 0.5 + 0.4 * np.sin(2 * np.pi * x)
    Y = np.stack([Y1, 1.0 - Y1])
    Rbar = mixture_R(tab, Y)
    T = 1.0 / (rho * Rbar)
    vel = np.stack([np.ones(nx), np.zeros(nx), np.zeros(nx)])
    interior = assemble(tab, rho, vel, T, Y).reshape(6, 1, 1, nx)
    U, g = _padded((nx, 1, 1), 6)
    _place(U, g, interior)
    return Case("wave1d", (nx, 1, 1), (1.0 / nx, 1.0, 1.0), (0,) * 6, tab, U)


def inert_sbi(n=128, seed=1):
    """3D inert shock-bubble on [0,1]^3: air ambient (p = 101325 Pa, T = 300 K),
    Mach 1.22 shock at x = 0.15, helium-like bubble at (0.35, 0.5, 0.5) with
    radius 0.15 perturbed by seeded real spherical harmonics up to degree 8 at
    1 % amplitude; outflow in x, periodic in y, z."""
    tab = perfect_gas_table([1.4, 1.667], [28.96, 4.003])
    rfn = _harmonic_radius_fn(seed)
    return _shock_bubble("inert_sbi", tab, (n, n, n), (0, 0, 0), (1, 1, 1),
                         [((0.35, 0.5, 0.5), 0.15)], [1.0, 0.0], [0.0, 1.0],
                         1.22, 0.15, radius_fn=rfn, perfect_gamma=1.4)


W9 = [2.0, 1.0, 16.0, 17.0, 18.0, 32.0, 33.0, 34.0, 28.0]
W5 = [2.0, 32.0, 18.0, 28.0, 40.0]


def nine_species_sbi(n=256, seed=0):
    """3D 9-species thermally perfect shock-bubble on [0,1]^3: ambient species 9
    at 300 K / 101325 Pa, bubble Y1/Y6/Y9 = 0.03/0.24/0.73 at (0.35, 0.5, 0.5),
    radius 0.15, Mach 2 shock at x = 0.15; outflow in x, periodic in y, z."""
    nn = (n, n, n) if np.isscalar(n) else tuple(n)
    tab = sampled_table(W9, seed)
    Yb = np.zeros(9)
    Yb[[0, 5, 8]] = [0.03, 0.24, 0.73]
    Ya = np.zeros(9)
    Ya[8] = 1.0
    return _shock_bubble("nine_species_sbi", tab, nn, (0, 0, 0), (1, 1, 1),
                         [((0.35, 0.5, 0.5), 0.15)], Ya, Yb, 2.0, 0.15)


def two_bubble_sbi(n=(512, 256, 256), seed=4):
    """3D 9-species Mach 2 shock with two bubbles on [0,2]x[0,1]x[0,1]; bubble
    centres drawn with seed in x in [0.4, 1.6], y, z in [0.3, 0.7], at least
    0.35 apart."""
    tab = sampled_table(W9, 0)
    rng = np.random.default_rng(seed)
    while True:
        c = [np.array([rng.uniform(0.4, 1.6), rng.uniform(0.3, 0.7), rng.uniform(0.3, 0.7)]) for _ in range(2)]
        if np.linalg.norm(c[0] - c[1]) >= 0.35:
            break
    Yb = np.zeros(9)
    Yb[[0, 5, 8]] = [0.03, 0.24, 0.73]
    Ya = np.zeros(9)
    Ya[8] = 1.0
    return _shock_bubble("two_bubble_sbi", tab, tuple(n), (0, 0, 0), (2, 1, 1),
                         [(tuple(c[0]), 0.15), (tuple(c[1]), 0.15)], Ya, Yb, 2.0, 0.15)


def _fourier_field(X, Y, Z, rng, kmax=4):
    """sum over integer wave vectors 1 <= |k| <= kmax of a_k cos(2 pi k.x + phi_k),
    a_k ~ N(0, 1), phi_k ~ U(0, 2 pi); normalised to max |delta| = 1"""
    f = np.zeros_like(X)
    r = range(-kmax, kmax + 1)
    for kx in r:
        for ky in r:
            for kz in r:
                k2 = kx * kx + ky * ky + kz * kz
                if k2 < 1 or k2 > kmax * kmax:
                    continue
                a = rng.standard_normal()
                ph = rng.uniform(0, 2 * np.pi)
                f += a * np.cos(2 * np.pi * (kx * X + ky * Y + kz * Z) + ph)
    return f / np.max(np.abs(f))


def periodic_mixture_fields(n=64, seed=2, thermo_seed=0, T_lo=20.0):
    """The primitive fields of periodic_mixture: (table, n, d, rho, vel, Y, p),
    interior arrays (rho (Z, Y, X), vel (3, ...), Y (5, ...)), p = 1e5 uniform."""
    nn = (n, n, n) if np.isscalar(n) else tuple(n)
    tab = sampled_table(W5, thermo_seed, T_lo=T_lo)
    d = tuple(1.0 / k for k in nn)
    xs, ys, zs = _centres(nn, (0, 0, 0), d)
    Z, Yc, X = np.meshgrid(zs, ys, xs, indexing="ij")
    rng = np.random.default_rng(seed)
    dr = _fourier_field(X, Yc, Z, rng)
    dv = [_fourier_field(X, Yc, Z, rng) for _ in range(3)]
    dY = [_fourier_field(X, Yc, Z, rng) for _ in range(5)]
    Y0 = np.full(5, 0.2)
    T_base = 1e5 / (1.2 * float(np.dot(Y0, R_UNIVERSAL / tab.W)))
    c0 = frozen_sound_speed(tab, Y0, T_base)
    rho = 1.2 * (1.0 + 0.05 * dr)
    vel = np.stack([0.05 * c0 * v for v in dv])
    Yf = np.stack([0.2 * (1.0 + 0.05 * v) for v in dY])
    Yf = Yf / np.sum(Yf, axis=0, keepdims=True)
    return tab, nn, d, rho, vel, Yf, 1e5, c0


def state_at_fixed_rho_u_p(tab, rho, vel, p, Y):
    """Conservative interior fields of mass fractions Y (any dtype, complex
    included) at given density, velocity and pressure: T = p / (rho R(Y)),
    partial densities rho Y_k (Y is not renormalised)."""
    T = p / (rho * mixture_R(tab, Y))
    return assemble(tab, rho, vel, T, Y)


def periodic_mixture(n=64, seed=2, thermo_seed=0, T_lo=20.0):
    """3D periodic 5-species thermally perfect mixture on [0,1]^3: rho = 1.2,
    p = 1e5, u = 0, Y = 0.2 each, plus seeded Fourier perturbations (|k| <= 4,
    5 % amplitude) of rho, u, v, w and every Y_k (renormalised); p uniform."""
    tab, nn, d, rho, vel, Yf, p, c0 = periodic_mixture_fields(n, seed, thermo_seed, T_lo)
    interior = state_at_fixed_rho_u_p(tab, rho, vel, p, Yf)
    U, g = _padded(nn, 9)
    _place(U, g, interior)
    return Case("periodic_mixture", nn, d, (0,) * 6, tab, U, meta=dict(c0=c0))


def sod(nx=400, gamma=1.4):
    """Sod shock tube on [0,1] (single calorically perfect gas):
    (rho, u, p) = (1, 0, 1) for x < 0.5 and (0.125, 0, 0.1) otherwise;
    outflow at both ends."""
    W = 28.96
    tab = perfect_gas_table([gamma], [W])
    x = (np.arange(nx) + 0.5) / nx
    left = x < 0.5
    rho = np.where(left, 1.0, 0.125)
    p = np.where(left, 1.0, 0.1)
    Rg = R_UNIVERSAL / tab.W[0]
    T = p / (rho * Rg)
    vel = np.zeros((3, nx))
    interior = assemble(tab, rho, vel, T, np.ones((1, nx))).reshape(5, 1, 1, nx)
    U, g = _padded((nx, 1, 1), 5)
    _place(U, g, interior)
    return Case("sod", (nx, 1, 1), (1.0 / nx, 1.0, 1.0), (1, 1, 1, 1, 1, 1), tab, U)


def species_interface_1d(nx=200):
    """Sharp two-gas slab advected through a periodic box: gas A
    (gamma, W) = (1.4, 28.96) on [0.25, 0.75), gas B (1.667, 4.003) elsewhere,
    u = 1, p = 1, T = 1e-3 (about 7x denser A); the mass fractions jump from 0
    to 1 in one cell, where WENO reconstruction undershoots."""
    tab = perfect_gas_table([1.4, 1.667], [28.96, 4.003])
    x = (np.arange(nx) + 0.5) / nx
    inside = (x >= 0.25) & (x < 0.75)
    Y = np.stack([np.where(inside, 1.0, 0.0), np.where(inside, 0.0, 1.0)])
    T = np.full(nx, 1e-3)
    Rm = mixture_R(tab, Y)
    rho = 1.0 / (Rm * T)
    vel = np.zeros((3, nx))
    vel[0] = 1.0
    interior = assemble(tab, rho, vel, T, Y).reshape(6, 1, 1, nx)
    U, g = _padded((nx, 1, 1), 6)
    _place(U, g, interior)
    return Case("species_interface_1d", (nx, 1, 1), (1.0 / nx, 1.0, 1.0), (0,) * 6, tab, U)


def species_slab(n=(48, 40, 1)):
    """Multi-dimensional sharp interface: gas A (1.4, 28.96) in the slab
    |x - 0.5 - 0.1 sin(2 pi y) - 0.05 sin(2 pi z)| < 0.25 of the periodic unit
    box, gas B (1.667, 4.003) elsewhere, u = (1, 0.5, 0.25) (components on
    inactive axes dropped), p = 1, T = 1e-3."""
    nn = tuple(n)
    tab = perfect_gas_table([1.4, 1.667], [28.96, 4.003])
    xs = [(np.arange(k) + 0.5) / k for k in nn]
    X, Yc, Z = np.meshgrid(xs[0], xs[1], xs[2], indexing="ij")
    X, Yc, Z = (np.transpose(a, (2, 1, 0)) for a in (X, Yc, Z))          # (z, y, x)
    inside = np.abs(X - 0.5 - 0.1 * np.sin(2 * np.pi * Yc) - 0.05 * np.sin(2 * np.pi * Z)) < 0.25
    Y = np.stack([np.where(inside, 1.0, 0.0), np.where(inside, 0.0, 1.0)])
    T = np.full(inside.shape, 1e-3)
    rho = 1.0 / (mixture_R(tab, Y) * T)
    vel = np.zeros((3,) + inside.shape)
    for k, v in enumerate((1.0, 0.5, 0.25)):
        if nn[k] > 1:
            vel[k] = v
    interior = assemble(tab, rho, vel, T, Y)
    U, g = _padded(nn, 6)
    _place(U, g, interior)
    return Case("species_slab", nn, tuple(1.0 / k for k in nn), (0,) * 6, tab, U)


def double_rarefaction_1d(nx=200, u0=3.0):
    """Two gases pulled apart: (rho, u, p) = (1, -u0, 0.4) with gas A
    (gamma 1.4, W 28.96) for x < 0.5 and (1, +u0, 0.4) with gas B (1.667,
    4.003) beyond; outflow at both ends.  Two strong rarefactions leave a
    near-vacuum between them (u0 = 2 is the classic '123' case)."""
    tab = perfect_gas_table([1.4, 1.667], [28.96, 4.003])
    x = (np.arange(nx) + 0.5) / nx
    left = x < 0.5
    Y = np.stack([np.where(left, 1.0, 0.0), np.where(left, 0.0, 1.0)])
    rho = np.ones(nx)
    p = np.full(nx, 0.4)
    T = p / (rho * mixture_R(tab, Y))
    vel = np.zeros((3, nx))
    vel[0] = np.where(left, -u0, u0)
    interior = assemble(tab, rho, vel, T, Y).reshape(6, 1, 1, nx)
    U, g = _padded((nx, 1, 1), 6)
    _place(U, g, interior)
    return Case("double_rarefaction_1d", (nx, 1, 1), (1.0 / nx, 1.0, 1.0), (1,) * 6, tab, U)


def random_smooth_state(tab, n, seed, amp=0.05, u_scale=50.0, T0=300.0, p0=1e5, bc=(0,) * 6,
                        jump=False):
    """A generic random state on a small grid for parity tests: smooth Fourier
    perturbations (and optionally a contact/shock-like jump in x) of a
    quiescent mixture with equal mass fractions."""
    rng = np.random.default_rng(seed)
    nn = tuple(n)
    ns = tab.ns
    d = tuple(1.0 / k for k in nn)
    xs, ys, zs = _centres(nn, (0, 0, 0), d)
    Z, Yc, X = np.meshgrid(zs, ys, xs, indexing="ij")

    def fld():
        f = np.zeros_like(X)
        for _ in range(4):
            k = rng.integers(-2, 3, size=3)
            f += rng.standard_normal() * np.cos(2 * np.pi * (k[0] * X + k[1] * Yc + k[2] * Z) + rng.uniform(0, 6.3))
        m = np.max(np.abs(f))
        return f / m if m > 0 else f

    Yf = np.stack([(1.0 + 0.5 * fld()) for _ in range(ns)])
    Yf = np.abs(Yf) + 0.05
    Yf = Yf / np.sum(Yf, axis=0, keepdims=True)
    T = T0 * (1.0 + amp * fld())
    p = p0 * (1.0 + amp * fld())
    vel = np.stack([u_scale * fld() for _ in range(3)])
    for k in range(3):
        if nn[k] == 1:
            vel[k] = 0.0
    if jump:
        sel = X > 0.5
        p = np.where(sel, 1.8 * p, p)
        T = np.where(sel, 1.3 * T, T)
        vel[0] = np.where(sel, vel[0] + 80.0, vel[0])
    rho = p / (mixture_R(tab, Yf) * T)
    interior = assemble(tab, rho, vel, T, Yf)
    U, g = _padded(nn, ns + 4)
    _place(U, g, interior)
    return Case("random", nn, d, tuple(bc), tab, U)
