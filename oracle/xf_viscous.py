"""Plain CPU oracle of the viscous and diffusive fluxes F_v of Eq. 2.

TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the CPU-baseline leg
of the benchmark import this module; the library's product path never does,
and it imports nothing from the library.  It shares no code with the HIP
kernels: every formula here is written out independently from the paper
(XFluids, arXiv 2403.05910).

What it computes, in the paper's order and notation:
  * pure-species viscosity mu_s, conductivity kappa_s and binary diffusion
    coefficients D_st from the fitted polynomials
    ln eta = sum_n a_n (ln T)^(n-1)                          (Sec. IV.4, Eq. 29)
  * mixture viscosity and conductivity by the semi-empirical
    mixing rule                                             (Sec. II.C.3, Eq. 22)
  * effective diffusion coefficient of each species into the
    mixture                                                  (Sec. II.C.3, Eq. 26)
  * Newtonian stress, Fourier conduction, diffusional enthalpy
    flux and mass-corrected Fickian diffusion                 (Sec. II.A, Eq. 2-6)
  * their divergence added to the residual with fourth-order central
    differences (the Fourth option of VISCOSITY_ORDER, Table I)

Readings of points the paper leaves open:
  * Fits: four coefficients per property (cubic in ln T).  The binary
    diffusion fits are taken at a reference pressure p_ref and scaled by
    p_ref / p (Eq. 25 has D_st proportional to 1/p).
  * Eq. 22 is applied literally to both properties: Phi^alpha uses the ratio
    of the property being mixed (mu_s/mu_t for the viscosity, kappa_s/kappa_t
    for the conductivity).
  * Eq. 26, whose numerator over Wbar equals 1 - Y_s, is undefined (0/0) in a
    pure species; the mole fractions inside it carry a floor of 1e-12
    (X_t + 1e-12), which changes a mixture's value by O(1e-12) and gives a
    pure species the finite limit of a trace admixture of all the others.
  * Eq. 6 is garbled (its sum runs over j but differentiates Y_s): it is read
    as J_s = -rho (D_sm grad Y_s - Y_s sum_j D_jm grad Y_j), the
    mixture-averaged flux with the correction that makes sum_s J_s = 0.
  * Sign of the species entry of F_v: Eq. 1 puts div F_v on the right-hand
    side and Eq. 6 defines J_s with Fick's sign (down the gradient), as q_c
    of Eq. 4 is; the energy entry subtracts q_c and q_d = sum h_s J_s, so the
    species entry consistent with it (and with diffusion rather than
    anti-diffusion) is -J_s.  F_v = (-J_s, tau, tau . u - q_c - q_d).
  * h_s in Eq. 5 is the species enthalpy per unit mass at the cell's T.
  * Discretisation (the paper names the order only), fourth order and
    conservative: first the point value of F_v at every face from
    fourth-order face values, (-f_{i-1} + 9 f_i + 9 f_{i+1} - f_{i+2}) / 16,
    normal derivatives (f_{i-1} - 27 f_i + 27 f_{i+1} - f_{i+2}) / (24 dx),
    and tangential derivatives interpolated the same way from the
    cell-centred differences (f_{j-2} - 8 f_{j-1} + 8 f_{j+1} - f_{j+2}) /
    (12 dy); transport coefficients, rho, Y_s, u and h_s are interpolated
    cell values; an inactive axis contributes no derivative.  The residual
    is then the staggered fourth-order difference of those point fluxes,
    (F_{i-3/2} - 27 F_{i-1/2} + 27 F_{i+1/2} - F_{i+3/2}) / (24 dx), i.e. the
    conservative difference of the numerical flux
    F^_{i+1/2} = (-F_{i-1/2} + 26 F_{i+1/2} - F_{i+3/2}) / 24 (the plain
    difference of point fluxes would be second order only).  The point
    fluxes one face beyond each end read the third ghost layer.
  * Terms can be switched separately (Visc, Visc_Heat, Visc_Diffu of
    Table I): STRESS (tau and its work tau . u), HEAT (q_c), DIFFUSION (J_s
    and q_d).
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from .xf_oracle import h_over_R, primitives

STRESS, HEAT, DIFFUSION = 1, 2, 4
ALL_TERMS = STRESS | HEAT | DIFFUSION
DIFF_X_FLOOR = 1e-12


@dataclass
class Transport:
    """Fitted transport tables (Eq. 29): mu (ns, 4) and kappa (ns, 4) give
    ln(mu_s / (Pa s)) and ln(kappa_s / (W/(m K))) as cubics in ln T; D
    (ns, ns, 4), symmetric in its first two indices, gives ln(D_st / (m^2/s))
    at the pressure p_ref (Pa)."""
    mu: np.ndarray
    kappa: np.ndarray
    D: np.ndarray
    p_ref: float = 101325.0

    def __post_init__(self):
        self.mu = np.asarray(self.mu, dtype=np.float64)
        self.kappa = np.asarray(self.kappa, dtype=np.float64)
        self.D = np.asarray(self.D, dtype=np.float64)


def fit_eval(coef, T):
    """eta(T) = exp(sum_n a_n (ln T)^n) for coef (..., 4) and T (cells);
    returns (cells..., ...) with the coefficient sets along the last axes"""
    lt = np.log(np.asarray(T)).reshape(np.shape(T) + (1,) * (coef.ndim - 1))
    out = np.zeros(np.shape(T) + coef.shape[:-1])
    for n in range(coef.shape[-1]):
        out = out + coef[..., n] * lt ** n
    return np.exp(out)


def species_transport(tr, T, p):
    """mu_s, kappa_s (cells..., ns) and D_st (cells..., ns, ns) at T, p"""
    mu = fit_eval(tr.mu, T)
    kappa = fit_eval(tr.kappa, T)
    D = fit_eval(tr.D, T) * (tr.p_ref / np.asarray(p))[..., None, None]
    return mu, kappa, D


def mole_fractions(W, Y):
    """X_s = (Y_s / W_s) / sum_t Y_t / W_t; Y (cells..., ns)"""
    n = Y / W
    return n / np.sum(n, axis=-1, keepdims=True)


def wilke_phi(W, alpha):
    """Phi_st of Eq. 22 for the pure-species property alpha (cells..., ns):
    (cells..., ns, ns) with s the row and t the column"""
    ns = len(W)
    phi = np.zeros(alpha.shape + (ns,))
    for s in range(ns):
        for t in range(ns):
            phi[..., s, t] = (1.0 / np.sqrt(8.0) * (1.0 + W[s] / W[t]) ** -0.5
                              * (1.0 + np.sqrt(alpha[..., s] / alpha[..., t]) * (W[t] / W[s]) ** 0.25) ** 2)
    return phi


def wilke_mix(W, X, alpha):
    """mixture value of Eq. 22: sum_s X_s alpha_s / sum_t X_t Phi_st"""
    phi = wilke_phi(W, alpha)
    ns = len(W)
    out = 0.0
    for s in range(ns):
        den = 0.0
        for t in range(ns):
            den = den + X[..., t] * phi[..., s, t]
        out = out + X[..., s] * alpha[..., s] / den
    return out


def diffusion_into_mixture(W, X, D):
    """D_sm of Eq. 26: sum_{t != s} X_t W_t / (Wbar sum_{t != s} X_t / D_st),
    Wbar = sum_s X_s W_s, with the floor X_t + 1e-12 inside the two sums
    (cells..., ns)"""
    ns = len(W)
    Wbar = np.sum(X * W, axis=-1)
    out = np.zeros(X.shape)
    if ns == 1:               # the sums over t != s are empty: a single species does not diffuse
        return out
    for s in range(ns):
        num = 0.0
        den = 0.0
        for t in range(ns):
            if t == s:
                continue
            Xt = X[..., t] + DIFF_X_FLOOR
            num = num + Xt * W[t]
            den = den + Xt / D[..., s, t]
        out[..., s] = num / (Wbar * den)
    return out


def mixture_transport(th, tr, prim):
    """mu_bar, kappa_bar (cells...) and D_sm (cells..., ns) of every cell"""
    mu, kappa, D = species_transport(tr, prim["T"], prim["p"])
    X = mole_fractions(th.W, prim["Y"])
    return wilke_mix(th.W, X, mu), wilke_mix(th.W, X, kappa), diffusion_into_mixture(th.W, X, D)


# ---------------------------------------------------------------------------
# fourth-order central operators on padded arrays
# ---------------------------------------------------------------------------
def _face_slices(n, g, ax, ndim):
    """the four cell slices (i-1, i, i+1, i+2) of faces k = -1..n+1 along
    array axis ax (face k lies between padded cells g+k-1 and g+k)"""
    out = []
    for m in range(4):
        sl = [slice(None)] * ndim
        sl[ax] = slice(g - 3 + m, g - 3 + m + n + 3)
        out.append(tuple(sl))
    return out


def face_value(q, n, g, ax):
    """(-q_{i-1} + 9 q_i + 9 q_{i+1} - q_{i+2}) / 16 at the faces along ax"""
    s = _face_slices(n, g, ax, q.ndim)
    return (-q[s[0]] + 9.0 * q[s[1]] + 9.0 * q[s[2]] - q[s[3]]) / 16.0


def face_normal_derivative(q, n, g, ax, h):
    """(q_{i-1} - 27 q_i + 27 q_{i+1} - q_{i+2}) / (24 h) at the faces along ax"""
    s = _face_slices(n, g, ax, q.ndim)
    return (q[s[0]] - 27.0 * q[s[1]] + 27.0 * q[s[2]] - q[s[3]]) / (24.0 * h)


def cell_derivative(q, ax, h):
    """(q_{j-2} - 8 q_{j-1} + 8 q_{j+1} - q_{j+2}) / (12 h) at the cells with
    two neighbours on each side along ax; NaN on the two outer layers"""
    out = np.full(q.shape, np.nan, dtype=q.dtype)
    L = q.shape[ax]

    def sl(a, b):
        s = [slice(None)] * q.ndim
        s[ax] = slice(a, b)
        return tuple(s)
    out[sl(2, L - 2)] = (q[sl(0, L - 4)] - 8.0 * q[sl(1, L - 3)] + 8.0 * q[sl(3, L - 1)] - q[sl(4, L)]) / (12.0 * h)
    return out


# ---------------------------------------------------------------------------
# viscous residual
# ---------------------------------------------------------------------------
def viscous_fluxes(th, tr, grid, U, terms=ALL_TERMS):
    """Point values of F_v (Eq. 2) at the faces of every active direction.
    U: padded state with every ghost cell filled (edges and corners included:
    the tangential derivatives at the face stencils' ghost columns read
    them).  Returns a dict d -> (Nv, faces...) over faces k = -1..n_d+1
    along d and the interior of the other axes."""
    ns = th.ns
    with np.errstate(all="ignore"):
        prim = primitives(th, U)
        mu, kappa, Dm = mixture_transport(th, tr, prim)
    rho, Y, u, T = prim["rho"], prim["Y"], prim["u"], prim["T"]
    h = (th.R * h_over_R(th, T))                      # (Z, Y, X, ns) J/kg
    iz, iy, ix = grid.interior()
    inner = [iz, iy, ix]
    # cell-centred velocity gradient G[a][b] = d u_b / d x_a (zero on inactive axes)
    G = [[None] * 3 for _ in range(3)]
    for a in range(3):
        for b in range(3):
            if grid.n[a] > 1:
                G[a][b] = cell_derivative(u[b], 2 - a, grid.d[a])
            else:
                G[a][b] = np.zeros_like(u[b])
    out = {}
    for d in grid.active():
        ax = 2 - d
        g, n, hd = grid.g(d), grid.n[d], grid.d[d]
        sel = list(inner)
        sel[ax] = slice(None)
        sel = tuple(sel)

        def F(q):                 # face value, transverse axes restricted to the interior
            return face_value(q, n, g, ax)[sel]

        def N(q):
            return face_normal_derivative(q, n, g, ax, hd)[sel]

        # velocity gradient at the faces: normal derivatives along d, the
        # interpolated cell-centred ones along the other axes
        Gf = [[None] * 3 for _ in range(3)]
        for a in range(3):
            for b in range(3):
                Gf[a][b] = N(u[b]) if a == d else F(G[a][b])
        div = Gf[0][0] + Gf[1][1] + Gf[2][2]
        muf, kf = F(mu), F(kappa)
        uf = [F(u[k]) for k in range(3)]
        Fv = np.zeros((ns + 4,) + div.shape)
        if terms & STRESS:
            for k in range(3):
                tau = muf * (Gf[k][d] + Gf[d][k])
                if k == d:
                    tau = tau - 2.0 / 3.0 * muf * div
                Fv[ns + k] = tau
                Fv[ns + 3] = Fv[ns + 3] + tau * uf[k]
        if terms & HEAT:
            Fv[ns + 3] = Fv[ns + 3] + kf * N(T)           # - q_c = kappa dT/dx_d
        if terms & DIFFUSION:
            rf = F(rho)
            Yf = [F(Y[..., s]) for s in range(ns)]
            Df = [F(Dm[..., s]) for s in range(ns)]
            dY = [N(Y[..., s]) for s in range(ns)]
            corr = 0.0
            for j in range(ns):
                corr = corr + Df[j] * dY[j]
            for s in range(ns):
                J = -rf * (Df[s] * dY[s] - Yf[s] * corr)     # Eq. 6
                Fv[s] = -J
                Fv[ns + 3] = Fv[ns + 3] - F(h[..., s]) * J   # - q_d = - sum_s h_s J_s
        out[d] = Fv
    return out


def numerical_flux(Fv, ax):
    """F^_{i+1/2} = (-F_{i-1/2} + 26 F_{i+1/2} - F_{i+3/2}) / 24 for faces
    k = 0..n from point fluxes at k = -1..n+1 along array axis ax"""
    L = Fv.shape[ax]

    def sl(a, b):
        s = [slice(None)] * Fv.ndim
        s[ax] = slice(a, b)
        return tuple(s)
    return (-Fv[sl(0, L - 2)] + 26.0 * Fv[sl(1, L - 1)] - Fv[sl(2, L)]) / 24.0


def viscous_rhs(th, tr, grid, U, terms=ALL_TERMS, return_aux=False):
    """Viscous part of the residual: + sum_d (F^_{i+1/2} - F^_{i-1/2}) / dx_d
    with the numerical flux F^ of the point fluxes F_v (Eq. 1 with F_v on the
    right-hand side), on the interior; ghosts zero.  aux["scale"]: per field
    max |F^| / min_d dx_d, the scale round-off of this residual is judged
    against."""
    nv = th.ns + 4
    out = np.zeros_like(U)
    iz, iy, ix = grid.interior()
    fmax = np.zeros(nv)
    fl = viscous_fluxes(th, tr, grid, U, terms)
    for d, Fv in fl.items():
        ax = 2 - d
        Fh = numerical_flux(Fv, ax + 1)
        out[(slice(None), iz, iy, ix)] += np.diff(Fh, axis=ax + 1) / grid.d[d]
        fmax = np.maximum(fmax, np.abs(Fh).reshape(nv, -1).max(axis=1))
    dmin = min([grid.d[d] for d in grid.active()] or [1.0])
    aux = {"scale": fmax / dmin, "fluxes": fl}
    return (out, aux) if return_aux else out
