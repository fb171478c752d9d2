"""Plain CPU oracle of the multicomponent convective right-hand side.

TEST INFRASTRUCTURE ONLY.  The tests, the smoke check and the CPU-baseline leg
of the benchmark import this module; the library's product path never does, and
this module imports nothing from the library.  It shares no code with the HIP
kernels: every formula here is written out independently from the paper
(XFluids, arXiv 2403.05910).

What it computes, in the paper's order and notation (Sec. II.C):
  * mixture ideal-gas EOS p = rho Rbar T                        (Sec. II.A, Eq. 7)
  * temperature from internal energy by Newton iteration        (Sec. II.C.3, Eq. 21)
  * per-face Roe-averaged eigensystem Lambda = L A R           (Sec. II.C.1, text of Eq. 13-15)
  * characteristic flux splitting F_m^pm = 1/2 L (F_m +- Lam U_m)  (Eq. 14)
  * WENO5-JS reconstruction and back-projection F^ = R (F+ + F-)   (Eq. 15)
    (or the scheme's other REC options: WENO-CU6, WENO7-JS)
  * conservative flux difference (F^_{i+1/2} - F^_{i-1/2}) / dx    (Eq. 13)
  * SSP-RK3 time march                                          (Eq. 16)
  * CFL time step lambda = dt/dx = CFL / Lambda                 (Eq. 17)
  * positivity-preserving blend of the face flux with the
    Lax-Friedrichs flux, for rho and the partial densities      (Sec. II.C.2, Eq. 17-20)

The arithmetic is deliberately plain: dense L and R matrices per face, dense
matrix-vector products, the three-division WENO form, no fusion or reordering.
All arrays are float64, or complex128 for complex-step differentiation; every
comparison (max, abs, bracket tests, convergence tests) acts on real parts, so a
complex-step derivative automatically holds the LLF wave speeds fixed.

Readings of points the paper leaves open (each is stated where it is used):
  * Roe average: sqrt(rho) weights on u, H, Y_s and T; the face sound speed is
    defined by the pressure-derivative identity so that L R = I exactly.
  * LLF: component-wise wave speed, the max over the stencil cells (six, or
    eight for WENO7) of the
    cell eigenvalue |u_n - c|, |u_n| or |u_n + c| of that characteristic field;
    ROE: |u~_n - c~|, |u~_n|, |u~_n + c~| of the face's Roe state; GLF: the
    largest LLF speed of the field over all faces of the direction.
  * Eigenbasis of the repeated eigenvalue u_n: partial-density waves
    d(rho_s) - Y_s dp / c^2 and the two tangential momentum waves.
  * Finite-difference point values (Shu-Osher flux splitting), cell centres at
    (i + 1/2) dx.
  * WENO5-JS with d = (1/10, 6/10, 3/10), p = 2, absolute eps = 1e-6;
    WENO-CU6 (the paper's other six-cell option) as stated at weno_cu6;
    WENO7-JS (eight-cell stencils, 4 ghost layers) as stated at weno7.
  * Eq. 21 calls C_v the constant-pressure heat capacity; it is the
    constant-volume one (C_v = sum Y_s C_p,s - Rbar, as the same equation says).
  * Eq. 17 writes U^{n+1} = U^n + lambda (F_{i+1/2} - F_{i-1/2}); the residual
    of Eq. 13 carries the opposite sign, which is the one used here.
  * Positivity preserving (Eq. 17-20; the limiting factor follows the cited
    method, which the paper does not restate): see positivity_limit.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

RU = 8.314462618  # universal gas constant, J/(mol K)

# status bits (the oracle's own copy; the library defines the same meanings)
FLAG_RHO = 1       # rho <= 0
FLAG_Y = 2         # Y_s < -1e-12
FLAG_P = 4         # p <= 0 or T <= 0
FLAG_TRANGE = 8    # T outside [T_lo, T_hi]
FLAG_NEWTON = 16   # Newton did not converge in NEWTON_MAXIT iterations
FLAG_C2 = 32       # face sound speed squared <= 0
FLAG_NAN = 64      # NaN or Inf

NEWTON_TOL = 1e-11
NEWTON_MAXIT = 50
WENO_EPS = 1e-6
BC_PERIODIC = 0
BC_OUTFLOW = 1


# ---------------------------------------------------------------------------
# grid and thermo descriptions
# ---------------------------------------------------------------------------
@dataclass
class Grid:
    """Uniform Cartesian grid with ng ghost layers in every active dimension
    (the block/halo layout of Sec. III.A, Fig. 3): 3 for the six-cell
    stencils of WENO5 and WENO-CU6, 4 for the eight-cell stencils of WENO7.
    bc = (-x,+x,-y,+y,-z,+z)."""
    nx: int
    ny: int
    nz: int
    dx: float
    dy: float
    dz: float
    bc: tuple = (0, 0, 0, 0, 0, 0)
    ng: int = 3

    @property
    def n(self):
        return (self.nx, self.ny, self.nz)

    @property
    def d(self):
        return (self.dx, self.dy, self.dz)

    def g(self, axis):
        """ghost width of spatial axis 0=x,1=y,2=z"""
        return self.ng if self.n[axis] > 1 else 0

    def active(self):
        return [a for a in range(3) if self.n[a] > 1]

    @property
    def padded(self):
        """array shape (z, y, x) of one padded field"""
        return tuple(self.n[a] + 2 * self.g(a) for a in (2, 1, 0))

    def interior(self):
        """slices (z, y, x) of the interior block of one padded field"""
        return tuple(slice(self.g(a), self.g(a) + self.n[a]) for a in (2, 1, 0))


@dataclass
class Thermo:
    """Per-species thermo: molar mass W_s (kg/mol) and the polynomial
    cp_s/R_s = a0 + a1 T + a2 T^2 + a3 T^3 + a4 T^4, with the enthalpy
    h_s/R_s = a0 T + a1 T^2/2 + a2 T^3/3 + a3 T^4/4 + a4 T^5/5 + a5 its integral
    (the NASA-polynomial form named after Eq. 12 and in Sec. II.C.3).  The
    Newton bracket is [T_lo, T_hi]; T_hi <= 0 means no bracket."""
    W: np.ndarray
    a: np.ndarray
    T_lo: float = 0.0
    T_hi: float = 0.0

    def __post_init__(self):
        self.W = np.asarray(self.W, dtype=np.float64)
        self.a = np.asarray(self.a, dtype=np.float64).reshape(len(self.W), 6)

    @property
    def ns(self):
        return len(self.W)

    @property
    def R(self):
        """specific gas constant of each species, R_s = R_u / W_s (Eq. 7)"""
        return RU / self.W

    @property
    def bracket(self):
        return self.T_hi > 0.0


# ---------------------------------------------------------------------------
# thermodynamics (Eq. 7 and Eq. 21)
# ---------------------------------------------------------------------------
def cp_over_R(th, T):
    """cp_s(T)/R_s for every species; T (...) -> (..., ns)"""
    a = th.a
    T = np.asarray(T)[..., None]
    return a[:, 0] + a[:, 1] * T + a[:, 2] * T**2 + a[:, 3] * T**3 + a[:, 4] * T**4


def h_over_R(th, T):
    """h_s(T)/R_s, the integral of cp_s/R_s plus the constant a5"""
    a = th.a
    T = np.asarray(T)[..., None]
    return (a[:, 0] * T + a[:, 1] * T**2 / 2 + a[:, 2] * T**3 / 3
            + a[:, 3] * T**4 / 4 + a[:, 4] * T**5 / 5 + a[:, 5])


def species_e(th, T):
    """species internal energy e_s = h_s - R_s T (Eq. 21); (..., ns)"""
    return th.R * (h_over_R(th, T) - np.asarray(T)[..., None])


def species_cv(th, T):
    """species constant-volume heat capacity C_v,s = C_p,s - R_s; (..., ns)"""
    return th.R * (cp_over_R(th, T) - 1.0)


def mixture_e(th, Y, T):
    """e(T) = sum_s Y_s e_s(T) (Eq. 21); Y (..., ns)"""
    return np.sum(Y * species_e(th, T), axis=-1)


def mixture_cv(th, Y, T):
    """C_v(T) = sum_s Y_s C_p,s(T) - Rbar (Eq. 21)"""
    return np.sum(Y * species_cv(th, T), axis=-1)


def mixture_R(th, Y):
    """Rbar = R_u sum_s Y_s / W_s (Eq. 7)"""
    return np.sum(Y * th.R, axis=-1)


def temperature_newton(th, Y, e):
    """Temperature from specific internal energy by Newton's method (Eq. 21).

    T^{k+1} = T^k + (e - e(T^k)) / C_v(T^k).  Cold start (no history):
    T^0 = e / C_v(T_ref), T_ref the bracket midpoint (or 1 K without bracket),
    clamped into the bracket.  Safeguard: e(T) is strictly increasing
    (C_v > 0), so every evaluation narrows the bracket [lo, hi] (e(T) > e moves
    hi down to T, otherwise lo up to T); a Newton step that leaves the closed
    bracket is replaced by bisection.  Stop when |dT| <= 1e-11 T and then
    apply one more Newton update; at most 50 iterations.

    Y (..., ns), e (...) -> (T (...), not_converged (...) bool)
    """
    Y = np.asarray(Y)
    e = np.asarray(e)
    T_ref = 0.5 * (th.T_lo + th.T_hi) if th.bracket else 1.0
    T = e / mixture_cv(th, Y, np.full(e.shape, T_ref))
    lo = np.full(e.shape, th.T_lo)
    hi = np.full(e.shape, th.T_hi)
    if th.bracket:
        T = np.where(T.real < th.T_lo, th.T_lo, np.where(T.real > th.T_hi, th.T_hi, T))
    active = np.ones(e.shape, dtype=bool)
    for _ in range(NEWTON_MAXIT):
        f = mixture_e(th, Y, T) - e
        cv = mixture_cv(th, Y, T)
        Tn = T - f / cv
        if th.bracket:
            hi = np.where(active & (f.real > 0), np.minimum(hi, T.real), hi)
            lo = np.where(active & (f.real <= 0), np.maximum(lo, T.real), lo)
            # a step that lands on a bracket end is kept: at the root f = 0
            # makes lo = T, and the converged step T -> T must not bisect
            outside = (Tn.real < lo) | (Tn.real > hi)
            Tn = np.where(outside, 0.5 * (lo + hi), Tn)
        conv = np.abs(Tn.real - T.real) <= NEWTON_TOL * np.abs(T.real)
        T = np.where(active, Tn, T)
        done = active & conv
        if done.any():
            Tp = T - (mixture_e(th, Y, T) - e) / mixture_cv(th, Y, T)
            T = np.where(done, Tp, T)
        active = active & ~conv
        if not active.any():
            break
    return T, active


def primitives(th, U):
    """Primitive state of every cell of U (Nv, ...): Eq. 7 and Eq. 21.

    Conservative fields in order rho Y_1..rho Y_N, rho u, rho v, rho w, rho E.
    Returns a dict with rho, Y (..., ns), u (3, ...), E, e, T, p, c, H, Rbar, cv
    and a status-bit array flags (...).
    """
    ns = th.ns
    rs = U[:ns]
    rho = np.sum(rs, axis=0)
    Y = np.moveaxis(rs / rho, 0, -1)
    u = U[ns:ns + 3] / rho
    E = U[ns + 3]
    e = E / rho - 0.5 * (u[0] ** 2 + u[1] ** 2 + u[2] ** 2)
    T, nonconv = temperature_newton(th, Y, e)
    Rbar = mixture_R(th, Y)
    cv = mixture_cv(th, Y, T)
    p = rho * Rbar * T
    c = np.sqrt((1.0 + Rbar / cv) * Rbar * T)
    H = (E + p) / rho
    flags = np.zeros(np.shape(rho), dtype=np.int64)
    flags |= np.where(rho.real <= 0, FLAG_RHO, 0)
    flags |= np.where(np.any(Y.real < -1e-12, axis=-1), FLAG_Y, 0)
    flags |= np.where((p.real <= 0) | (T.real <= 0), FLAG_P, 0)
    if th.bracket:
        flags |= np.where((T.real < th.T_lo) | (T.real > th.T_hi), FLAG_TRANGE, 0)
    flags |= np.where(nonconv, FLAG_NEWTON, 0)
    bad = ~np.isfinite(np.asarray(U).real).all(axis=0) | ~np.isfinite(T.real) | ~np.isfinite(c.real)
    flags |= np.where(bad, FLAG_NAN, 0)
    return dict(rho=rho, Y=Y, u=u, E=E, e=e, T=T, p=p, c=c, H=H, Rbar=Rbar, cv=cv, flags=flags)


def conservative(th, rho, u, T, Y):
    """U from rho, velocity (3, ...), T and Y (ns, ...): E = rho e(T) + rho|u|^2/2.
    A helper for building test states inside the oracle's own tests."""
    Yl = np.moveaxis(np.asarray(Y), 0, -1)
    e = mixture_e(th, Yl, T)
    E = rho * e + 0.5 * rho * (u[0] ** 2 + u[1] ** 2 + u[2] ** 2)
    return np.concatenate([rho * np.asarray(Y), rho * np.asarray(u), E[None]], axis=0)


# ---------------------------------------------------------------------------
# physical flux and eigensystem (Sec. II.C.1)
# ---------------------------------------------------------------------------
NORMALS = {0: (np.array([1.0, 0, 0]), np.array([0, 1.0, 0]), np.array([0, 0, 1.0])),
           1: (np.array([0, 1.0, 0]), np.array([1.0, 0, 0]), np.array([0, 0, 1.0])),
           2: (np.array([0, 0, 1.0]), np.array([1.0, 0, 0]), np.array([0, 1.0, 0]))}


def physical_flux(th, U, prim, d):
    """Convective flux of Eq. 2 in direction d: (rho_s u_n, m u_n + p n, (E+p) u_n)."""
    ns = th.ns
    n = NORMALS[d][0]
    un = prim["u"][d]
    F = np.empty_like(U)
    F[:ns] = U[:ns] * un
    for k in range(3):
        F[ns + k] = U[ns + k] * un + prim["p"] * n[k]
    F[ns + 3] = (U[ns + 3] + prim["p"]) * un
    return F


def roe_state(th, pL, pR):
    """Multicomponent Roe-averaged face state (Sec. II.C.1, the Roe treatment
    cited after Eq. 15).  Reading: sqrt(rho) weights w_L = sqrt(rho_L) /
    (sqrt(rho_L) + sqrt(rho_R)), w_R = 1 - w_L, applied to u, H, Y_s and T.
    Species thermo is taken at the averaged T:
        Gamma = Rbar / C_v,   chi_s = Gamma (|u|^2/2 - e_s) + R_s T,
        c^2   = sum_s Y_s chi_s + Gamma (H - |u|^2)
    (the last is the identity that pressure derivatives of p = sum rho_s R_s T
    satisfy; defining the face c^2 by it makes L R = I hold exactly)."""
    sL = np.sqrt(pL["rho"])
    sR = np.sqrt(pR["rho"])
    wL = sL / (sL + sR)
    wR = 1.0 - wL
    u = wL * pL["u"] + wR * pR["u"]
    H = wL * pL["H"] + wR * pR["H"]
    Y = wL[..., None] * pL["Y"] + wR[..., None] * pR["Y"]
    T = wL * pL["T"] + wR * pR["T"]
    es = species_e(th, T)
    Rbar = mixture_R(th, Y)
    cv = mixture_cv(th, Y, T)
    Gam = Rbar / cv
    q2 = u[0] ** 2 + u[1] ** 2 + u[2] ** 2
    chi = Gam[..., None] * (0.5 * q2[..., None] - es) + th.R * T[..., None]
    c2 = np.sum(Y * chi, axis=-1) + Gam * (H - q2)
    c = np.sqrt(c2)
    return dict(u=u, H=H, Y=Y, T=T, Gam=Gam, chi=chi, c2=c2, c=c, q2=q2)


def eigen_R(th, roe, d):
    """Right eigenvectors (columns) of the convective flux Jacobian in direction
    d at the Roe state; column order: u_n - c, species 1..N, tangent t1,
    tangent t2, u_n + c.  Component order rho_1..rho_N, m_x, m_y, m_z, E.
        r_-+ = (Y, u -+ c n, H -+ u_n c)
        r_s  = (e_s, u, |u|^2 - chi_s / Gamma)
        r_ta = (0, t_a, u . t_a)
    Returns (..., Nv, Nv)."""
    ns = th.ns
    nv = ns + 4
    n, t1, t2 = NORMALS[d]
    u, c, H, Y, Gam, chi, q2 = roe["u"], roe["c"], roe["H"], roe["Y"], roe["Gam"], roe["chi"], roe["q2"]
    shape = np.shape(c)
    R = np.zeros(shape + (nv, nv), dtype=np.result_type(c, u))
    un = n[0] * u[0] + n[1] * u[1] + n[2] * u[2]
    for col, sgn in ((0, -1.0), (nv - 1, 1.0)):
        R[..., :ns, col] = Y
        for k in range(3):
            R[..., ns + k, col] = u[k] + sgn * c * n[k]
        R[..., ns + 3, col] = H + sgn * un * c
    for s in range(ns):
        col = 1 + s
        R[..., s, col] = 1.0
        for k in range(3):
            R[..., ns + k, col] = u[k]
        R[..., ns + 3, col] = q2 - chi[..., s] / Gam
    for a, t in ((0, t1), (1, t2)):
        col = ns + 1 + a
        for k in range(3):
            R[..., ns + k, col] = t[k]
        R[..., ns + 3, col] = t[0] * u[0] + t[1] * u[1] + t[2] * u[2]
    return R


def eigen_L(th, roe, d):
    """Left eigenvectors (rows), same order as the columns of eigen_R.
    With sigma(v) = sum_s v_rho_s and dp(v) = sum_s chi_s v_rho_s - Gamma u.v_m
    + Gamma v_E (the pressure differential):
        l_-+ . v = [dp(v) -+ c (n.v_m - u_n sigma(v))] / (2 c^2)
        l_s  . v = v_rho_s - Y_s dp(v) / c^2
        l_ta . v = t_a . v_m - (u . t_a) sigma(v)
    Written out as a dense (..., Nv, Nv) matrix."""
    ns = th.ns
    nv = ns + 4
    n, t1, t2 = NORMALS[d]
    u, c, c2, Y, Gam, chi = roe["u"], roe["c"], roe["c2"], roe["Y"], roe["Gam"], roe["chi"]
    shape = np.shape(c)
    L = np.zeros(shape + (nv, nv), dtype=np.result_type(c, u))
    un = n[0] * u[0] + n[1] * u[1] + n[2] * u[2]
    # dp row coefficients
    dp = np.zeros(shape + (nv,), dtype=L.dtype)
    dp[..., :ns] = chi
    for k in range(3):
        dp[..., ns + k] = -Gam * u[k]
    dp[..., ns + 3] = Gam
    # (n . v_m - u_n sigma) row coefficients
    nm = np.zeros(shape + (nv,), dtype=L.dtype)
    nm[..., :ns] = -un[..., None]
    for k in range(3):
        nm[..., ns + k] = n[k]
    for row, sgn in ((0, -1.0), (nv - 1, 1.0)):
        L[..., row, :] = (dp + sgn * c[..., None] * nm) / (2.0 * c2[..., None])
    for s in range(ns):
        row = 1 + s
        L[..., row, :] = -Y[..., s, None] * dp / c2[..., None]
        L[..., row, s] += 1.0
    for a, t in ((0, t1), (1, t2)):
        row = ns + 1 + a
        ut = t[0] * u[0] + t[1] * u[1] + t[2] * u[2]
        L[..., row, :ns] = -ut[..., None]
        for k in range(3):
            L[..., row, ns + k] = t[k]
    return L


def eigenvalues(th, prim, d):
    """Cell eigenvalues per characteristic field: u_n - c, u_n (N + 2 times),
    u_n + c; returns (nv, ...)."""
    un = prim["u"][d]
    c = prim["c"]
    nv = th.ns + 4
    lam = [un - c] + [un] * (nv - 2) + [un + c]
    return np.stack(lam, axis=0)


# ---------------------------------------------------------------------------
# WENO5-JS (Eq. 15 with the fifth-order scheme it cites)
# ---------------------------------------------------------------------------
WENO_D = (0.1, 0.6, 0.3)


def weno5_candidates(a, b, c, d, e):
    """The three third-order candidate values q_k at the right edge of the cell
    holding c, from the sub-stencils (a,b,c), (b,c,d), (c,d,e)."""
    q0 = (2.0 * a - 7.0 * b + 11.0 * c) / 6.0
    q1 = (-b + 5.0 * c + 2.0 * d) / 6.0
    q2 = (2.0 * c + 5.0 * d - e) / 6.0
    return q0, q1, q2


def weno5_smoothness(a, b, c, d, e):
    """Jiang-Shu smoothness indicators beta_k of the three sub-stencils."""
    b0 = 13.0 / 12.0 * (a - 2.0 * b + c) ** 2 + 0.25 * (a - 4.0 * b + 3.0 * c) ** 2
    b1 = 13.0 / 12.0 * (b - 2.0 * c + d) ** 2 + 0.25 * (b - d) ** 2
    b2 = 13.0 / 12.0 * (c - 2.0 * d + e) ** 2 + 0.25 * (3.0 * c - 4.0 * d + e) ** 2
    return b0, b1, b2


def weno5(a, b, c, d, e):
    """Fifth-order WENO-JS value at the right edge of the cell holding c, from
    the five point values a..e (the fifth-order scheme REC of Eq. 15):
    alpha_k = d_k / (eps + beta_k)^2 with linear weights d = (1/10, 6/10, 3/10)
    and absolute eps = 1e-6; result sum_k alpha_k q_k / sum_k alpha_k, written
    in the plain three-division form."""
    q = weno5_candidates(a, b, c, d, e)
    beta = weno5_smoothness(a, b, c, d, e)
    al = [WENO_D[k] / (WENO_EPS + beta[k]) ** 2 for k in range(3)]
    s = al[0] + al[1] + al[2]
    return (al[0] / s) * q[0] + (al[1] / s) * q[1] + (al[2] / s) * q[2]


# ---------------------------------------------------------------------------
# WENO-CU6: the central-upwind sixth-order WENO the paper offers as REC in
# Eq. 15 (its reference [34]; the paper restates none of its formulas)
# ---------------------------------------------------------------------------
CU6_D = (1.0 / 20.0, 9.0 / 20.0, 9.0 / 20.0, 1.0 / 20.0)
CU6_C = 20.0
CU6_EPS = 1e-6


def smoothness_parts(offsets):
    """Pieces of the Jiang-Shu smoothness indicator
    beta = sum_{l >= 1} dx^(2l-1) int_{cell i} (p^(l))^2 dx of the polynomial p
    whose averages over the cells at `offsets` (relative to cell i, dx = 1)
    are the data f: for l = 1..n-1 the matrix D_l giving the coefficients of
    p^(l) from f and the Gram matrix G_l of the monomials on [-1/2, 1/2], so
    beta = sum_l (D_l f)^T G_l (D_l f).  Built in floating point from the
    cell-average moment matrix and exact monomial integrals."""
    n = len(offsets)
    A = np.array([[((c + 0.5) ** (k + 1) - (c - 0.5) ** (k + 1)) / (k + 1) for k in range(n)] for c in offsets])
    D = np.linalg.solve(A, np.eye(n))          # polynomial coefficients = D @ f
    parts = []
    for _ in range(1, n):
        D = np.array([k * D[k] for k in range(1, D.shape[0])])     # coefficients of the next derivative
        m = D.shape[0]
        G = np.array([[(0.5 ** (i + j + 1) - (-0.5) ** (i + j + 1)) / (i + j + 1) for j in range(m)]
                      for i in range(m)])
        parts.append((D, G))
    return parts


def smoothness_form(offsets):
    """the same indicator as one quadratic form: beta = f^T B f"""
    return sum(D.T @ G @ D for D, G in smoothness_parts(offsets))


CU6_PARTS = smoothness_parts(range(-2, 4))
CU6_B6 = smoothness_form(range(-2, 4))


def smoothness_gram(parts, w):
    """sum over the parts (D_l, G_l) of (D_l w)^T G_l (D_l w) for values w
    (n, ...): the indicator as a sum of positive Gram forms"""
    out = 0.0
    for D, G in parts:
        Dw = np.einsum("kj,j...->k...", D, w)
        out = out + np.einsum("k...,kj,j...->...", Dw, G, Dw)
    return out


def smoothness6(v):
    """beta of the six-cell quintic for values v (6, ...): the data are first
    shifted by the centre value (beta ignores constants), then the positive
    Gram forms of the derivatives are summed, so no large terms cancel"""
    return smoothness_gram(CU6_PARTS, v - v[2])


def weno_cu6(a, b, c, d, e, f):
    """Sixth-order central-upwind WENO value at the right edge of the cell
    holding c, from the six point values a..f (cells i-2..i+3).  Reading of
    the cited scheme: the three WENO5 candidates plus the downwind candidate
    of (d, e, f); linear weights (1, 9, 9, 1)/20, which give the sixth-order
    central value; smoothness beta_0..2 of the three upwind sub-stencils and
    beta_6 of the whole stencil for the downwind one;
    tau_6 = beta_6 - (beta_0 + 4 beta_1 + beta_2)/6;
    alpha_k = d_k (C + tau_6 / (beta_k + eps)), C = 20, eps = 1e-6 absolute
    (as in the WENO5 reading: with a vanishing eps a sub-stencil that is flat
    to round-off takes all the weight, which drops the scheme to third order
    on a smooth entropy wave, and 1e-40 also underflows in FP32);
    result sum_k alpha_k q_k / sum_k alpha_k."""
    q0, q1, q2 = weno5_candidates(a, b, c, d, e)
    q3 = (11.0 * d - 7.0 * e + 2.0 * f) / 6.0
    b0, b1, b2 = weno5_smoothness(a, b, c, d, e)
    b6 = smoothness6(np.stack(np.broadcast_arrays(a, b, c, d, e, f), axis=0))
    tau = b6 - (b0 + 4.0 * b1 + b2) / 6.0
    al = [CU6_D[k] * (CU6_C + tau / (bk + CU6_EPS)) for k, bk in enumerate((b0, b1, b2, b6))]
    s = al[0] + al[1] + al[2] + al[3]
    return (al[0] / s) * q0 + (al[1] / s) * q1 + (al[2] / s) * q2 + (al[3] / s) * q3


# ---------------------------------------------------------------------------
# WENO7: the seventh-order WENO-JS the paper also offers as REC in Eq. 15
# (Balsara and Shu's extension of the Jiang-Shu weights to four cubic
# sub-stencils; the paper restates none of its formulas)
# ---------------------------------------------------------------------------
WENO7_D = (1.0 / 35.0, 12.0 / 35.0, 18.0 / 35.0, 4.0 / 35.0)
WENO7_PARTS = [smoothness_parts(range(k - 3, k + 1)) for k in range(4)]


def weno7_candidates(a, b, c, d, e, f, g):
    """The four fourth-order candidate values at the right edge of the cell
    holding d (cell i), from the sub-stencils of cells i-3..i, i-2..i+1,
    i-1..i+2 and i..i+3: the value at x_{i+1/2} of the cubic whose cell
    averages are the data."""
    q0 = (-3.0 * a + 13.0 * b - 23.0 * c + 25.0 * d) / 12.0
    q1 = (b - 5.0 * c + 13.0 * d + 3.0 * e) / 12.0
    q2 = (-c + 7.0 * d + 7.0 * e - f) / 12.0
    q3 = (3.0 * d + 13.0 * e - 5.0 * f + g) / 12.0
    return q0, q1, q2, q3


def weno7_smoothness(a, b, c, d, e, f, g):
    """Jiang-Shu indicators of the four cubic sub-stencils (the integral
    definition, as positive Gram forms of data shifted by the value of cell i,
    which lies in every sub-stencil)"""
    v = np.stack(np.broadcast_arrays(a, b, c, d, e, f, g), axis=0)
    w = v - v[3]
    return tuple(smoothness_gram(WENO7_PARTS[k], w[k:k + 4]) for k in range(4))


def weno7(a, b, c, d, e, f, g):
    """Seventh-order WENO-JS value at the right edge of the cell holding d,
    from the seven point values a..g (cells i-3..i+3): alpha_k = d_k /
    (eps + beta_k)^2 with linear weights (1, 12, 18, 4)/35, which combine the
    four candidates into the seven-cell value, and absolute eps = 1e-6 as in
    the WENO5 reading; result sum_k alpha_k q_k / sum_k alpha_k."""
    q = weno7_candidates(a, b, c, d, e, f, g)
    beta = weno7_smoothness(a, b, c, d, e, f, g)
    al = [WENO7_D[k] / (WENO_EPS + beta[k]) ** 2 for k in range(4)]
    s = al[0] + al[1] + al[2] + al[3]
    return (al[0] / s) * q[0] + (al[1] / s) * q[1] + (al[2] / s) * q[2] + (al[3] / s) * q[3]


RECON_TYPES = ("WENO5", "CU6", "WENO7")


def stencil_radius(recon):
    """half width of the stencil of one face: 3 (six cells i-2..i+3) for
    WENO5 and WENO-CU6, 4 (eight cells i-3..i+4) for WENO7"""
    return 4 if recon == "WENO7" else 3


# ---------------------------------------------------------------------------
# face flux (Eq. 14-15) and right-hand side (Eq. 13)
# ---------------------------------------------------------------------------
def _take(prim, idx):
    """primitive dict restricted to stencil slot idx (leading axis)"""
    out = {}
    for k, v in prim.items():
        if k == "u":
            out[k] = v[:, idx]
        else:
            out[k] = v[idx]
    return out


VISC_TYPES = ("LLF", "ROE", "GLF")


def face_flux(th, d, Ust, Pst, alpha=None, visc="LLF", recon="WENO5"):
    """Numerical flux at faces i+1/2 from the stencils of 2r cells
    m = i-r+1..i+r (r = stencil_radius(recon): six cells i-2..i+3 for WENO5
    and CU6, eight cells i-3..i+4 for WENO7).

    Ust: (Nv, 2r, F) conservative values of the stencil cells (slot r-1 =
    cell i, slot r = cell i+1); Pst: primitives of the same cells (values
    (2r, F); u (3, 2r, F); Y (2r, F, ns)).  alpha, if given, is the (Nv, F) array of
    wave speeds to use instead of computing them (a frozen dissipation; the
    global GLF speeds arrive this way).  visc: the artificial viscosity of
    Eq. 14 (Table I): "LLF" as below, or "ROE", |lambda_n| of the face's Roe
    state (u~_n - c~, u~_n, u~_n + c~), no entropy fix.
    Returns (Fhat (Nv, F), alpha (Nv, F), c2 of the Roe state (F,)).

    Steps: Roe state of cells i, i+1; dense L, R; component-wise LLF speed
    alpha_n = max_m |lambda_n(U_m)| over the stencil's cells; F_m^pm = 1/2 L
    (F_m +- alpha U_m) (Eq. 14); plus side from the 2r - 1 cells m <= i+r-1,
    minus side mirrored from m = i+r..i-r+2; Fhat = R (F^+ + F^-) (Eq. 15)."""
    nv = th.ns + 4
    r = stencil_radius(recon)
    assert Ust.shape[1] == 2 * r, (Ust.shape, recon)
    pL = _take(Pst, r - 1)
    pR = _take(Pst, r)
    roe = roe_state(th, pL, pR)
    L = eigen_L(th, roe, d)          # (F, nv, nv)
    R = eigen_R(th, roe, d)
    if alpha is None and visc == "ROE":
        un, c = roe["u"][d], roe["c"]
        alpha = np.abs(np.stack([un - c] + [un] * (nv - 2) + [un + c], axis=0).real)
    elif alpha is None:
        lam = eigenvalues(th, Pst, d)            # (nv, 2r, F)
        alpha = np.max(np.abs(lam.real), axis=1)  # (nv, F)
    Fm = physical_flux(th, Ust, Pst, d)          # (nv, 2r, F)
    # characteristic projections, dense: f[m, F, n] = sum_j L[F, n, j] Fm[j, m, F]
    f = np.einsum("Fnj,jmF->mFn", L, Fm)
    v = np.einsum("Fnj,jmF->mFn", L, Ust)
    al = alpha.T                                 # (F, nv)
    gp = 0.5 * (f + al * v)
    gm = 0.5 * (f - al * v)
    if recon == "CU6":
        hp = weno_cu6(gp[0], gp[1], gp[2], gp[3], gp[4], gp[5])
        hm = weno_cu6(gm[5], gm[4], gm[3], gm[2], gm[1], gm[0])
    elif recon == "WENO7":
        hp = weno7(gp[0], gp[1], gp[2], gp[3], gp[4], gp[5], gp[6])
        hm = weno7(gm[7], gm[6], gm[5], gm[4], gm[3], gm[2], gm[1])
    else:
        hp = weno5(gp[0], gp[1], gp[2], gp[3], gp[4])
        hm = weno5(gm[5], gm[4], gm[3], gm[2], gm[1])
    Fhat = np.einsum("Fjn,Fn->jF", R, hp + hm)
    return Fhat, alpha, roe["c2"]


# ---------------------------------------------------------------------------
# Positivity-preserving flux blend (Sec. II.C.2, Eq. 17-20)
# ---------------------------------------------------------------------------
PP_RHO_FLOOR = 1e-13   # total density floor, relative to min(rho_L, rho_R)
PP_Y_FLOOR = 1e-13     # partial densities may reach -1e-13 rho of their own cell


def lax_friedrichs_flux(th, d, Ust, Pst, lf):
    """Eq. 19 at faces i+1/2: 1/2 [F(U_i) + F(U_i+1) + lf (U_i - U_i+1)],
    U_i, U_i+1 the stencil's two middle slots; lf (F,) the dissipation
    coefficient."""
    Fm = physical_flux(th, Ust, Pst, d)
    r = Ust.shape[1] // 2
    return 0.5 * (Fm[:, r - 1] + Fm[:, r] + lf * (Ust[:, r - 1] - Ust[:, r]))


def positivity_limit(th, d, Ust, Pst, Fhat, alpha, lam):
    """Blend F* = F^LF + theta (F^ - F^LF) of Eq. 20 at faces i+1/2.

    Eq. 18 writes the Euler update of cell i as the mean of the half-step
    states U_i - 2 lam F_{i+1/2} and U_i + 2 lam F_{i-1/2}.  Readings (the
    paper defers the limiting factor to the method it cites):
      * the components kept positive are the total density and every partial
        density rho_s (the paper extends the density limiter to the mass
        fractions): floors 1e-13 min(rho_i, rho_i+1) for rho and
        -1e-13 rho of the half-state's own cell for rho_s (a vanishing species
        tolerates round-off of that size; the new state, a mean of half-states,
        then keeps Y_s above -1e-12);
      * the Lax-Friedrichs coefficient of Eq. 19 is the face's largest LLF
        wave speed, i.e. the larger acoustic one;
      * in D active dimensions the update is the mean of D one-dimensional
        updates with lam = D dt / dx_d each (lam is passed in);
      * per face and component, theta is the largest value in [0, 1] for which
        the half-states of both neighbouring cells stay at or above the floor;
        the face's theta is the minimum over components and both cells, and
        theta = 1 leaves F^ untouched.
    Ust (Nv, 2r, F), Pst as in face_flux; Fhat (Nv, F); alpha (Nv, F) the
    face's LLF speeds (rows u-c, ..., u+c); lam a scalar.
    Returns (Fstar (Nv, F), theta (F,))."""
    ns = th.ns
    lf = np.maximum(alpha[0].real, alpha[-1].real)
    FLF = lax_friedrichs_flux(th, d, Ust, Pst, lf)

    def comps(V):                      # rows: rho, rho_1 .. rho_ns
        return np.concatenate([V[:ns].sum(axis=0, keepdims=True), V[:ns]], axis=0)

    r = Ust.shape[1] // 2
    qL, qR = comps(Ust[:, r - 1]), comps(Ust[:, r])
    qH, qLF = comps(Fhat), comps(FLF)
    rhoL, rhoR = qL[0].real, qR[0].real
    floor_rho = PP_RHO_FLOOR * np.minimum(rhoL, rhoR)
    epsL = np.concatenate([floor_rho[None], np.broadcast_to(-PP_Y_FLOOR * rhoL, (ns,) + rhoL.shape)], axis=0)
    epsR = np.concatenate([floor_rho[None], np.broadcast_to(-PP_Y_FLOOR * rhoR, (ns,) + rhoR.shape)], axis=0)
    theta = np.ones(Fhat.shape[1])
    for q0, sgn, eps in ((qL, -1.0, epsL), (qR, 1.0, epsR)):
        w_hi = (q0 + sgn * 2.0 * lam * qH).real          # half-state with the high-order flux
        w_lo = (q0 + sgn * 2.0 * lam * qLF).real         # ... with the Lax-Friedrichs flux
        gap = w_lo - w_hi
        with np.errstate(all="ignore"):
            t = np.where(w_hi >= eps, 1.0, np.where(gap > 0, (w_lo - eps) / gap, 0.0))
        theta = np.minimum(theta, np.clip(t, 0.0, 1.0).min(axis=0))
    Fstar = np.where(theta == 1.0, Fhat, FLF + theta * (Fhat - FLF))
    return Fstar, theta


def _stencils(Q, axis, g, n, r=3):
    """the 2r stencil slices along `axis` for faces k = 0..n (face k lies
    between padded cells g+k-1 and g+k; slot m holds cell g+k-r+m)"""
    return np.stack([np.take(Q, np.arange(g - r + m, g - r + m + n + 1), axis=axis) for m in range(2 * r)],
                    axis=0)


def rhs(th, grid, U, alpha=None, return_aux=False, pp_dt=None, visc="LLF", recon="WENO5"):
    """Convective residual L(U) = -sum_d (F^_{i+1/2} - F^_{i-1/2}) / dx_d
    (Eq. 13) on the interior of the padded state U (Nv, Z, Y, X); ghost cells
    of U must already hold their boundary values; ghost cells of the result are
    zero.  alpha, if given, is a dict d -> frozen LLF speeds (Nv, faces).
    pp_dt, if given, is the time step of the Euler stage the residual is used
    in: the face fluxes are then blended by positivity_limit with
    lam = D pp_dt / dx_d (D active dimensions).  visc: "LLF", "ROE" or "GLF"
    (Table I).  Reading of GLF: per direction and characteristic field, the
    largest LLF speed over all faces of that direction (the device-wide
    maximum the paper reduces across processes).  recon: "WENO5" (WENO5-JS
    on the five cells of each side), "CU6" (WENO-CU6 on all six) or "WENO7"
    (WENO7-JS on seven of eight cells; needs a grid with 4 ghost layers)."""
    assert visc in VISC_TYPES, visc
    assert recon in RECON_TYPES, recon
    r = stencil_radius(recon)
    assert grid.ng >= r, (grid.ng, recon)
    nv = th.ns + 4
    assert U.shape == (nv,) + grid.padded, (U.shape, grid.padded)
    with np.errstate(all="ignore"):
        prim = primitives(th, U)
    out = np.zeros_like(U)
    iz, iy, ix = grid.interior()
    aux = {"alpha": {}, "flags": 0, "fmax": np.zeros(nv)}
    flags = np.zeros(grid.padded, dtype=np.int64)
    # flags only from cells the stencils read (interior + face ghost slabs)
    read = np.zeros(grid.padded, dtype=bool)
    for d in grid.active():
        sl = [iz, iy, ix]
        sl[2 - d] = slice(None)
        read[tuple(sl)] = True
    if not grid.active():
        read[iz, iy, ix] = True
    flags = np.where(read, prim["flags"], 0)
    aux_flags = int(np.bitwise_or.reduce(flags.ravel())) if flags.size else 0
    for d in grid.active():
        ax = 2 - d                    # array axis of spatial direction d in (z, y, x)
        g = grid.g(d)
        n = grid.n[d]
        # restrict the transverse axes to the interior, keep the sweep axis whole
        sl = [iz, iy, ix]
        sl[ax] = slice(None)
        sl = tuple(sl)
        Ud = U[(slice(None),) + sl]
        Pd = {}
        for k, v in prim.items():
            if k == "flags":
                continue
            if k == "u":
                Pd[k] = v[(slice(None),) + sl]
            elif k == "Y":
                Pd[k] = v[sl + (slice(None),)]
            else:
                Pd[k] = v[sl]
        # stencils: (2r, ...) with the face index along the sweep axis
        W = 2 * r
        Ust = _stencils(Ud, ax + 1, g, n, r)            # (2r, nv, z', y', x'')
        tshape = Ust.shape[2:]
        nf = int(np.prod(tshape))
        Ust = np.moveaxis(Ust, 0, 1).reshape(nv, W, nf)
        Pst = {}
        for k, v in Pd.items():
            if k == "u":
                s = _stencils(v, ax + 1, g, n, r)       # (2r, 3, ...)
                Pst[k] = np.moveaxis(s, 0, 1).reshape(3, W, nf)
            elif k == "Y":
                s = _stencils(v, ax, g, n, r)           # (2r, ..., ns)
                Pst[k] = s.reshape(W, nf, th.ns)
            else:
                s = _stencils(v, ax, g, n, r)
                Pst[k] = s.reshape(W, nf)
        a_in = None if alpha is None else alpha[d]
        if a_in is None and visc == "GLF":
            lam_c = eigenvalues(th, Pst, d)                           # (nv, 2r, F)
            glf = np.max(np.abs(lam_c.real), axis=(1, 2))             # (nv,)
            a_in = np.broadcast_to(glf[:, None], (nv, nf)).copy()
        with np.errstate(all="ignore"):
            Fh, al, c2 = face_flux(th, d, Ust, Pst, a_in, visc, recon)
        aux["alpha"][d] = al
        if pp_dt is not None:
            lam = len(grid.active()) * pp_dt / grid.d[d]
            # the Lax-Friedrichs coefficient stays the LLF speed whatever the
            # splitting's viscosity (Eq. 19 is positive only with a bound on
            # the neighbouring cells' wave speeds)
            al_lf = al if (visc == "LLF" and a_in is None) else np.max(np.abs(eigenvalues(th, Pst, d).real), axis=1)
            with np.errstate(all="ignore"):
                Fh, theta = positivity_limit(th, d, Ust, Pst, Fh, al_lf, lam)
            aux.setdefault("theta", {})[d] = theta
        aux["fmax"] = np.maximum(aux["fmax"], np.max(np.abs(Fh.real), axis=1))
        if np.any(c2.real <= 0):
            aux_flags |= FLAG_C2
        Fh = Fh.reshape((nv,) + tshape)
        dF = np.diff(Fh, axis=ax + 1)                    # F_{i+1/2} - F_{i-1/2}
        out[(slice(None), iz, iy, ix)] -= dF / grid.d[d]
    if not np.all(np.isfinite(out.real)):
        aux_flags |= FLAG_NAN
    aux["flags"] = aux_flags
    # per-field flux-divergence scale S_f = max |F^_f| / min_d dx_d (the scale
    # against which round-off of this residual is judged), and the same with
    # a floor at the size of the LLF dissipation term, max_i (|u| + c)_i |U_f,i|
    # (a field whose flux vanishes, e.g. a species at rest, still carries
    # round-off of that size)
    dmin = min([grid.d[d] for d in grid.active()] or [1.0])
    aux["scale"] = aux["fmax"] / dmin
    aux["scale_llf"] = np.maximum(aux["fmax"], dissipation_scale(th, grid, U, prim)) / dmin
    return (out, aux) if return_aux else out


def dissipation_scale(th, grid, U, prim=None):
    """per field, max over interior cells of (max_d |u_d| + c) |U_f|"""
    iz, iy, ix = grid.interior()
    if prim is None:
        with np.errstate(all="ignore"):
            prim = primitives(th, U)
    lam = prim["c"].real.copy()
    lam = lam + np.max(np.abs(prim["u"].real), axis=0)
    v = lam[None] * np.abs(U.real)
    return v[:, iz, iy, ix].reshape(U.shape[0], -1).max(axis=1)


def rhs_at(th, grid, U, cells, return_fmax=False, recon="WENO5"):
    """L(U) at selected interior cells only.  cells: (K, 3) integer array of
    interior indices (i, j, k) = (x, y, z).  Computes the two faces of each
    cell in every active direction from their own stencils (LLF speeds).
    Returns (Nv, K) and, with return_fmax, the per-field max |F^| over those
    faces."""
    r = stencil_radius(recon)
    assert grid.ng >= r, (grid.ng, recon)
    cells = np.asarray(cells, dtype=np.int64).reshape(-1, 3)
    nv = th.ns + 4
    K = len(cells)
    out = np.zeros((nv, K))
    fmax = np.zeros(nv)
    gx, gy, gz = grid.g(0), grid.g(1), grid.g(2)
    pz, py, px = cells[:, 2] + gz, cells[:, 1] + gy, cells[:, 0] + gx
    for d in grid.active():
        unit = np.zeros(3, dtype=np.int64)
        unit[d] = 1
        fl = []
        for side in (0, 1):                      # face i-1/2, then i+1/2
            idx = []
            for m in range(2 * r):
                off = side - r + m               # stencil of face between cells (side-1) and side
                idx.append((pz + off * unit[2], py + off * unit[1], px + off * unit[0]))
            Ust = np.stack([U[:, z, y, x] for (z, y, x) in idx], axis=1)   # (nv, 2r, K)
            with np.errstate(all="ignore"):
                P = primitives(th, Ust)
            Pst = {k: v for k, v in P.items() if k != "flags"}
            with np.errstate(all="ignore"):
                Fh, _, _ = face_flux(th, d, Ust, Pst, recon=recon)
            fl.append(Fh)
            fmax = np.maximum(fmax, np.max(np.abs(Fh.real), axis=1))
        out -= (fl[1] - fl[0]) / grid.d[d]
    return (out, fmax) if return_fmax else out


# ---------------------------------------------------------------------------
# boundary ghosts, CFL and SSP-RK3
# ---------------------------------------------------------------------------
def fill_ghosts(grid, U):
    """Fill the ghost layers of every active side (boundary conditions of Sec. III.B.4):
    periodic = wrap-around copy of the opposite interior layers; outflow =
    zero-gradient copy of the nearest interior cell.  Dimensions are filled in
    the order x, y, z over the whole padded extent of the other axes, so edge
    and corner ghosts end up consistent as well.  Returns a new array."""
    U = np.array(U, copy=True)
    for d in grid.active():
        ax = 3 - d                     # array axis of direction d in (nv, z, y, x)
        g, n = grid.g(d), grid.n[d]
        for side in (0, 1):
            bc = grid.bc[2 * d + side]
            for layer in range(g):
                if side == 0:
                    dst = layer
                    src = (n + layer) if bc == BC_PERIODIC else g
                else:
                    dst = g + n + layer
                    src = (g + layer) if bc == BC_PERIODIC else g + n - 1
                sd = [slice(None)] * 4
                ss = [slice(None)] * 4
                sd[ax] = dst
                ss[ax] = src
                U[tuple(sd)] = U[tuple(ss)]
    return U


def cfl_dt(th, grid, U, cfl):
    """dt = CFL / max_i sum_{d active} (|u_d| + c)_i / dx_d over interior cells
    (Eq. 17 read per direction and summed for a multidimensional grid)."""
    with np.errstate(all="ignore"):
        prim = primitives(th, U)
    iz, iy, ix = grid.interior()
    s = 0.0
    for d in grid.active():
        s = s + (np.abs(prim["u"][d].real) + prim["c"].real) / grid.d[d]
    return cfl / np.max(s[iz, iy, ix])


def ssp_rk3(L, U, dt):
    """One SSP-RK3 step of dU/dt = L(U) (Eq. 16):
    U1 = U + dt L(U); U2 = 3/4 U + 1/4 (U1 + dt L(U1));
    U^{n+1} = 1/3 U + 2/3 (U2 + dt L(U2))."""
    U1 = U + dt * L(U)
    U2 = 0.75 * U + 0.25 * (U1 + dt * L(U1))
    return U / 3.0 + 2.0 / 3.0 * (U2 + dt * L(U2))


def rk3_step(th, grid, U, dt, alpha=None, pp=False, visc="LLF", recon="WENO5", transport=None,
             viscous_terms=7, mechanism=None, n_sub=1, splitting="strang"):
    """One SSP-RK3 step of the convective system with ghosts refilled before
    every stage.  alpha: optional list of three frozen-speed dicts, one per
    stage (in stage order).  pp: blend every stage's face fluxes for
    positivity (each SSP-RK3 stage is a convex combination of Euler steps of
    size dt).  transport: an xf_viscous.Transport to add the viscous and
    diffusive fluxes (Eq. 1-6; the terms selected by viscous_terms) to every
    stage's residual.  mechanism: an xf_reaction.Mechanism to split the
    reaction source off the flow step (Sec. II.C.4): "strang" takes
    R(dt/2) F(dt) R(dt/2), "lie" F(dt) R(dt), each R with n_sub alpha-QSS
    sub-steps."""
    if mechanism is not None:
        from .xf_reaction import react
        U0 = fill_ghosts(grid, U)
        if splitting == "strang":
            U0 = fill_ghosts(grid, react(th, mechanism, grid, U0, 0.5 * dt, n_sub))
        flow = rk3_step(th, grid, U0, dt, alpha, pp, visc, recon, transport, viscous_terms)
        return fill_ghosts(grid, react(th, mechanism, grid, flow, dt if splitting == "lie" else 0.5 * dt, n_sub))
    a = list(alpha) if alpha is not None else [None, None, None]
    stage = [0]

    def L(V):
        V = fill_ghosts(grid, V)
        r = rhs(th, grid, V, a[stage[0]], pp_dt=dt if pp else None, visc=visc, recon=recon)
        if transport is not None:
            from .xf_viscous import viscous_rhs
            r = r + viscous_rhs(th, transport, grid, V, viscous_terms)
        stage[0] += 1
        return r

    return fill_ghosts(grid, ssp_rk3(L, fill_ghosts(grid, U), dt))
