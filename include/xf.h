/*
 * xf.h -- C ABI of libxf.so: the convective right-hand side of the
 * multicomponent compressible Euler/Navier-Stokes system of XFluids
 * (arXiv 2403.05910), hand-written HIP for gfx950 (MI355X).
 *
 * What the library computes (paper section / equation):
 *   state U = (rho Y_1..rho Y_N, rho u, rho v, rho w, rho E)   Sec. II.A, Eq. 1-2
 *   mixture EOS p = rho Rbar T                                  Eq. 7
 *   T from internal energy by Newton iteration                  Sec. II.C.3, Eq. 21
 *   Roe-averaged characteristic projection, LLF splitting       Sec. II.C.1, Eq. 14
 *   WENO5-JS reconstruction, back-projection                    Eq. 15
 *   flux difference L(U) = -sum_d (F^_{i+1/2} - F^_{i-1/2})/dx_d  Eq. 13
 *   SSP-RK3 update                                              Eq. 16
 *   CFL time step                                               Eq. 17
 * plus a hand-written vector-Jacobian product of the right-hand side (the
 * LLF wave speeds held fixed), which the paper does not have.
 *
 * Layout.  Every state-shaped buffer is FP64, structure of arrays,
 * field-major: [Nv][Z][Y][X] with x fastest, Nv = N + 4.  Each dimension with
 * n_d > 1 is active and carries 3 ghost layers on both sides
 * (X = nx + 6, ...); an inactive dimension (n_d == 1) has no ghosts and no
 * flux.  Cell (i, j, k) of the interior sits at padded (i+gx, j+gy, k+gz).
 * Ghost layers follow the block/halo layout of Sec. III.A (Fig. 3).
 *
 * Ownership.  The caller owns every device buffer (state, rhs, cotangents,
 * workspace).  The library allocates device memory only inside xf_create (a
 * status word); no call after that allocates device memory (HIP events for
 * the optional per-kernel timing are created only while timing is enabled).
 * Workspace sizes come from
 * xf_workspace_bytes; workspace contents need not be initialised and are not
 * preserved between calls.
 *
 * Streams.  `stream` is a hipStream_t passed as void*; NULL means the null
 * stream.  Every call except xf_create, xf_destroy and xf_status is
 * asynchronous on that stream and never synchronises the host.
 *
 * Errors (the error catching of Sec. III.B.6: the solver detects
 * non-physical states and stops with a report instead of running on).
 * Functions return an int status: XF_OK (0) or a negative code.
 * Argument errors are detected on the host before anything is enqueued.
 * Non-physical states met by the kernels (rho <= 0, p <= 0, T out of its
 * bracket, Newton not converged, Roe c^2 <= 0, NaN) set bits in a device
 * status word that xf_status reads (and clears); the kernels never trap.
 * Kernel launch failures return XF_EDEVICE.
 */
#ifndef XF_H
#define XF_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct xf_ctx xf_ctx;

enum {
    XF_OK = 0,
    XF_EINVAL = -1,        /* bad argument (null pointer, size, enum value)       */
    XF_EDEVICE = -2,       /* HIP runtime error (launch, copy, no device)          */
    XF_ENOMEM = -3,        /* allocation inside xf_create failed                  */
    XF_ENONPHYS = -4,      /* xf_status: a non-physical state was flagged          */
    XF_EUNSUPPORTED = -5,  /* valid request this build does not provide (e.g. N)  */
    XF_ETOOLARGE = -6      /* xf_rhs_noalloc: workspace exceeds XF_NOALLOC_BYTES   */
};

enum { XF_BC_PERIODIC = 0, XF_BC_OUTFLOW = 1 };
enum { XF_PREC_FP64 = 0, XF_PREC_MIXED = 1 };
enum { XF_OP_RHS = 0, XF_OP_RK3 = 1, XF_OP_VJP = 2, XF_OP_RK3_VJP = 3 };

/* status-word bits (xf_status) */
enum {
    XF_FLAG_RHO = 1,       /* rho <= 0 in a cell the stencils read               */
    XF_FLAG_Y = 2,         /* some Y_s < -1e-12                                  */
    XF_FLAG_P = 4,         /* p <= 0 or T <= 0                                   */
    XF_FLAG_TRANGE = 8,    /* T outside [T_lo, T_hi] (bracketed tables only)    */
    XF_FLAG_NEWTON = 16,   /* Newton not converged in 50 iterations              */
    XF_FLAG_C2 = 32,       /* Roe-averaged face c^2 <= 0                         */
    XF_FLAG_NAN = 64       /* NaN or Inf in the state or a result                */
};

#define XF_MAX_SPECIES 9

/* Uniform Cartesian grid (Sec. III.A, Fig. 3).  1 <= n_d <= 65535 (the
 * launch grids put single axes on the y and z grid dimensions); a dimension
 * with n_d > 1 needs n_d >= the ghost width (3, or 4 for xf_create_ghosts
 * with 4).  bc order: -x, +x, -y, +y, -z, +z; XF_BC_PERIODIC
 * wraps, XF_BC_OUTFLOW copies the nearest interior cell (zero gradient).
 * Periodic sides must come in pairs. */
typedef struct {
    int nx, ny, nz;
    double dx, dy, dz;
    int bc[6];
} xf_grid;

/* Per-species thermo tables (Sec. II.C.3; the NASA-polynomial form named
 * there): molar mass W[s] in kg/mol and a[s*6 + k], k = 0..5, with
 *   cp_s/R_s = a0 + a1 T + a2 T^2 + a3 T^3 + a4 T^4,
 *   h_s/R_s  = a0 T + a1 T^2/2 + a2 T^3/3 + a3 T^4/4 + a4 T^5/5 + a5,
 *   e_s = h_s - R_s T,  R_s = 8.314462618 / W_s.
 * [T_lo, T_hi] brackets the Newton temperature solve; T_hi <= 0 means no
 * bracket (use it for calorically perfect tables).  Host pointers; the
 * library copies them in xf_create. 1 <= ns <= XF_MAX_SPECIES. */
typedef struct {
    int ns;
    const double *W;
    const double *a;
    double T_lo, T_hi;
} xf_thermo;

/* Create a context on the current HIP device.  precision: XF_PREC_FP64, or
 * XF_PREC_MIXED (characteristic projection, WENO weights and fluxes in FP32;
 * internal energy, Newton T, pressure and all stored values in FP64).
 * Allocates the device status word.  On error *out is NULL. */
int xf_create(const xf_grid *grid, const xf_thermo *thermo, int precision, xf_ctx **out);
int xf_destroy(xf_ctx *ctx);

/* xf_create with a chosen ghost width: the number of ghost layers on each
 * side of every active dimension of the padded state (the halo of Fig. 3).
 * ghost_width 3 (what xf_create uses) serves the six-cell face stencils of
 * WENO5 and WENO-CU6; 4 is needed by the eight-cell stencils of WENO7
 * (XF_RECON_WENO7) and serves the six-cell schemes too, with identical
 * results.  Every padded array of the context (state, rhs, cotangents,
 * primitives) takes this width.  Returns XF_EINVAL for another width. */
int xf_create_ghosts(const xf_grid *grid, const xf_thermo *thermo, int precision, int ghost_width,
                     xf_ctx **out);

/* Number of doubles in one padded state: Nv * Z * Y * X. */
size_t xf_state_elems(const xf_ctx *ctx);

/* Bytes of device workspace needed by an operation (XF_OP_*). */
size_t xf_workspace_bytes(const xf_ctx *ctx, int op);

/* Fill the ghost layers of every active side of U in place: periodic wrap
 * or zero-gradient outflow (the boundary treatment of Sec. III.B.4), for all
 * fields; dimensions in the order x, y, z over the full padded extent of the
 * other axes, so edges and corners are filled consistently. */
int xf_fill_ghosts(xf_ctx *ctx, double *U, void *stream);

/* rhs = L(U) = -sum_d (F^_{i+1/2} - F^_{i-1/2}) / dx_d on the interior (Eq. 13
 * with the flux of Eq. 14-15); ghost cells of rhs are set to zero.  U's ghost
 * layers must be valid (xf_fill_ghosts).  U and rhs must not overlap.
 * ws: xf_workspace_bytes(ctx, XF_OP_RHS) bytes. */
int xf_rhs(xf_ctx *ctx, const double *U, double *rhs, void *ws, void *stream);

/* xf_rhs for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid allocation): the
 * same residual, bit for bit, with the workspace taken from a static device
 * array of the library (XF_NOALLOC_BYTES, held on every device the library
 * runs on until the process ends) instead of a caller buffer.  The call
 * itself allocates nothing and creates no event (per-kernel timing does not
 * record it).  The caller still owns U and rhs (device, layout as xf_rhs).
 * The current device must be the context's.  Every call on one device shares
 * that device's array, whose contents the next call overwrites: calls that
 * overlap on one device (different streams or host threads) race, and must
 * be serialised by the caller.  Returns XF_ETOOLARGE when
 * xf_workspace_bytes(ctx, XF_OP_RHS) exceeds XF_NOALLOC_BYTES (about
 * 2 million padded cells in FP64, 260 thousand in a mixed nine-species
 * context), XF_EINVAL for null, overlapping or misaligned buffers or another
 * current device. */
#define XF_NOALLOC_BYTES ((size_t)64 << 20)
int xf_rhs_noalloc(xf_ctx *ctx, const double *U, double *rhs, void *stream);

/* xf_rhs with the dissipation speeds of the flux splitting (the Lambda~ of
 * Eq. 14; Table I's artificial-viscosity options) passed in and out, for
 * checks of the linearisation at fixed speeds (the VJPs hold them fixed).
 * Layout of both alpha buffers (FP64, device): for each active direction in
 * the order x, y, z, a block [3][nf_d] holding the speeds of the u-c field,
 * of the middle fields and of the u+c field at every face of the direction,
 * nf_x = (nx+1) ny nz, nf_y = nx (ny+1) nz, nf_z = nx ny (nz+1) (0 for an
 * inactive direction), face index x: i + (nx+1)(j + ny k), y:
 * i + nx (j + (ny+1) k), z: i + nx (j + ny k) (i, j, k from 0; the face
 * with index i along its direction lies before interior cell i); total
 * 3 (nf_x + nf_y + nf_z) doubles.  alpha_out (may be NULL) receives, in
 * FP64, the speeds the context's scheme takes at U (LLF stencil maxima,
 * the ROE face speeds or the GLF direction maxima); alpha_in (may be
 * NULL) replaces them in the flux splitting (both may be the same buffer:
 * the speeds are written before they are read).  With both NULL this is
 * xf_rhs.  The residual is otherwise computed as by xf_rhs (its precision,
 * reconstruction and viscous terms); with alpha_in, directions are summed in
 * the order z, y, x as there.  ws: xf_workspace_bytes(ctx, XF_OP_RHS) bytes.
 * Caller-owned buffers; returns XF_EINVAL for null or misaligned pointers. */
int xf_rhs_alpha(xf_ctx *ctx, const double *U, const double *alpha_in, double *alpha_out, double *rhs,
                 void *ws, void *stream);

/* Primitive variables of every cell (interior and ghosts): prim is
 * [4][cells] FP64 (cells = xf_state_elems / Nv, the padded extent), holding
 * T from the Newton iteration on the mixture internal energy (Eq. 21), p from
 * the mixture equation of state (Eq. 7), the frozen sound speed c, and 1/rho.
 * Non-physical cells set the status bits as in xf_rhs.  U's ghost layers
 * must be valid for the ghost entries to be meaningful.  Caller-owned prim;
 * no workspace.  Computed in FP64 in both precisions. */
int xf_primitives(xf_ctx *ctx, const double *U, double *prim, void *stream);

/* dt = cfl / max_i sum_{d active} (|u_d| + c)_i / dx_d over the interior
 * (Eq. 17 per direction, summed), written to the device double *dt_dev.
 * ws: xf_workspace_bytes(ctx, XF_OP_RHS) bytes. */
int xf_cfl_dt(xf_ctx *ctx, const double *U, double cfl, double *dt_dev, void *ws, void *stream);

/* One SSP-RK3 step of Eq. 16 in place on U (ghosts are filled before each
 * stage and after the step).  The step is dt, or *dt_dev when dt_dev is not
 * NULL (a device scalar, e.g. from xf_cfl_dt, so no host round trip).
 * Stage combinations are accumulated in FP64 in both precisions.
 * ws: xf_workspace_bytes(ctx, XF_OP_RK3) bytes. */
int xf_rk3_step(xf_ctx *ctx, double *U, double dt, const double *dt_dev, void *ws, void *stream);

/* Artificial viscosity of the flux splitting of Eq. 14 (the options of
 * Table I): XF_VISC_LLF (default), per face and characteristic field the
 * largest |lambda| of the field over the stencil cells (six, or eight for
 * WENO7); XF_VISC_ROE,
 * |lambda| of the face's Roe state (u~_n - c~, u~_n, u~_n + c~), no entropy
 * fix; XF_VISC_GLF, per direction and field the largest LLF speed over all
 * faces of the direction, reduced on the device after every primitive pass.
 * Applies to every later call on the context; the VJPs hold the chosen speeds
 * fixed.  The positivity blend keeps the LLF speeds as its Lax-Friedrichs
 * coefficient.  Returns XF_EINVAL for another type. */
enum { XF_VISC_LLF = 0, XF_VISC_ROE = 1, XF_VISC_GLF = 2 };
int xf_set_dissipation(xf_ctx *ctx, int type);

/* Reconstruction REC of Eq. 15: XF_RECON_WENO5 (default; WENO5-JS, linear
 * weights (1, 6, 3)/10, eps = 1e-6), or XF_RECON_CU6, the sixth-order
 * central-upwind WENO the paper also offers (four candidates on the six
 * stencil cells, the downwind one (11 f_i+1 - 7 f_i+2 + 2 f_i+3)/6, linear
 * weights (1, 9, 9, 1)/20, alpha_k = d_k (20 + tau6 / (beta_k + 1e-6)),
 * beta_3 = beta6 the Jiang-Shu smoothness of the six-cell quintic,
 * tau6 = beta6 - (beta_0 + 4 beta_1 + beta_2)/6), or XF_RECON_WENO7, the
 * seventh-order WENO-JS (four cubic candidates on cells i-3..i+3 for the
 * plus side and i+4..i-2 for the minus side, linear weights
 * (1, 12, 18, 4)/35, alpha_k = d_k / (1e-6 + beta_k)^2), which needs a
 * context with 4 ghost layers (XF_EUNSUPPORTED otherwise).  Applies to
 * every later call; the VJPs differentiate WENO5 and CU6 with the
 * dissipation speeds held fixed and return XF_EUNSUPPORTED for WENO7.
 * Returns XF_EINVAL for another type. */
enum { XF_RECON_WENO5 = 0, XF_RECON_CU6 = 1, XF_RECON_WENO7 = 2 };
int xf_set_reconstruction(xf_ctx *ctx, int type);

/* Positivity-preserving flux blend (Sec. II.C.2, Eq. 17-20) in the SSP-RK3
 * steps of this context (xf_rk3_step, xf_rk3_step_cfl), off by default.
 * Each face flux becomes F_LF + theta (F^ - F_LF), F_LF the Lax-Friedrichs
 * flux of Eq. 19 (coefficient: the face's larger acoustic LLF speed) and
 * theta in [0, 1] the largest value keeping the Euler half-states
 * U_i -+ 2 lam F of Eq. 18 (lam = D dt / dx_d, D active dimensions) at or
 * above 1e-13 min(rho_i, rho_i+1) in total density and -1e-13 rho of the
 * cell in every partial density (-1e-6 rho in XF_PREC_MIXED, above FP32
 * round-off).  Stages use the step's dt.  xf_rhs and
 * xf_rhs_vjp are unaffected (the blend needs a time step); xf_rk3_step_vjp
 * returns XF_EUNSUPPORTED while the blend is on.  enable: 0 or 1. */
int xf_set_positivity(xf_ctx *ctx, int enable);

/* Viscous and diffusive fluxes F_v of Eq. 2 (Eq. 3-6: Newtonian stress and
 * its work, Fourier conduction, mass-corrected mixture-averaged species
 * diffusion -rho (D_sm grad Y_s - Y_s sum_j D_jm grad Y_j) with its enthalpy
 * flux), added to every residual of the context (xf_rhs, xf_rk3_step,
 * xf_rk3_step_cfl) as + div F_v (Eq. 1).  Transport per cell from the
 * fitted form of Eq. 29 with four coefficients per property:
 *   ln(mu_s / Pa s) = sum_k mu[s*4 + k] (ln T)^k, likewise kappa (W/(m K)),
 *   ln(D_st / (m^2/s)) = sum_k D[(s*ns + t)*4 + k] (ln T)^k at p_ref, and
 *   D_st(T, p) = D_st(T, p_ref) p_ref / p (D must be symmetric in s, t);
 * mixture viscosity and conductivity by the rule of Eq. 22 (Phi from the
 * ratio of the property being mixed), D_sm by Eq. 26 with the mole
 * fractions in its sums floored at X_t + 1e-12 (a pure species stays
 * finite).  Discretisation: fourth order and conservative (face values
 * (-1, 9, 9, -1)/16, normal derivatives (1, -27, 27, -1)/(24 dx),
 * tangential ones interpolated from (1, -8, 8, -1)/(12 dy) cell
 * differences; residual = staggered fourth-order difference of the face
 * point fluxes).  Computed in FP64 in both precisions.  terms: a bit set of
 * XF_VISCOUS_*; 0 switches the fluxes off (tr may then be NULL).  Host
 * tables are copied to the device (the first call allocates that copy; the
 * call synchronises the device).  The workspaces grow while the fluxes are
 * on: query xf_workspace_bytes after this call.  The VJPs return
 * XF_EUNSUPPORTED while they are on; the CFL step stays convective.
 * Returns XF_EINVAL for a table of another species count, a non-symmetric
 * D, p_ref <= 0, non-finite coefficients or unknown bits. */
typedef struct {
    int ns;
    const double *mu;      /* [ns][4]      */
    const double *kappa;   /* [ns][4]      */
    const double *D;       /* [ns][ns][4]  */
    double p_ref;          /* Pa           */
} xf_transport;
enum { XF_VISCOUS_STRESS = 1, XF_VISCOUS_HEAT = 2, XF_VISCOUS_DIFFUSION = 4 };
int xf_set_viscous(xf_ctx *ctx, const xf_transport *tr, int terms);

/* Reaction source of Eq. 1 (S: Eq. 8-12) split off the flow step
 * (Sec. II.C.4).  Mass-action kinetics with [X_s] = rho Y_s / W_s,
 * k_f = A T^B exp(-E / (R_u T)), k_b = k_f / K_c for reversible reactions
 * with K_c = (p0 / (R_u T))^(sum nu) exp(sum_s nu_s (S_s/R_s - h_s/(R_s T)))
 * (p0 = 1 atm, S_s/R_s = a0 ln T + a1 T + a2 T^2/2 + a3 T^3/3 + a4 T^4/4 +
 * s0[s], a0..a5 the context's thermo table), third bodies
 * sum_s eff[r*ns + s] [X_s] on both directions.  The reaction step keeps
 * rho, momentum and E (formation enthalpies live in a5, so the heat release
 * of Eq. 8 shows as a change of T) and advances the mass fractions by
 * `substeps` equal alpha-QSS predictor-corrector steps (Eq. 27-28, alpha(r)
 * = 1/(1 - e^-r) - 1/r), renormalised to unit sum after each.  splitting
 * XF_SPLIT_STRANG: xf_rk3_step and xf_rk3_step_cfl take R(dt/2) F(dt)
 * R(dt/2); XF_SPLIT_LIE: F(dt) R(dt) (F the SSP-RK3 flow step; with the
 * CFL variant dt comes from U^n before the first reaction step).  A NULL
 * mechanism or substeps = 0 switches reactions off.  Stoichiometric
 * coefficients 0..3, at most seven molecules on each side of a reaction
 * (sum_s nu' <= 7, sum_s nu'' <= 7); 1 <= nr <= XF_MAX_REACTIONS; every reaction must
 * conserve mass (sum_s W_s (nu'' - nu') = 0 within 1e-9 W_max).  Tables are
 * copied to the device (the first call allocates that copy and the call
 * synchronises).  The VJPs return XF_EUNSUPPORTED while reactions are on.
 * Returns XF_EINVAL for bad tables, counts or flags. */
#define XF_MAX_REACTIONS 32
typedef struct {
    int ns, nr;
    const int *nu_f, *nu_b;       /* [nr][ns] nu' and nu''           */
    const double *A, *B, *E;      /* [nr]: SI, -, J/mol              */
    const int *third;             /* [nr] 0/1                        */
    const double *eff;            /* [nr][ns] third-body efficiency  */
    const int *reversible;        /* [nr] 0/1                        */
    const double *s0;             /* [ns] entropy constants (a6)     */
} xf_mechanism;
enum { XF_SPLIT_STRANG = 0, XF_SPLIT_LIE = 1 };
int xf_set_reactions(xf_ctx *ctx, const xf_mechanism *mech, int substeps, int splitting);

/* One reaction step over dt (or *dt_dev when not NULL) on the interior of U,
 * in place, with the context's mechanism and substeps; the ghosts are filled
 * afterwards.  Returns XF_EUNSUPPORTED when no mechanism is set. */
int xf_react(xf_ctx *ctx, double *U, double dt, const double *dt_dev, void *stream);

/* xf_rk3_step with the time step of Eq. 17 computed on the device from U^n
 * (the same reduction as xf_cfl_dt, reusing the first stage's primitives)
 * and written to the device double *dt_dev before the stages use it.  This
 * is one full time step of the convective system with no host round trip.
 * ws: xf_workspace_bytes(ctx, XF_OP_RK3) bytes. */
int xf_rk3_step_cfl(xf_ctx *ctx, double *U, double cfl, double *dt_dev, void *ws, void *stream);

/* Vector-Jacobian product of the right-hand side: U_bar += J(U)^T rhs_bar,
 * J = d rhs / dU on the padded state with ghost values treated as independent
 * inputs (compose with xf_fill_ghosts_vjp for the map from the interior).
 * The LLF wave speeds are held fixed (their dependence on U is not
 * differentiated); T(U) is differentiated through the converged Newton
 * solve by the implicit-function rule dT = (de - sum_s e_s dY_s) / C_v.
 * rhs_bar ghost entries are ignored.  U_bar is read and updated.
 * ws: xf_workspace_bytes(ctx, XF_OP_VJP) bytes. */
int xf_rhs_vjp(xf_ctx *ctx, const double *U, const double *rhs_bar, double *U_bar,
               void *ws, void *stream);

/* Adjoint of xf_fill_ghosts: adds every ghost entry of U_bar onto the
 * interior cell it was copied from (reverse order z, y, x) and zeroes the
 * ghost entries. */
int xf_fill_ghosts_vjp(xf_ctx *ctx, double *U_bar, void *stream);

/* Adjoint of one xf_rk3_step with a fixed dt: given U_n (the state before
 * the step, ghosts need not be valid) and U_bar = dJ/dU_{n+1} (padded), it
 * recomputes the stage states from U_n and overwrites U_bar with dJ/dU_n.
 * The LLF wave speeds of every stage are held fixed.
 * ws: xf_workspace_bytes(ctx, XF_OP_RK3_VJP) bytes. */
int xf_rk3_step_vjp(xf_ctx *ctx, const double *U_n, double dt, double *U_bar,
                    void *ws, void *stream);

/* Kernel classes of the per-kernel timing below. */
enum {
    XF_K_PRIMS = 0,        /* primitives + Newton temperature                    */
    XF_K_SWEEP_X = 1,      /* x flux difference                                  */
    XF_K_SWEEP_Y = 2,      /* y flux difference                                  */
    XF_K_SWEEP_Z = 3,      /* z flux difference                                  */
    XF_K_FILL = 4,         /* ghost fill (all active directions of one call)     */
    XF_K_STAGE = 5,        /* SSP-RK3 stage combination                          */
    XF_K_CFL = 6,          /* CFL reduction                                      */
    XF_K_ZERO = 7,         /* zeroing of rhs ghosts / VJP scratch                */
    XF_K_VJP_X = 8,        /* x flux-difference VJP                              */
    XF_K_VJP_Y = 9,
    XF_K_VJP_Z = 10,
    XF_K_PRIMS_VJP = 11,   /* implicit-function VJP of (p, T)(U)                  */
    XF_K_FILL_VJP = 12,    /* adjoint of the ghost fill                          */
    XF_K_TRANSPORT = 13,   /* transport properties and velocity gradient         */
    XF_K_VISCOUS_X = 14,   /* x viscous flux difference                          */
    XF_K_VISCOUS_Y = 15,
    XF_K_VISCOUS_Z = 16,
    XF_K_REACT = 17,       /* reaction step (alpha-QSS sub-steps)                */
    XF_K_COUNT = 18
};

/* Per-kernel timing for profiling.  While enabled, every kernel launch of
 * this context is bracketed by two HIP events recorded on the launch stream
 * (events are created on demand and reused; nothing else changes).
 * xf_timing_read synchronises `stream`, adds the elapsed time of every
 * completed launch of class k to ms[k] and its count to launches[k]
 * (arrays of XF_K_COUNT entries, overwritten), and forgets the records. */
int xf_timing(xf_ctx *ctx, int enable);
int xf_timing_read(xf_ctx *ctx, void *stream, double *ms, long long *launches);

/* Synchronise `stream`, return the accumulated status bits in *flags_out
 * and clear them.  Returns XF_ENONPHYS when any bit was set, else XF_OK.
 * This is the report of the error catching of Sec. III.B.6 (a
 * non-physical state stops the run with a message instead of going on):
 * the kernels flag, the caller decides. */
int xf_status(xf_ctx *ctx, void *stream, unsigned *flags_out);

/* Static description of a status code (the messages of the error catching
 * of Sec. III.B.6). */
const char *xf_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* XF_H */
