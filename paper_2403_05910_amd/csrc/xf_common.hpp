// xf_common.hpp -- host/device shared definitions of libxf (gfx950).
//
// Kernel-argument structs (grid geometry, thermo coefficient tables) and the
// per-species-count operation table the C ABI dispatches through.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/xf.h"

namespace xf {

constexpr double kRu = 8.314462618;      // J/(mol K)
constexpr double kP0 = 101325.0;         // Pa, the reference pressure of the equilibrium constants
constexpr int kMaxNs = XF_MAX_SPECIES;
constexpr double kNewtonTol = 1e-11;
constexpr int kNewtonMaxIt = 50;

// Geometry of one padded SoA field: x fastest, 3 or 4 ghost layers per active axis.
struct Geo {
    int nx, ny, nz;      // interior cells
    int gx, gy, gz;      // ghost widths (3 or 4; 0 on an inactive axis)
    int px, py, pz;      // padded extents
    long long sy, sz;    // strides of y and z in a field
    long long cells;     // px * py * pz: stride between fields
    double dx, dy, dz;
    double idx, idy, idz;
    int bc[6];
};

// Padded source index (along the ghost's axis) of ghost layer l on side sd
// (0 low, 1 high), n interior cells, ng ghost layers per side: periodic wraps,
// outflow copies the nearest interior cell (n >= ng, so every source is an
// interior cell).
__device__ __forceinline__ int ghost_src(int bc, int sd, int l, int n, int ng) {
    if (sd == 0) return bc == XF_BC_PERIODIC ? n + l : ng;
    return bc == XF_BC_PERIODIC ? ng + l : ng + n - 1;
}

// Species thermo in the form the kernels evaluate (Horner in T):
//   cv_s(T) = sum_k cv[s][k] T^k  (k = 0..4),  C_v,s = C_p,s - R_s
//   e_s(T)  = sum_k e[s][k] T^k   (k = 0..5),  e_s = h_s - R_s T
// For a table a[0..5] (cp/R = sum a_k T^k, h/R = sum a_k T^(k+1)/(k+1) + a5):
//   cv = R_s (a0 - 1, a1, a2, a3, a4),  e = R_s (a5, a0 - 1, a1/2, a2/3, a3/4, a4/5).
template <typename R>
struct ThermoK {
    R Rs[kMaxNs];
    R cv[kMaxNs][5];
    R e[kMaxNs][6];
    double T_lo, T_hi, T_ref;
    int bracket;
};

// Fitted transport (Eq. 29) and the species constants of the mixing rules
// (Eq. 22, 26), in device memory (too large for kernel arguments):
//   ln mu_s = sum_k mu[s][k] (ln T)^k, likewise kappa_s, and
//   ln D_st(T, p_ref) = sum_k D[s][t][k] (ln T)^k, D_st(T, p) = D_st(T, p_ref) p_ref / p;
//   wa[s][t] = (1 + W_s/W_t)^(-1/2) / sqrt(8), wb[s][t] = (W_t/W_s)^(1/4).
struct TransportK {
    double mu[kMaxNs][4];
    double kappa[kMaxNs][4];
    double D[kMaxNs][kMaxNs][4];
    double wa[kMaxNs][kMaxNs];
    double wb[kMaxNs][kMaxNs];
    double W[kMaxNs];       // kg/mol
    double iW[kMaxNs];
    double ip_ref;          // 1 / p_ref
};
// Viscous terms (bit set): stress with its work, Fourier conduction,
// species diffusion with its enthalpy flux.
constexpr int kViscousStress = 1, kViscousHeat = 2, kViscousDiffusion = 4;
// Per-cell fields of the transport pass: mu_bar, kappa_bar, u, v, w, D_sm (NS).
inline int transport_fields(int ns) { return 5 + ns; }

// Reaction mechanism (Eq. 9-12) in device memory: stoichiometric
// coefficients nu' (nf) and nu'' (nb), Arrhenius ln A, B and E / R_u, third
// bodies with efficiencies, reversibility, and per species the thermo
// coefficients a0..a5 with the entropy constant a6 (for Eq. 12).
constexpr int kMaxReactions = XF_MAX_REACTIONS;
struct ReactK {
    int nr;
    int nf[kMaxReactions][kMaxNs], nb[kMaxReactions][kMaxNs];
    int dn[kMaxReactions];          // sum_s (nu'' - nu')
    int third[kMaxReactions], rev[kMaxReactions];
    double lnA[kMaxReactions], B[kMaxReactions], ER[kMaxReactions];
    double eff[kMaxReactions][kMaxNs];
    // sum_s (nu'' - nu') g_s(T), with g_s = S_s/R_s - h_s/(R_s T) linear in the
    // species' NASA coefficients, folded per reaction:
    // dg = G0 (ln T - 1) + G1 T + G2 T^2 + G3 T^3 + G4 T^4 + G5 / T + G6
    double G[kMaxReactions][7];
    double W[kMaxNs], iW[kMaxNs];
    // per reaction, for scalar loads ahead of the species work: the reactant
    // and product lists (the count in bits 0..2, then up to seven species
    // indices of four bits each, a species listed nu times), and nu' and
    // nu'' as doubles for the accumulation of q and p
    unsigned fl[kMaxReactions], bl[kMaxReactions];
    double fd[kMaxReactions][kMaxNs], bd[kMaxReactions][kMaxNs];
    ThermoK<double> th;   // the context's species tables, for the temperature solves
    double lp0;           // ln(p0 / R_u)
};

// Step size seen by the sweeps, for the positivity blend: dt, or *dt_dev
// when dt_dev is set; pp switches the blend on.  With Uout set, the x sweep
// finishes the SSP-RK3 stage of Eq. 16 itself instead of writing its
// residual: Uout = a U0 + b (Uin + h L), L = ((L_x + L_y) + L_z) + L_v with
// its own L_x and the other terms read where their pointers are set (the
// FP64 or the FP32 per-direction buffers, by the sweep's type), exactly as
// the separate stage kernel sums them.
struct StageArgs {
    double dt;
    const double *dt_dev;
    int pp;   // blend the face fluxes for positivity with the step dt (or *dt_dev)
    double *Uout = nullptr;
    const double *U0 = nullptr, *Uin = nullptr;
    const double *Ly64 = nullptr, *Lz64 = nullptr;
    const float *Ly32 = nullptr, *Lz32 = nullptr;
    const double *Lv = nullptr;
    double a = 0.0, b = 1.0;
};

// Everything a launch needs besides buffers.
struct LaunchCtx {
    Geo g;
    ThermoK<double> th64;
    ThermoK<float> th32;
    unsigned *status;    // device status word (atomicOr of XF_FLAG_*)
    int precision;       // XF_PREC_*
    int visc;            // artificial viscosity: kViscLlf, kViscRoe or kViscGlf
    int recon;           // reconstruction: kReconWeno5 or kReconCu6
};

// Per species-count entry points (one translation unit per N).
struct NsOps {
    // primitive variables (T, p, c, 1/rho) of every cell a stencil reads (of
    // every padded cell with all_cells); with Uf, Pf also FP32 copies of U
    // and P for the mixed-precision sweeps.  With Ug (= U) the ghosts of U
    // the pass covers are filled on the way, each from its boundary source as
    // the ghost fill does (without all_cells: the face ghosts; the edge and
    // corner ghosts lie outside every stencil and are left)
    // With cfl, the pass also folds the CFL rate of its interior cells
    // (Eq. 17, as the cfl entry) into *cfl, which the caller has zeroed.
    hipError_t (*prims)(const LaunchCtx &, const double *U, double *P, float *Uf, float *Pf, int all_cells,
                        double *Ug, unsigned long long *cfl, hipStream_t);
    // one direction of the convective flux difference.  FP64 sweeps read U,
    // P and write rhs (accumulate: rhs +=, else rhs =); mixed-precision
    // sweeps read Uf, Pf and write the FP32 differences to rhs32 (no
    // accumulation: every direction has its own buffer).
    // glf: the direction's three GLF speeds (device) when lc.visc is GLF
    hipError_t (*sweep)(const LaunchCtx &, int dir, int accumulate, const double *U, const double *P,
                        const float *Uf, const float *Pf, double *rhs, float *rhs32, const StageArgs &stage,
                        const double *glf, hipStream_t);
    // VJP of one direction: Ubar += (dF/dU)^T ..., Pbar += (dF/d(p, T, rho))^T ...
    // (Pbar: [3][cells], the cotangents of each cell's p, T and rho)
    hipError_t (*sweep_vjp)(const LaunchCtx &, int dir, const double *U, const double *P,
                            const double *rbar, double *Ubar, double *Pbar, const double *glf, hipStream_t);
    // one direction of the flux difference with the dissipation speeds of
    // every face given (alpha [3][astride], astride the direction's face
    // count); otherwise as sweep with no stage
    hipError_t (*sweep_frozen)(const LaunchCtx &, int dir, int accumulate, const double *U, const double *P,
                               const float *Uf, const float *Pf, double *rhs, float *rhs32, const double *alpha,
                               long long astride, hipStream_t);
    // the dissipation speeds the context's scheme takes at every face of one
    // direction, FP64, into alpha [3][astride] (glf: the direction's GLF speeds)
    hipError_t (*face_speeds)(const LaunchCtx &, int dir, const double *U, const double *P, const double *glf,
                              double *alpha, long long astride, hipStream_t);
    // GLF speeds of one direction: atomicMax of |u_d - c|, |u_d|, |u_d + c|
    // (uint64 bits of positive doubles) into mx[0..2], which must start at 0
    hipError_t (*glf)(const LaunchCtx &, int dir, const double *U, const double *P, unsigned long long *mx,
                      hipStream_t);
    // VJP of the primitive map: Ubar += (d(p, T, rho)/dU)^T Pbar
    hipError_t (*prims_vjp)(const LaunchCtx &, const double *U, const double *P,
                            const double *Pbar, double *Ubar, hipStream_t);
    // CFL reduction: max_i sum_d (|u_d| + c)/dx_d -> atomicMax on *mx (uint64 bits)
    hipError_t (*cfl)(const LaunchCtx &, const double *U, const double *P,
                      unsigned long long *mx, hipStream_t);
    // transport pass at every padded cell: Q[transport_fields(ns)][cells]
    hipError_t (*transport)(const LaunchCtx &, const double *U, const double *P, double *Q, const TransportK *tk,
                            hipStream_t);
    // viscous fluxes of one direction, added to rhs on the interior; G the
    // cell-centred velocity gradient [9][cells] (G[3 a + b] = d u_b / d x_a)
    hipError_t (*viscous)(const LaunchCtx &, int dir, const double *U, const double *P, const double *Q,
                          const double *G, double *rhs, int terms, hipStream_t);
    // reaction step on the interior cells, in place: n_sub alpha-QSS
    // sub-steps over scale * (dt_dev ? *dt_dev : dt)
    hipError_t (*react)(const LaunchCtx &, double *U, const ReactK *rk, double dt, const double *dt_dev,
                        double scale, int n_sub, hipStream_t);
    // SSP-RK3 stage on the interior: Uout = a U0 + b (Uin + h (((Lx + Ly) + Lz) + Lv)),
    // h = dt_dev ? *dt_dev : dt, a == 0 skipping U0; L[d] null for an
    // inactive direction, FP64 (L64) in FP64 contexts and FP32 (L32) in mixed
    // ones, Lv (FP64, may be null) the viscous residual of a mixed context.
    // Uout may alias U0.
    hipError_t (*stage)(const LaunchCtx &, double *Uout, const double *U0, const double *Uin,
                        const double *const L64[3], const float *const L32[3], const double *Lv, double a, double b,
                        double dt, const double *dt_dev, hipStream_t);
};

// The reaction launcher of one species count, from its own translation unit
// (xf_react.hip, built with different code-motion settings).
template <int N>
hipError_t react_launch(const LaunchCtx &, double *U, const ReactK *rk, double dt, const double *dt_dev, double scale,
                        int n_sub, hipStream_t);

const NsOps *ops_for_ns(int ns);

// Faces of direction d (0 when the direction is inactive): the interior
// count plus one along d.
inline long long face_count(const Geo &g, int d) {
    const int n[3] = {g.nx, g.ny, g.nz};
    if (n[d] <= 1) return 0;
    return (long long)(g.nx + (d == 0)) * (g.ny + (d == 1)) * (g.nz + (d == 2));
}

// Launch geometry of the face VJP in x: waves of 64 consecutive faces in
// one z-plane, launch groups of every second wave, blocks of up to 4 waves.
constexpr int kVjpGroups = 2;
inline long long vjp_x_waves_per_plane(const Geo &g) { return ((long long)(g.nx + 1) * g.ny + 63) / 64; }

// Species-independent launches (xf_misc.hip).
hipError_t launch_fill_ghosts(const LaunchCtx &, int nv, double *U, hipStream_t);
hipError_t launch_fill_ghosts_vjp(const LaunchCtx &, int nv, double *Ubar, hipStream_t);
hipError_t launch_zero_ghosts(const LaunchCtx &, int nv, double *A, hipStream_t);
hipError_t launch_rk3_stage_vjp(const LaunchCtx &, int nv, int stage, double *lam, double *lam0,
                                double *mu, const double *dt_dev, double dt, hipStream_t);
// rhs = ((Lz + Ly) + Lx) on the interior (FP32 per-direction differences of
// a mixed context, summed in FP64 in the order of the FP64 sweeps; null for
// an inactive direction)
hipError_t launch_sum_dirs(const LaunchCtx &, int nv, double *rhs, const float *const L[3], hipStream_t);
hipError_t launch_axpy_state(long long n, double a, const double *x, double b, double *y,
                             hipStream_t);
hipError_t launch_cfl_reset(unsigned long long *mx, hipStream_t);
// cell-centred velocity gradient from the velocity fields Q[2..4] of the
// transport pass: G[3 a + b][cells], fourth-order differences along every
// active axis a at the cells two or more layers inside the padded extent
hipError_t launch_vel_grad(const LaunchCtx &, const double *Q, double *G, hipStream_t);
hipError_t launch_reset_u64(unsigned long long *p, int n, hipStream_t);
hipError_t launch_cfl_finish(const unsigned long long *mx, double cfl, double *dt_dev,
                             hipStream_t);
hipError_t launch_copy(long long n, const double *src, double *dst, hipStream_t);
hipError_t launch_zero(long long n, double *dst, hipStream_t);

}  // namespace xf
