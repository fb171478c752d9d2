// xf_ns.hip -- launchers of the species-templated kernels for one species
// count.  Compiled once per N with -DXF_NS=N; each object exports
// xf::ops_ns<N>(), which the C ABI collects into its dispatch table.
#include "xf_forward.hpp"
#include "xf_viscous.hpp"
#include "xf_vjp.hpp"

#ifndef XF_NS
#error "compile with -DXF_NS=<species count>"
#endif

namespace xf {
namespace {

constexpr int NS = XF_NS;

unsigned blocks_for(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

hipError_t prims(const LaunchCtx &c, const double *U, double *P, float *Uf, float *Pf, int all_cells, double *Ug,
                 unsigned long long *cfl, hipStream_t s) {
    if (Ug && Ug != U) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_prims<NS>, dim3(blocks_for(c.g.cells, 256)), dim3(256), 0, s, U, P, c.g, c.th64,
                       c.status, Uf, Pf, all_cells, Ug, cfl);
    return hipGetLastError();
}

template <typename R, typename S, bool PP, int SPD, int REC>
hipError_t launch_face_sweep(const LaunchCtx &c, const ThermoK<R> &th, int dir, int accumulate, const S *U,
                             const S *P, R *rhs, const StageArgs &sa, const Dissip &ds, hipStream_t s) {
    const Geo &g = c.g;
    if (dir == 0) {
        const long long nfx = (long long)g.nx + 1, nf = nfx * g.ny * g.nz;
        const int fpb = x_faces_per_block<stencil_radius(REC)>(nfx);
        // blocks overlap by one face; the count is rounded up to a multiple
        // of the XCD count so that each XCD takes one contiguous range
        unsigned nb = (unsigned)((nf - 1 + (fpb - 2)) / (fpb - 1));
        nb = (nb + kNumXcd - 1) / kNumXcd * kNumXcd;
        hipLaunchKernelGGL((k_sweep_x<NS, R, S, PP, SPD, REC>), dim3(nb), dim3(kXBlock), 0, s, U, P, rhs, g, th,
                           accumulate, sa, c.status, ds, fpb);
        return hipGetLastError();
    }
    const int ntr = dir == 1 ? g.nz : g.ny;
    const int nsw = dir == 1 ? g.ny : g.nz;
    constexpr int TX = TileShape<R, REC, PP>::x, TS = TileShape<R, REC, PP>::s;
    const unsigned tiles = (unsigned)((nsw + TS - 2) / (TS - 1));
    dim3 grid((g.nx + TX - 1) / TX, tiles, ntr), block(TX, TS);
    if (dir == 1)
        hipLaunchKernelGGL((k_sweep_tile<NS, R, 1, S, PP, SPD, REC>), grid, block, 0, s, U, P, rhs, g, th, accumulate,
                           sa, c.status, ds);
    else
        hipLaunchKernelGGL((k_sweep_tile<NS, R, 2, S, PP, SPD, REC>), grid, block, 0, s, U, P, rhs, g, th, accumulate,
                           sa, c.status, ds);
    return hipGetLastError();
}

// One instance per (positivity blend, artificial viscosity, reconstruction).
template <typename R, typename S, bool PP, int SPD>
hipError_t face_sweep_rec(const LaunchCtx &c, const ThermoK<R> &th, int dir, int accumulate, const S *U, const S *P,
                          R *rhs, const StageArgs &sa, const Dissip &ds, hipStream_t s) {
    switch (ds.recon) {
        case kReconCu6: return launch_face_sweep<R, S, PP, SPD, kReconCu6>(c, th, dir, accumulate, U, P, rhs, sa, ds, s);
        case kReconWeno7:
            return launch_face_sweep<R, S, PP, SPD, kReconWeno7>(c, th, dir, accumulate, U, P, rhs, sa, ds, s);
        default: return launch_face_sweep<R, S, PP, SPD, kReconWeno5>(c, th, dir, accumulate, U, P, rhs, sa, ds, s);
    }
}

template <typename R, typename S, bool PP>
hipError_t face_sweep_spd(const LaunchCtx &c, const ThermoK<R> &th, int dir, int accumulate, const S *U, const S *P,
                          R *rhs, const StageArgs &sa, const Dissip &ds, hipStream_t s) {
    if constexpr (!PP) {   // given speeds: right-hand sides only, never the blended step
        if (ds.type == kViscFrozen) return face_sweep_rec<R, S, PP, kViscFrozen>(c, th, dir, accumulate, U, P, rhs, sa, ds, s);
    } else {
        if (ds.type == kViscFrozen) return hipErrorInvalidValue;
    }
    switch (ds.type) {
        case kViscRoe: return face_sweep_rec<R, S, PP, kViscRoe>(c, th, dir, accumulate, U, P, rhs, sa, ds, s);
        case kViscGlf: return face_sweep_rec<R, S, PP, kViscGlf>(c, th, dir, accumulate, U, P, rhs, sa, ds, s);
        default: return face_sweep_rec<R, S, PP, kViscLlf>(c, th, dir, accumulate, U, P, rhs, sa, ds, s);
    }
}

template <typename R, typename S>
hipError_t face_sweep_scheme(const LaunchCtx &c, const ThermoK<R> &th, int dir, int accumulate, const S *U,
                             const S *P, R *rhs, const StageArgs &sa, const Dissip &ds, hipStream_t s) {
    return sa.pp ? face_sweep_spd<R, S, true>(c, th, dir, accumulate, U, P, rhs, sa, ds, s)
                 : face_sweep_spd<R, S, false>(c, th, dir, accumulate, U, P, rhs, sa, ds, s);
}

hipError_t sweep(const LaunchCtx &c, int dir, int accumulate, const double *U, const double *P, const float *Uf,
                 const float *Pf, double *rhs, float *rhs32, const StageArgs &sa, const double *glf, hipStream_t s) {
    const Dissip ds{c.visc, glf, c.recon};
    if (c.visc == kViscGlf && !glf) return hipErrorInvalidValue;
    if (c.precision == XF_PREC_MIXED) {
        if (!rhs32 || accumulate) return hipErrorInvalidValue;   // FP32 differences: one buffer per direction
        return face_sweep_scheme<float, float>(c, c.th32, dir, 0, Uf, Pf, rhs32, sa, ds, s);
    }
    return face_sweep_scheme<double, double>(c, c.th64, dir, accumulate, U, P, rhs, sa, ds, s);
}

hipError_t sweep_frozen(const LaunchCtx &c, int dir, int accumulate, const double *U, const double *P, const float *Uf,
                        const float *Pf, double *rhs, float *rhs32, const double *alpha, long long astride,
                        hipStream_t s) {
    Dissip ds{kViscFrozen, nullptr, c.recon};
    ds.alpha = alpha;
    ds.astride = astride;
    const StageArgs off{};
    if (c.precision == XF_PREC_MIXED) {
        if (!rhs32 || accumulate) return hipErrorInvalidValue;
        return face_sweep_rec<float, float, false, kViscFrozen>(c, c.th32, dir, 0, Uf, Pf, rhs32, off, ds, s);
    }
    return face_sweep_rec<double, double, false, kViscFrozen>(c, c.th64, dir, accumulate, U, P, rhs, off, ds, s);
}

hipError_t stage(const LaunchCtx &c, double *Uout, const double *U0, const double *Uin, const double *const L64[3],
                 const float *const L32[3], const double *Lv, double a, double b, double dt, const double *dt_dev,
                 hipStream_t s) {
    const dim3 grid((unsigned)c.g.ny * c.g.nz, NS + 4), block(256);
    if (c.precision == XF_PREC_MIXED)
        hipLaunchKernelGGL(k_stage_sum<float>, grid, block, 0, s, Uout, U0, Uin, L32[0], L32[1], L32[2], Lv, c.g, a,
                           b, dt, dt_dev);
    else
        hipLaunchKernelGGL(k_stage_sum<double>, grid, block, 0, s, Uout, U0, Uin, L64[0], L64[1], L64[2], Lv, c.g, a,
                           b, dt, dt_dev);
    return hipGetLastError();
}

hipError_t face_speeds(const LaunchCtx &c, int dir, const double *U, const double *P, const double *glf,
                       double *alpha, long long astride, hipStream_t s) {
    if (c.visc == kViscGlf && !glf) return hipErrorInvalidValue;
    const dim3 grid(blocks_for(astride, 256)), block(256);
    const bool w7 = c.recon == kReconWeno7;
#define XF_SPEEDS(D)                                                                                              \
    if (w7)                                                                                                    \
        hipLaunchKernelGGL((k_face_speeds<NS, D, 4>), grid, block, 0, s, U, P, c.g, c.th64, c.visc, glf, alpha, \
                           astride);                                                                           \
    else                                                                                                       \
        hipLaunchKernelGGL((k_face_speeds<NS, D, 3>), grid, block, 0, s, U, P, c.g, c.th64, c.visc, glf, alpha, \
                           astride);
    if (dir == 0) {
        XF_SPEEDS(0)
    } else if (dir == 1) {
        XF_SPEEDS(1)
    } else {
        XF_SPEEDS(2)
    }
#undef XF_SPEEDS
    return hipGetLastError();
}

// LDS a block of the x face VJP may take (of the CU's 160 KB).
constexpr size_t kVjpLdsBytes = 160 * 1024;

template <typename R, bool CU6>
hipError_t launch_vjp_group(const LaunchCtx &c, const ThermoK<R> &th, int dir, int grp, const double *U,
                            const double *P, const double *rbar, double *Ubar, double *Pbar, const Dissip &ds,
                            hipStream_t s) {
    const Geo &g = c.g;
    if (dir == 0) {
        // consecutive faces per wave with private LDS areas of W cells
        const int rowf = g.nx + 1;
        const int bounds = (63 + rowf - 1) / rowf;               // row boundaries 64 faces can cross
        const int W = 69 + 5 * bounds;
        const size_t per_wave = vjp_x_lds_per_wave<NS, R>(W);
        // FP64: one wave per block, so the waves of a CU (one per SIMD) run
        // their staging, faces and window merge out of step (12.3 -> 12.0 ms
        // per direction at 256^3, nine species, against four-wave blocks)
        const int wpb = sizeof(R) == 8 ? 1 : (per_wave * 4 <= kVjpLdsBytes ? 4 : 1);
        if (per_wave * wpb > kVjpLdsBytes) return hipErrorInvalidValue;
        const long long waves = (vjp_x_waves_per_plane(g) - grp + kVjpGroups - 1) / kVjpGroups;
        dim3 grid((unsigned)((waves + wpb - 1) / wpb), g.nz), block(64 * wpb);
        // dynamic LDS above 64 KB must be allowed for the kernel
        const hipError_t e = hipFuncSetAttribute((const void *)k_face_vjp_x<NS, R, CU6>,
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)kVjpLdsBytes);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL((k_face_vjp_x<NS, R, CU6>), grid, block, per_wave * wpb, s, U, P, rbar, Ubar, Pbar, g, th,
                           W, grp, ds);
    } else {
        const int nsw = dir == 1 ? g.ny : g.nz;
        const int xt = (g.nx + kVjpTX - 1) / kVjpTX;
        const int nfb = (nsw + 1 + vjp_yz_faces<R>() - 1) / vjp_yz_faces<R>();
        const int nb = (nfb - grp + kVjpGroups - 1) / kVjpGroups;
        dim3 grid((unsigned)(xt * nb), dir == 1 ? g.nz : g.ny), block(64 * vjp_yz_waves<R>());
        if (dir == 1)
            hipLaunchKernelGGL((k_face_vjp_yz<NS, R, 1, CU6>), grid, block, 0, s, U, P, rbar, Ubar, Pbar, g, th, grp,
                               ds);
        else
            hipLaunchKernelGGL((k_face_vjp_yz<NS, R, 2, CU6>), grid, block, 0, s, U, P, rbar, Ubar, Pbar, g, th, grp,
                               ds);
    }
    return hipGetLastError();
}

// Two launch groups per direction (x: waves w = grp mod 2; y/z: face
// blocks b = grp mod 2), one kernel each: neighbours share window cells,
// next-but-one neighbours none (measured at 256^3, nine species, the RHS VJP
// took 46.4 ms with six groups and 45.6 ms with two).
template <typename R>
hipError_t sweep_vjp_t(const LaunchCtx &c, const ThermoK<R> &th, int dir, const double *U, const double *P,
                       const double *rbar, double *Ubar, double *Pbar, const Dissip &ds, hipStream_t s) {
    const Geo &g = c.g;
    const int nsw = dir == 1 ? g.ny : g.nz;
    const long long ngrp = dir == 0 ? vjp_x_waves_per_plane(g) : (nsw + 1 + vjp_yz_faces<R>() - 1) / vjp_yz_faces<R>();
    for (int grp = 0; grp < kVjpGroups && grp < ngrp; ++grp) {
        const hipError_t e = ds.recon == kReconCu6
                                 ? launch_vjp_group<R, true>(c, th, dir, grp, U, P, rbar, Ubar, Pbar, ds, s)
                                 : launch_vjp_group<R, false>(c, th, dir, grp, U, P, rbar, Ubar, Pbar, ds, s);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t sweep_vjp(const LaunchCtx &c, int dir, const double *U, const double *P, const double *rbar,
                     double *Ubar, double *Pbar, const double *glf, hipStream_t s) {
    const Dissip ds{c.visc, glf, c.recon};
    if (c.visc == kViscGlf && !glf) return hipErrorInvalidValue;
    if (c.recon == kReconWeno7) return hipErrorInvalidValue;   // six-cell stencils only
    if (c.precision == XF_PREC_MIXED)
        return sweep_vjp_t<float>(c, c.th32, dir, U, P, rbar, Ubar, Pbar, ds, s);
    return sweep_vjp_t<double>(c, c.th64, dir, U, P, rbar, Ubar, Pbar, ds, s);
}

hipError_t glf(const LaunchCtx &c, int dir, const double *U, const double *P, unsigned long long *mx,
               hipStream_t s) {
    const Geo &g = c.g;
    const long long n = (long long)(dir == 0 ? g.px : g.nx) * (dir == 1 ? g.py : g.ny) * (dir == 2 ? g.pz : g.nz);
    long long nb = blocks_for(n, 256);
    if (nb > 2048) nb = 2048;   // grid-stride: three atomics per block
    hipLaunchKernelGGL(k_glf<NS>, dim3((unsigned)nb), dim3(256), 0, s, U, P, g, dir, mx);
    return hipGetLastError();
}

hipError_t prims_vjp(const LaunchCtx &c, const double *U, const double *P, const double *Pbar, double *Ubar,
                     hipStream_t s) {
    hipLaunchKernelGGL(k_prims_vjp<NS>, dim3(blocks_for(c.g.cells, 256)), dim3(256), 0, s, U, P, Pbar, Ubar, c.g,
                       c.th64);
    return hipGetLastError();
}

hipError_t cfl(const LaunchCtx &c, const double *U, const double *P, unsigned long long *mx, hipStream_t s) {
    const long long n = (long long)c.g.nx * c.g.ny * c.g.nz;
    long long nb = blocks_for(n, 256);
    if (nb > 2048) nb = 2048;   // grid-stride: one atomic per block
    hipLaunchKernelGGL(k_cfl<NS>, dim3((unsigned)nb), dim3(256), 0, s, U, P, c.g, mx);
    return hipGetLastError();
}

hipError_t transport(const LaunchCtx &c, const double *U, const double *P, double *Q, const TransportK *tk,
                     hipStream_t s) {
    hipLaunchKernelGGL(k_transport<NS>, dim3(blocks_for(c.g.cells, 256)), dim3(256), 0, s, U, P, Q, c.g, tk);
    return hipGetLastError();
}

hipError_t viscous(const LaunchCtx &c, int dir, const double *U, const double *P, const double *Q, const double *G,
                   double *rhs, int terms, hipStream_t s) {
    const Geo &g = c.g;
    if (dir == 0) {
        const long long nf = ((long long)g.nx + 3) * g.ny * g.nz;
        unsigned nb = (unsigned)((nf - 3 + (kViscXBlock - 4)) / (kViscXBlock - 3));   // blocks overlap by three
        nb = (nb + kNumXcd - 1) / kNumXcd * kNumXcd;
        hipLaunchKernelGGL(k_visc_x<NS>, dim3(nb), dim3(kViscXBlock), 0, s, U, P, Q, G, rhs, g, c.th64, terms);
        return hipGetLastError();
    }
    const int nsw = dir == 1 ? g.ny : g.nz;
    const int ntr = dir == 1 ? g.nz : g.ny;
    dim3 grid((g.nx + kViscTX - 1) / kViscTX, (nsw + kViscTS - 4) / (kViscTS - 3), ntr), block(kViscTX, kViscTS);
    if (dir == 1)
        hipLaunchKernelGGL((k_visc_tile<NS, 1>), grid, block, 0, s, U, P, Q, G, rhs, g, c.th64, terms);
    else
        hipLaunchKernelGGL((k_visc_tile<NS, 2>), grid, block, 0, s, U, P, Q, G, rhs, g, c.th64, terms);
    return hipGetLastError();
}

const NsOps kOps = {prims, sweep, sweep_vjp, sweep_frozen, face_speeds, glf, prims_vjp, cfl, transport, viscous, react_launch<NS>,
                    stage};

}  // namespace

template <int N>
const NsOps *ops_ns();

template <>
const NsOps *ops_ns<NS>() {
    return &kOps;
}

}  // namespace xf
