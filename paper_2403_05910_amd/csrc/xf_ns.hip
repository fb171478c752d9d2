// xf_ns.hip -- launchers of the species-templated kernels for one species
// count.  Compiled once per N with -DXF_NS=N; each object exports
// xf::ops_ns<N>(), which the C ABI collects into its dispatch table.
#include "xf_forward.hpp"
#include "xf_vjp.hpp"

#ifndef XF_NS
#error "compile with -DXF_NS=<species count>"
#endif

namespace xf {
namespace {

constexpr int NS = XF_NS;

unsigned blocks_for(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

hipError_t prims(const LaunchCtx &c, const double *U, double *P, float *Uf, float *Pf, int all_cells,
                 hipStream_t s) {
    hipLaunchKernelGGL(k_prims<NS>, dim3(blocks_for(c.g.cells, 256)), dim3(256), 0, s, U, P, c.g, c.th64,
                       c.status, Uf, Pf, all_cells);
    return hipGetLastError();
}

template <typename R, typename S>
hipError_t sweep_t(const LaunchCtx &c, const ThermoK<R> &th, int dir, int accumulate, const S *U, const S *P,
                   double *rhs, const StageArgs &sa, hipStream_t s) {
    const Geo &g = c.g;
    if (dir == 0) {
        const long long nf = (long long)(g.nx + 1) * g.ny * g.nz;
        const unsigned nb = (unsigned)((nf - 1 + (kXBlock - 2)) / (kXBlock - 1));   // blocks overlap by one face
        hipLaunchKernelGGL((k_sweep_x<NS, R, S>), dim3(nb), dim3(kXBlock), 0, s, U, P, rhs, g, th, accumulate, sa,
                           c.status);
        return hipGetLastError();
    }
    const int ntr = dir == 1 ? g.nz : g.ny;
    const int nsw = dir == 1 ? g.ny : g.nz;
    const unsigned tiles = (unsigned)((nsw + kTileS - 2) / (kTileS - 1));
    // c.variant (measurement only): 0 default = tiled, 1 = marching with the
    // previous flux in registers, 2 = marching with it in LDS
    if (c.variant == 0 && ntr <= 65535 && tiles <= 65535u) {
        dim3 grid((g.nx + kTileX - 1) / kTileX, tiles, ntr), block(kTileX, kTileS);
        if (dir == 1)
            hipLaunchKernelGGL((k_sweep_tile<NS, R, 1, S>), grid, block, 0, s, U, P, rhs, g, th, accumulate, sa,
                               c.status);
        else
            hipLaunchKernelGGL((k_sweep_tile<NS, R, 2, S>), grid, block, 0, s, U, P, rhs, g, th, accumulate, sa,
                               c.status);
        return hipGetLastError();
    }
    int nseg, seglen;
    march_shape(g, dir, &nseg, &seglen);
    dim3 grid((g.nx + 63) / 64, (ntr + 3) / 4, nseg), block(64, 4);
    const bool regs = c.variant != 2;
    if (dir == 1) {
        if (regs)
            hipLaunchKernelGGL((k_sweep_march<NS, R, 1, 1, S>), grid, block, 0, s, U, P, rhs, g, th, seglen,
                               accumulate, sa, c.status);
        else
            hipLaunchKernelGGL((k_sweep_march<NS, R, 1, 0, S>), grid, block, 0, s, U, P, rhs, g, th, seglen,
                               accumulate, sa, c.status);
    } else {
        if (regs)
            hipLaunchKernelGGL((k_sweep_march<NS, R, 2, 1, S>), grid, block, 0, s, U, P, rhs, g, th, seglen,
                               accumulate, sa, c.status);
        else
            hipLaunchKernelGGL((k_sweep_march<NS, R, 2, 0, S>), grid, block, 0, s, U, P, rhs, g, th, seglen,
                               accumulate, sa, c.status);
    }
    return hipGetLastError();
}

hipError_t sweep(const LaunchCtx &c, int dir, int accumulate, const double *U, const double *P, const float *Uf,
                 const float *Pf, double *rhs, const StageArgs &sa, hipStream_t s) {
    if (c.precision == XF_PREC_MIXED) return sweep_t<float, float>(c, c.th32, dir, accumulate, Uf, Pf, rhs, sa, s);
    return sweep_t<double, double>(c, c.th64, dir, accumulate, U, P, rhs, sa, s);
}

MarchGeo march_geo(const Geo &g, int dir) {
    MarchGeo m;
    m.origin = (long long)g.gz * g.sz + (long long)g.gy * g.sy + g.gx;
    if (dir == 0) {
        m.sl = g.sy; m.nl = g.ny;
        m.st = g.sz; m.nt = g.nz;
        m.ss = 1;    m.nsw = g.nx;
    } else if (dir == 1) {
        m.sl = 1;    m.nl = g.nx;
        m.st = g.sz; m.nt = g.nz;
        m.ss = g.sy; m.nsw = g.ny;
    } else {
        m.sl = 1;    m.nl = g.nx;
        m.st = g.sy; m.nt = g.ny;
        m.ss = g.sz; m.nsw = g.nz;
    }
    return m;
}

template <typename R>
hipError_t sweep_vjp_t(const LaunchCtx &c, const ThermoK<R> &th, int dir, const double *U, const double *P,
                       const double *rbar, double *Ubar, double *Pbar, hipStream_t s) {
    const Geo &g = c.g;
    const MarchGeo mg = march_geo(g, dir);
    const double id = dir == 0 ? g.idx : (dir == 1 ? g.idy : g.idz);
    // segments of at least 8 faces (two segments a column apart never touch
    // the same cell); enough of them to fill the chip
    const long long cols = (long long)mg.nl * mg.nt;
    const int nfaces = mg.nsw + 1;
    int seglen = nfaces;
    const long long want = 16384;   // threads in flight per launch
    if (cols < want) {
        const long long segs = (want + cols - 1) / cols;
        seglen = (int)((nfaces + segs - 1) / segs);
        if (seglen < 8) seglen = 8;
    }
    const int nseg = (nfaces + seglen - 1) / seglen;
    dim3 grid((mg.nl + 63) / 64, (mg.nt + 3) / 4, (nseg + 1) / 2), block(64, 4);
    for (int parity = 0; parity < 2; ++parity) {
        if (dir == 0)
            hipLaunchKernelGGL((k_sweep_vjp<NS, R, 0>), grid, block, 0, s, U, P, rbar, Ubar, Pbar, g.cells, mg,
                               th, id, seglen, parity);
        else if (dir == 1)
            hipLaunchKernelGGL((k_sweep_vjp<NS, R, 1>), grid, block, 0, s, U, P, rbar, Ubar, Pbar, g.cells, mg,
                               th, id, seglen, parity);
        else
            hipLaunchKernelGGL((k_sweep_vjp<NS, R, 2>), grid, block, 0, s, U, P, rbar, Ubar, Pbar, g.cells, mg,
                               th, id, seglen, parity);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t sweep_vjp(const LaunchCtx &c, int dir, const double *U, const double *P, const double *rbar,
                     double *Ubar, double *Pbar, hipStream_t s) {
    if (c.precision == XF_PREC_MIXED) return sweep_vjp_t<float>(c, c.th32, dir, U, P, rbar, Ubar, Pbar, s);
    return sweep_vjp_t<double>(c, c.th64, dir, U, P, rbar, Ubar, Pbar, s);
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

const NsOps kOps = {prims, sweep, sweep_vjp, prims_vjp, cfl};

}  // namespace

template <int N>
const NsOps *ops_ns();

template <>
const NsOps *ops_ns<NS>() {
    return &kOps;
}

}  // namespace xf
