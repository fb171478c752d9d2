// xf_misc.hip -- species-independent kernels: boundary ghosts and their
// adjoint, ghost zeroing, SSP-RK3 stage combinations (Eq. 16) and their
// adjoint, CFL finish, copies.
#include "xf_common.hpp"

namespace xf {
namespace {

unsigned blocks_for(long long n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// Ghost layers of direction d: one thread per (field, other two padded
// coordinates), both sides and all ghost layers in that thread.  The other
// two coordinates are enumerated with the faster one first so that y and z
// fills are coalesced along x.
__device__ __forceinline__ void ghost_geometry(const Geo &g, int d, long long o, long long &base, long long &step,
                                               int &n) {
    if (d == 0) {
        const long long y = o % g.py, z = o / g.py;
        base = z * g.sz + y * g.sy;
        step = 1;
        n = g.nx;
    } else if (d == 1) {
        const long long x = o % g.px, z = o / g.px;
        base = z * g.sz + x;
        step = g.sy;
        n = g.ny;
    } else {
        const long long x = o % g.px, y = o / g.px;
        base = y * g.sy + x;
        step = g.sz;
        n = g.nz;
    }
}

__device__ __forceinline__ long long others(const Geo &g, int d) {
    return d == 0 ? (long long)g.py * g.pz : (d == 1 ? (long long)g.px * g.pz : (long long)g.px * g.py);
}

__device__ __forceinline__ int ghost_dst(int sd, int l, int n, int ng) { return sd == 0 ? l : ng + n + l; }
__device__ __forceinline__ int ghost_width(const Geo &g, int d) { return d == 0 ? g.gx : (d == 1 ? g.gy : g.gz); }

template <typename T>
__global__ __launch_bounds__(256) void k_fill(T *U, Geo g, int nv, int d) {
    const long long no = others(g, d);
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= no * nv) return;
    const long long f = q / no, o = q - f * no;
    long long base, step;
    int n;
    ghost_geometry(g, d, o, base, step, n);
    T *u = U + f * g.cells + base;
    const int ng = ghost_width(g, d);
#pragma unroll
    for (int sd = 0; sd < 2; ++sd) {
        const int bc = g.bc[2 * d + sd];
#pragma unroll
        for (int l = 0; l < 4; ++l)   // ng <= 4 layers
            if (l < ng) u[ghost_dst(sd, l, n, ng) * step] = u[ghost_src(bc, sd, l, n, ng) * step];
    }
}

// The x ghosts, one thread per ghost cell: a row's 2 ng ghost cells are
// consecutive lanes, so one instruction touches each row's two ends once
// (the per-row form of k_fill touches a different row in every lane).  The
// sources are interior cells, so the copies are independent.
template <typename T>
__global__ __launch_bounds__(256) void k_fill_x(T *U, Geo g, int nv) {
    const int ng = g.gx, w = 2 * ng;
    const long long rows = (long long)g.py * g.pz;
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= rows * w * nv) return;
    const int k = (int)(q % w);
    const long long r = q / w;
    const long long o = r % rows, f = r / rows;
    const int sd = k / ng, l = k - sd * ng;
    T *u = U + f * g.cells + (o / g.py) * g.sz + (o % g.py) * g.sy;
    u[ghost_dst(sd, l, g.nx, ng)] = u[ghost_src(g.bc[sd], sd, l, g.nx, ng)];
}

// Adjoint of k_fill: every ghost cotangent is added to its source and zeroed,
// in the reverse order of the forward copies.
__global__ __launch_bounds__(256) void k_fill_vjp(double *Ub, Geo g, int nv, int d) {
    const long long no = others(g, d);
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= no * nv) return;
    const long long f = q / no, o = q - f * no;
    long long base, step;
    int n;
    ghost_geometry(g, d, o, base, step, n);
    double *u = Ub + f * g.cells + base;
    const int ng = ghost_width(g, d);
#pragma unroll
    for (int sd = 1; sd >= 0; --sd) {
        const int bc = g.bc[2 * d + sd];
#pragma unroll
        for (int l = 3; l >= 0; --l) {   // ng <= 4 layers
            if (l >= ng) continue;
            const long long dst = ghost_dst(sd, l, n, ng) * step;
            const double v = u[dst];
            u[dst] = 0.0;
            u[ghost_src(bc, sd, l, n, ng) * step] += v;
        }
    }
}

__global__ __launch_bounds__(256) void k_zero_ghosts(double *A, Geo g, int nv) {
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= g.cells * nv) return;
    const long long idx = q % g.cells;
    const int x = (int)(idx % g.px);
    const long long r = idx / g.px;
    const int y = (int)(r % g.py), z = (int)(r / g.py);
    const bool ghost = x < g.gx || x >= g.gx + g.nx || y < g.gy || y >= g.gy + g.ny || z < g.gz ||
                       z >= g.gz + g.nz;
    if (ghost) A[q] = 0.0;
}

// rhs = ((Lz + Ly) + Lx) on the interior cells from FP32 per-direction
// differences (the order in which the FP64 sweeps accumulate).
__global__ __launch_bounds__(256) void k_sum_dirs(double *rhs, const float *Lx, const float *Ly, const float *Lz,
                                                  Geo g, int nv) {
    const long long nint = (long long)g.nx * g.ny * g.nz;
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nint * nv) return;
    const long long f = q / nint, r = q - f * nint;
    const int i = (int)(r % g.nx);
    const long long r2 = r / g.nx;
    const int j = (int)(r2 % g.ny), k = (int)(r2 / g.ny);
    const long long o = f * g.cells + (long long)(g.gz + k) * g.sz + (long long)(g.gy + j) * g.sy + (g.gx + i);
    double L = 0.0;
    bool first = true;
    if (Lz) {
        L = (double)Lz[o];
        first = false;
    }
    if (Ly) {
        L = first ? (double)Ly[o] : L + (double)Ly[o];
        first = false;
    }
    if (Lx) L = first ? (double)Lx[o] : L + (double)Lx[o];
    rhs[o] = L;
}

// y = a x + b y (b == 0 ignores the old y, so y may hold anything)
__global__ __launch_bounds__(256) void k_axpby(long long n, double a, const double *x, double b, double *y) {
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    y[q] = b == 0.0 ? a * x[q] : a * x[q] + b * y[q];
}

// Adjoint of one stage given the stage cotangent lam (of the stage output)
// and mu = J(V)^T lam (the rhs-VJP at that stage's input V):
//   stage 3 (U = 1/3 V0 + 2/3 (V2 + dt L(V2))): lam0 = lam/3;      lam = 2/3 (lam + dt mu)
//   stage 2 (U = 3/4 V0 + 1/4 (V1 + dt L(V1))): lam0 += 3/4 lam;   lam = 1/4 (lam + dt mu)
//   stage 1 (U = V0 + dt L(V0)):                lam0 += lam + dt mu
__global__ __launch_bounds__(256) void k_rk3_stage_vjp(double *lam, double *lam0, const double *mu, long long n,
                                                       int stage, double dt, const double *dt_dev) {
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= n) return;
    const double h = dt_dev ? *dt_dev : dt;
    const double l = lam[q];
    if (stage == 3) {
        lam0[q] = l / 3.0;
        lam[q] = 2.0 / 3.0 * (l + h * mu[q]);
    } else if (stage == 2) {
        lam0[q] += 0.75 * l;
        lam[q] = 0.25 * (l + h * mu[q]);
    } else {
        lam0[q] += l + h * mu[q];
    }
}

__global__ void k_cfl_reset(unsigned long long *mx) { *mx = 0ull; }

__global__ void k_reset_u64(unsigned long long *p, int n) {
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0ull;
}

__global__ void k_cfl_finish(const unsigned long long *mx, double cfl, double *dt) {
    *dt = cfl / __longlong_as_double((long long)*mx);
}

__global__ __launch_bounds__(256) void k_copy(long long n, const double *src, double *dst) {
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) dst[q] = src[q];
}

// Cell-centred velocity gradient G[3 a + b] = d u_b / d x_a by the
// fourth-order difference (u_{-2} - 8 u_{-1} + 8 u_{+1} - u_{+2}) / (12 dx_a)
// at every cell two or more layers inside the padded extent along an active
// axis a (the velocity u_b is Q[2 + b] of the transport pass); the other
// entries are left as they are (no face stencil reads them).
__global__ __launch_bounds__(256) void k_vel_grad(const double *__restrict__ Q, double *__restrict__ G, Geo g) {
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= g.cells) return;
    const long long C = g.cells;
    const int x = (int)(idx % g.px);
    const long long r = idx / g.px;
    const int co[3] = {x, (int)(r % g.py), (int)(r / g.py)};
    const int n[3] = {g.nx, g.ny, g.nz}, p[3] = {g.px, g.py, g.pz};
    const long long st[3] = {1, g.sy, g.sz};
    const double ih[3] = {g.idx, g.idy, g.idz};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        if (n[a] <= 1 || co[a] < 2 || co[a] >= p[a] - 2) continue;
        const long long s = st[a];
        const double f = ih[a] * (1.0 / 12.0);
#pragma unroll
        for (int b = 0; b < 3; ++b) {
            const double *u = Q + (2 + b) * C + idx;
            G[(3 * a + b) * C + idx] = (u[-2 * s] - 8.0 * u[-s] + 8.0 * u[s] - u[2 * s]) * f;
        }
    }
}

__global__ __launch_bounds__(256) void k_zero(long long n, double *dst) {
    const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q < n) dst[q] = 0.0;
}

}  // namespace

template <typename T>
hipError_t fill_ghosts_t(const LaunchCtx &c, int nv, T *U, hipStream_t s) {
    const Geo &g = c.g;
    const int n[3] = {g.nx, g.ny, g.nz};
    for (int d = 0; d < 3; ++d) {
        if (n[d] <= 1) continue;
        const long long no = d == 0 ? (long long)g.py * g.pz : (d == 1 ? (long long)g.px * g.pz : (long long)g.px * g.py);
        if (d == 0 && g.gx > 0)
            hipLaunchKernelGGL(k_fill_x<T>, dim3(blocks_for(no * 2 * g.gx * nv, 256)), dim3(256), 0, s, U, g, nv);
        else
            hipLaunchKernelGGL(k_fill<T>, dim3(blocks_for(no * nv, 256)), dim3(256), 0, s, U, g, nv, d);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_fill_ghosts(const LaunchCtx &c, int nv, double *U, hipStream_t s) {
    return fill_ghosts_t(c, nv, U, s);
}

hipError_t launch_fill_ghosts_vjp(const LaunchCtx &c, int nv, double *Ub, hipStream_t s) {
    const Geo &g = c.g;
    const int n[3] = {g.nx, g.ny, g.nz};
    for (int d = 2; d >= 0; --d) {
        if (n[d] <= 1) continue;
        const long long no = d == 0 ? (long long)g.py * g.pz : (d == 1 ? (long long)g.px * g.pz : (long long)g.px * g.py);
        hipLaunchKernelGGL(k_fill_vjp, dim3(blocks_for(no * nv, 256)), dim3(256), 0, s, Ub, g, nv, d);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t launch_zero_ghosts(const LaunchCtx &c, int nv, double *A, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_ghosts, dim3(blocks_for(c.g.cells * nv, 256)), dim3(256), 0, s, A, c.g, nv);
    return hipGetLastError();
}

hipError_t launch_rk3_stage_vjp(const LaunchCtx &c, int nv, int stage, double *lam, double *lam0, double *mu,
                                const double *dt_dev, double dt, hipStream_t s) {
    const long long n = c.g.cells * nv;
    hipLaunchKernelGGL(k_rk3_stage_vjp, dim3(blocks_for(n, 256)), dim3(256), 0, s, lam, lam0, mu, n, stage, dt,
                       dt_dev);
    return hipGetLastError();
}

hipError_t launch_sum_dirs(const LaunchCtx &c, int nv, double *rhs, const float *const L[3], hipStream_t s) {
    const long long n = (long long)c.g.nx * c.g.ny * c.g.nz * nv;
    hipLaunchKernelGGL(k_sum_dirs, dim3(blocks_for(n, 256)), dim3(256), 0, s, rhs, L[0], L[1], L[2], c.g, nv);
    return hipGetLastError();
}

hipError_t launch_axpy_state(long long n, double a, const double *x, double b, double *y, hipStream_t s) {
    hipLaunchKernelGGL(k_axpby, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, a, x, b, y);
    return hipGetLastError();
}

hipError_t launch_vel_grad(const LaunchCtx &c, const double *Q, double *G, hipStream_t s) {
    hipLaunchKernelGGL(k_vel_grad, dim3(blocks_for(c.g.cells, 256)), dim3(256), 0, s, Q, G, c.g);
    return hipGetLastError();
}

hipError_t launch_cfl_reset(unsigned long long *mx, hipStream_t s) {
    hipLaunchKernelGGL(k_cfl_reset, dim3(1), dim3(1), 0, s, mx);
    return hipGetLastError();
}

hipError_t launch_reset_u64(unsigned long long *p, int n, hipStream_t s) {
    if (n < 1 || n > 64) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_reset_u64, dim3(1), dim3(64), 0, s, p, n);
    return hipGetLastError();
}

hipError_t launch_cfl_finish(const unsigned long long *mx, double cfl, double *dt_dev, hipStream_t s) {
    hipLaunchKernelGGL(k_cfl_finish, dim3(1), dim3(1), 0, s, mx, cfl, dt_dev);
    return hipGetLastError();
}

hipError_t launch_copy(long long n, const double *src, double *dst, hipStream_t s) {
    hipLaunchKernelGGL(k_copy, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, src, dst);
    return hipGetLastError();
}

hipError_t launch_zero(long long n, double *dst, hipStream_t s) {
    hipLaunchKernelGGL(k_zero, dim3(blocks_for(n, 256)), dim3(256), 0, s, n, dst);
    return hipGetLastError();
}

}  // namespace xf
