// xf_forward.hpp -- forward kernels of the convective right-hand side.
//
//   k_prims       primitive recovery with the Newton temperature (Eq. 7, 21)
//   k_sweep_x     x-direction flux difference, one face per thread
//   k_sweep_tile  y/z-direction flux difference, tiles of one face per thread
//   k_cfl         CFL reduction (Eq. 17), wavefront max + one 64-bit atomic
//   k_stage_sum   SSP-RK3 stage (Eq. 16) from the per-direction residuals
#pragma once

#include "xf_face.hpp"

namespace xf {

// ---------------------------------------------------------------------------
// primitive variables and Newton temperature (always FP64)
// ---------------------------------------------------------------------------
// The mixture's internal energy and C_v at fixed Y as polynomials in T:
// e(T) = sum_k E_k T^k (k = 0..5), C_v(T) = sum_k C_k T^k (k = 0..4), the
// species tables weighted by Y once per solve, so that a Newton iteration
// costs two Horner evaluations instead of one per species.
struct MixPoly {
    double E[6], C[5];
    __device__ __forceinline__ double e(double T) const {
        return ((((E[5] * T + E[4]) * T + E[3]) * T + E[2]) * T + E[1]) * T + E[0];
    }
    __device__ __forceinline__ double cv(double T) const {
        return (((C[4] * T + C[3]) * T + C[2]) * T + C[1]) * T + C[0];
    }
};

// Newton on e(T) = e (Eq. 21) with the mixture polynomials m:
// T <- T + (e - e(T)) / C_v(T) from the start T clamped into the bracket
// [T_lo, T_hi] where there is one; every evaluation narrows the bracket
// (e(T) > e: hi = T, else lo = T) and a step that leaves the closed bracket
// is replaced by bisection.  Stop when |dT| <= 1e-11 |T|, then one more
// Newton update.  Returns false if not converged in 50 iterations.  The
// primitive pass starts from the cold start e / C_v(T_ref); the reaction
// step from the cell's previous temperature (the root does not depend on
// the start).
__device__ __forceinline__ bool newton_poly(bool bracket, double T_lo, double T_hi, const MixPoly &m, double e,
                                            double &T) {
    double lo = T_lo, hi = T_hi;
    if (bracket) T = T < lo ? lo : (T > hi ? hi : T);
    for (int it = 0; it < kNewtonMaxIt; ++it) {
        const double f = m.e(T) - e;
        double Tn = T - f / m.cv(T);
        if (bracket) {
            if (f > 0.0)
                hi = fmin(hi, T);
            else
                lo = fmax(lo, T);
            if (Tn < lo || Tn > hi) Tn = 0.5 * (lo + hi);
        }
        const bool conv = fabs(Tn - T) <= kNewtonTol * fabs(T);
        T = Tn;
        if (conv) {
            T = T - (m.e(T) - e) / m.cv(T);
            return true;
        }
    }
    return false;
}

// The fold of the species tables with Y (the table at hand, by value or
// in kernel arguments).
template <int NS>
__device__ __forceinline__ void mix_poly_of(const ThermoK<double> &th, const double *Y, MixPoly &m) {
#pragma unroll
    for (int k = 0; k < 6; ++k) m.E[k] = 0.0;
#pragma unroll
    for (int k = 0; k < 5; ++k) m.C[k] = 0.0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
#pragma unroll
        for (int k = 0; k < 6; ++k) m.E[k] += Y[s] * th.e[s][k];
#pragma unroll
        for (int k = 0; k < 5; ++k) m.C[k] += Y[s] * th.cv[s][k];
    }
}

// The primitive variables of one cell from its conserved values u(f)
// (f = 0..N+3): T by Newton (Eq. 21) on the mixture polynomials,
// p = rho Rbar T, c^2 = (1 + Rbar / C_v) Rbar T, 1/rho; returns the cell's
// status flags.
template <int NS, class Get>
__device__ __forceinline__ unsigned cell_prims(const Get &u, const ThermoK<double> &th, double &T, double &p,
                                               double &c, double &rinv) {
    double Y[NS];
    double rho = 0.0;
    bool finite = true;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        Y[s] = u(s);
        rho += Y[s];
        finite = finite && isfinite(Y[s]);
    }
    rinv = 1.0 / rho;
    unsigned flags = 0;
    bool yneg = false;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        Y[s] *= rinv;
        yneg = yneg || (Y[s] < -1e-12);
    }
    const double mx = u(NS), my = u(NS + 1), mz = u(NS + 2);
    const double E = u(NS + 3);
    finite = finite && isfinite(mx) && isfinite(my) && isfinite(mz) && isfinite(E);
    const double uu = mx * rinv, v = my * rinv, w = mz * rinv;
    const double e = E * rinv - 0.5 * (uu * uu + v * v + w * w);
    // Newton on the mixture's folded polynomials from the cold start
    // e / C_v(T_ref)
    MixPoly m;
    mix_poly_of<NS>(th, Y, m);
    T = e / m.cv(th.T_ref);
    const bool conv = newton_poly(th.bracket, th.T_lo, th.T_hi, m, e, T);
    double Rb = 0.0;
#pragma unroll
    for (int s = 0; s < NS; ++s) Rb += Y[s] * th.Rs[s];
    const double cv = m.cv(T);
    p = rho * Rb * T;
    c = sqrt((1.0 + Rb / cv) * Rb * T);
    if (rho <= 0.0) flags |= XF_FLAG_RHO;
    if (yneg) flags |= XF_FLAG_Y;
    if (p <= 0.0 || T <= 0.0) flags |= XF_FLAG_P;
    if (th.bracket && (T < th.T_lo || T > th.T_hi)) flags |= XF_FLAG_TRANGE;
    if (!conv) flags |= XF_FLAG_NEWTON;
    if (!finite || !isfinite(T) || !isfinite(c)) flags |= XF_FLAG_NAN;
    return flags;
}

// P[0..3][cell] = (T, p, c, 1/rho) for every cell with at most one
// coordinate in a ghost layer (the cells axis-aligned stencils read).
// Uf, Pf (optional): FP32 copies of U and of (T, p, c, 1/rho) for the
// mixed-precision sweeps, written for the same cells; P may be null when
// only they are needed.
template <int NS>
__global__ __launch_bounds__(256) void k_prims(const double *U, double *__restrict__ P, Geo g,
                                               ThermoK<double> th, unsigned *status, float *__restrict__ Uf,
                                               float *__restrict__ Pf, int all_cells, double *Ug,
                                               unsigned long long *cfl) {
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    double sv = 0.0;   // with cfl: the cell's rate sum_d (|u_d| + c) / dx_d of Eq. 17 (interior cells)
    if (idx < g.cells) {
        const int x = (int)(idx % g.px);
        const long long r = idx / g.px;
        const int y = (int)(r % g.py);
        const int z = (int)(r / g.py);
        const int ng = (x < g.gx || x >= g.gx + g.nx) + (y < g.gy || y >= g.gy + g.ny) +
                       (z < g.gz || z >= g.gz + g.nz);
        // edge and corner ghosts lie outside every stencil
        if (ng <= 1 || all_cells) {
            const long long C = g.cells;
            // with Ug (= U): a ghost takes its boundary source's state, written
            // to the ghost as the ghost fill would.  Each ghost coordinate maps
            // to its source on its own axis (the axis-by-axis fill gives an edge
            // or corner ghost the state of the interior cell all its
            // coordinates map to); sources are interior cells, which this pass
            // does not write.
            long long src = idx;
            if (Ug && ng > 0) {
                auto map = [](int c, int n, int gw, int lo, int hi) {
                    if (c < gw) return ghost_src(lo, 0, c, n, gw);
                    if (c >= gw + n) return ghost_src(hi, 1, c - gw - n, n, gw);
                    return c;
                };
                const int sx = map(x, g.nx, g.gx, g.bc[0], g.bc[1]), sy = map(y, g.ny, g.gy, g.bc[2], g.bc[3]),
                          sz = map(z, g.nz, g.gz, g.bc[4], g.bc[5]);
                src = sx + (long long)g.px * (sy + (long long)g.py * sz);
            }
            double u[NS + 4];
#pragma unroll
            for (int f = 0; f < NS + 4; ++f) u[f] = U[f * C + src];
            if (src != idx) {
#pragma unroll
                for (int f = 0; f < NS + 4; ++f) Ug[f * C + idx] = u[f];
            }
            // the FP32 copies go out before the Newton solve, from the loaded
            // values (read again after it, the state was partly evicted from
            // the L2 and fetched twice: 2.43 against 1.92 GB per launch at
            // 256^3, nine species)
            if (Uf) {
#pragma unroll
                for (int f = 0; f < NS + 4; ++f) Uf[f * C + idx] = (float)u[f];
            }
            double T, p, c, rinv;
            const unsigned flags = cell_prims<NS>([&](int f) { return u[f]; }, th, T, p, c, rinv);
            if (P) {
                P[idx] = T;
                P[C + idx] = p;
                P[2 * C + idx] = c;
                P[3 * C + idx] = rinv;
            }
            if (Uf) {
                Pf[idx] = (float)T;
                Pf[C + idx] = (float)p;
                Pf[2 * C + idx] = (float)c;
                Pf[3 * C + idx] = (float)rinv;
            }
            if (cfl && ng == 0) {   // the same sum, in the same order, as k_cfl
                double v = 0.0;
                if (g.nx > 1) v += (fabs(u[NS] * rinv) + c) * g.idx;
                if (g.ny > 1) v += (fabs(u[NS + 1] * rinv) + c) * g.idy;
                if (g.nz > 1) v += (fabs(u[NS + 2] * rinv) + c) * g.idz;
                if (v > sv) sv = v;   // NaN never wins (it is flagged)
            }
            if (flags) atomicOr(status, flags);
        }
    }
    if (cfl) {
        // block max, then one 64-bit atomicMax (positive doubles order like
        // their bit patterns), skipped when the running max is already larger
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) sv = fmax(sv, __shfl_xor(sv, off, 64));
        __shared__ double wmax[4];
        if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = sv;
        __syncthreads();
        if (threadIdx.x == 0) {
            const double m = fmax(fmax(wmax[0], wmax[1]), fmax(wmax[2], wmax[3]));
            const unsigned long long bits = (unsigned long long)__double_as_longlong(m);
            if (bits > __atomic_load_n(cfl, __ATOMIC_RELAXED)) atomicMax(cfl, bits);
        }
    }
}

// SSP-RK3 stage of Eq. 16 on the interior cells: Uout = a U0 + b (Uin + h L),
// L = ((Lx + Ly) + Lz) + Lv.  A block takes one interior row of one field
// (blockIdx.x = j + ny k, blockIdx.y = field), its threads the cells along
// x, so no index needs a 64-bit division.
template <typename LT>
__global__ __launch_bounds__(256) void k_stage_sum(double *Uout, const double *U0, const double *Uin, const LT *Lx,
                                                   const LT *Ly, const LT *Lz, const double *Lv, Geo g, double a,
                                                   double b, double dt, const double *dt_dev) {
    const int row = blockIdx.x;
    const int j = row % g.ny, k = row / g.ny;
    const long long base = (long long)blockIdx.y * g.cells + (long long)(g.gz + k) * g.sz +
                           (long long)(g.gy + j) * g.sy + g.gx;
    const double h = dt_dev ? *dt_dev : dt;
    for (int i = threadIdx.x; i < g.nx; i += blockDim.x) {
        const long long o = base + i;
        double L = 0.0;
        if (Lx) L = (double)Lx[o];
        if (Ly) L = L + (double)Ly[o];
        if (Lz) L = L + (double)Lz[o];
        if (Lv) L = L + Lv[o];
        const double v = Uin[o] + h * L;
        Uout[o] = a == 0.0 ? b * v : a * U0[o] + b * v;
    }
}

// ---------------------------------------------------------------------------
// Phase fences, loop form and occupancy per kernel flavour, chosen from the
// compiler's resource report and timings at 256^3, nine species:
// * the x sweeps run the species loops rolled (face_flux_to ROLL): FP64 at
//   three waves per SIMD without spill (168 registers; 2.20 -> 2.00 ms per
//   launch), FP32 1.74 -> 1.33 ms;
// * the y/z tiles roll their species loops too (their shapes, LDS and
//   waves per SIMD are at TileShape);
// * the positivity-blend instances stay at two waves (at three the FP64
//   blended step went from 37.5 to 47.7 ms), the FP64 WENO7 instances at
//   one (at two they spilled 324-460 bytes per lane; at one they keep their
//   overflow in the accumulation registers, 61.7 -> 50.3 ms per step).
template <typename R>
struct SweepTune {
    static constexpr bool fence_face = false;   // face-per-thread sweeps (x, tiled y/z)
    static constexpr bool roll_tile = true;     // species loops rolled in the y/z tiles
};
template <>
struct SweepTune<double> {
    static constexpr bool fence_face = true;
    static constexpr bool roll_tile = true;
};
// Waves per SIMD asked of a face-per-thread sweep (X: the x sweep).
template <typename R, int REC, bool X, bool PP>
constexpr int sweep_waves() {
    if (sizeof(R) == 4) return X ? 4 : 1;
    if (REC == kReconWeno7) return 1;
    if (!X && !PP && REC == kReconWeno5) return 3;     // the exchanging FP64 tiles (CU6 spills at three)
    return (X && !PP && REC == kReconWeno5) ? 3 : 2;   // the rolled CU6 x face spills ~100 bytes at three
}

// lam = D dt / dx_d of the positivity blend (D active dimensions).
template <typename R>
__device__ __forceinline__ R pp_lambda(const Geo &g, const StageArgs &sa, double idx) {
    const double h = sa.dt_dev ? *sa.dt_dev : sa.dt;
    const int D = (g.nx > 1) + (g.ny > 1) + (g.nz > 1);
    return R(D * h * idx);
}

// Write the finished residual d of one field at one cell: rhs = d, or
// rhs += d when accumulating (FP64 output only; an FP32 difference is stored
// as computed, exactly).
template <typename OT>
__device__ __forceinline__ void put_result(OT *__restrict__ rhs, long long o, double d, int accumulate) {
    rhs[o] = accumulate ? OT(rhs[o] + d) : OT(d);
}

// ---------------------------------------------------------------------------
// x sweep: faces linearised over interior rows (face i of row r = the face
// between interior cells i-1 and i, i = 0..nx).  A block of 256 threads takes
// fpb <= 256 consecutive faces and blocks overlap by one face, so every cell
// whose two faces lie in a block gets (F^_{i-1/2} - F^_{i+1/2}) / dx there.
// The block first copies U and the primitives of its stencil cells to LDS,
// row segment by row segment: the faces of one row need their own cells plus
// 2 RAD - 1 more, so a block touching nseg rows stages fpb + nseg (2 RAD - 1)
// cells.  Unstaged, the six overlapping stencil loads of each field went to
// the caches, and at three blocks per CU the working set outgrew the L2:
// 4.0 GB fetched per launch at 256^3, nine species, against 2.33 GB of
// stencil inputs.  fpb is 256 whenever a row holds at least 255 faces; for
// shorter rows the launch lowers it until the staged cells fit x_stage_cells.
// The FP64 WENO5 instances without the blend hand each flux component to
// the cell below as soon as it is final, taking the neighbouring face's
// value from the next lane down; the first lane of each wave takes it
// through LDS.  The others keep the block's fluxes in LDS (the blend limits
// whole flux vectors).  A mixed RK3 step's x sweep also finishes the stage (sa.Uout).
// ---------------------------------------------------------------------------
constexpr int kXBlock = 256;

template <int RAD>
constexpr int x_stage_cells() { return kXBlock + 2 * (2 * RAD - 1); }

// Faces per x-sweep block for rows of nfx faces: the largest count whose
// worst-case staging (a window of fpb faces spans at most
// ceil((fpb - 1) / nfx) + 1 rows) fits x_stage_cells.
template <int RAD>
inline int x_faces_per_block(long long nfx) {
    constexpr int gap = 2 * RAD - 1;
    int fpb = kXBlock;
    while (fpb > 2 && fpb + ((fpb - 1 + nfx - 1) / nfx + 1) * gap > x_stage_cells<RAD>()) --fpb;
    return fpb;
}

// Exchanging x sweeps: FP64 WENO5 (three waves per SIMD).  The CU6 and
// WENO7 faces (two and one waves per SIMD) took 3.09 ms per x sweep
// exchanging against 2.62 and 2.65 ms with the fluxes in LDS.
template <typename R, int REC>
struct XShape {
    static constexpr bool exchange = sizeof(R) == 8 && REC == kReconWeno5;
};

template <int NS, typename R, typename S, bool PP, int SPD, int REC>
__global__ __launch_bounds__(kXBlock) __attribute__((amdgpu_waves_per_eu(sweep_waves<R, REC, true, PP>()))) void k_sweep_x(
    const S *__restrict__ U, const S *__restrict__ P, R *__restrict__ rhs, Geo g, ThermoK<R> th, int accumulate,
    StageArgs sa, unsigned *status, Dissip ds, int fpb) {
    constexpr int NV = NS + 4;
    constexpr int RAD = stencil_radius(REC);
    constexpr int GAP = 2 * RAD - 1;
    constexpr int XC = x_stage_cells<RAD>();
    constexpr bool EXCH = XShape<R, REC>::exchange && !PP;
    constexpr int NW = kXBlock / 64;
    __shared__ R sF[EXCH ? 1 : NV][EXCH ? 1 : kXBlock];
    __shared__ R sEdge[2][EXCH ? NW : 1][EXCH ? NV : 1];
    __shared__ S xf_xstage[(NV + 4) * XC];
    unsigned lb, u1, u2;
    xcd_block(lb, u1, u2);
    const int t = threadIdx.x;
    const long long nfx = (long long)g.nx + 1;
    const long long nfaces = nfx * g.ny * g.nz;
    const long long f0 = (long long)lb * (fpb - 1);
    if (f0 >= nfaces) return;   // blocks that round the grid up to a multiple of 8
    const long long flast = min(f0 + fpb - 1, nfaces - 1);
    // the block's first face: face i0 of row row0 = (j0, k0); its faces lie
    // in rows row0 .. row0 + nseg - 1 (segment sg = row row0 + sg), so the
    // per-cell and per-face indexing below needs 32-bit divisions only
    const long long row0 = f0 / nfx;
    const int i0 = (int)(f0 - row0 * nfx);
    const int j0 = (int)(row0 % g.ny);
    const long long k0 = row0 / g.ny;
    const int nfx32 = g.nx + 1;
    auto row_base = [&](int sg) {
        int j = j0 + sg;
        long long k = k0;
        if (j >= g.ny) {
            k += j / g.ny;
            j %= g.ny;
        }
        return (g.gz + k) * g.sz + (long long)(g.gy + j) * g.sy + g.gx;
    };
    {
        // staged cell e: segment sg = (e + i0) / W, W = nfx + GAP, x index
        // e + i0 - sg W - RAD of that row (segment 0 starts at face i0, the
        // others at face 0)
        const int nseg = (int)(flast / nfx - row0) + 1;
        const int ncell = (int)(flast - f0 + 1) + nseg * GAP;
        const int W = nfx32 + GAP;
        for (int e = t; e < ncell; e += kXBlock) {
            const int sg = (e + i0) / W;
            const int cx = e + i0 - sg * W - RAD;
            const long long cell = row_base(sg) + cx;
#pragma unroll
            for (int q = 0; q < NV; ++q) xf_xstage[q * XC + e] = U[q * g.cells + cell];
#pragma unroll
            for (int q = 0; q < 4; ++q) xf_xstage[(NV + q) * XC + e] = P[q * g.cells + cell];
        }
    }
    __syncthreads();
    const long long f = f0 + t;
    const bool valid = t < fpb && f < nfaces;
    const int lane = t & 63, w = t >> 6;
    int i = 0;
    unsigned flags = 0;
    long long rowbase = 0;
    const R id = R(g.idx);
    // the result of interior cell `cell` from its flux difference L (x part)
    auto emit = [&](int q, long long cell, double L) {
        const long long o = q * g.cells + cell;
        if (sa.Uout) {
            const double h = sa.dt_dev ? *sa.dt_dev : sa.dt;
            if constexpr (sizeof(R) == 8) {
                if (sa.Ly64) L = L + sa.Ly64[o];
                if (sa.Lz64) L = L + sa.Lz64[o];
            } else {
                if (sa.Ly32) L = L + (double)sa.Ly32[o];
                if (sa.Lz32) L = L + (double)sa.Lz32[o];
            }
            if (sa.Lv) L = L + sa.Lv[o];
            const double v = sa.Uin[o] + h * L;
            sa.Uout[o] = sa.a == 0.0 ? sa.b * v : sa.a * sa.U0[o] + sa.b * v;
        } else {
            put_result(rhs, o, L, accumulate);
        }
    };
    if (valid) {
        const int sg = (t + i0) / nfx32;
        i = t + i0 - sg * nfx32;
        rowbase = row_base(sg);
        // stencil cell m of face i (cell i - RAD + m of its row) is staged at
        // t + sg GAP + m
        StencilLds<NV, S> st{(const __attribute__((address_space(3))) S *)xf_xstage, t + sg * GAP, 1, XC};
        if constexpr (SPD == kViscFrozen) ds.fidx = f;   // x faces: i + (nx + 1) (j + ny k)
        if constexpr (EXCH) {
            face_flux_to<NS, R, 0, SweepTune<R>::fence_face, SPD, REC, true, true>(
                st, th,
                [&](int q, R v) {
                    // face f - 1 is lane t - 1, valid wherever face f is
                    const R vb = __shfl_up(v, 1);
                    if (lane > 0 && i > 0) emit(q, rowbase + i - 1, double((vb - v) * id));
                    if (lane == 63) sEdge[0][w][q] = v;
                    if (lane == 0) sEdge[1][w][q] = v;
                },
                flags, ds);
        } else {
            face_flux_to<NS, R, 0, SweepTune<R>::fence_face, SPD, REC, !PP, true>(
                st, th, [&](int q, R v) { sF[q][t] = v; }, flags, ds);
            if constexpr (PP) {
                R Fq[NV];
#pragma unroll
                for (int q = 0; q < NV; ++q) Fq[q] = sF[q][t];
                pp_limit<NS, R, 0, RAD>(st, pp_lambda<R>(g, sa, g.idx), Fq);
#pragma unroll
                for (int q = 0; q < NV; ++q) sF[q][t] = Fq[q];
            }
        }
    }
    __syncthreads();
    if constexpr (EXCH) {
        // the cell between the last face of wave w - 1 and the first of w
        if (valid && lane == 0 && w > 0 && i > 0) {
#pragma unroll
            for (int q = 0; q < NV; ++q)
                emit(q, rowbase + i - 1, double((sEdge[0][w - 1][q] - sEdge[1][w][q]) * id));
        }
    } else if (valid && t > 0 && i > 0) {
#pragma unroll
        for (int q = 0; q < NV; ++q) emit(q, rowbase + i - 1, double((sF[q][t - 1] - sF[q][t]) * id));
    }
    if (flags) atomicOr(status, flags);
}

// ---------------------------------------------------------------------------
// Tiled y/z sweep: one face per thread, like the x sweep.  A block is a tile
// of TileShape::x x-columns by TileShape::s consecutive faces along the
// sweep axis (in one plane of the third axis); tiles overlap by one face
// along the sweep axis, so each finishes s - 1 cells per column.  Lanes run
// along x, so the staging loads of a wave read whole row segments.  Tiles
// that are neighbours along x or the sweep axis share stencil rows and are
// numbered to run on the same XCD.
// ---------------------------------------------------------------------------
// Tile shape per instance.  Every tile stages its stencils in LDS: the block
// copies U and the primitives of its (s + 2 RAD - 1) x x stencil cells once,
// in whole rows, and every face reads its stencil from there (a face's
// stencil is six rows apart in memory, so unstaged each wave issues twice
// the loads of the x sweep, one per row and field).  The WENO5 tiles
// without the blend are 8 x 32 and exchange their fluxes across lanes
// instead of holding them in LDS (FP64: 46.9 KB per block, three blocks,
// three waves per SIMD, in 146 registers; FP32: 23.5 KB, five waves in 95
// registers); the other instances are 16 x 16 with the fluxes in LDS (FP64:
// 72 KB, two waves; the CU6 and WENO7 faces need more than the 168
// registers of three waves; FP32: 36 KB, four waves).  Measured at 256^3,
// nine species, y/z: FP64 WENO5 2.92/3.01 ms unstaged, 2.10/2.19 staged at
// 16 x 16, 1.92/1.97 exchanging at 8 x 32 (CU6 and WENO7 ran 5 % slower at
// 8 x 32 than at 16 x 16); FP32 1.43/1.49 unstaged at 32 x 8, 1.36/1.37
// staged at 32 x 8 or 32 x 16, 1.15/1.16 staged at 16 x 16, 1.12/1.11
// exchanging at 8 x 32 (1.12/1.12 exchanging at 16 x 16).
template <typename R, int REC, bool PP>
struct TileShape {
    static constexpr bool exchange = REC == kReconWeno5 && !PP;
    static constexpr int x = exchange ? 8 : 16, s = exchange ? 32 : 16;
};

template <int NS, typename R, int DIR, typename S, bool PP, int SPD, int REC>
__global__ __launch_bounds__((TileShape<R, REC, PP>::x * TileShape<R, REC, PP>::s)) __attribute__((amdgpu_waves_per_eu(sweep_waves<R, REC, false, PP>()))) void
k_sweep_tile(const S *__restrict__ U, const S *__restrict__ P, R *__restrict__ rhs, Geo g, ThermoK<R> th,
             int accumulate, StageArgs sa, unsigned *status, Dissip ds) {
    constexpr int NV = NS + 4;
    using Shape = TileShape<R, REC, PP>;
    constexpr int kTileX = Shape::x, kTileS = Shape::s;
    constexpr int RAD = stencil_radius(REC);
    constexpr bool STAGE = true;
    constexpr int kRows = kTileS + 2 * RAD - 1;        // stencil rows of the tile's faces
    constexpr int TSZ = kRows * kTileX;                // staged cells
    // EXCH: each flux component goes to the cell below as soon as it is
    // final, the neighbouring face's value taken across lanes (the face
    // below is kTileX lanes down in the same wave); only the first and last
    // face rows of each wave pass theirs through LDS, for the cell between
    // two waves.  Otherwise (the blend, which limits the whole flux vector
    // at once) the fluxes wait in LDS for the block.
    constexpr bool EXCH = Shape::exchange;
    constexpr int RPW = 64 / kTileX;                   // face rows per wave
    constexpr int NWV = kTileS / RPW;                  // waves per block
    __shared__ R sF[EXCH ? 1 : NV][EXCH ? 1 : kTileS][EXCH ? 1 : kTileX];
    __shared__ R sEdge[2][EXCH ? NWV : 1][EXCH ? NV : 1][EXCH ? kTileX : 1];
    __shared__ S xf_ftile[STAGE ? (NV + 4) * TSZ : 1];
    unsigned bx, by, bz;
    xcd_block(bx, by, bz);
    const int tx = threadIdx.x, ts = threadIdx.y;
    const int x = bx * kTileX + tx;
    const int j0 = by * (kTileS - 1);                 // the tile's first face
    const int j = j0 + ts;                            // face j: between cells j-1 and j of the sweep axis
    const int nsw = (DIR == 1) ? g.ny : g.nz;
    const bool valid = x < g.nx && j <= nsw;
    const long long step = (DIR == 1) ? g.sy : g.sz;
    const int gs = (DIR == 1) ? g.gy : g.gz;
    const long long plane = (DIR == 1) ? (long long)(g.gz + bz) * g.sz : (long long)(g.gy + bz) * g.sy;
    const long long col = (long long)(g.gx + x) + plane;
    unsigned flags = 0;
    if constexpr (STAGE) {
        // tile row r = padded sweep row gs + j0 - RAD + r, for the tile's x
        // columns; rows past the padded extent and columns past the interior
        // are never read
        const int npad = nsw + 2 * gs;
        for (int e = ts * kTileX + tx; e < TSZ; e += kTileX * kTileS) {
            const int r = e / kTileX, cx = bx * kTileX + (e % kTileX);
            const int row = gs + j0 - RAD + r;
            if (cx >= g.nx || row >= npad) continue;
            const long long cell = plane + g.gx + cx + (long long)row * step;
#pragma unroll
            for (int q = 0; q < NV; ++q) xf_ftile[q * TSZ + e] = U[q * g.cells + cell];
#pragma unroll
            for (int k = 0; k < 4; ++k) xf_ftile[(NV + k) * TSZ + e] = P[k * g.cells + cell];
        }
        __syncthreads();
    }
    if (valid) {
        if constexpr (SPD == kViscFrozen)   // y faces: i + nx (j + (ny + 1) k); z faces: i + nx (j + ny k)
            ds.fidx = DIR == 1 ? x + (long long)g.nx * (j + (long long)(g.ny + 1) * bz)
                               : x + (long long)g.nx * (bz + (long long)g.ny * j);
        auto face = [&](const auto &st) {
            if constexpr (EXCH) {
                const R id = R((DIR == 1) ? g.idy : g.idz);
                const int r = ts % RPW, w = ts / RPW;
                const long long below = col + (long long)(gs + j - 1) * step;
                face_flux_to<NS, R, DIR, SweepTune<R>::fence_face, SPD, REC, !PP, SweepTune<R>::roll_tile>(
                    st, th,
                    [&](int q, R v) {
                        // face j - 1 of this column, valid wherever face j is
                        const R vb = __shfl_up(v, kTileX);
                        if (r > 0) put_result(rhs, q * g.cells + below, double((vb - v) * id), accumulate);
                        if (r == RPW - 1) sEdge[0][w][q][tx] = v;
                        if (r == 0) sEdge[1][w][q][tx] = v;
                    },
                    flags, ds);
                return;
            }
            face_flux_to<NS, R, DIR, SweepTune<R>::fence_face, SPD, REC, !PP, SweepTune<R>::roll_tile>(
                st, th, [&](int q, R v) { sF[q][ts][tx] = v; }, flags, ds);
            if constexpr (PP) {
                R Fq[NV];
#pragma unroll
                for (int q = 0; q < NV; ++q) Fq[q] = sF[q][ts][tx];
                pp_limit<NS, R, DIR, RAD>(st, pp_lambda<R>(g, sa, DIR == 1 ? g.idy : g.idz), Fq);
#pragma unroll
                for (int q = 0; q < NV; ++q) sF[q][ts][tx] = Fq[q];
            }
        };
        if constexpr (STAGE) {
            // stencil cell m of face j is tile row j - j0 + m
            face(StencilLds<NV, S>{(const __attribute__((address_space(3))) S *)xf_ftile, ts * kTileX + tx, kTileX,
                                   TSZ});
        } else {
            face(StencilT<S>{U, P, col + (long long)(gs + j - RAD) * step, step, g.cells});
        }
    }
    __syncthreads();
    if constexpr (EXCH) {
        // the cell between the last face row of wave w - 1 and the first of w
        const int r = ts % RPW, w = ts / RPW;
        if (valid && r == 0 && w > 0) {
            const R id = R((DIR == 1) ? g.idy : g.idz);
            const long long cell = col + (long long)(gs + j - 1) * step;
#pragma unroll
            for (int q = 0; q < NV; ++q)
                put_result(rhs, q * g.cells + cell, double((sEdge[0][w - 1][q][tx] - sEdge[1][w][q][tx]) * id),
                           accumulate);
        }
    } else if (valid && ts > 0) {
        const R id = R((DIR == 1) ? g.idy : g.idz);
        const long long cell = col + (long long)(gs + j - 1) * step;
#pragma unroll
        for (int q = 0; q < NV; ++q)
            put_result(rhs, q * g.cells + cell, double((sF[q][ts - 1][tx] - sF[q][ts][tx]) * id), accumulate);
    }
    if (flags) atomicOr(status, flags);
}

// ---------------------------------------------------------------------------
// CFL: max over interior cells of sum_d (|u_d| + c) / dx_d; positive doubles
// order like their bit patterns, so the max is one 64-bit atomicMax per wave.
// ---------------------------------------------------------------------------
template <int NS>
__global__ __launch_bounds__(256) void k_cfl(const double *__restrict__ U, const double *__restrict__ P, Geo g,
                                             unsigned long long *mx) {
    const long long n = (long long)g.nx * g.ny * g.nz;
    double s = 0.0;
    for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(q % g.nx);
        const long long r = q / g.nx;
        const int j = (int)(r % g.ny), k = (int)(r / g.ny);
        const long long idx = (long long)(g.gz + k) * g.sz + (long long)(g.gy + j) * g.sy + (g.gx + i);
        const double rinv = P[3 * g.cells + idx], c = P[2 * g.cells + idx];
        double v = 0.0;
        if (g.nx > 1) v += (fabs(U[NS * g.cells + idx] * rinv) + c) * g.idx;
        if (g.ny > 1) v += (fabs(U[(NS + 1) * g.cells + idx] * rinv) + c) * g.idy;
        if (g.nz > 1) v += (fabs(U[(NS + 2) * g.cells + idx] * rinv) + c) * g.idz;
        if (v > s) s = v;   // NaN never wins (it is flagged by k_prims)
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) s = fmax(s, __shfl_xor(s, off, 64));
    __shared__ double wmax[4];
    if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        const double m = fmax(fmax(wmax[0], wmax[1]), fmax(wmax[2], wmax[3]));
        atomicMax(mx, (unsigned long long)__double_as_longlong(m));
    }
}

// ---------------------------------------------------------------------------
// GLF speeds of direction d: max of |u_d - c|, |u_d|, |u_d + c| over every
// cell the direction's stencils read (interior in the other axes, the full
// padded extent along d), three 64-bit atomicMax per block into mx[0..2]
// (positive doubles order like their bit patterns).
// ---------------------------------------------------------------------------
template <int NS>
__global__ __launch_bounds__(256) void k_glf(const double *__restrict__ U, const double *__restrict__ P, Geo g,
                                             int dir, unsigned long long *mx) {
    const int ex = dir == 0 ? g.px : g.nx, ey = dir == 1 ? g.py : g.ny, ez = dir == 2 ? g.pz : g.nz;
    const int ox = dir == 0 ? 0 : g.gx, oy = dir == 1 ? 0 : g.gy, oz = dir == 2 ? 0 : g.gz;
    const long long n = (long long)ex * ey * ez;
    double m0 = 0.0, m1 = 0.0, m2 = 0.0;
    for (long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x; q < n;
         q += (long long)gridDim.x * blockDim.x) {
        const int i = (int)(q % ex);
        const long long r = q / ex;
        const int j = (int)(r % ey), k = (int)(r / ey);
        const long long idx = (long long)(oz + k) * g.sz + (long long)(oy + j) * g.sy + (ox + i);
        const double rinv = P[3 * g.cells + idx], c = P[2 * g.cells + idx];
        const double un = U[(NS + dir) * g.cells + idx] * rinv;
        m0 = fmax(m0, fabs(un - c));
        m1 = fmax(m1, fabs(un));
        m2 = fmax(m2, fabs(un + c));
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        m0 = fmax(m0, __shfl_xor(m0, off, 64));
        m1 = fmax(m1, __shfl_xor(m1, off, 64));
        m2 = fmax(m2, __shfl_xor(m2, off, 64));
    }
    __shared__ double wmax[3][4];
    if ((threadIdx.x & 63) == 0) {
        wmax[0][threadIdx.x >> 6] = m0;
        wmax[1][threadIdx.x >> 6] = m1;
        wmax[2][threadIdx.x >> 6] = m2;
    }
    __syncthreads();
    if (threadIdx.x < 3) {
        const double *w = wmax[threadIdx.x];
        const double m = fmax(fmax(w[0], w[1]), fmax(w[2], w[3]));
        atomicMax(mx + threadIdx.x, (unsigned long long)__double_as_longlong(m));
    }
}

}  // namespace xf
