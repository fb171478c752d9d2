// xf_viscous.hpp -- viscous and diffusive fluxes F_v of Eq. 2 (Eq. 3-6) with
// the fitted transport of Eq. 29, the mixing rule of Eq. 22 and the
// effective diffusion coefficients of Eq. 26; fourth order, FP64.
//
// Per cell (k_transport): mole fractions, mu_s, kappa_s and 1/D_st from the
// fits, mu_bar and kappa_bar by Eq. 22, D_sm by Eq. 26 (mole fractions
// floored at X_t + 1e-12 inside its sums, which keeps a pure species
// finite), and the velocity.  Per face (k_visc_x, k_visc_tile): the point
// value of F_v = (-J_s, tau . n, tau . u . n - q_c - q_d) from the four cells
// i-1..i+2 across the face: face values (-f0 + 9 f1 + 9 f2 - f3)/16, normal
// derivatives (f0 - 27 f1 + 27 f2 - f3)/(24 dx), tangential derivatives
// interpolated from the cell-centred (1, -8, 8, -1)/(12 dy) differences;
// J_s = -rho (D_sm dY_s - Y_s sum_j D_jm dY_j) (Eq. 6 with the correction
// that makes the fluxes sum to zero).  The residual of cell i is the
// difference of the numerical fluxes F^_{i+1/2} = (-F_{i-1/2} + 26 F_{i+1/2}
// - F_{i+3/2})/24, i.e. the staggered fourth-order difference of the point
// fluxes (a plain difference of point fluxes is second order).
#pragma once

#include "xf_face.hpp"

namespace xf {

// ---------------------------------------------------------------------------
// transport pass
// ---------------------------------------------------------------------------
template <int NS>
__global__ __launch_bounds__(256) void k_transport(const double *__restrict__ U, const double *__restrict__ P,
                                                   double *__restrict__ Q, Geo g,
                                                   const TransportK *__restrict__ tk) {
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= g.cells) return;
    const long long C = g.cells;
    const double rinv = P[3 * C + idx], T = P[idx], p = P[C + idx];
    double X[NS];
    double nsum = 0.0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        X[s] = U[s * C + idx] * rinv * tk->iW[s];
        nsum += X[s];
    }
    const double inv = 1.0 / nsum;
    double Wbar = 0.0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        X[s] *= inv;
        Wbar += X[s] * tk->W[s];
    }
    const double lt = log(T);
    auto fit = [&](const double *a) { return ((a[3] * lt + a[2]) * lt + a[1]) * lt + a[0]; };
    // Eq. 22 for one property: sum_s X_s a_s / sum_t X_t Phi_st with
    // Phi_st = wa_st (1 + sqrt(a_s / a_t) wb_st)^2
    auto mix = [&](const double (*coef)[4]) {
        double a[NS], sa[NS], isa[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            a[s] = exp(fit(coef[s]));
            sa[s] = sqrt(a[s]);
            isa[s] = 1.0 / sa[s];
        }
        double out = 0.0;
        // one row of the pair tables at a time (unrolled, all 2 NS^2
        // table values are loaded up front and spill the scalar registers)
#pragma unroll 1
        for (int s = 0; s < NS; ++s) {
            double den = 0.0;
#pragma unroll
            for (int t = 0; t < NS; ++t) {
                const double f = 1.0 + sa[s] * isa[t] * tk->wb[s][t];
                den += X[t] * (tk->wa[s][t] * f * f);
            }
            out += X[s] * a[s] / den;
        }
        return out;
    };
    Q[idx] = mix(tk->mu);
    Q[C + idx] = mix(tk->kappa);
    Q[2 * C + idx] = U[NS * C + idx] * rinv;
    Q[3 * C + idx] = U[(NS + 1) * C + idx] * rinv;
    Q[4 * C + idx] = U[(NS + 2) * C + idx] * rinv;
    // Eq. 26: D_sm = sum_{t != s} X_t W_t / (Wbar sum_{t != s} X_t / D_st),
    // 1 / D_st = exp(-fit) p / p_ref
    double num[NS], den[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) num[s] = den[s] = 0.0;
    const double pr = p * tk->ip_ref;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
#pragma unroll
        for (int t = s + 1; t < NS; ++t) {
            const double iD = exp(-fit(tk->D[s][t])) * pr;
            const double Xs = X[s] + 1e-12, Xt = X[t] + 1e-12;
            num[s] += Xt * tk->W[t];
            den[s] += Xt * iD;
            num[t] += Xs * tk->W[s];
            den[t] += Xs * iD;
        }
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) Q[(5 + s) * C + idx] = NS > 1 ? num[s] / (Wbar * den[s]) : 0.0;
}

// ---------------------------------------------------------------------------
// point value of F_v at one face
// ---------------------------------------------------------------------------
XF_HD double fv_face(double a0, double a1, double a2, double a3) {
    return (-a0 + 9.0 * a1 + 9.0 * a2 - a3) * 0.0625;
}
XF_HD double fv_normal(double a0, double a1, double a2, double a3, double i24h) {
    return (a0 - 27.0 * a1 + 27.0 * a2 - a3) * i24h;
}

// cells m = 0..3 at c0 + m step (cells i-1..i+2 of the face between i and
// i+1); F[0..NS+3] receives the point flux in conservative field order
template <int NS, int DIR>
__device__ __forceinline__ void visc_point_flux(const double *__restrict__ U, const double *__restrict__ P,
                                                const double *__restrict__ Q, const double *__restrict__ G,
                                                long long c0, long long step, const Geo &g,
                                                const ThermoK<double> &th, double i24h, int terms, double *F) {
    const long long C = g.cells;
    constexpr int T1 = Axes<DIR>::t1, T2 = Axes<DIR>::t2;
    const bool a1 = (T1 == 0 ? g.nx : T1 == 1 ? g.ny : g.nz) > 1;
    const bool a2 = (T2 == 0 ? g.nx : T2 == 1 ? g.ny : g.nz) > 1;
    long long c[4];
#pragma unroll
    for (int m = 0; m < 4; ++m) c[m] = c0 + m * step;
    auto fc = [&](const double *A) { return fv_face(A[c[0]], A[c[1]], A[c[2]], A[c[3]]); };
    auto nd = [&](const double *A) { return fv_normal(A[c[0]], A[c[1]], A[c[2]], A[c[3]], i24h); };
#pragma unroll
    for (int q = 0; q < NS + 4; ++q) F[q] = 0.0;
    if (terms & kViscousStress) {
        const double mu = fc(Q);
        double uf[3], dn[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            uf[k] = fc(Q + (2 + k) * C);
            dn[k] = nd(Q + (2 + k) * C);      // d u_k / d x_DIR
        }
        // tangential derivatives at the face: d u_DIR / d x_t and d u_t / d x_t
        const double t1n = a1 ? fc(G + (3 * T1 + DIR) * C) : 0.0, t1t = a1 ? fc(G + (3 * T1 + T1) * C) : 0.0;
        const double t2n = a2 ? fc(G + (3 * T2 + DIR) * C) : 0.0, t2t = a2 ? fc(G + (3 * T2 + T2) * C) : 0.0;
        double Gf[3][3] = {};                   // Gf[a][b] = d u_b / d x_a, the entries used
        Gf[DIR][0] = dn[0];
        Gf[DIR][1] = dn[1];
        Gf[DIR][2] = dn[2];
        Gf[T1][DIR] = t1n;
        Gf[T1][T1] = t1t;
        Gf[T2][DIR] = t2n;
        Gf[T2][T2] = t2t;
        const double div = Gf[0][0] + Gf[1][1] + Gf[2][2];
        double work = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            double tau = mu * (Gf[k][DIR] + Gf[DIR][k]);
            if (k == DIR) tau = tau - 2.0 / 3.0 * mu * div;
            F[NS + k] = tau;
            work = work + tau * uf[k];
        }
        F[NS + 3] = work;
    }
    if (terms & kViscousHeat) F[NS + 3] = F[NS + 3] + fc(Q + C) * nd(P);     // - q_c = kappa dT/dx
    if (terms & kViscousDiffusion) {
        double rho[4], Tm[4], rinv[4];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            double r = 0.0;
#pragma unroll
            for (int s = 0; s < NS; ++s) r += U[s * C + c[m]];
            rho[m] = r;
            rinv[m] = P[3 * C + c[m]];
            Tm[m] = P[c[m]];
        }
        const double rf = fv_face(rho[0], rho[1], rho[2], rho[3]);
        double Yf[NS], Df[NS], dY[NS];
        double corr = 0.0;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            double y[4];
#pragma unroll
            for (int m = 0; m < 4; ++m) y[m] = U[s * C + c[m]] * rinv[m];
            Yf[s] = fv_face(y[0], y[1], y[2], y[3]);
            dY[s] = fv_normal(y[0], y[1], y[2], y[3], i24h);
            Df[s] = fc(Q + (5 + s) * C);
            corr = corr + Df[s] * dY[s];
        }
        double e = F[NS + 3];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const double J = -rf * (Df[s] * dY[s] - Yf[s] * corr);
            F[s] = -J;
            double hm[4];
#pragma unroll
            for (int m = 0; m < 4; ++m) hm[m] = e_species(th, s, Tm[m]) + th.Rs[s] * Tm[m];
            e = e - fv_face(hm[0], hm[1], hm[2], hm[3]) * J;                     // - q_d
        }
        F[NS + 3] = e;
    }
}

// ---------------------------------------------------------------------------
// x direction: point faces k = -1..nx+1 of every interior row, linearised
// (nx + 3 per row); a block of 256 threads takes 256 consecutive faces and
// blocks overlap by three, so each cell's four point faces meet in one block.
// The block count is a multiple of the XCD count and each XCD takes one
// contiguous range of faces (neighbouring blocks share their edge cells in
// one L2).
// The point fluxes go to LDS; a thread whose face closes a cell's window
// (the cell's last point face) adds that cell's residual.
// ---------------------------------------------------------------------------
constexpr int kViscXBlock = 256;

// Both viscous face kernels ask for at least five waves per SIMD: the
// compiler's default of four left them latency-bound (at nine species the x
// kernel then keeps 96 registers with a few dozen bytes of spill, the tile
// kernel 80 registers with none, which gives it six).
template <int NS>
__global__ __launch_bounds__(kViscXBlock) __attribute__((amdgpu_waves_per_eu(5))) void k_visc_x(const double *__restrict__ U, const double *__restrict__ P,
                                                       const double *__restrict__ Q, const double *__restrict__ G,
                                                       double *__restrict__ rhs, Geo g, ThermoK<double> th,
                                                       int terms) {
    constexpr int NV = NS + 4;
    __shared__ double sF[NV][kViscXBlock];
    unsigned lb, u1, u2;
    xcd_block(lb, u1, u2);
    const int t = threadIdx.x;
    const long long per_row = (long long)g.nx + 3;
    const long long nfaces = per_row * g.ny * g.nz;
    const long long f0 = (long long)lb * (kViscXBlock - 3);
    if (f0 >= nfaces) return;   // blocks that round the grid up to a multiple of 8
    const long long f = f0 + t;
    const bool valid = f < nfaces;
    long long row = 0, rowbase = 0;
    int kk = 0;
    if (valid) {
        row = f / per_row;
        kk = (int)(f - row * per_row);           // point face k = kk - 1, between cells kk - 2 and kk - 1
        const int j = (int)(row % g.ny), k = (int)(row / g.ny);
        rowbase = (long long)(g.gz + k) * g.sz + (long long)(g.gy + j) * g.sy + g.gx;
        double F[NV];
        visc_point_flux<NS, 0>(U, P, Q, G, rowbase + kk - 3, 1, g, th, g.idx / 24.0, terms, F);
#pragma unroll
        for (int q = 0; q < NV; ++q) sF[q][t] = F[q];
    }
    __syncthreads();
    if (valid && t >= 3 && kk >= 3) {
        const long long cell = rowbase + kk - 3;
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            const double hl = (-sF[q][t - 3] + 26.0 * sF[q][t - 2] - sF[q][t - 1]) * (1.0 / 24.0);
            const double hr = (-sF[q][t - 2] + 26.0 * sF[q][t - 1] - sF[q][t]) * (1.0 / 24.0);
            rhs[q * g.cells + cell] += (hr - hl) * g.idx;
        }
    }
}

// ---------------------------------------------------------------------------
// y/z directions: tiles of 16 x-columns by 16 consecutive point faces along
// the sweep axis; tiles overlap by three faces, so each finishes 13 cells per
// column.  Lanes run along x (coalesced loads).
// ---------------------------------------------------------------------------
constexpr int kViscTX = 16, kViscTS = 16;

template <int NS, int DIR>
__global__ __launch_bounds__(kViscTX *kViscTS) __attribute__((amdgpu_waves_per_eu(5))) void k_visc_tile(const double *__restrict__ U,
                                                               const double *__restrict__ P,
                                                               const double *__restrict__ Q,
                                                               const double *__restrict__ G,
                                                               double *__restrict__ rhs, Geo g,
                                                               ThermoK<double> th, int terms) {
    constexpr int NV = NS + 4;
    __shared__ double sF[NV][kViscTS][kViscTX];
    unsigned bx, by, bz;
    xcd_block(bx, by, bz);
    const int tx = threadIdx.x, ts = threadIdx.y;
    const int x = bx * kViscTX + tx;
    const int kk = by * (kViscTS - 3) + ts;       // point face k = kk - 1
    const int nsw = DIR == 1 ? g.ny : g.nz;
    const bool valid = x < g.nx && kk <= nsw + 2;
    const long long step = DIR == 1 ? g.sy : g.sz;
    const int gs = DIR == 1 ? g.gy : g.gz;
    const long long col = (long long)(g.gx + x) +
                          (DIR == 1 ? (long long)(g.gz + bz) * g.sz : (long long)(g.gy + bz) * g.sy);
    const double id = DIR == 1 ? g.idy : g.idz;
    if (valid) {
        double F[NV];
        visc_point_flux<NS, DIR>(U, P, Q, G, col + (long long)(gs + kk - 3) * step, step, g, th, id / 24.0, terms,
                                 F);
#pragma unroll
        for (int q = 0; q < NV; ++q) sF[q][ts][tx] = F[q];
    }
    __syncthreads();
    if (valid && ts >= 3) {
        const long long cell = col + (long long)(gs + kk - 3) * step;
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            const double hl = (-sF[q][ts - 3][tx] + 26.0 * sF[q][ts - 2][tx] - sF[q][ts - 1][tx]) * (1.0 / 24.0);
            const double hr = (-sF[q][ts - 2][tx] + 26.0 * sF[q][ts - 1][tx] - sF[q][ts][tx]) * (1.0 / 24.0);
            rhs[q * g.cells + cell] += (hr - hl) * id;
        }
    }
}

}  // namespace xf
