// xf_reaction.hpp -- the reaction source (Eq. 9-12) and its alpha-QSS time
// integration (Eq. 27-28), one thread per interior cell, FP64.
//
// Per cell the step keeps rho, the momentum and the total energy (the
// species enthalpies carry the formation enthalpy a5, so the heat release
// of Eq. 8 shows as a change of T at fixed internal energy) and advances the
// mass fractions through n_sub equal sub-steps of the predictor-corrector
// of Eq. 28:
//   Y^p = Y^0 + h (q^0 - p^0 Y^0) / (1 + alpha(p^0 h) p^0 h),
//   Y^c = Y^0 + h (q_l - p_bar Y^0) / (1 + alpha_bar p_bar h),
//   p_bar = (p^0 + p^p)/2, alpha_bar = alpha(p_bar h), q_l = alpha_bar q^p + (1 - alpha_bar) q^0,
// with alpha(r) = 1/(1 - e^-r) - 1/r (exact for constant p and q; the
// series 1/2 + r/12 - r^3/720 below r = 1e-3), T from the internal energy by
// Newton wherever rates are evaluated, and the mass fractions renormalised
// to unit sum after each sub-step.  Rates: [X_s] = rho Y_s / W_s,
// k_f = A T^B exp(-E / (R_u T)), k_b = k_f / K_c with
// K_c = (p0 / (R_u T))^(sum nu) exp(sum_s nu_s (S_s/R_s - h_s/(R_s T))),
// p0 = 1 atm, S/R = a0 ln T + a1 T + a2 T^2/2 + a3 T^3/3 + a4 T^4/4 + a6
// (the sum over species folded per reaction on the host);
// third bodies Gamma_r = sum_s eff_rs [X_s]; production q_s from the
// creation terms and loss p_s Y_s from the destruction terms of both
// directions, p_s = loss / Y_s (0 where Y_s <= 0).
#pragma once

#include "xf_forward.hpp"

namespace xf {

constexpr double kP0 = 101325.0;

__device__ __forceinline__ double qss_alpha(double r) {
    if (r < 1e-3) return 0.5 + r * (1.0 / 12.0) - r * r * r * (1.0 / 720.0);
    return 1.0 / (-expm1(-r)) - 1.0 / r;
}

// production q_s and loss rate p_s (1/s) at (rho, Y, T); the species' Gibbs
// functions enter only through each reaction's net sum, whose coefficients
// the host folds (ReactK::G), so no per-species thermo table is held here
template <int NS>
__device__ __forceinline__ void qss_rates(const ReactK *__restrict__ rk, double rho, const double *Y, double T,
                                          double *q, double *p) {
    const double lt = log(T), iT = 1.0 / T, lt1 = lt - 1.0;
    const double lp = log(kP0 / (kRu * T));
    double conc[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        conc[s] = rho * Y[s] * rk->iW[s];
        q[s] = 0.0;
        p[s] = 0.0;   // the loss p_s Y_s until the end
    }
    const int nr = rk->nr;
    for (int r = 0; r < nr; ++r) {
        const double lkf = rk->lnA[r] + rk->B[r] * lt - rk->ER[r] * iT;
        double gam = 1.0;
        if (rk->third[r]) {
            gam = 0.0;
#pragma unroll
            for (int s = 0; s < NS; ++s) gam += rk->eff[r][s] * conc[s];
        }
        double pf = 1.0, pb = 1.0;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int f = rk->nf[r][s], b = rk->nb[r][s];
            for (int k = 0; k < f; ++k) pf *= conc[s];
            for (int k = 0; k < b; ++k) pb *= conc[s];
        }
        const double Rf = gam * exp(lkf) * pf;
        double Rb = 0.0;
        if (rk->rev[r]) {
            const double *G = rk->G[r];
            const double dg = G[0] * lt1 + (((G[4] * T + G[3]) * T + G[2]) * T + G[1]) * T + G[5] * iT + G[6];
            Rb = gam * exp(lkf - (rk->dn[r] * lp + dg)) * pb;
        }
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int f = rk->nf[r][s], b = rk->nb[r][s];
            if (f | b) {
                q[s] += b * Rf + f * Rb;
                p[s] += f * Rf + b * Rb;
            }
        }
    }
    const double ir = 1.0 / rho;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        q[s] *= rk->W[s] * ir;
        const double l = p[s] * rk->W[s] * ir;
        p[s] = Y[s] > 0.0 ? l / Y[s] : 0.0;
    }
}

// The predictor's rates q0 and p0 wait out the corrector's rate evaluation in
// LDS (one slot per thread, conflict-free rows of 256 doubles) instead of 2 NS
// registers, and the kernel is held to 128 registers per lane (four waves per
// SIMD) so that more waves hide the FP64 latency; at nine species that costs
// a few hundred bytes of spill per lane and still wins over two or three waves.
template <int NS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_react(double *__restrict__ U, Geo g, ThermoK<double> th,
                                               const ReactK *__restrict__ rk, double dt, const double *dt_dev,
                                               double scale, int n_sub, unsigned *status) {
    __shared__ double held[2 * NS][256];
    const int t = threadIdx.x;
    const long long q = (long long)blockIdx.x * blockDim.x + t;
    const long long nint = (long long)g.nx * g.ny * g.nz;
    if (q >= nint) return;
    const int i = (int)(q % g.nx);
    const long long r2 = q / g.nx;
    const int j = (int)(r2 % g.ny), k = (int)(r2 / g.ny);
    const long long idx = (long long)(g.gz + k) * g.sz + (long long)(g.gy + j) * g.sy + (g.gx + i);
    const long long C = g.cells;
    double Y[NS];
    double rho = 0.0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        Y[s] = U[s * C + idx];
        rho += Y[s];
    }
    const double irho = 1.0 / rho;
#pragma unroll
    for (int s = 0; s < NS; ++s) Y[s] *= irho;
    const double u = U[NS * C + idx] * irho, v = U[(NS + 1) * C + idx] * irho, w = U[(NS + 2) * C + idx] * irho;
    const double e = U[(NS + 3) * C + idx] * irho - 0.5 * (u * u + v * v + w * w);
    const double h = (dt_dev ? *dt_dev : dt) * scale / n_sub;
    unsigned flags = 0;
    for (int it = 0; it < n_sub; ++it) {
        double T0, Tp, qp[NS], pp[NS], Yp[NS];
        {
            double q0[NS], p0[NS];
            if (!newton_T<NS>(th, Y, e, T0)) flags |= XF_FLAG_NEWTON;
            qss_rates<NS>(rk, rho, Y, T0, q0, p0);
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const double a0 = qss_alpha(p0[s] * h);
                Yp[s] = Y[s] + h * (q0[s] - p0[s] * Y[s]) / (1.0 + a0 * p0[s] * h);
                held[s][t] = q0[s];
                held[NS + s][t] = p0[s];
            }
        }
        // each thread reads back only its own slots; the fence keeps the
        // compiler from carrying the stored values in registers instead
        asm volatile("" ::: "memory");
        if (!newton_T<NS>(th, Yp, e, Tp)) flags |= XF_FLAG_NEWTON;
        qss_rates<NS>(rk, rho, Yp, Tp, qp, pp);
        asm volatile("" ::: "memory");
        double sum = 0.0;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const double q0 = held[s][t], p0 = held[NS + s][t];
            const double pb = 0.5 * (p0 + pp[s]);
            const double ab = qss_alpha(pb * h);
            const double ql = ab * qp[s] + (1.0 - ab) * q0;
            Y[s] = Y[s] + h * (ql - pb * Y[s]) / (1.0 + ab * pb * h);
            sum += Y[s];
        }
        const double is = 1.0 / sum;
#pragma unroll
        for (int s = 0; s < NS; ++s) Y[s] *= is;
    }
    bool finite = true;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        U[s * C + idx] = rho * Y[s];
        finite = finite && isfinite(Y[s]);
    }
    if (!finite) flags |= XF_FLAG_NAN;
    if (flags) atomicOr(status, flags);
}

}  // namespace xf
