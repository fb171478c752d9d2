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

// The mechanism and the species tables are read through constant-address
// pointers (scalar loads).
template <class T>
using cptr = const __attribute__((address_space(4))) T *;

// exp and expm1 of the rate evaluations.  x = k ln2 + r with k = rint(x /
// ln2) and r reduced in two FMA steps against ln2 split into its double and
// the remainder, so |r| <= ln2 / 2; e^r from its Taylor series through r^13
// (truncation below 5e-18 relative), scaled by 2^k.  For expm1 the series
// starts at r, P(r) = e^r - 1, and expm1(x) = 2^k P(r) + (2^k - 1), which is
// P(r) itself wherever |x| < ln2 / 2 (k = 0), so small arguments keep their
// relative accuracy.  The constants come by scalar loads from a table in
// constant memory, read at every call (the pointer is laundered), so that
// they enter the FMAs as scalar operands rather than being copied into
// vector registers first.  Infinite or NaN arguments give NaN.
__constant__ double kExpTab[17] = {
    1.4426950408889634,                            // 1 / ln2
    0.6931471805599453,    2.3190468138462996e-17,  // ln2 as a double, and the remainder
    1.6059043836821613e-10, 2.08767569878681e-09,   // 1/13!, 1/12!
    2.505210838544172e-08, 2.755731922398589e-07,   // 1/11!, 1/10!
    2.7557319223985893e-06, 2.48015873015873e-05,   // 1/9!, 1/8!
    0.0001984126984126984, 0.001388888888888889,    // 1/7!, 1/6!
    0.008333333333333333,  0.041666666666666664,    // 1/5!, 1/4!
    0.16666666666666666,   0.5,                     // 1/3!, 1/2!
    1.0,                   1.0};                    // 1/1!, 1/0!

// a * b + c with c in scalar registers, as one VOP3 instruction: written out
// because the compiler otherwise copies c into the destination's vector
// registers (two moves) to use the two-operand form
__device__ __forceinline__ double fma_sc(double a, double b, double c) {
    double d;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "s"(c));
    return d;
}

__device__ __forceinline__ cptr<double> exp_table() {
    cptr<double> c = (cptr<double>)kExpTab;
    asm volatile("" : "+s"(c));
    return c;
}

__device__ __forceinline__ double rx_exp(double x, cptr<double> c) {
    const double k = rint(x * c[0]);
    double r = fma(-k, c[1], x);
    r = fma(-k, c[2], r);
    double p = fma_sc(r, c[3], c[4]);
#pragma unroll
    for (int i = 5; i < 17; ++i) p = fma_sc(p, r, c[i]);
    return ldexp(p, (int)k);
}

__device__ __forceinline__ double rx_expm1(double x, cptr<double> c) {
    const double k = rint(x * c[0]);
    double r = fma(-k, c[1], x);
    r = fma(-k, c[2], r);
    double q = fma_sc(r, c[3], c[4]);
#pragma unroll
    for (int i = 5; i < 16; ++i) q = fma_sc(q, r, c[i]);
    const int ki = (int)k;
    return fma(ldexp(r, ki), q, ldexp(1.0, ki) - 1.0);
}

__device__ __forceinline__ double qss_alpha(double r) {
    if (r < 1e-3) return 0.5 + r * (1.0 / 12.0) - r * r * r * (1.0 / 720.0);
    return 1.0 / (-rx_expm1(-r, exp_table())) - 1.0 / r;
}

// The table pointer is laundered on every call, so that the table comes in
// where it is used instead of being held in scalar registers across the
// sub-steps, where it would crowd out everything else.

template <int NS>
__device__ __forceinline__ void mix_poly(cptr<ThermoK<double>> thp, const double *Y, MixPoly &m) {
    asm volatile("" : "+s"(thp));
    const auto &th = *thp;
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

// production q_s and loss rate p_s (1/s) at (rho, Y, T); the species' Gibbs
// functions enter only through each reaction's net sum, whose coefficients
// the host folds (ReactK::G), so no per-species thermo table is held here.
// Each reaction's concentration products run over its reactant and product
// lists (a uniform register index per molecule), and q and p accumulate over
// all species with nu' and nu'' as scalar operands (zero for bystanders), so
// that the per-reaction work has no per-species branches.  p_s = loss_s /
// [X_s] (= loss W_s / (rho Y_s)), 0 where Y_s <= 0.
template <int NS>
__device__ __forceinline__ void qss_rates(cptr<ReactK> rk, double rho, const double *Y, double T, double *q,
                                          double *p) {
    // a fresh pointer per call: nothing read from the mechanism (W_s / rho,
    // rho / W_s) is kept live across the sub-steps
    asm volatile("" : "+s"(rk));
    const double lt = log(T), iT = 1.0 / T, lt1 = lt - 1.0;
    const double lp = rk->lp0 - lt;   // ln(p0 / (R_u T))
    double conc[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        conc[s] = rho * Y[s] * rk->iW[s];
        q[s] = 0.0;
        p[s] = 0.0;   // the loss p_s Y_s until the end
    }
    const int nr = rk->nr;
    for (int r = 0; r < nr; ++r) {
        const unsigned fl = rk->fl[r], bl = rk->bl[r];
        const cptr<double> ec = exp_table();
        const double lkf = rk->lnA[r] + rk->B[r] * lt - rk->ER[r] * iT;
        double gam = 1.0;
        if (rk->third[r]) {
            gam = 0.0;
#pragma unroll
            for (int s = 0; s < NS; ++s) gam += rk->eff[r][s] * conc[s];
        }
        // the loops end at the list's count (a uniform branch; the empty
        // statement keeps the compiler from running all seven slots under
        // per-lane selects)
        double pf = 1.0, pb = 1.0;
#pragma unroll
        for (unsigned k = 0; k < 7; ++k) {
            if (k >= (fl & 7u)) break;
            asm volatile("");
            pf *= conc[fl >> (3 + 4 * k) & 15u];
        }
#pragma unroll
        for (unsigned k = 0; k < 7; ++k) {
            if (k >= (bl & 7u)) break;
            asm volatile("");
            pb *= conc[bl >> (3 + 4 * k) & 15u];
        }
        const double Rf = gam * rx_exp(lkf, ec) * pf;
        const auto *fd = rk->fd[r], *bd = rk->bd[r];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            q[s] = fma(bd[s], Rf, q[s]);
            p[s] = fma(fd[s], Rf, p[s]);
        }
        if (rk->rev[r]) {
            const auto *G = rk->G[r];
            const double dg = G[0] * lt1 + (((G[4] * T + G[3]) * T + G[2]) * T + G[1]) * T + G[5] * iT + G[6];
            const double Rb = gam * rx_exp(lkf - (rk->dn[r] * lp + dg), ec) * pb;
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                q[s] = fma(fd[s], Rb, q[s]);
                p[s] = fma(bd[s], Rb, p[s]);
            }
        }
    }
    const double ir = 1.0 / rho;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        q[s] *= rk->W[s] * ir;
        p[s] = conc[s] > 0.0 ? p[s] / conc[s] : 0.0;
    }
}

// The predictor's rates q0 and p0 wait out the corrector's rate evaluation in
// LDS (one slot per thread, conflict-free rows of 256 doubles) instead of 2 NS
// registers.  Each temperature solve starts from the cell's previous one
// (the first from e / C_v(T_ref)).
template <int NS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) void k_react(double *__restrict__ U, Geo g, const ReactK *__restrict__ rk,
                                               double dt, const double *dt_dev, double scale, int n_sub,
                                               unsigned *status) {
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
    const cptr<ReactK> rc = (cptr<ReactK>)rk;
    const cptr<ThermoK<double>> th = &rc->th;
    const bool bracket = th->bracket;
    const double T_lo = th->T_lo, T_hi = th->T_hi;
    double T;
    {
        MixPoly m;
        mix_poly<NS>(th, Y, m);
        T = e / m.cv(th->T_ref);
    }
    for (int it = 0; it < n_sub; ++it) {
        double qp[NS], pp[NS];
        {
            double Yp[NS];
            {
                double q0[NS], p0[NS];
                {
                    MixPoly m;
                    mix_poly<NS>(th, Y, m);
                    if (!newton_poly(bracket, T_lo, T_hi, m, e, T)) flags |= XF_FLAG_NEWTON;
                }
                qss_rates<NS>(rc, rho, Y, T, q0, p0);
#pragma unroll
                for (int s = 0; s < NS; ++s) {
                    const double a0 = qss_alpha(p0[s] * h);
                    Yp[s] = Y[s] + h * (q0[s] - p0[s] * Y[s]) / (1.0 + a0 * p0[s] * h);
                    held[s][t] = q0[s];
                    held[NS + s][t] = p0[s];
                    // one species at a time: interleaving the nine alpha and
                    // division chains would only raise the register count
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
            // each thread reads back only its own slots; the fence keeps the
            // compiler from carrying the stored values in registers instead
            asm volatile("" ::: "memory");
            {
                MixPoly m;
                mix_poly<NS>(th, Yp, m);
                if (!newton_poly(bracket, T_lo, T_hi, m, e, T)) flags |= XF_FLAG_NEWTON;
            }
            qss_rates<NS>(rc, rho, Yp, T, qp, pp);
        }
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
            __builtin_amdgcn_sched_barrier(0);
        }
        const double is = 1.0 / sum;
#pragma unroll
        for (int s = 0; s < NS; ++s) Y[s] *= is;
    }
    // the addresses are formed again here rather than held through the loop
    long long o = idx;
    asm volatile("" : "+v"(o));
    bool finite = true;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        U[s * C + o] = rho * Y[s];
        finite = finite && isfinite(Y[s]);
    }
    if (!finite) flags |= XF_FLAG_NAN;
    if (flags) atomicOr(status, flags);
}

}  // namespace xf
