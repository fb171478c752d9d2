// xf_face.hpp -- device code of one face of the convective flux (gfx950).
//
// Computes the numerical flux F^_{i+1/2} of Eq. 14-15 of XFluids (arXiv
// 2403.05910) at one face from the six cells m = i-2..i+3 of its stencil:
//
//   1. Roe-averaged face state of cells i, i+1 (sqrt(rho) weights on u, H,
//      Y_s and T), species thermo at the averaged T, Gamma = Rbar / C_v,
//      chi_s = Gamma (|u|^2/2 - e_s) + R_s T and the face sound speed
//      c^2 = sum_s Y_s chi_s + Gamma (H - |u|^2).
//   2. Component-wise LLF speeds: max over the six cells of |u_n - c|,
//      |u_n|, |u_n + c| for the u-c, middle and u+c characteristic fields.
//   3. Projection of F_m and U_m onto the characteristic fields, split
//      F_m^pm = 1/2 (L F_m +- alpha L U_m) (Eq. 14).
//   4. WENO5-JS of the plus side over m = i-2..i+2 and of the minus side
//      mirrored over m = i+3..i-1 (Eq. 15).
//   5. Back-projection F^ = R (F^+ + F^-) (Eq. 15).
//
// The left/right eigenvectors are never stored.  They are identity plus a few
// rank-one terms, so each projection costs O(N):
//   dp(v)     = sum_s chi_s v_rho_s - Gamma u.v_m + Gamma v_E
//   l_-+ . v  = [dp(v) -+ c (n.v_m - u_n sigma(v))] / (2 c^2),  sigma = sum_s v_rho_s
//   l_s  . v  = v_rho_s - Y_s dp(v) / c^2
//   l_ta . v  = t_a . v_m - (u.t_a) sigma(v)
//   r_-+ = (Y, u -+ c n, H -+ u_n c),  r_s = (e_s, u, |u|^2 - chi_s/Gamma),
//   r_ta = (0, t_a, u.t_a).
// Field order of the characteristic vector: u-c, species 1..N, t1, t2, u+c,
// with (t1, t2) = (y, z) for an x face, (x, z) for y, (x, y) for z.  The
// characteristic fields are streamed one at a time (acoustic pair first, then
// the tangential pair, then the species), so registers hold O(N) values.
#pragma once

#include <cmath>

#include "xf_common.hpp"

// Face code is compiled for the device and, for CPU checks of its arithmetic,
// for the host as well.
#define XF_HD __host__ __device__ __forceinline__
// Compiler-only fence between phases of the face computation: keeps the
// compiler from hoisting every stencil load to the top of the routine (which
// holds ~100 loaded values in registers at once); emits no instruction.
#ifdef __HIP_DEVICE_COMPILE__
#define XF_FENCE() asm volatile("" ::: "memory")
#else
#define XF_FENCE() ((void)0)
#endif

namespace xf {

XF_HD double xsqrt(double a) { return sqrt(a); }
XF_HD float xsqrt(float a) { return sqrtf(a); }

template <typename R>
XF_HD R rmax(R a, R b) { return a > b ? a : b; }
template <typename R>
XF_HD R rmin(R a, R b) { return a < b ? a : b; }

template <typename R>
XF_HD R rabs(R a) { return a < R(0) ? -a : a; }

// Horner evaluations of the species tables.
template <typename R>
XF_HD R cv_species(const ThermoK<R> &th, int s, R T) {
    return (((th.cv[s][4] * T + th.cv[s][3]) * T + th.cv[s][2]) * T + th.cv[s][1]) * T + th.cv[s][0];
}
template <typename R>
XF_HD R e_species(const ThermoK<R> &th, int s, R T) {
    return ((((th.e[s][5] * T + th.e[s][4]) * T + th.e[s][3]) * T + th.e[s][2]) * T + th.e[s][1]) * T
           + th.e[s][0];
}

// WENO5-JS value at the right edge of the cell holding c (linear weights
// 1/10, 6/10, 3/10; absolute eps = 1e-6; weights (eps + beta)^-2).  Written
// with one division and with the constant factors gathered where they cost
// least, none of which changes the weights in exact arithmetic: the
// smoothness indicators are taken times 12 (13 t^2 + 3 u^2, eps 12e-6), the
// linear weights times 10 (1, 6, 3), and the candidates times 6, their 1/6
// applied once to the denominator;
// alpha_k / sum alpha = d_k prod_{j!=k} s_j / sum(...), s_k = (eps + beta_k)^2.
// The value as numerator over denominator, N / D.
XF_HD void weno5_nd(double a, double b, double c, double d, double e, double &N, double &D) {
    const double q0 = 2.0 * a - 7.0 * b + 11.0 * c;
    const double q1 = -b + 5.0 * c + 2.0 * d;
    const double q2 = 2.0 * c + 5.0 * d - e;
    const double t0 = a - 2.0 * b + c, u0 = a - 4.0 * b + 3.0 * c;
    const double t1 = b - 2.0 * c + d, u1 = b - d;
    const double t2 = c - 2.0 * d + e, u2 = 3.0 * c - 4.0 * d + e;
    double s0 = (13.0 * t0) * t0 + ((3.0 * u0) * u0 + 12e-6);
    double s1 = (13.0 * t1) * t1 + ((3.0 * u1) * u1 + 12e-6);
    double s2 = (13.0 * t2) * t2 + ((3.0 * u2) * u2 + 12e-6);
    s0 *= s0;
    s1 *= s1;
    s2 *= s2;
    const double w0 = s1 * s2, w1 = 6.0 * (s0 * s2), w2 = 3.0 * (s0 * s1);
    N = w0 * q0 + w1 * q1 + w2 * q2;
    D = 6.0 * (w0 + w1 + w2);
}

XF_HD double weno5(double a, double b, double c, double d, double e) {
    double N, D;
    weno5_nd(a, b, c, d, e, N, D);
    return N / D;
}

// FP64 reciprocal of a positive normal number: the hardware estimate refined
// by two Newton-Raphson steps r <- r + r (1 - x r) (each step squares the
// relative error), about 1 ulp, in 5 instructions where the IEEE division
// sequence takes 11.
XF_HD double rcp_nr(double x) {
#ifdef __HIP_DEVICE_COMPILE__
    double r = __builtin_amdgcn_rcp(x);
#else
    double r = 1.0 / x;
#endif
    double e = fma(-x, r, 1.0);
    r = fma(e, r, r);
    e = fma(-x, r, 1.0);
    return fma(e, r, r);
}

// Both sides of one characteristic field: weno5(a..e) + weno5(f..j) with one
// reciprocal, N_p / D_p + N_m / D_m = (N_p D_m + N_m D_p) / (D_p D_m).  With
// |values| <= v each D lies between 1e-19 ((12e-6)^4) and about 1.5e12 v^8,
// so D_p D_m and N_p D_m stay finite for v up to about 1e16; past a product
// of 1e280 (never reached by fluxes at SI scales) the two sides are divided
// separately.
XF_HD double weno5_pair(double a, double b, double c, double d, double e, double f, double g, double h,
                        double i, double j) {
    double Np, Dp, Nm, Dm;
    weno5_nd(a, b, c, d, e, Np, Dp);
    weno5_nd(f, g, h, i, j, Nm, Dm);
    const double P = Dp * Dm;
    if (P < 1e280) return (Np * Dm + Nm * Dp) * rcp_nr(P);
    return Np / Dp + Nm / Dm;
}

// FP32 form.  The (eps + beta)^2 products can overflow FP32, so the three
// (eps + beta) are first scaled by the same power of two (exact, no rounding),
// which leaves the weights unchanged.
XF_HD float weno5(float a, float b, float c, float d, float e) {
    const float q0 = 2.0f * a - 7.0f * b + 11.0f * c;
    const float q1 = -b + 5.0f * c + 2.0f * d;
    const float q2 = 2.0f * c + 5.0f * d - e;
    const float t0 = a - 2.0f * b + c, u0 = a - 4.0f * b + 3.0f * c;
    const float t1 = b - 2.0f * c + d, u1 = b - d;
    const float t2 = c - 2.0f * d + e, u2 = 3.0f * c - 4.0f * d + e;
    float s0 = (13.0f * t0) * t0 + ((3.0f * u0) * u0 + 12e-6f);
    float s1 = (13.0f * t1) * t1 + ((3.0f * u1) * u1 + 12e-6f);
    float s2 = (13.0f * t2) * t2 + ((3.0f * u2) * u2 + 12e-6f);
    const float smax = fmaxf(s0, fmaxf(s1, s2));
    int ex;
    frexpf(smax, &ex);
    s0 = ldexpf(s0, -ex);
    s1 = ldexpf(s1, -ex);
    s2 = ldexpf(s2, -ex);
    s0 *= s0;
    s1 *= s1;
    s2 *= s2;
    const float w0 = s1 * s2, w1 = 6.0f * (s0 * s2), w2 = 3.0f * (s0 * s1);
    return (w0 * q0 + w1 * q1 + w2 * q2) / (6.0f * (w0 + w1 + w2));
}

// WENO-CU6 value at the right edge of the cell holding c, from the six
// point values a..f (cells i-2..i+3): the three WENO5 candidates plus the
// downwind one (11 d - 7 e + 2 f)/6, linear weights (1, 9, 9, 1)/20,
// alpha_k = d_k (20 + tau6 / (beta_k + 1e-6)) with beta_3 = beta6, the
// smoothness of the whole six-cell stencil, and tau6 = beta6 -
// (beta_0 + 4 beta_1 + beta_2)/6.  beta6 is the Jiang-Shu integral of the
// stencil's quintic over cell i, a quadratic form that vanishes on
// constants; it is evaluated as sum_k D_k z_k^2 over the first differences
// (z_k = sum_{i >= k} L_ik (f_{i+1} - f_i), the exact LDL^T factors of the
// form rounded to double), which has no cancellation.  One division: all
// alpha_k are multiplied by prod_j (beta_j + eps).
template <typename R>
XF_HD R cu6_beta6(R a, R b, R c, R d, R e, R f) {
    const R d0 = b - a, d1 = c - b, d2 = d - c, d3 = e - d, d4 = f - e;
    const R z0 = d0 + R(-3.3800293620919937) * d1 + R(4.137755308541131) * d2 + R(-2.2318538224071762) * d3 +
                 R(0.4518745009732172) * d4;
    const R z1 = d1 + R(-1.8788632502196132) * d2 + R(1.2398246217680282) * d3 + R(-0.2835945203123665) * d4;
    const R z2 = d2 + R(-0.8641384480158466) * d3 + R(0.22441845180562248) * d4;
    const R z3 = d3 + R(-0.3841978250666033) * d4;
    return R(2.2468501984126985) * z0 * z0 + R(3.6320275079835525) * z1 * z1 + R(4.213886137822353) * z2 * z2 +
           R(1.0316113515772065) * z3 * z3 + R(0.03897812227306876) * d4 * d4;
}

XF_HD double weno_cu6(double a, double b, double c, double d, double e, double f) {
    const double q0 = (2.0 * a - 7.0 * b + 11.0 * c) * (1.0 / 6.0);
    const double q1 = (-b + 5.0 * c + 2.0 * d) * (1.0 / 6.0);
    const double q2 = (2.0 * c + 5.0 * d - e) * (1.0 / 6.0);
    const double q3 = (11.0 * d - 7.0 * e + 2.0 * f) * (1.0 / 6.0);
    const double t0 = a - 2.0 * b + c, u0 = a - 4.0 * b + 3.0 * c;
    const double t1 = b - 2.0 * c + d, u1 = b - d;
    const double t2 = c - 2.0 * d + e, u2 = 3.0 * c - 4.0 * d + e;
    const double b0 = (13.0 / 12.0) * t0 * t0 + 0.25 * u0 * u0;
    const double b1 = (13.0 / 12.0) * t1 * t1 + 0.25 * u1 * u1;
    const double b2 = (13.0 / 12.0) * t2 * t2 + 0.25 * u2 * u2;
    const double b6 = cu6_beta6(a, b, c, d, e, f);
    const double tau = b6 - (b0 + 4.0 * b1 + b2) * (1.0 / 6.0);
    const double e0 = b0 + 1e-6, e1 = b1 + 1e-6, e2 = b2 + 1e-6, e3 = b6 + 1e-6;
    const double p01 = e0 * e1, p23 = e2 * e3;
    const double w0 = (1.0 / 20.0) * (20.0 * e0 + tau) * (e1 * p23);
    const double w1 = (9.0 / 20.0) * (20.0 * e1 + tau) * (e0 * p23);
    const double w2 = (9.0 / 20.0) * (20.0 * e2 + tau) * (p01 * e3);
    const double w3 = (1.0 / 20.0) * (20.0 * e3 + tau) * (p01 * e2);
    return (w0 * q0 + w1 * q1 + w2 * q2 + w3 * q3) / (w0 + w1 + w2 + w3);
}

// FP32 form: beta_k + eps and tau are scaled by one power of two (exact),
// which leaves the weights unchanged and keeps the fourth-degree products in
// range.
XF_HD float weno_cu6(float a, float b, float c, float d, float e, float f) {
    const float q0 = (2.0f * a - 7.0f * b + 11.0f * c) * (1.0f / 6.0f);
    const float q1 = (-b + 5.0f * c + 2.0f * d) * (1.0f / 6.0f);
    const float q2 = (2.0f * c + 5.0f * d - e) * (1.0f / 6.0f);
    const float q3 = (11.0f * d - 7.0f * e + 2.0f * f) * (1.0f / 6.0f);
    const float t0 = a - 2.0f * b + c, u0 = a - 4.0f * b + 3.0f * c;
    const float t1 = b - 2.0f * c + d, u1 = b - d;
    const float t2 = c - 2.0f * d + e, u2 = 3.0f * c - 4.0f * d + e;
    const float b0 = (13.0f / 12.0f) * t0 * t0 + 0.25f * u0 * u0;
    const float b1 = (13.0f / 12.0f) * t1 * t1 + 0.25f * u1 * u1;
    const float b2 = (13.0f / 12.0f) * t2 * t2 + 0.25f * u2 * u2;
    const float b6 = cu6_beta6(a, b, c, d, e, f);
    float tau = b6 - (b0 + 4.0f * b1 + b2) * (1.0f / 6.0f);
    float e0 = b0 + 1e-6f, e1 = b1 + 1e-6f, e2 = b2 + 1e-6f, e3 = b6 + 1e-6f;
    int ex;
    frexpf(fmaxf(fmaxf(e0, e1), fmaxf(e2, e3)), &ex);
    e0 = ldexpf(e0, -ex);
    e1 = ldexpf(e1, -ex);
    e2 = ldexpf(e2, -ex);
    e3 = ldexpf(e3, -ex);
    tau = ldexpf(tau, -ex);
    const float p01 = e0 * e1, p23 = e2 * e3;
    const float w0 = (1.0f / 20.0f) * (20.0f * e0 + tau) * (e1 * p23);
    const float w1 = (9.0f / 20.0f) * (20.0f * e1 + tau) * (e0 * p23);
    const float w2 = (9.0f / 20.0f) * (20.0f * e2 + tau) * (p01 * e3);
    const float w3 = (1.0f / 20.0f) * (20.0f * e3 + tau) * (p01 * e2);
    return (w0 * q0 + w1 * q1 + w2 * q2 + w3 * q3) / (w0 + w1 + w2 + w3);
}


// WENO7-JS value at the right edge of the cell holding d, from the seven
// point values a..g (cells i-3..i+3): four cubic candidates (the edge values
// of the cubics whose cell averages are the data on i-3..i, ..., i..i+3),
// linear weights (1, 12, 18, 4)/35, alpha_k = d_k / (1e-6 + beta_k)^2.
// beta_k is the Jiang-Shu integral of sub-stencil k's cubic over cell i, a
// quadratic form that vanishes on constants; it is evaluated as
// D0 z0^2 + D1 z1^2 + D2 z2^2 over the sub-stencil's three first differences
// (z_j = sum_{l >= j} L_lj delta_l with L, D the exact LDL^T factors of the
// form, rational constants rounded once), so no large terms cancel.  The
// candidates are taken times 12 and the linear weights times 35.
template <typename R>
XF_HD void weno7_parts(R a, R b, R c, R d, R e, R f, R g, R *q, R *beta) {
    q[0] = R(-3) * a + R(13) * b - R(23) * c + R(25) * d;
    q[1] = b - R(5) * c + R(13) * d + R(3) * e;
    q[2] = -c + R(7) * d + R(7) * e - f;
    q[3] = R(3) * d + R(13) * e - R(5) * f + g;
    const R d0 = b - a, d1 = c - b, d2 = d - c, d3 = e - d, d4 = f - e, d5 = g - f;
    {
        const R z0 = d0 + R(-1394.0 / 547.0) * d1 + R(927.0 / 547.0) * d2, z1 = d1 + R(-3167.0 / 2126.0) * d2;
        beta[0] = R(547.0 / 240.0) * z0 * z0 + R(1063.0 / 1641.0) * z1 * z1 + R(10153.0 / 12756.0) * d2 * d2;
    }
    {
        const R z0 = d1 + R(-554.0 / 267.0) * d2 + R(247.0 / 267.0) * d3, z1 = d2 + R(-1345.0 / 2126.0) * d3;
        beta[1] = R(89.0 / 80.0) * z0 * z0 + R(1063.0 / 801.0) * z1 * z1 + R(10153.0 / 12756.0) * d3 * d3;
    }
    {
        const R z0 = d2 + R(-714.0 / 547.0) * d3 + R(247.0 / 547.0) * d4, z1 = d3 + R(-3167.0 / 7330.0) * d4;
        beta[2] = R(547.0 / 240.0) * z0 * z0 + R(3665.0 / 1641.0) * z1 * z1 + R(10153.0 / 43980.0) * d4 * d4;
    }
    {
        const R z0 = d3 + R(-2594.0 / 2107.0) * d4 + R(927.0 / 2107.0) * d5, z1 = d4 + R(-13313.0 / 27098.0) * d5;
        beta[3] = R(2107.0 / 240.0) * z0 * z0 + R(13549.0 / 6321.0) * z1 * z1 + R(10153.0 / 162588.0) * d5 * d5;
    }
}

// FP64: one division; alpha_k / sum alpha = d_k prod_{j!=k} s_j / sum(...),
// s_k = (eps + beta_k)^2, after the four (eps + beta_k) are scaled by one
// power of two (exact; weights unchanged) so that every product is <= 1.
XF_HD double weno7(double a, double b, double c, double d, double e, double f, double g) {
    double q[4], be[4];
    weno7_parts(a, b, c, d, e, f, g, q, be);
    double e0 = be[0] + 1e-6, e1 = be[1] + 1e-6, e2 = be[2] + 1e-6, e3 = be[3] + 1e-6;
    int ex;
    frexp(fmax(fmax(e0, e1), fmax(e2, e3)), &ex);
    e0 = ldexp(e0, -ex);
    e1 = ldexp(e1, -ex);
    e2 = ldexp(e2, -ex);
    e3 = ldexp(e3, -ex);
    const double s0 = e0 * e0, s1 = e1 * e1, s2 = e2 * e2, s3 = e3 * e3;
    const double p01 = s0 * s1, p23 = s2 * s3;
    const double w0 = s1 * p23, w1 = 12.0 * (s0 * p23), w2 = 18.0 * (p01 * s3), w3 = 4.0 * (p01 * s2);
    return (w0 * q[0] + w1 * q[1] + w2 * q[2] + w3 * q[3]) / (12.0 * (w0 + w1 + w2 + w3));
}

// FP32: the three-factor products of the FP64 form can underflow FP32 when
// one sub-stencil is far rougher than the others, so the weights are taken
// as d_k / (eps + beta_k)^2 directly, after the (eps + beta_k) are scaled by
// the power of two of the smallest (exact): every 1 / (eps + beta_k) is then
// at most 2 and the smoothest at least 1.
XF_HD float weno7(float a, float b, float c, float d, float e, float f, float g) {
    float q[4], be[4];
    weno7_parts(a, b, c, d, e, f, g, q, be);
    float e0 = be[0] + 1e-6f, e1 = be[1] + 1e-6f, e2 = be[2] + 1e-6f, e3 = be[3] + 1e-6f;
    int ex;
    frexpf(fminf(fminf(e0, e1), fminf(e2, e3)), &ex);
    const float i0 = 1.0f / ldexpf(e0, -ex), i1 = 1.0f / ldexpf(e1, -ex), i2 = 1.0f / ldexpf(e2, -ex),
                i3 = 1.0f / ldexpf(e3, -ex);
    const float w0 = i0 * i0, w1 = 12.0f * (i1 * i1), w2 = 18.0f * (i2 * i2), w3 = 4.0f * (i3 * i3);
    return (w0 * q[0] + w1 * q[1] + w2 * q[2] + w3 * q[3]) / (12.0f * (w0 + w1 + w2 + w3));
}

// Blocks are dealt to the 8 XCDs of the chip round robin in dispatch order.
// xcd_block renumbers them so that each XCD receives a contiguous range of
// logical blocks (blocks that share stencil rows then share one L2).
constexpr int kNumXcd = 8;

__device__ __forceinline__ void xcd_block(unsigned &bx, unsigned &by, unsigned &bz) {
    const unsigned gx = gridDim.x, gy = gridDim.y, gz = gridDim.z;
    const unsigned n = gx * gy * gz;
    const unsigned b = blockIdx.x + gx * (blockIdx.y + gy * blockIdx.z);
    // dispatch order b goes to XCD b % 8; give consecutive logical ids to the
    // blocks one XCD receives (only when the count divides evenly)
    unsigned l = b;
    if (n % kNumXcd == 0) l = (b % kNumXcd) * (n / kNumXcd) + b / kNumXcd;
    bx = l % gx;
    by = (l / gx) % gy;
    bz = l / (gx * gy);
}

// Read-only view of the stencil of one face along one axis (2 RAD cells:
// six, or eight for WENO7); S is the storage type (FP64 state, or the FP32
// copies the mixed path sweeps read).
template <typename S>
struct StencilT {
    const S *__restrict__ U;
    const S *__restrict__ P;        // [4][cells]: T, p, c, 1/rho
    long long base;                 // padded index of stencil cell 0 (= i-RAD+1)
    long long step;                 // index stride along the sweep axis
    long long cells;                // field stride
    XF_HD S u(int f, int m) const { return U[f * cells + base + m * step]; }
    XF_HD S p(int k, int m) const { return P[k * cells + base + m * step]; }
};
using Stencil = StencilT<double>;

// Stencil values staged in LDS: field f of stencil cell m at
// t[f * fs + base + m * step]; fields 0..NV-1 are U, NV..NV+3 the primitives
// (T, p, c, 1/rho).  The pointer carries the LDS address space, so no
// generic-address checks are generated.
typedef __attribute__((address_space(3))) double lds_double;
template <int NV, typename T = double>
struct StencilLds {
    const __attribute__((address_space(3))) T *t;
    int base, step, fs;
    XF_HD T u(int f, int m) const { return t[f * fs + base + m * step]; }
    XF_HD T p(int k, int m) const { return t[(NV + k) * fs + base + m * step]; }
};

template <int DIR>
struct Axes {
    // momentum component of the normal and of the two tangents
    static constexpr int n = DIR;
    static constexpr int t1 = (DIR == 0) ? 1 : 0;
    static constexpr int t2 = (DIR == 2) ? 1 : 2;
};

// Numerical flux at one face.  Each component of F^ is handed to out(q, v)
// as soon as it is final (species first, then momentum and energy), so the
// caller decides where it lives.  flags collects XF_FLAG_C2 if the face c^2
// is not positive.  FENCE inserts compiler fences between the phases.
// Artificial viscosity of the flux splitting (Eq. 14; Table I): LLF, the
// max over the stencil cells of each field's |lambda|; ROE, |lambda| of
// the face's Roe state (u~_n - c~, u~_n, u~_n + c~); GLF, each field's
// largest LLF speed over all faces of the direction (glf: the three speeds
// u_n - c, u_n, u_n + c, reduced beforehand).
// kViscFrozen is no scheme of its own: the three speeds of every face are
// given (alpha[k * astride + fidx], k = u-c, u, u+c fields; fidx the face's
// index in its direction), for checks of the linearisation at fixed speeds.
constexpr int kViscLlf = 0, kViscRoe = 1, kViscGlf = 2, kViscFrozen = 3;
constexpr int kReconWeno5 = 0, kReconCu6 = 1, kReconWeno7 = 2;
struct Dissip {
    int type;
    const double *glf;
    int recon;   // kReconWeno5, kReconCu6 or kReconWeno7
    const double *alpha = nullptr;   // kViscFrozen: [3][astride] speeds of the direction's faces
    long long astride = 0, fidx = 0;
};

// Stencil half width of a reconstruction: 3 (six cells i-2..i+3; WENO5,
// CU6) or 4 (eight cells i-3..i+4; WENO7).
constexpr int stencil_radius(int rec) { return rec == kReconWeno7 ? 4 : 3; }

// Reconstruction of one characteristic field at the face from the split
// values of the stencil cells: WENO5-JS of g+ on cells i-2..i+2 plus g-
// mirrored on i+3..i-1; WENO-CU6 of both on all six cells; WENO7-JS of g+
// on i-3..i+3 plus g- mirrored on i+4..i-2.
template <int REC, bool PAIR, typename R>
XF_HD R recon_pair(const R *gp, const R *gm) {
    if constexpr (REC == kReconWeno7)
        return weno7(gp[0], gp[1], gp[2], gp[3], gp[4], gp[5], gp[6]) +
               weno7(gm[7], gm[6], gm[5], gm[4], gm[3], gm[2], gm[1]);
    else if constexpr (REC == kReconCu6)
        return weno_cu6(gp[0], gp[1], gp[2], gp[3], gp[4], gp[5]) +
               weno_cu6(gm[5], gm[4], gm[3], gm[2], gm[1], gm[0]);
    else if constexpr (sizeof(R) == 8 && PAIR)
        return weno5_pair(gp[0], gp[1], gp[2], gp[3], gp[4], gm[5], gm[4], gm[3], gm[2], gm[1]);
    else
        return weno5(gp[0], gp[1], gp[2], gp[3], gp[4]) + weno5(gm[5], gm[4], gm[3], gm[2], gm[1]);
}

// SPD (kVisc*) and REC (kRecon*) select the artificial viscosity and the
// reconstruction at compile time, so every combination is its own code with
// no run-time switch left in it (ROE and GLF skip the stencil maxima
// altogether); ds supplies the GLF speeds.  PAIR takes both sides of an
// FP64 WENO5 field with one reciprocal (off where the extra live values
// spill, as next to the positivity blend).  ROLL runs the species loops as
// loops (the Roe Y_s and chi_s recomputed where used, the per-cell sums
// taken species by species) instead of unrolling them, which frees the
// per-species registers at the cost of three evaluations of e_s(T~) per
// species instead of one.
template <int NS, typename R, int DIR, bool FENCE = false, int SPD = kViscLlf, int REC = kReconWeno5,
          bool PAIR = true, bool ROLL = false, class St, class Out>
XF_HD void face_flux_to(const St &st, const ThermoK<R> &th, Out &&out, unsigned &flags, const Dissip &ds) {
    constexpr int RAD = stencil_radius(REC);
    constexpr int W = 2 * RAD;       // stencil cells
    constexpr int CL = RAD - 1;      // slot of cell i (left of the face)
    constexpr int CR = RAD;          // slot of cell i+1
    constexpr int IM = NS;
    constexpr int IE = NS + 3;
    constexpr int IN = NS + Axes<DIR>::n;
    constexpr int I1 = NS + Axes<DIR>::t1;
    constexpr int I2 = NS + Axes<DIR>::t2;

    // ---- 1. Roe-averaged face state ------------------------------------
    R rL = R(0), rR = R(0);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        rL += R(st.u(s, CL));
        rR += R(st.u(s, CR));
    }
    const R sL = xsqrt(rL), sR = xsqrt(rR);
    const R wL = sL / (sL + sR);
    const R wR = R(1) - wL;
    const R aL = wL * R(st.p(3, CL)), aR = wR * R(st.p(3, CR));   // weights on conservative values
    R ut[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) ut[k] = aL * R(st.u(IM + k, CL)) + aR * R(st.u(IM + k, CR));
    const R Ht = aL * (R(st.u(IE, CL)) + R(st.p(1, CL))) + aR * (R(st.u(IE, CR)) + R(st.p(1, CR)));
    const R Tt = wL * R(st.p(0, CL)) + wR * R(st.p(0, CR));
    R Yt[ROLL ? 1 : NS], chi[ROLL ? 1 : NS];   // per-species Roe values (unrolled form only)
    R Rb = R(0), cvb = R(0), Se = R(0), S1 = R(0);
    if constexpr (ROLL) {
#pragma unroll 1
        for (int s = 0; s < NS; ++s) {
            const R Y = aL * R(st.u(s, CL)) + aR * R(st.u(s, CR));
            S1 += Y;
            Rb += Y * th.Rs[s];
            cvb += Y * cv_species(th, s, Tt);
            Se += Y * e_species(th, s, Tt);
        }
    } else {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            Yt[s] = aL * R(st.u(s, CL)) + aR * R(st.u(s, CR));
            Rb += Yt[s] * th.Rs[s];
            cvb += Yt[s] * cv_species(th, s, Tt);
            chi[s] = e_species(th, s, Tt);   // e_s(T~) for now
        }
    }
    const R Gam = Rb / cvb;
    const R q2 = ut[0] * ut[0] + ut[1] * ut[1] + ut[2] * ut[2];
    R c2 = Gam * (Ht - q2);
    if constexpr (ROLL) {
        // sum_s Y_s chi_s with S1 = sum Y, Se = sum Y e_s(T~), Rb = sum Y R_s
        c2 += Gam * (R(0.5) * q2 * S1 - Se) + Tt * Rb;
    } else {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            chi[s] = Gam * (R(0.5) * q2 - chi[s]) + th.Rs[s] * Tt;
            c2 += Yt[s] * chi[s];
        }
    }
    if (!(c2 > R(0))) flags |= XF_FLAG_C2;
    const R ct = xsqrt(c2);
    const R ic2 = R(1) / c2;
    const R cih = R(0.5) * ct * ic2;      // c / (2 c^2)
    const R utn = ut[Axes<DIR>::n], ut1 = ut[Axes<DIR>::t1], ut2 = ut[Axes<DIR>::t2];

    if (FENCE) XF_FENCE();
    // ---- 2./3. per-cell scalars of the projections, LLF speeds ----------
    R un[W], DU[W], DF[W], rh[W];
    R aM = R(0), a0 = R(0), aP = R(0);
    R scm[ROLL ? W : 1];   // rolled form: sum_s chi_s rho_s of every cell, species outermost
    if constexpr (ROLL) {
#pragma unroll
        for (int m = 0; m < W; ++m) {
            scm[m] = R(0);
            rh[m] = R(0);
        }
#pragma unroll 1
        for (int s = 0; s < NS; ++s) {
            const R chis = Gam * (R(0.5) * q2 - e_species(th, s, Tt)) + th.Rs[s] * Tt;
#pragma unroll
            for (int m = 0; m < W; ++m) {
                const R r = R(st.u(s, m));
                scm[m] += chis * r;
                rh[m] += r;
            }
        }
    }
#pragma unroll
    for (int m = 0; m < W; ++m) {
        R sc = R(0), sr = R(0);
        if constexpr (ROLL) {
            sc = scm[m];
            sr = rh[m];
        } else {
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const R r = R(st.u(s, m));
                sc += chi[s] * r;
                sr += r;
            }
        }
        const R rinv = R(st.p(3, m)), pm = R(st.p(1, m)), cm = R(st.p(2, m));
        const R E = R(st.u(IE, m));
        const R unm = R(st.u(IN, m)) * rinv;
        const R um = ut[0] * R(st.u(IM, m)) + ut[1] * R(st.u(IM + 1, m)) + ut[2] * R(st.u(IM + 2, m));
        // dp of U_m and of F_m = (rho_s u_n, m u_n + p n, (E + p) u_n)
        const R dpU = sc - Gam * um + Gam * E;
        const R dpF = unm * sc - Gam * (unm * um + pm * utn) + Gam * ((E + pm) * unm);
        un[m] = unm;
        DU[m] = dpU * ic2;
        DF[m] = dpF * ic2;
        rh[m] = sr;
        if constexpr (SPD == kViscLlf) {
            aM = rmax(aM, rabs(unm - cm));
            a0 = rmax(a0, rabs(unm));
            aP = rmax(aP, rabs(unm + cm));
        } else {
            (void)cm;
        }
    }
    if constexpr (SPD == kViscRoe) {
        aM = rabs(utn - ct);
        a0 = rabs(utn);
        aP = rabs(utn + ct);
    } else if constexpr (SPD == kViscGlf) {
        aM = R(ds.glf[0]);
        a0 = R(ds.glf[1]);
        aP = R(ds.glf[2]);
    } else if constexpr (SPD == kViscFrozen) {
        aM = R(ds.alpha[ds.fidx]);
        a0 = R(ds.alpha[ds.astride + ds.fidx]);
        aP = R(ds.alpha[2 * ds.astride + ds.fidx]);
    }

    if (FENCE) XF_FENCE();
    // ---- acoustic pair ----------------------------------------------------
    R hm, hp;
    {
        R gMp[W], gMm[W], gPp[W], gPm[W];
#pragma unroll
        for (int m = 0; m < W; ++m) {
            const R mn = R(st.u(IN, m));
            const R XU = mn - utn * rh[m];
            const R XF = (mn * un[m] + R(st.p(1, m))) - utn * (rh[m] * un[m]);
            const R wUm = R(0.5) * DU[m] - cih * XU, wFm = R(0.5) * DF[m] - cih * XF;
            const R wUp = R(0.5) * DU[m] + cih * XU, wFp = R(0.5) * DF[m] + cih * XF;
            gMp[m] = R(0.5) * (wFm + aM * wUm);
            gMm[m] = R(0.5) * (wFm - aM * wUm);
            gPp[m] = R(0.5) * (wFp + aP * wUp);
            gPm[m] = R(0.5) * (wFp - aP * wUp);
        }
        hm = recon_pair<REC, PAIR>(gMp, gMm);
        hp = recon_pair<REC, PAIR>(gPp, gPm);
    }
    const R Asum = hm + hp, Dif = hp - hm;

    if (FENCE) XF_FENCE();
    // ---- tangential pair --------------------------------------------------
    R h1, h2;
    {
        R gp[W], gm[W];
#pragma unroll
        for (int m = 0; m < W; ++m) {
            const R wU = R(st.u(I1, m)) - ut1 * rh[m];
            const R wF = un[m] * wU;
            gp[m] = R(0.5) * (wF + a0 * wU);
            gm[m] = R(0.5) * (wF - a0 * wU);
        }
        h1 = recon_pair<REC, PAIR>(gp, gm);
#pragma unroll
        for (int m = 0; m < W; ++m) {
            const R wU = R(st.u(I2, m)) - ut2 * rh[m];
            const R wF = un[m] * wU;
            gp[m] = R(0.5) * (wF + a0 * wU);
            gm[m] = R(0.5) * (wF - a0 * wU);
        }
        h2 = recon_pair<REC, PAIR>(gp, gm);
    }

    // ---- species fields, back-projected as they come ----------------------
    const R iGam = R(1) / Gam;
    R gsum = R(0), gE = R(0);
    // one species field: its Roe mass fraction Ys and chi_s given
    auto species = [&](int s, R Ys, R chis) {
        R gp[W], gm[W];
#pragma unroll
        for (int m = 0; m < W; ++m) {
            const R r = R(st.u(s, m));
            const R wU = r - Ys * DU[m];
            const R wF = r * un[m] - Ys * DF[m];
            gp[m] = R(0.5) * (wF + a0 * wU);
            gm[m] = R(0.5) * (wF - a0 * wU);
        }
        const R hs = recon_pair<REC, PAIR>(gp, gm);
        out(s, Ys * Asum + hs);
        gsum += hs;
        gE += (q2 - chis * iGam) * hs;
    };
    if constexpr (ROLL) {
#pragma unroll 1
        for (int s = 0; s < NS; ++s) {
            if (FENCE) XF_FENCE();
            const R Ys = aL * R(st.u(s, CL)) + aR * R(st.u(s, CR));
            species(s, Ys, Gam * (R(0.5) * q2 - e_species(th, s, Tt)) + th.Rs[s] * Tt);
        }
    } else {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            if (FENCE) XF_FENCE();
            species(s, Yt[s], chi[s]);
        }
    }

    // ---- momentum and energy of F^ = R h ----------------------------------
    R Fm[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) Fm[k] = ut[k] * (Asum + gsum);
    Fm[Axes<DIR>::n] += ct * Dif;
    Fm[Axes<DIR>::t1] += h1;
    Fm[Axes<DIR>::t2] += h2;
    out(IM + 0, Fm[0]);
    out(IM + 1, Fm[1]);
    out(IM + 2, Fm[2]);
    out(IE, Ht * Asum + utn * ct * Dif + ut1 * h1 + ut2 * h2 + gE);
}

// Numerical flux at one face into Fh[0..NS+3] (conservative field order).
template <int NS, typename R, int DIR>
XF_HD void face_flux(const Stencil &st, const ThermoK<R> &th, R *__restrict__ Fh, unsigned &flags) {
    face_flux_to<NS, R, DIR>(st, th, [&](int q, R v) { Fh[q] = v; }, flags, Dissip{kViscLlf, nullptr});
}

// ---------------------------------------------------------------------------
// Positivity-preserving blend of one face flux (Sec. II.C.2, Eq. 17-20):
// F* = F_LF + theta (F^ - F_LF), F_LF the Lax-Friedrichs flux of Eq. 19 with
// the face's larger acoustic LLF speed as its coefficient, theta the largest
// value in [0, 1] that keeps the Euler half-states U_i - 2 lam F* and
// U_i+1 + 2 lam F* of Eq. 18 at or above the floors: total density
// 1e-13 min(rho_i, rho_i+1), each partial density -1e-13 rho of its own cell
// in FP64 (-1e-6 rho in FP32, above that precision's round-off of a
// vanishing species' flux); the minimum over the components and both cells;
// theta = 1 leaves F^ untouched.  lam = D dt / dx for D active dimensions (the multi-dimensional
// Euler step is the mean of D one-dimensional ones).  F holds F^ on entry and
// F* on return.
// ---------------------------------------------------------------------------
constexpr double kPpRhoFloor = 1e-13;
template <typename R>
struct PpFloor {
    static constexpr double y = 1e-6;
};
template <>
struct PpFloor<double> {
    static constexpr double y = 1e-13;
};

template <int NS, typename R, int DIR, int RAD = 3, class St>
XF_HD void pp_limit(const St &st, R lam, R *F) {
    constexpr int NV = NS + 4, IE = NS + 3, IN = NS + Axes<DIR>::n;
    constexpr int CL = RAD - 1, CR = RAD;   // slots of cells i and i+1
    R aM = R(0), aP = R(0);
#pragma unroll
    for (int m = 0; m < 2 * RAD; ++m) {
        const R rinv = R(st.p(3, m)), cm = R(st.p(2, m));
        const R unm = R(st.u(IN, m)) * rinv;
        aM = rmax(aM, rabs(unm - cm));
        aP = rmax(aP, rabs(unm + cm));
    }
    const R lf = rmax(aM, aP);
    const R pL = R(st.p(1, CL)), pR = R(st.p(1, CR));
    const R unL = R(st.u(IN, CL)) * R(st.p(3, CL)), unR = R(st.u(IN, CR)) * R(st.p(3, CR));
    R FLF[NV];
#pragma unroll
    for (int f = 0; f < NV; ++f) {
        const R uL = R(st.u(f, CL)), uR = R(st.u(f, CR));
        R fL, fR;
        if (f == IE) {
            fL = (uL + pL) * unL;
            fR = (uR + pR) * unR;
        } else if (f == IN) {
            fL = uL * unL + pL;
            fR = uR * unR + pR;
        } else {
            fL = uL * unL;
            fR = uR * unR;
        }
        FLF[f] = R(0.5) * ((fL + fR) + lf * (uL - uR));
    }
    // components kept positive: rho (row 0), rho_1 .. rho_NS
    R rhoL = R(0), rhoR = R(0), qH = R(0), qLF = R(0);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        rhoL += R(st.u(s, CL));
        rhoR += R(st.u(s, CR));
        qH += F[s];
        qLF += FLF[s];
    }
    const R two_lam = R(2) * lam;
    const R floor_rho = R(kPpRhoFloor) * rmin(rhoL, rhoR);
    R theta = R(1);
    auto bound = [&](R q0, R sgn, R h, R lo, R eps) {
        const R w_hi = q0 + sgn * two_lam * h;       // half-state with the high-order flux
        const R w_lo = q0 + sgn * two_lam * lo;      // ... with the Lax-Friedrichs flux
        const R gap = w_lo - w_hi;
        R t = R(1);
        if (!(w_hi >= eps)) t = gap > R(0) ? (w_lo - eps) / gap : R(0);
        t = rmin(rmax(t, R(0)), R(1));
        theta = rmin(theta, t);
    };
    bound(rhoL, R(-1), qH, qLF, floor_rho);
    bound(rhoR, R(1), qH, qLF, floor_rho);
    const R epsL = -R(PpFloor<R>::y) * rhoL, epsR = -R(PpFloor<R>::y) * rhoR;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        bound(R(st.u(s, CL)), R(-1), F[s], FLF[s], epsL);
        bound(R(st.u(s, CR)), R(1), F[s], FLF[s], epsR);
    }
    if (theta < R(1)) {
#pragma unroll
        for (int f = 0; f < NV; ++f) F[f] = FLF[f] + theta * (F[f] - FLF[f]);
    }
}

}  // namespace xf
