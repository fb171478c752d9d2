// xf_vjp.hpp -- hand-written vector-Jacobian product of the convective flux.
//
// For one face, face_vjp recomputes the forward flux of xf_face.hpp and then
// runs it backwards, given the cotangent Fb of F^_{i+1/2}.  It adds the
// cotangents of the six stencil cells' conservative values (directly, and
// through 1/rho = 1/sum_s rho_s) and of the cells' pressure and temperature
// (into a separate two-field buffer; the per-cell map (p, T)(U) is
// differentiated afterwards by k_prims_vjp).  The LLF speeds alpha are held
// fixed.  Every step of the forward is differentiated: back-projection,
// WENO5-JS weights (through the smoothness indicators), the characteristic
// projections and their dependence on the Roe state, the Roe average with
// species thermo at the averaged temperature, and the sqrt(rho) weights.
#pragma once

#include "xf_face.hpp"

namespace xf {

// Phase boundary of the face VJP: besides the compiler fence, the stencil's
// base index passes through an empty asm statement, so loads of one phase
// cannot be merged with the same loads of an earlier one (which would keep
// every loaded stencil value live across the whole routine).
#ifdef __HIP_DEVICE_COMPILE__
#define XF_PHASE(st) asm volatile("" : "+v"(st.base) : : "memory")
#else
#define XF_PHASE(st) ((void)0)
#endif

// Reciprocal of a positive normal number: rcp_nr (about 1 ulp, 5
// instructions) in FP64, IEEE division in FP32.
XF_HD double vjp_recip(double x) { return rcp_nr(x); }
XF_HD float vjp_recip(float x) { return 1.0f / x; }

// WENO5-JS backward.  Adds hb * dW/d(a..e) to (ab..eb), W the value of
// weno5(a..e):  dW/dx = sum_k w_k dq_k/dx - 2 sum_k w_k (q_k - W)/(eps + beta_k)
// dbeta_k/dx, w_k the normalised nonlinear weights.
template <typename R>
XF_HD R weno5_bwd(R a, R b, R c, R d, R e, R hb, R &ab, R &bb, R &cb, R &db, R &eb) {
    const R q0 = (R(2) * a - R(7) * b + R(11) * c) * R(1.0 / 6.0);
    const R q1 = (-b + R(5) * c + R(2) * d) * R(1.0 / 6.0);
    const R q2 = (R(2) * c + R(5) * d - e) * R(1.0 / 6.0);
    const R t0 = a - R(2) * b + c, u0 = a - R(4) * b + R(3) * c;
    const R t1 = b - R(2) * c + d, u1 = b - d;
    const R t2 = c - R(2) * d + e, u2 = R(3) * c - R(4) * d + e;
    const R i0 = vjp_recip(R(1e-6) + (R(13.0 / 12.0) * t0 * t0 + R(0.25) * u0 * u0));
    const R i1 = vjp_recip(R(1e-6) + (R(13.0 / 12.0) * t1 * t1 + R(0.25) * u1 * u1));
    const R i2 = vjp_recip(R(1e-6) + (R(13.0 / 12.0) * t2 * t2 + R(0.25) * u2 * u2));
    const R al0 = R(0.1) * i0 * i0, al1 = R(0.6) * i1 * i1, al2 = R(0.3) * i2 * i2;
    const R iS = vjp_recip(al0 + al1 + al2);
    const R w0 = al0 * iS, w1 = al1 * iS, w2 = al2 * iS;
    const R W = w0 * q0 + w1 * q1 + w2 * q2;
    const R g0 = hb * w0, g1 = hb * w1, g2 = hb * w2;
    const R z0 = R(-2) * g0 * (q0 - W) * i0;
    const R z1 = R(-2) * g1 * (q1 - W) * i1;
    const R z2 = R(-2) * g2 * (q2 - W) * i2;
    const R A0 = R(13.0 / 6.0) * t0 * z0, B0 = R(0.5) * u0 * z0;
    const R A1 = R(13.0 / 6.0) * t1 * z1, B1 = R(0.5) * u1 * z1;
    const R A2 = R(13.0 / 6.0) * t2 * z2, B2 = R(0.5) * u2 * z2;
    ab += g0 * R(2.0 / 6.0) + A0 + B0;
    bb += g0 * R(-7.0 / 6.0) - g1 * R(1.0 / 6.0) - R(2) * A0 - R(4) * B0 + A1 + B1;
    cb += g0 * R(11.0 / 6.0) + g1 * R(5.0 / 6.0) + g2 * R(2.0 / 6.0) + A0 + R(3) * B0 - R(2) * A1 + A2 + R(3) * B2;
    db += g1 * R(2.0 / 6.0) + g2 * R(5.0 / 6.0) + A1 - B1 - R(2) * A2 - R(4) * B2;
    eb += g2 * R(-1.0 / 6.0) + A2 + B2;
    return W;
}

// Forward and backward of h = W(g+_{0..4}) + W(g-_{5..1}) with
// g+- = (wF +- al wU)/2: returns h and the cotangents of wF and wU at the six
// stencil cells for the output cotangent hb.
// WENO-CU6 backward (forms as in weno_cu6 of the face code).  Adds
// hb * dW/d(a..f) to (ab..fb), W the value of weno_cu6(a..f):
// W = sum_k w_k q_k, w_k = alpha_k / S, alpha_k = d_k (C + tau / e_k),
// e_k = beta_k + eps (beta_3 = beta6), so
// dW = sum_k w_k dq_k + sum_k (q_k - W) / S * d_k / e_k (dtau - tau dbeta_k / e_k).
template <typename R>
XF_HD R cu6_bwd(R a, R b, R c, R d, R e, R f, R hb, R &ab, R &bb, R &cb, R &db, R &eb, R &fb) {
    const R q0 = (R(2) * a - R(7) * b + R(11) * c) * R(1.0 / 6.0);
    const R q1 = (-b + R(5) * c + R(2) * d) * R(1.0 / 6.0);
    const R q2 = (R(2) * c + R(5) * d - e) * R(1.0 / 6.0);
    const R q3 = (R(11) * d - R(7) * e + R(2) * f) * R(1.0 / 6.0);
    const R t0 = a - R(2) * b + c, u0 = a - R(4) * b + R(3) * c;
    const R t1 = b - R(2) * c + d, u1 = b - d;
    const R t2 = c - R(2) * d + e, u2 = R(3) * c - R(4) * d + e;
    const R b0 = R(13.0 / 12.0) * t0 * t0 + R(0.25) * u0 * u0;
    const R b1 = R(13.0 / 12.0) * t1 * t1 + R(0.25) * u1 * u1;
    const R b2 = R(13.0 / 12.0) * t2 * t2 + R(0.25) * u2 * u2;
    // beta6 = sum_k D_k z_k^2 over first differences (constants of cu6_beta6)
    const R d0 = b - a, d1 = c - b, d2 = d - c, d3 = e - d, d4 = f - e;
    const R L10 = R(-3.3800293620919937), L20 = R(4.137755308541131), L30 = R(-2.2318538224071762),
            L40 = R(0.4518745009732172), L21 = R(-1.8788632502196132), L31 = R(1.2398246217680282),
            L41 = R(-0.2835945203123665), L32 = R(-0.8641384480158466), L42 = R(0.22441845180562248),
            L43 = R(-0.3841978250666033);
    const R D0 = R(2.2468501984126985), D1 = R(3.6320275079835525), D2 = R(4.213886137822353),
            D3 = R(1.0316113515772065), D4 = R(0.03897812227306876);
    const R z0 = d0 + L10 * d1 + L20 * d2 + L30 * d3 + L40 * d4;
    const R z1 = d1 + L21 * d2 + L31 * d3 + L41 * d4;
    const R z2 = d2 + L32 * d3 + L42 * d4;
    const R z3 = d3 + L43 * d4;
    const R b6 = D0 * z0 * z0 + D1 * z1 * z1 + D2 * z2 * z2 + D3 * z3 * z3 + D4 * d4 * d4;
    const R tau = b6 - (b0 + R(4) * b1 + b2) * R(1.0 / 6.0);
    const R ie0 = vjp_recip(b0 + R(1e-6)), ie1 = vjp_recip(b1 + R(1e-6)), ie2 = vjp_recip(b2 + R(1e-6)),
            ie3 = vjp_recip(b6 + R(1e-6));
    const R al0 = R(1.0 / 20.0) * (R(20) + tau * ie0), al1 = R(9.0 / 20.0) * (R(20) + tau * ie1);
    const R al2 = R(9.0 / 20.0) * (R(20) + tau * ie2), al3 = R(1.0 / 20.0) * (R(20) + tau * ie3);
    const R iS = vjp_recip(al0 + al1 + al2 + al3);
    const R W = (al0 * q0 + al1 * q1 + al2 * q2 + al3 * q3) * iS;
    // cotangents of the candidates, of tau and of the betas
    const R g0 = hb * (q0 - W) * iS * R(1.0 / 20.0) * ie0, g1 = hb * (q1 - W) * iS * R(9.0 / 20.0) * ie1;
    const R g2 = hb * (q2 - W) * iS * R(9.0 / 20.0) * ie2, g3 = hb * (q3 - W) * iS * R(1.0 / 20.0) * ie3;
    const R tau_b = g0 + g1 + g2 + g3;
    const R b0_b = -g0 * tau * ie0 - tau_b * R(1.0 / 6.0);
    const R b1_b = -g1 * tau * ie1 - tau_b * R(4.0 / 6.0);
    const R b2_b = -g2 * tau * ie2 - tau_b * R(1.0 / 6.0);
    const R b6_b = -g3 * tau * ie3 + tau_b;
    const R w0 = hb * al0 * iS, w1 = hb * al1 * iS, w2 = hb * al2 * iS, w3 = hb * al3 * iS;
    // candidates
    ab += w0 * R(2.0 / 6.0);
    bb += w0 * R(-7.0 / 6.0) - w1 * R(1.0 / 6.0);
    cb += w0 * R(11.0 / 6.0) + w1 * R(5.0 / 6.0) + w2 * R(2.0 / 6.0);
    db += w1 * R(2.0 / 6.0) + w2 * R(5.0 / 6.0) + w3 * R(11.0 / 6.0);
    eb += -w2 * R(1.0 / 6.0) - w3 * R(7.0 / 6.0);
    fb += w3 * R(2.0 / 6.0);
    // Jiang-Shu indicators of the three upwind sub-stencils
    const R A0 = R(13.0 / 6.0) * t0 * b0_b, B0 = R(0.5) * u0 * b0_b;
    const R A1 = R(13.0 / 6.0) * t1 * b1_b, B1 = R(0.5) * u1 * b1_b;
    const R A2 = R(13.0 / 6.0) * t2 * b2_b, B2 = R(0.5) * u2 * b2_b;
    ab += A0 + B0;
    bb += -R(2) * A0 - R(4) * B0 + A1 + B1;
    cb += A0 + R(3) * B0 - R(2) * A1 + A2 + R(3) * B2;
    db += A1 - B1 - R(2) * A2 - R(4) * B2;
    eb += A2 + B2;
    // beta6 through its squares and the first differences
    const R y0 = R(2) * D0 * z0 * b6_b, y1 = R(2) * D1 * z1 * b6_b, y2 = R(2) * D2 * z2 * b6_b,
            y3 = R(2) * D3 * z3 * b6_b, y4 = R(2) * D4 * d4 * b6_b;
    const R d0b = y0;
    const R d1b = L10 * y0 + y1;
    const R d2b = L20 * y0 + L21 * y1 + y2;
    const R d3b = L30 * y0 + L31 * y1 + L32 * y2 + y3;
    const R d4b = L40 * y0 + L41 * y1 + L42 * y2 + L43 * y3 + y4;
    ab -= d0b;
    bb += d0b - d1b;
    cb += d1b - d2b;
    db += d2b - d3b;
    eb += d3b - d4b;
    fb += d4b;
    return W;
}

// split_weno_fb for WENO-CU6: h = CU6(g+_{0..5}) + CU6(g-_{5..0}).
template <typename R>
XF_HD R split_cu6_fb(const R *gp, const R *gm, R al, R hb, R *wFb, R *wUb) {
    R pb[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
    R mb[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
    const R h = cu6_bwd(gp[0], gp[1], gp[2], gp[3], gp[4], gp[5], hb, pb[0], pb[1], pb[2], pb[3], pb[4], pb[5]) +
                cu6_bwd(gm[5], gm[4], gm[3], gm[2], gm[1], gm[0], hb, mb[5], mb[4], mb[3], mb[2], mb[1], mb[0]);
#pragma unroll
    for (int m = 0; m < 6; ++m) {
        wFb[m] = R(0.5) * (pb[m] + mb[m]);
        wUb[m] = R(0.5) * al * (pb[m] - mb[m]);
    }
    return h;
}

template <typename R>
XF_HD R split_weno_fb(const R *gp, const R *gm, R al, R hb, R *wFb, R *wUb) {
    R pb[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
    R mb[6] = {R(0), R(0), R(0), R(0), R(0), R(0)};
    const R h = weno5_bwd(gp[0], gp[1], gp[2], gp[3], gp[4], hb, pb[0], pb[1], pb[2], pb[3], pb[4]) +
                weno5_bwd(gm[5], gm[4], gm[3], gm[2], gm[1], hb, mb[5], mb[4], mb[3], mb[2], mb[1]);
#pragma unroll
    for (int m = 0; m < 6; ++m) {
        wFb[m] = R(0.5) * (pb[m] + mb[m]);
        wUb[m] = R(0.5) * al * (pb[m] - mb[m]);
    }
    return h;
}

template <typename R>
XF_HD R dcv_species(const ThermoK<R> &th, int s, R T) {
    return ((R(4) * th.cv[s][4] * T + R(3) * th.cv[s][3]) * T + R(2) * th.cv[s][2]) * T + th.cv[s][1];
}

// Where the cotangents of one stencil go: a wave's private LDS window of the
// padded cells its faces touch ([NV + 3][W], field-major; stencil cell 0 of
// this thread's face at window index off).  Rows NV.. hold the cotangents of
// the cell's pressure, of its temperature and of its density rho = sum_s
// rho_s (added to every partial density by k_prims_vjp).  Lanes of a wave
// share window cells through different (field, cell) calls, so the
// read-modify-writes must stay in program order even where one thread's
// addresses differ: the accesses are volatile (LDS executes a wave's
// instructions in order).  The pointer carries the LDS address space, so no
// generic-address checks are generated.
constexpr int kSinkP = 0, kSinkT = 1, kSinkRho = 2, kSinkExtra = 3;
struct SinkLds {
    volatile lds_double *w;
    int W, off, mstep, pofs;   // window length, offset of stencil cell 0, cell stride, start of the extra rows
    XF_HD void u(int f, int m, double v) const { w[f * W + off + m * mstep] += v; }
    XF_HD void p(int k, int m, double v) const { w[pofs + k * W + off + m * mstep] += v; }
};

// Cotangent of the face flux, (rbar_R - rbar_L) / dx of the residual's
// cotangent at the face's two cells (zero outside the interior); read from
// memory where it is used.
struct FaceBar {
    const double *__restrict__ rbar;
    long long C, cr, cl;   // field stride, right and left cell
    bool hr, hl;           // the right / left cell is interior
    double id;             // 1 / dx of the direction
    XF_HD double operator()(int q) const {
        const double r = hr ? rbar[q * C + cr] : 0.0;
        const double l = hl ? rbar[q * C + cl] : 0.0;
        return (r - l) * id;
    }
};

// Forward Roe state of one face (the dissipation speeds of the ROE scheme).
template <int NS, typename R>
struct RoeFwd {
    R ut[3], ct;
    XF_HD RoeFwd(const Stencil &st, const ThermoK<R> &th) {
        constexpr int IM = NS;
        constexpr int IE = NS + 3;
        R rL = R(0), rR = R(0);
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            rL += R(st.u(s, 2));
            rR += R(st.u(s, 3));
        }
        const R sL = xsqrt(rL), sR = xsqrt(rR);
        const R wL = sL / (sL + sR), wR = R(1) - wL;
        const R aL = wL * R(st.p(3, 2)), aR = wR * R(st.p(3, 3));
#pragma unroll
        for (int k = 0; k < 3; ++k) ut[k] = aL * R(st.u(IM + k, 2)) + aR * R(st.u(IM + k, 3));
        const R Ht = aL * (R(st.u(IE, 2)) + R(st.p(1, 2))) + aR * (R(st.u(IE, 3)) + R(st.p(1, 3)));
        const R Tt = wL * R(st.p(0, 2)) + wR * R(st.p(0, 3));
        R Rb = R(0), cvb = R(0), chi[NS];
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const R Y = aL * R(st.u(s, 2)) + aR * R(st.u(s, 3));
            Rb += Y * th.Rs[s];
            cvb += Y * cv_species(th, s, Tt);
            chi[s] = e_species(th, s, Tt);
        }
        const R Gam = Rb / cvb;
        const R q2 = ut[0] * ut[0] + ut[1] * ut[1] + ut[2] * ut[2];
        R c2 = Gam * (Ht - q2);
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const R Y = aL * R(st.u(s, 2)) + aR * R(st.u(s, 3));
            c2 += Y * (Gam * (R(0.5) * q2 - chi[s]) + th.Rs[s] * Tt);
        }
        ct = xsqrt(c2);
    }
};

// VJP of one face in one pass: the forward recomputed (Roe state, per-cell
// projection scalars, LLF speeds), then backwards through the
// back-projection, the reconstruction of each characteristic field (acoustic
// pair, tangential pair, species), the projections and the Roe state.  No
// per-species array is kept: the averaged Y_s, chi_s and the species thermo
// at T~ are recomputed where they are used, and each contribution to the
// cotangent of Y_s or chi_s is passed on at once (to the partial densities
// of the face's two cells, and to Gamma, |u|^2 and T~), so the live state is
// the per-cell scalars (u_n, DU, DF and their cotangents) and a few dozen
// scalars of the Roe state.  Fb(q) gives the face flux cotangent.
//
// Names: DU = dp(U_m)/c^2, DF = dp(F_m)/c^2 with dp(v) = sum_s chi_s v_s -
// Gamma u.v_m + Gamma v_E; XU = n.m - u_n rho, XF = n.F_m - u_n F_rho
// (acoustic rows l_-+ . v = DU/2 -+ c XU/(2 c^2), likewise for F).
template <int NS, typename R, int DIR, bool CU6, class St, class Bar, class Out>
XF_HD void face_vjp(St st, const ThermoK<R> &th, const Bar &Fb, const Out &out, const Dissip &ds) {
    constexpr int IM = NS;
    constexpr int IE = NS + 3;
    constexpr int KN = Axes<DIR>::n, K1 = Axes<DIR>::t1, K2 = Axes<DIR>::t2;
    constexpr int IN = NS + KN, I1 = NS + K1, I2 = NS + K2;

    // ================= forward: Roe state ===================================
    R ut[3], Ht, Tt, aL, aR, Gam, q2, c2, ct, ic2, cih, iGam, S1, Se, Rb, cvb;
    {
        R rL = R(0), rR = R(0);
#pragma unroll 1
        for (int s = 0; s < NS; ++s) {
            rL += R(st.u(s, 2));
            rR += R(st.u(s, 3));
        }
        const R sL = xsqrt(rL), sR = xsqrt(rR);
        const R wL = sL / (sL + sR), wR = R(1) - wL;
        aL = wL * R(st.p(3, 2));
        aR = wR * R(st.p(3, 3));
#pragma unroll
        for (int k = 0; k < 3; ++k) ut[k] = aL * R(st.u(IM + k, 2)) + aR * R(st.u(IM + k, 3));
        Ht = aL * (R(st.u(IE, 2)) + R(st.p(1, 2))) + aR * (R(st.u(IE, 3)) + R(st.p(1, 3)));
        Tt = wL * R(st.p(0, 2)) + wR * R(st.p(0, 3));
    }
    Rb = R(0);
    cvb = R(0);
    Se = R(0);
    S1 = R(0);
#pragma unroll 1
    for (int s = 0; s < NS; ++s) {
        const R Y = aL * R(st.u(s, 2)) + aR * R(st.u(s, 3));
        S1 += Y;
        Rb += Y * th.Rs[s];
        cvb += Y * cv_species(th, s, Tt);
        Se += Y * e_species(th, s, Tt);
    }
    Gam = Rb / cvb;
    q2 = ut[0] * ut[0] + ut[1] * ut[1] + ut[2] * ut[2];
    // c^2 = Gamma (H - q^2) + sum_s Y_s chi_s, the sum written with S1 = sum Y,
    // Se = sum Y e_s(T~), Rb = sum Y R_s
    c2 = Gam * (Ht - q2) + Gam * (R(0.5) * q2 * S1 - Se) + Tt * Rb;
    ct = xsqrt(c2);
    ic2 = R(1) / c2;
    cih = R(0.5) * ct * ic2;
    iGam = R(1) / Gam;
    const R utn = ut[KN];

    // ================= forward: per-cell projection scalars =================
    R un[6], DU[6], DF[6], rh[6];
    R aM = R(0), a0 = R(0), aP = R(0);
    {
        R sc[6];
#pragma unroll
        for (int m = 0; m < 6; ++m) {
            sc[m] = R(0);
            rh[m] = R(0);
        }
#pragma unroll 1
        for (int s = 0; s < NS; ++s) {
            const R chis = Gam * (R(0.5) * q2 - e_species(th, s, Tt)) + th.Rs[s] * Tt;
#pragma unroll
            for (int m = 0; m < 6; ++m) {
                const R r = R(st.u(s, m));
                sc[m] += chis * r;
                rh[m] += r;
            }
        }
#pragma unroll
        for (int m = 0; m < 6; ++m) {
            const R rinv = R(st.p(3, m)), pm = R(st.p(1, m)), cm = R(st.p(2, m));
            const R E = R(st.u(IE, m));
            const R unm = R(st.u(IN, m)) * rinv;
            const R um = ut[0] * R(st.u(IM, m)) + ut[1] * R(st.u(IM + 1, m)) + ut[2] * R(st.u(IM + 2, m));
            const R dpU = sc[m] - Gam * um + Gam * E;
            const R dpF = unm * sc[m] - Gam * (unm * um + pm * utn) + Gam * ((E + pm) * unm);
            un[m] = unm;
            DU[m] = dpU * ic2;
            DF[m] = dpF * ic2;
            aM = rmax(aM, rabs(unm - cm));
            a0 = rmax(a0, rabs(unm));
            aP = rmax(aP, rabs(unm + cm));
        }
    }
    if (ds.type == kViscRoe) {   // speeds of the Roe state, held fixed like the LLF ones
        aM = rabs(utn - ct);
        a0 = rabs(utn);
        aP = rabs(utn + ct);
    } else if (ds.type == kViscGlf) {
        aM = R(ds.glf[0]);
        a0 = R(ds.glf[1]);
        aP = R(ds.glf[2]);
    }

    XF_PHASE(st);
    // ================= back-projection cotangents known from Fb ============
    // F_s = Y_s A + h_s; F_m = u (A + gsum) + c n D + t1 h1 + t2 h2;
    // F_E = H A + u_n c D + u_t1 h1 + u_t2 h2 + sum_s (q2 - chi_s / Gam) h_s,
    // A = h_- + h_+, D = h_+ - h_-, gsum = sum_s h_s.
    const R FbE = R(Fb(IE));
    const R Fbm[3] = {R(Fb(IM)), R(Fb(IM + 1)), R(Fb(IM + 2))};
    const R gsum_b = ut[0] * Fbm[0] + ut[1] * Fbm[1] + ut[2] * Fbm[2];
    R Asum_b = gsum_b + Ht * FbE;
#pragma unroll 1
    for (int s = 0; s < NS; ++s) Asum_b += (aL * R(st.u(s, 2)) + aR * R(st.u(s, 3))) * R(Fb(s));
    const R Dif_b = ct * Fbm[KN] + utn * ct * FbE;
    R ut_b[3] = {R(0), R(0), R(0)};
    R ct_b = R(0), Ht_b = R(0), q2_b = R(0), iGam_b = R(0), cih_b = R(0), Gam_b = R(0), Tt_b = R(0);
    R aL_b = R(0), aR_b = R(0);
    R un_b[6], DU_b[6], DF_b[6];
#pragma unroll
    for (int m = 0; m < 6; ++m) {
        un_b[m] = R(0);
        DU_b[m] = R(0);
        DF_b[m] = R(0);
    }

    // ================= acoustic fields, one at a time =======================
    // The cotangents of each cell's normal momentum, pressure and density
    // go to the sink as they arise.
    R Asum = R(0), Dif = R(0);
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        XF_PHASE(st);
        const R sg = a == 0 ? R(-1) : R(1);
        const R al = a == 0 ? aM : aP;
        const R hb = Asum_b + sg * Dif_b;
        R gp[6], gm[6], wFb[6], wUb[6];
#pragma unroll
        for (int m = 0; m < 6; ++m) {
            const R mn = R(st.u(IN, m));
            const R XU = mn - utn * rh[m];
            const R XF = (mn * un[m] + R(st.p(1, m))) - utn * (rh[m] * un[m]);
            const R wU = R(0.5) * DU[m] + sg * cih * XU, wF = R(0.5) * DF[m] + sg * cih * XF;
            gp[m] = R(0.5) * (wF + al * wU);
            gm[m] = R(0.5) * (wF - al * wU);
        }
        const R h = CU6 ? split_cu6_fb(gp, gm, al, hb, wFb, wUb) : split_weno_fb(gp, gm, al, hb, wFb, wUb);
        Asum += h;
        Dif += sg * h;
        XF_PHASE(st);
#pragma unroll
        for (int m = 0; m < 6; ++m) {
            const R mn = R(st.u(IN, m));
            const R XU = mn - utn * rh[m];
            const R XF = (mn * un[m] + R(st.p(1, m))) - utn * (rh[m] * un[m]);
            DU_b[m] += R(0.5) * wUb[m];
            DF_b[m] += R(0.5) * wFb[m];
            const R XUb = sg * cih * wUb[m];
            const R XFb = sg * cih * wFb[m];
            cih_b += sg * (XU * wUb[m] + XF * wFb[m]);
            const R xb = XUb + un[m] * XFb;
            ut_b[KN] -= rh[m] * xb;
            un_b[m] += (mn - utn * rh[m]) * XFb;
            out.u(IN, m, double(xb));
            out.p(kSinkRho, m, double(-utn * xb));
            out.p(kSinkP, m, double(XFb));
        }
    }
    ct_b += Dif * Fbm[KN] + utn * Dif * FbE;
    ut_b[KN] += ct * Dif * FbE;
    Ht_b += Asum * FbE;

    // ================= tangential pair =====================================
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        XF_PHASE(st);
        const int I = a == 0 ? I1 : I2;
        const int K = a == 0 ? K1 : K2;
        const R uta = ut[K];
        const R hb = Fbm[K] + uta * FbE;
        R gp[6], gm[6], wU[6], wFb[6], wUb[6];
#pragma unroll
        for (int m = 0; m < 6; ++m) {
            wU[m] = R(st.u(I, m)) - uta * rh[m];
            gp[m] = R(0.5) * (un[m] * wU[m] + a0 * wU[m]);
            gm[m] = R(0.5) * (un[m] * wU[m] - a0 * wU[m]);
        }
        const R ha = CU6 ? split_cu6_fb(gp, gm, a0, hb, wFb, wUb) : split_weno_fb(gp, gm, a0, hb, wFb, wUb);
        ut_b[K] += ha * FbE;
#pragma unroll
        for (int m = 0; m < 6; ++m) {
            un_b[m] += wU[m] * wFb[m];
            const R wUt = wUb[m] + un[m] * wFb[m];
            out.u(I, m, double(wUt));
            ut_b[K] -= rh[m] * wUt;
            out.p(kSinkRho, m, double(-uta * wUt));
        }
    }

    // ================= species fields ======================================
    R gsum = R(0);
#pragma unroll 1
    for (int s = 0; s < NS; ++s) {
        XF_PHASE(st);
        const R r2s = R(st.u(s, 2)), r3s = R(st.u(s, 3));
        const R Ys = aL * r2s + aR * r3s;
        const R es = e_species(th, s, Tt);
        const R chis = Gam * (R(0.5) * q2 - es) + th.Rs[s] * Tt;
        const R Fbs = R(Fb(s));
        const R hsb = Fbs + gsum_b + (q2 - chis * iGam) * FbE;
        R gp[6], gm[6], wFb[6], wUb[6];
#pragma unroll
        for (int m = 0; m < 6; ++m) {
            const R r = R(st.u(s, m));
            const R wU = r - Ys * DU[m];
            const R wF = r * un[m] - Ys * DF[m];
            gp[m] = R(0.5) * (wF + a0 * wU);
            gm[m] = R(0.5) * (wF - a0 * wU);
        }
        const R hs = CU6 ? split_cu6_fb(gp, gm, a0, hsb, wFb, wUb) : split_weno_fb(gp, gm, a0, hsb, wFb, wUb);
        gsum += hs;
        q2_b += hs * FbE;
        iGam_b -= chis * hs * FbE;
        R ytb = Asum * Fbs;   // cotangent of Y_s from this field
#pragma unroll
        for (int m = 0; m < 6; ++m) {
            const R r = R(st.u(s, m));
            out.u(s, m, double(wUb[m] + un[m] * wFb[m]));
            un_b[m] += r * wFb[m];
            ytb -= DU[m] * wUb[m] + DF[m] * wFb[m];
            DU_b[m] -= Ys * wUb[m];
            DF_b[m] -= Ys * wFb[m];
        }
        // chi_s = Gamma (q^2/2 - e_s(T~)) + R_s T~, its cotangent -hs FbE / Gamma
        const R chb = -iGam * hs * FbE;
        Gam_b += (R(0.5) * q2 - es) * chb;
        q2_b += R(0.5) * Gam * chb;
        Tt_b += (th.Rs[s] - Gam * cv_species(th, s, Tt)) * chb;
        // Y_s = aL rho_s(2) + aR rho_s(3)
        out.u(s, 2, double(aL * ytb));
        out.u(s, 3, double(aR * ytb));
        aL_b += r2s * ytb;
        aR_b += r3s * ytb;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) ut_b[k] += (Asum + gsum) * Fbm[k];

    // ================= per-cell projections: DU = dpU / c^2, DF = dpF / c^2
    R ic2_b = R(0), scb[6];
#pragma unroll
    for (int m = 0; m < 6; ++m) {
        XF_PHASE(st);
        const R rinv = R(st.p(3, m)), pm = R(st.p(1, m));
        const R E = R(st.u(IE, m));
        const R M0 = R(st.u(IM, m)), M1 = R(st.u(IM + 1, m)), M2 = R(st.u(IM + 2, m));
        const R mn = R(st.u(IN, m));
        const R unm = un[m];
        const R um = ut[0] * M0 + ut[1] * M1 + ut[2] * M2;
        const R dpU = DU[m] * c2, dpF = DF[m] * c2;
        const R dpU_b = ic2 * DU_b[m], dpF_b = ic2 * DF_b[m];
        ic2_b += dpU * DU_b[m] + dpF * DF_b[m];
        const R sc_b = dpU_b + unm * dpF_b;
        scb[m] = sc_b;
        const R um_b = -Gam * sc_b;
        Gam_b += (E - um) * dpU_b + ((E + pm) * unm - unm * um - pm * utn) * dpF_b;
        const R un_bt = un_b[m] + (dpU + Gam * pm) * dpF_b;
        ut_b[KN] -= Gam * pm * dpF_b;
        ut_b[0] += M0 * um_b;
        ut_b[1] += M1 * um_b;
        ut_b[2] += M2 * um_b;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            R v = ut[k] * um_b;
            if (k == KN) v += rinv * un_bt;
            out.u(IM + k, m, double(v));
        }
        out.u(IE, m, double(Gam * sc_b));
        out.p(kSinkP, m, double(Gam * (unm - utn) * dpF_b));
        out.p(kSinkRho, m, double(-rinv * rinv * mn * un_bt));   // through 1/rho
    }
    // sc = sum_s chi_s rho_s of each cell
#pragma unroll 1
    for (int s = 0; s < NS; ++s) {
        XF_PHASE(st);
        const R es = e_species(th, s, Tt);
        const R chis = Gam * (R(0.5) * q2 - es) + th.Rs[s] * Tt;
        R chb = R(0);
#pragma unroll
        for (int m = 0; m < 6; ++m) {
            chb += R(st.u(s, m)) * scb[m];
            out.u(s, m, double(chis * scb[m]));
        }
        Gam_b += (R(0.5) * q2 - es) * chb;
        q2_b += R(0.5) * Gam * chb;
        Tt_b += (th.Rs[s] - Gam * cv_species(th, s, Tt)) * chb;
    }

    XF_PHASE(st);
    // ================= Roe state: c^2, Gamma, chi_s, thermo at T~, averages
    ct_b += R(0.5) * ic2 * cih_b;
    ic2_b += R(0.5) * ct * cih_b;
    const R c2_b = -ic2 * ic2 * ic2_b + ct_b / (R(2) * ct);
    Gam_b += (Ht - q2) * c2_b - iGam * iGam * iGam_b;
    Ht_b += Gam * c2_b;
    q2_b -= Gam * c2_b;
    // the cotangent Y_s c2_b of every chi_s, summed over s
    Gam_b += (R(0.5) * q2 * S1 - Se) * c2_b;
    q2_b += R(0.5) * Gam * S1 * c2_b;
    Tt_b += (Rb - Gam * cvb) * c2_b;
    // Gamma = Rb / cvb
    const R Rb_b = Gam_b / cvb;
    const R cvb_b = -Gam / cvb * Gam_b;
#pragma unroll 1
    for (int s = 0; s < NS; ++s) {
        XF_PHASE(st);
        const R r2s = R(st.u(s, 2)), r3s = R(st.u(s, 3));
        const R Ys = aL * r2s + aR * r3s;
        const R chis = Gam * (R(0.5) * q2 - e_species(th, s, Tt)) + th.Rs[s] * Tt;
        const R ytb = chis * c2_b + th.Rs[s] * Rb_b + cv_species(th, s, Tt) * cvb_b;
        Tt_b += Ys * dcv_species(th, s, Tt) * cvb_b;
        out.u(s, 2, double(aL * ytb));
        out.u(s, 3, double(aR * ytb));
        aL_b += r2s * ytb;
        aR_b += r3s * ytb;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) ut_b[k] += R(2) * ut[k] * q2_b;

    XF_PHASE(st);
    aL_b += (R(st.u(IE, 2)) + R(st.p(1, 2))) * Ht_b;
    aR_b += (R(st.u(IE, 3)) + R(st.p(1, 3))) * Ht_b;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        aL_b += R(st.u(IM + k, 2)) * ut_b[k];
        aR_b += R(st.u(IM + k, 3)) * ut_b[k];
        out.u(IM + k, 2, double(aL * ut_b[k]));
        out.u(IM + k, 3, double(aR * ut_b[k]));
    }
    out.u(IE, 2, double(aL * Ht_b));
    out.u(IE, 3, double(aR * Ht_b));
    out.p(kSinkP, 2, double(aL * Ht_b));
    out.p(kSinkP, 3, double(aR * Ht_b));
    // the sqrt(rho) weights, again from the two cells' densities
    R rL = R(0), rR = R(0);
#pragma unroll 1
    for (int s = 0; s < NS; ++s) {
        rL += R(st.u(s, 2));
        rR += R(st.u(s, 3));
    }
    const R sL = xsqrt(rL), sR = xsqrt(rR), Ssum = sL + sR;
    const R wL = sL / Ssum, wR = R(1) - wL;
    const R r2 = R(st.p(3, 2)), r3 = R(st.p(3, 3));
    out.p(kSinkT, 2, double(wL * Tt_b));
    out.p(kSinkT, 3, double(wR * Tt_b));
    // aL = wL / rho_L, aR = wR / rho_R, T~ = wL T_L + wR T_R
    R wL_b = R(st.p(0, 2)) * Tt_b + r2 * aL_b;
    const R wR_b = R(st.p(0, 3)) * Tt_b + r3 * aR_b;
    const R r2_b = wL * aL_b, r3_b = wR * aR_b;
    wL_b -= wR_b;
    const R iS2 = R(1) / (Ssum * Ssum);
    const R rL_b = wL_b * sR * iS2 / (R(2) * sL);
    const R rR_b = -wL_b * sL * iS2 / (R(2) * sR);
    out.p(kSinkRho, 2, double(rL_b - r2 * r2 * r2_b));
    out.p(kSinkRho, 3, double(rR_b - r3 * r3 * r3_b));
}

// Waves per SIMD the face VJP kernels are compiled for: the FP32 face keeps
// its state in 256 registers (two waves); the FP64 one needs up to 512 (one
// wave; at two it spills 744 bytes per lane).  At one wave per SIMD a block
// has its CU's LDS to itself, so the FP64 kernels first copy the stencil
// values of all their faces (U and the primitives) into LDS, and the face
// computation waits on no global load; the FP32 kernels, two blocks per CU,
// read the stencil through the caches.
template <typename R>
constexpr int vjp_waves() { return sizeof(R) == 4 ? 2 : 1; }
template <typename R>
constexpr bool vjp_staged() { return sizeof(R) == 8; }

// ---------------------------------------------------------------------------
// The face VJP runs as one kernel per launch group of faces.
//
// x direction: lanes take consecutive x faces, linearised over the rows of
// one z-plane (face f of the plane: row f / (nx + 1), face f % (nx + 1)).
// The padded rows of a plane are contiguous, so the cells the 64 faces of a
// wave touch form one run of at most W = 69 + 5 b padded cells (b = row
// boundaries the wave crosses; face k of the wave has its stencil at offset
// k + 5 b_k).  Each wave accumulates its cotangents in a private LDS window
// over that run: within one instruction the 64 lanes address 64 distinct
// cells, and the window accesses keep program order, so no atomics are
// needed.  The window is then added to Ubar / Pbar with coalesced
// read-modify-writes.  Runs of waves w and w + 1 can share up to five cells,
// those of w and w + 2 cannot; launch `grp` takes the waves w = grp mod 2.
// Staged (FP64): the wave first copies the run's U and primitives into a
// second private LDS area of (NV + 4) W values.
// ---------------------------------------------------------------------------
template <int NS, typename R, bool CU6>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(vjp_waves<R>()))) void k_face_vjp_x(
    const double *__restrict__ U, const double *__restrict__ P, const double *__restrict__ rbar,
    double *__restrict__ Ubar, double *__restrict__ Pbar, Geo g, ThermoK<R> th, int W, int grp, Dissip ds) {
    constexpr int NV = NS + 4;
    constexpr int NW = NV + kSinkExtra;                    // window rows
    constexpr int NT = vjp_staged<R>() ? NV + 4 : 0;       // staged rows
    extern __shared__ double xf_win[];
    const int wpb = blockDim.x >> 6, wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const long long rowf = (long long)g.nx + 1;          // faces per row
    const long long nfp = rowf * g.ny;                   // faces per plane
    const long long wpp = (nfp + 63) / 64;               // waves per plane
    const long long wid = kVjpGroups * ((long long)blockIdx.x * wpb + wv) + grp;
    const long long C = g.cells;
    const long long zb = (long long)(g.gz + blockIdx.y) * g.sz + (long long)g.gy * g.sy;   // plane's first row
    double *w = xf_win + (size_t)wv * (NW + NT) * W;
    double *tile = w + (size_t)NW * W;
    const long long f0 = wid * 64, f = f0 + lane;
    const long long r0 = f0 / rowf;
    const long long base0 = zb + r0 * g.sy + (f0 - r0 * rowf);   // stencil cell 0 of the wave's first face
    int span = 0;                                                 // cells of the wave's run
    if (wid < wpp) {
        const long long fl = min(f0 + 63, nfp - 1);
        const long long rl = fl / rowf;
        span = (int)(zb + rl * g.sy + (fl - rl * rowf) - base0) + 6;
    }
    for (int i = lane; i < NW * W; i += 64) w[i] = 0.0;
    if constexpr (NT > 0) {
        for (int c = lane; c < span; c += 64) {
#pragma unroll
            for (int q = 0; q < NV; ++q) tile[q * W + c] = U[q * C + base0 + c];
#pragma unroll
            for (int k = 0; k < 4; ++k) tile[(NV + k) * W + c] = P[k * C + base0 + c];
        }
    }
    __syncthreads();
    if (wid < wpp && f < nfp) {
        const long long r = f / rowf;
        const int i = (int)(f - r * rowf);
        const long long row = zb + r * g.sy + g.gx;             // interior cell 0 of the row
        const FaceBar fb{rbar, C, row + i, row + i - 1, i < g.nx, i > 0, g.idx};
        bool any = false;
#pragma unroll
        for (int q = 0; q < NV; ++q) any = any || (fb(q) != 0.0);
        if (any) {
            const long long base = row + i - 3;
            SinkLds sk{(volatile lds_double *)w, W, (int)(base - base0), 1, NV * W};
            if constexpr (NT > 0) {
                const StencilLds<NV> st{(const lds_double *)tile, (int)(base - base0), 1, W};
                face_vjp<NS, R, 0, CU6>(st, th, fb, sk, ds);
            } else {
                const Stencil st{U, P, base, 1, C};
                face_vjp<NS, R, 0, CU6>(st, th, fb, sk, ds);
            }
        }
    }
    __syncthreads();
    for (int c = lane; c < span; c += 64) {
#pragma unroll
        for (int q = 0; q < NV; ++q) Ubar[q * C + base0 + c] += w[q * W + c];
#pragma unroll
        for (int k = 0; k < kSinkExtra; ++k) Pbar[k * C + base0 + c] += w[(NV + k) * W + c];
    }
}

// LDS bytes per wave of k_face_vjp_x for a run of W cells.
template <int NS, typename R>
constexpr size_t vjp_x_lds_per_wave(int W) {
    return (size_t)(NS + 4 + kSinkExtra + (vjp_staged<R>() ? NS + 8 : 0)) * W * sizeof(double);
}

// ---------------------------------------------------------------------------
// y and z directions, blocked: a block of WY waves takes 16 x-columns by
// F = 4 WY consecutive faces j0..j0+F-1 of the sweep axis (j0 = F b) in one
// plane of the third axis; wave w of the block takes faces j0+4w..j0+4w+3
// (lane = 16 ts + tx), so each stencil load of a wave reads four whole
// 128-byte rows.  Wave w accumulates in a private LDS window of sweep rows
// j0+4w-3..j0+4w+5 (within one instruction its lanes address distinct
// cells); the block then adds, for each of its (F + 5) x 16 cells, the
// windows that cover it in wave order to Ubar / Pbar (one coalesced
// read-modify-write per cell and field).  Blocks b and b + 1 share five
// rows, blocks b and b + 2 none: launch `phase` takes the blocks
// b = phase mod 2.  Staged (FP64): the block first copies the U and
// primitives of its (F + 5) x 16 cells into LDS.
// ---------------------------------------------------------------------------
constexpr int kVjpTX = 16, kVjpWin = kVjpTX * 9;
// Waves per y/z block (four faces each): two in FP64, so that two blocks of
// 65 KB share a CU and one block's staging and window merge overlap the
// other's faces (RHS VJP at 256^3, nine species, 45.6 -> 44.8 ms against
// four-wave blocks of 119 KB, one per CU); four in FP32, whose blocks hold
// no staged tile (there two-wave blocks measured 35.3 -> 36.2 ms).  Blocks
// of at least five faces keep next-but-one neighbours disjoint (two launch
// groups).
template <typename R>
constexpr int vjp_yz_waves() { return sizeof(R) == 8 ? 2 : 4; }
template <typename R>
constexpr int vjp_yz_faces() { return 4 * vjp_yz_waves<R>(); }
static_assert(vjp_yz_faces<double>() >= 5 && vjp_yz_faces<float>() >= 5, "windows of blocks b and b + 2 must not meet");

template <int NS, typename R, int DIR, bool CU6>
__global__ __launch_bounds__(64 * vjp_yz_waves<R>()) __attribute__((amdgpu_waves_per_eu(vjp_waves<R>()))) void k_face_vjp_yz(
    const double *__restrict__ U, const double *__restrict__ P, const double *__restrict__ rbar,
    double *__restrict__ Ubar, double *__restrict__ Pbar, Geo g, ThermoK<R> th, int phase, Dissip ds) {
    constexpr int NV = NS + 4;
    constexpr int NW = NV + kSinkExtra;                    // window rows
    constexpr int NT = vjp_staged<R>() ? NV + 4 : 0;       // staged rows
    constexpr int WY = vjp_yz_waves<R>(), kVjpFB = vjp_yz_faces<R>(), kVjpRows = kVjpFB + 5;
    constexpr int TS = kVjpRows * kVjpTX;                  // staged cells
    __shared__ double xf_wyz[WY][NW * kVjpWin];
    __shared__ double xf_tile[NT > 0 ? NT * TS : 1];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int tx = lane & (kVjpTX - 1), ts = lane / kVjpTX;
    const int nsw = DIR == 1 ? g.ny : g.nz;
    const long long ss = DIR == 1 ? g.sy : g.sz;
    const int gs = DIR == 1 ? g.gy : g.gz;
    const int xt = (g.nx + kVjpTX - 1) / kVjpTX;                   // x tiles
    const int xi = blockIdx.x % xt;
    const int b = phase + kVjpGroups * (int)(blockIdx.x / xt);     // this block's face block
    const int tr = blockIdx.y;                                     // plane of the third axis
    const int j0 = b * kVjpFB;
    const int x = xi * kVjpTX + tx;
    const int j = j0 + 4 * wv + ts;
    const long long C = g.cells;
    // padded index of the cell at x = x0 + tx, interior sweep index 0, in this plane
    const long long col0 = (long long)g.gx + (DIR == 1 ? (long long)(g.gz + tr) * g.sz : (long long)(g.gy + tr) * g.sy) +
                           (long long)gs * ss;
    volatile double *w = xf_wyz[wv];
    for (int i = lane; i < NW * kVjpWin; i += 64) w[i] = 0.0;
    if constexpr (NT > 0) {
        // tile row r = sweep row j0 - 3 + r; cells past the padded extent are never read
        for (int e = threadIdx.x; e < TS; e += 64 * WY) {
            const int r = e / kVjpTX, cx = xi * kVjpTX + (e % kVjpTX);
            if (cx >= g.nx || j0 - 3 + r > nsw + 2) continue;
            const long long cell = col0 + cx + (long long)(j0 - 3 + r) * ss;
#pragma unroll
            for (int q = 0; q < NV; ++q) xf_tile[q * TS + e] = U[q * C + cell];
#pragma unroll
            for (int k = 0; k < 4; ++k) xf_tile[(NV + k) * TS + e] = P[k * C + cell];
        }
    }
    __syncthreads();
    if (x < g.nx && j <= nsw) {
        const long long col = col0 + x;
        const FaceBar fb{rbar, C, col + (long long)j * ss, col + (long long)(j - 1) * ss, j < nsw, j > 0,
                         DIR == 1 ? g.idy : g.idz};
        bool any = false;
#pragma unroll
        for (int q = 0; q < NV; ++q) any = any || (fb(q) != 0.0);
        if (any) {
            // window row r of wave w = sweep row j0 + 4w - 3 + r; stencil cell m is row ts + m
            SinkLds sk{(volatile lds_double *)xf_wyz[wv], kVjpWin, ts * kVjpTX + tx, kVjpTX, NV * kVjpWin};
            if constexpr (NT > 0) {
                // stencil cell m of face j is tile row j - j0 + m
                const StencilLds<NV> st{(const lds_double *)xf_tile, (4 * wv + ts) * kVjpTX + tx, kVjpTX, TS};
                face_vjp<NS, R, DIR, CU6>(st, th, fb, sk, ds);
            } else {
                const Stencil st{U, P, col + (long long)(j - 3) * ss, ss, C};
                face_vjp<NS, R, DIR, CU6>(st, th, fb, sk, ds);
            }
        }
    }
    __syncthreads();
    // block rows r = 0..20 (sweep rows j0-3 .. j0+17); wave w covers r in [4w, 4w+9)
    for (int c = threadIdx.x; c < kVjpTX * kVjpRows; c += 64 * WY) {
        const int r = c / kVjpTX, cx = xi * kVjpTX + (c % kVjpTX);
        const int row = j0 - 3 + r;                       // interior index along the sweep axis
        if (cx >= g.nx || row > nsw + 2) continue;
        const int wlo = r >= 8 ? (r - 8 + 3) / 4 : 0, whi = min(WY - 1, r / 4);
        const long long cell = col0 + cx + (long long)row * ss;
#pragma unroll
        for (int q = 0; q < NW; ++q) {
            double v = 0.0;
            for (int ww = wlo; ww <= whi; ++ww) v += xf_wyz[ww][q * kVjpWin + (r - 4 * ww) * kVjpTX + (c % kVjpTX)];
            if (q < NV)
                Ubar[q * C + cell] += v;
            else
                Pbar[(q - NV) * C + cell] += v;
        }
    }
}

// ---------------------------------------------------------------------------
// The dissipation speeds of every face of one direction, in FP64, as the
// context's scheme takes them (LLF: the stencil maxima of |u_n - c|, |u_n|,
// |u_n + c| over the 2 RAD cells; ROE: those of the face's Roe state; GLF:
// the direction's three reduced speeds), written to alpha[k * astride + f]
// with the face index f of the frozen-speed sweeps (x: i + (nx+1)(j + ny k),
// y: i + nx (j + (ny+1) k), z: i + nx (j + ny k)).  These are the speeds the
// VJP holds fixed.
// ---------------------------------------------------------------------------
template <int NS, int DIR, int RAD>
__global__ __launch_bounds__(256) void k_face_speeds(const double *__restrict__ U, const double *__restrict__ P, Geo g,
                                                     ThermoK<double> th, int type, const double *__restrict__ glf,
                                                     double *__restrict__ alpha, long long astride) {
    const long long f = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const int ex = g.nx + (DIR == 0), ey = g.ny + (DIR == 1);
    if (f >= astride) return;
    const int i = (int)(f % ex);
    const long long r = f / ex;
    const int j = (int)(r % ey), k = (int)(r / ey);
    const long long step = DIR == 0 ? 1 : DIR == 1 ? g.sy : g.sz;
    // left cell of the face: one back along the sweep axis
    const long long left = (long long)(g.gz + k) * g.sz + (long long)(g.gy + j) * g.sy + (g.gx + i) - step;
    double aM = 0.0, a0 = 0.0, aP = 0.0;
    if (type == kViscGlf) {
        aM = glf[0];
        a0 = glf[1];
        aP = glf[2];
    } else if (type == kViscRoe) {
        const Stencil st{U, P, left - 2 * step, step, g.cells};
        const RoeFwd<NS, double> rf(st, th);
        const double un = rf.ut[DIR];
        aM = fabs(un - rf.ct);
        a0 = fabs(un);
        aP = fabs(un + rf.ct);
    } else {
        for (int m = 1 - RAD; m <= RAD; ++m) {
            const long long q = left + m * step;
            const double un = U[(NS + DIR) * g.cells + q] * P[3 * g.cells + q], c = P[2 * g.cells + q];
            aM = fmax(aM, fabs(un - c));
            a0 = fmax(a0, fabs(un));
            aP = fmax(aP, fabs(un + c));
        }
    }
    alpha[f] = aM;
    alpha[astride + f] = a0;
    alpha[2 * astride + f] = aP;
}

// Per-cell backward of (p, T, rho)(U): p = T sum_s rho_s R_s, rho = sum_s
// rho_s, and T from rho e(T) = E - |m|^2 / (2 rho) by the implicit-function
// rule
//   dT = (dE - u.dm + |u|^2/2 sum_s drho_s - sum_s e_s(T) drho_s) / (rho C_v).
// u: the cell's conservative values (stride `stride`), T and 1/rho from the
// primitive pass, (pb, Tb, rb) the cotangents of p, T and rho; adds into ub.
template <int NS>
XF_HD void prims_vjp_cell(const ThermoK<double> &th, const double *u, long long stride, double T, double rinv,
                          double pb, double Tb, double rb, double *ub) {
    double rR = 0.0, cv = 0.0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const double r = u[s * stride];
        rR += r * th.Rs[s];
        cv += r * cv_species(th, s, T);
    }
    cv *= rinv;   // mixture C_v = sum_s Y_s C_v,s
    const double vx = u[NS * stride] * rinv, vy = u[(NS + 1) * stride] * rinv, vz = u[(NS + 2) * stride] * rinv;
    const double gT = (Tb + pb * rR) * rinv / cv;
    const double k2 = 0.5 * (vx * vx + vy * vy + vz * vz);
#pragma unroll
    for (int s = 0; s < NS; ++s) ub[s * stride] += rb + pb * T * th.Rs[s] + gT * (k2 - e_species(th, s, T));
    ub[NS * stride] -= gT * vx;
    ub[(NS + 1) * stride] -= gT * vy;
    ub[(NS + 2) * stride] -= gT * vz;
    ub[(NS + 3) * stride] += gT;
}

template <int NS>
__global__ __launch_bounds__(256) void k_prims_vjp(const double *__restrict__ U, const double *__restrict__ P,
                                                   const double *__restrict__ Pbar, double *__restrict__ Ubar,
                                                   Geo g, ThermoK<double> th) {
    const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= g.cells) return;
    const long long C = g.cells;
    const double pb = Pbar[idx], Tb = Pbar[C + idx], rb = Pbar[2 * C + idx];
    if (pb == 0.0 && Tb == 0.0 && rb == 0.0) return;
    prims_vjp_cell<NS>(th, U + idx, C, P[idx], P[3 * C + idx], pb, Tb, rb, Ubar + idx);
}

}  // namespace xf
