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

// Where the cotangents of one stencil go: FP64 padded buffers, added to.
struct Sink {
    double *__restrict__ Ub;   // [Nv][cells]
    double *__restrict__ Pb;   // [2][cells]: cotangent of p, of T
    long long base, step, cells;
    XF_HD void u(int f, int m, double v) const { Ub[f * cells + base + m * step] += v; }
    XF_HD void p(int k, int m, double v) const { Pb[k * cells + base + m * step] += v; }
};

// Where the cotangents of one stencil go, variant 2: a wave's private LDS
// window of the padded cells its faces touch ([NV + 2][W], field-major;
// stencil cell 0 of this thread's face at window index off).  Lanes of a wave
// share window cells through different (field, cell) calls, so the
// read-modify-writes must stay in program order even where one thread's
// addresses differ: the accesses are volatile (LDS executes a wave's
// instructions in order).  The pointer carries the LDS address space, so no
// generic-address checks are generated.
typedef __attribute__((address_space(3))) double lds_double;   // a pointer known to be LDS
struct SinkLds {
    volatile lds_double *w;
    int W, off, mstep, pofs;   // window length, offset of stencil cell 0, cell stride, start of the P rows
    XF_HD void u(int f, int m, double v) const { w[f * W + off + m * mstep] += v; }
    XF_HD void p(int k, int m, double v) const { w[pofs + k * W + off + m * mstep] += v; }
};

// Forward Roe state of one face (shared by both halves of the face VJP).
template <int NS, typename R>
struct RoeFwd {
    R sL, sR, Ssum, wL, wR, r2, r3, aL, aR, ut[3], Ht, Tt, Yt[NS], chi[NS], cvb, Gam, q2, c2, ct, ic2, cih, iGam;
    XF_HD RoeFwd(const Stencil &st, const ThermoK<R> &th) {
        constexpr int IM = NS;
        constexpr int IE = NS + 3;
        R rL = R(0), rR = R(0);
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            rL += R(st.u(s, 2));
            rR += R(st.u(s, 3));
        }
        sL = xsqrt(rL);
        sR = xsqrt(rR);
        Ssum = sL + sR;
        wL = sL / Ssum;
        wR = R(1) - wL;
        r2 = R(st.p(3, 2));
        r3 = R(st.p(3, 3));
        aL = wL * r2;
        aR = wR * r3;
#pragma unroll
        for (int k = 0; k < 3; ++k) ut[k] = aL * R(st.u(IM + k, 2)) + aR * R(st.u(IM + k, 3));
        Ht = aL * (R(st.u(IE, 2)) + R(st.p(1, 2))) + aR * (R(st.u(IE, 3)) + R(st.p(1, 3)));
        Tt = wL * R(st.p(0, 2)) + wR * R(st.p(0, 3));
        R Rb = R(0);
        cvb = R(0);
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            Yt[s] = aL * R(st.u(s, 2)) + aR * R(st.u(s, 3));
            Rb += Yt[s] * th.Rs[s];
            cvb += Yt[s] * cv_species(th, s, Tt);
            chi[s] = e_species(th, s, Tt);
        }
        Gam = Rb / cvb;
        q2 = ut[0] * ut[0] + ut[1] * ut[1] + ut[2] * ut[2];
        c2 = Gam * (Ht - q2);
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            chi[s] = Gam * (R(0.5) * q2 - chi[s]) + th.Rs[s] * Tt;
            c2 += Yt[s] * chi[s];
        }
        ct = xsqrt(c2);
        ic2 = R(1) / c2;
        cih = R(0.5) * ct * ic2;
        iGam = R(1) / Gam;
    }
};

// Record passed from the first half of the face VJP to the second: the
// per-cell cotangents of DU, DF, u_n, rho, p, m_n (6 each), those of the Roe
// Y_s and chi_s, of u~ and of c~, H~, q~^2, 1/Gamma, c~/(2 c~^2).
template <int NS>
struct VjpRec {
    static constexpr int N = 44 + 2 * NS;
    static constexpr int DUb = 0, DFb = 6, unb = 12, rhb = 18, pmb = 24, Mnb = 30, Ytb = 36, chib = 36 + NS,
                         utb = 36 + 2 * NS, ctb = utb + 3, Htb = ctb + 1, q2b = ctb + 2, iGamb = ctb + 3,
                         cihb = ctb + 4;
    double *__restrict__ r;
    long long stride, idx;
    XF_HD void put(int k, double v) const { r[k * stride + idx] = v; }
    XF_HD double get(int k) const { return r[k * stride + idx]; }
};

#define XF_ROE_UNPACK(rf)                                                                                   \
    const R sL = rf.sL, sR = rf.sR, Ssum = rf.Ssum, wL = rf.wL, wR = rf.wR, r2 = rf.r2, r3 = rf.r3,        \
            aL = rf.aL, aR = rf.aR, Ht = rf.Ht, Tt = rf.Tt, cvb = rf.cvb, Gam = rf.Gam, q2 = rf.q2,        \
            c2 = rf.c2, ct = rf.ct, ic2 = rf.ic2, cih = rf.cih, iGam = rf.iGam;                            \
    const R *ut = rf.ut, *Yt = rf.Yt, *chi = rf.chi;                                                       \
    (void)sL; (void)sR; (void)Ssum; (void)wL; (void)wR; (void)r2; (void)r3; (void)aL; (void)aR; (void)Ht; \
    (void)Tt; (void)cvb; (void)c2; (void)ct; (void)cih; (void)iGam

// First half: forward recompute, then the backward through the back-projection,
// the WENO5 reconstructions and the characteristic projections' dependence on
// each cell's own values; writes the direct cell cotangents to `out` and the
// accumulated ones to `rec`.
template <int NS, typename R, int DIR, bool CU6 = false, class Out>
XF_HD void face_vjp_a(const Stencil &st, const ThermoK<R> &th, const R *Fb, const Out &out, const VjpRec<NS> &rec,
                      const Dissip &ds) {
    constexpr int IM = NS;
    constexpr int IE = NS + 3;
    constexpr int KN = Axes<DIR>::n, K1 = Axes<DIR>::t1, K2 = Axes<DIR>::t2;
    constexpr int IN = NS + KN, I1 = NS + K1, I2 = NS + K2;

    // ================= forward: Roe state and per-cell scalars =================
    constexpr bool cu6 = CU6;   // WENO-CU6 reconstruction (else WENO5)
    const RoeFwd<NS, R> rf(st, th);
    XF_ROE_UNPACK(rf);
    const R utn = ut[KN], ut1 = ut[K1], ut2 = ut[K2];

    R un[6], DU[6], DF[6], rh[6];
    R aM = R(0), a0 = R(0), aP = R(0);
#pragma unroll
    for (int m = 0; m < 6; ++m) {
        R sc = R(0), sr = R(0);
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const R r = R(st.u(s, m));
            sc += chi[s] * r;
            sr += r;
        }
        const R rinv = R(st.p(3, m)), pm = R(st.p(1, m)), cm = R(st.p(2, m));
        const R E = R(st.u(IE, m));
        const R unm = R(st.u(IN, m)) * rinv;
        const R um = ut[0] * R(st.u(IM, m)) + ut[1] * R(st.u(IM + 1, m)) + ut[2] * R(st.u(IM + 2, m));
        const R dpU = sc - Gam * um + Gam * E;
        const R dpF = unm * sc - Gam * (unm * um + pm * utn) + Gam * ((E + pm) * unm);
        un[m] = unm;
        DU[m] = dpU * ic2;
        DF[m] = dpF * ic2;
        rh[m] = sr;
        aM = rmax(aM, rabs(unm - cm));
        a0 = rmax(a0, rabs(unm));
        aP = rmax(aP, rabs(unm + cm));
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

    XF_FENCE();
    // ================= back-projection cotangents known from Fb ============
    // F_s = Y_s A + h_s; F_m = u (A + gsum) + c n D + t1 h1 + t2 h2;
    // F_E = H A + u_n c D + u_t1 h1 + u_t2 h2 + sum_s (q2 - chi_s / Gam) h_s,
    // A = h_- + h_+, D = h_+ - h_-, gsum = sum_s h_s.
    const R FbE = Fb[IE];
    const R Fbm[3] = {Fb[IM], Fb[IM + 1], Fb[IM + 2]};
    const R gsum_b = ut[0] * Fbm[0] + ut[1] * Fbm[1] + ut[2] * Fbm[2];
    R Asum_b = gsum_b + Ht * FbE;
#pragma unroll
    for (int s = 0; s < NS; ++s) Asum_b += Yt[s] * Fb[s];
    const R Dif_b = ct * Fbm[KN] + utn * ct * FbE;
    R ut_b[3] = {R(0), R(0), R(0)};
    R ct_b = R(0), Ht_b = R(0), q2_b = R(0), iGam_b = R(0), cih_b = R(0);
    R Yt_b[NS], chi_b[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        Yt_b[s] = R(0);
        chi_b[s] = R(0);
    }
    R un_b[6], DU_b[6], DF_b[6], rh_b[6], pm_b[6], Mn_b[6];
#pragma unroll
    for (int m = 0; m < 6; ++m) {
        un_b[m] = R(0);
        DU_b[m] = R(0);
        DF_b[m] = R(0);
        rh_b[m] = R(0);
        pm_b[m] = R(0);
        Mn_b[m] = R(0);
    }

    XF_FENCE();
    // ================= acoustic pair: forward value and backward ===========
    R Asum, Dif;
    {
        R gMp[6], gMm[6], gPp[6], gPm[6];
#pragma unroll
        for (int m = 0; m < 6; ++m) {
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
        R wFmb[6], wUmb[6], wFpb[6], wUpb[6];
        const R hm = cu6 ? split_cu6_fb(gMp, gMm, aM, Asum_b - Dif_b, wFmb, wUmb)
                         : split_weno_fb(gMp, gMm, aM, Asum_b - Dif_b, wFmb, wUmb);
        const R hp = cu6 ? split_cu6_fb(gPp, gPm, aP, Asum_b + Dif_b, wFpb, wUpb)
                         : split_weno_fb(gPp, gPm, aP, Asum_b + Dif_b, wFpb, wUpb);
        Asum = hm + hp;
        Dif = hp - hm;
#pragma unroll
        for (int m = 0; m < 6; ++m) {
            const R mn = R(st.u(IN, m));
            const R XU = mn - utn * rh[m];
            const R XF = (mn * un[m] + R(st.p(1, m))) - utn * (rh[m] * un[m]);
            DU_b[m] += R(0.5) * (wUmb[m] + wUpb[m]);
            DF_b[m] += R(0.5) * (wFmb[m] + wFpb[m]);
            const R XUb = cih * (wUpb[m] - wUmb[m]);
            const R XFb = cih * (wFpb[m] - wFmb[m]);
            cih_b += XU * (wUpb[m] - wUmb[m]) + XF * (wFpb[m] - wFmb[m]);
            Mn_b[m] += XUb + un[m] * XFb;
            ut_b[KN] -= rh[m] * XUb + rh[m] * un[m] * XFb;
            rh_b[m] -= utn * XUb + utn * un[m] * XFb;
            un_b[m] += (mn - utn * rh[m]) * XFb;
            pm_b[m] += XFb;
        }
    }
    ct_b += Dif * Fbm[KN] + utn * Dif * FbE;
    ut_b[KN] += ct * Dif * FbE;
    Ht_b += Asum * FbE;

    // ================= tangential pair =====================================
#pragma unroll
    for (int a = 0; a < 2; ++a) {
        XF_FENCE();
        const int I = a == 0 ? I1 : I2;
        const int K = a == 0 ? K1 : K2;
        const R uta = a == 0 ? ut1 : ut2;
        const R hb = Fbm[K] + uta * FbE;
        R gp[6], gm[6], wU[6], wFb[6], wUb[6];
#pragma unroll
        for (int m = 0; m < 6; ++m) {
            wU[m] = R(st.u(I, m)) - uta * rh[m];
            gp[m] = R(0.5) * (un[m] * wU[m] + a0 * wU[m]);
            gm[m] = R(0.5) * (un[m] * wU[m] - a0 * wU[m]);
        }
        const R ha = cu6 ? split_cu6_fb(gp, gm, a0, hb, wFb, wUb) : split_weno_fb(gp, gm, a0, hb, wFb, wUb);
        ut_b[K] += ha * FbE;
#pragma unroll
        for (int m = 0; m < 6; ++m) {
            un_b[m] += wU[m] * wFb[m];
            const R wUt = wUb[m] + un[m] * wFb[m];
            out.u(I, m, double(wUt));
            ut_b[K] -= rh[m] * wUt;
            rh_b[m] -= uta * wUt;
        }
    }

    // ================= species fields ======================================
    R gsum = R(0);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        XF_FENCE();
        const R hsb = Fb[s] + gsum_b + (q2 - chi[s] * iGam) * FbE;
        R gp[6], gm[6], wFb[6], wUb[6];
#pragma unroll
        for (int m = 0; m < 6; ++m) {
            const R r = R(st.u(s, m));
            const R wU = r - Yt[s] * DU[m];
            const R wF = r * un[m] - Yt[s] * DF[m];
            gp[m] = R(0.5) * (wF + a0 * wU);
            gm[m] = R(0.5) * (wF - a0 * wU);
        }
        const R hs = cu6 ? split_cu6_fb(gp, gm, a0, hsb, wFb, wUb) : split_weno_fb(gp, gm, a0, hsb, wFb, wUb);
        gsum += hs;
        Yt_b[s] += Asum * Fb[s];
        q2_b += hs * FbE;
        chi_b[s] -= iGam * hs * FbE;
        iGam_b -= chi[s] * hs * FbE;
#pragma unroll
        for (int m = 0; m < 6; ++m) {
            const R r = R(st.u(s, m));
            out.u(s, m, double(wUb[m] + un[m] * wFb[m]));
            un_b[m] += r * wFb[m];
            Yt_b[s] -= DU[m] * wUb[m] + DF[m] * wFb[m];
            DU_b[m] -= Yt[s] * wUb[m];
            DF_b[m] -= Yt[s] * wFb[m];
        }
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) ut_b[k] += (Asum + gsum) * Fbm[k];

    using Rc = VjpRec<NS>;
#pragma unroll
    for (int m = 0; m < 6; ++m) {
        rec.put(Rc::DUb + m, double(DU_b[m]));
        rec.put(Rc::DFb + m, double(DF_b[m]));
        rec.put(Rc::unb + m, double(un_b[m]));
        rec.put(Rc::rhb + m, double(rh_b[m]));
        rec.put(Rc::pmb + m, double(pm_b[m]));
        rec.put(Rc::Mnb + m, double(Mn_b[m]));
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        rec.put(Rc::Ytb + s, double(Yt_b[s]));
        rec.put(Rc::chib + s, double(chi_b[s]));
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) rec.put(Rc::utb + k, double(ut_b[k]));
    rec.put(Rc::ctb, double(ct_b));
    rec.put(Rc::Htb, double(Ht_b));
    rec.put(Rc::q2b, double(q2_b));
    rec.put(Rc::iGamb, double(iGam_b));
    rec.put(Rc::cihb, double(cih_b));
}

// Second half: forward Roe state again, the record, then the backward through
// the per-cell projection scalars DU, DF, the Roe state (c~^2, Gamma~, chi_s
// and the species thermo at T~), the sqrt(rho) averages and their weights.
template <int NS, typename R, int DIR, class Out>
XF_HD void face_vjp_b(const Stencil &st, const ThermoK<R> &th, const Out &out, const VjpRec<NS> &rec) {
    constexpr int IM = NS;
    constexpr int IE = NS + 3;
    constexpr int KN = Axes<DIR>::n;
    constexpr int IN = NS + KN;
    using Rc = VjpRec<NS>;
    const RoeFwd<NS, R> rf(st, th);
    XF_ROE_UNPACK(rf);
    const R utn = ut[KN];
    R ut_b[3], Yt_b[NS], chi_b[NS];
#pragma unroll
    for (int k = 0; k < 3; ++k) ut_b[k] = R(rec.get(Rc::utb + k));
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        Yt_b[s] = R(rec.get(Rc::Ytb + s));
        chi_b[s] = R(rec.get(Rc::chib + s));
    }
    R ct_b = R(rec.get(Rc::ctb)), Ht_b = R(rec.get(Rc::Htb)), q2_b = R(rec.get(Rc::q2b));
    const R iGam_b = R(rec.get(Rc::iGamb)), cih_b = R(rec.get(Rc::cihb));

    // ================= per-cell projections: DU = dpU / c^2, DF = dpF / c^2
    R Gam_b = R(0), ic2_b = R(0);
#pragma unroll
    for (int m = 0; m < 6; ++m) {
        XF_FENCE();
        R sc = R(0);
#pragma unroll
        for (int s = 0; s < NS; ++s) sc += chi[s] * R(st.u(s, m));
        const R rinv = R(st.p(3, m)), pm = R(st.p(1, m));
        const R E = R(st.u(IE, m));
        const R M0 = R(st.u(IM, m)), M1 = R(st.u(IM + 1, m)), M2 = R(st.u(IM + 2, m));
        const R mn = R(st.u(IN, m));
        const R unm = mn * rinv;
        const R DUb = R(rec.get(Rc::DUb + m)), DFb = R(rec.get(Rc::DFb + m));
        const R um = ut[0] * M0 + ut[1] * M1 + ut[2] * M2;
        const R dpU = sc - Gam * um + Gam * E;
        const R dpF = unm * sc - Gam * (unm * um + pm * utn) + Gam * ((E + pm) * unm);
        const R dpU_b = ic2 * DUb, dpF_b = ic2 * DFb;
        ic2_b += dpU * DUb + dpF * DFb;
        const R sc_b = dpU_b + unm * dpF_b;
        const R um_b = -Gam * (dpU_b + unm * dpF_b);
        const R E_b = Gam * (dpU_b + unm * dpF_b);
        Gam_b += (E - um) * dpU_b + ((E + pm) * unm - unm * um - pm * utn) * dpF_b;
        const R un_bt = R(rec.get(Rc::unb + m)) + (sc - Gam * um + Gam * (E + pm)) * dpF_b;
        const R pm_bt = R(rec.get(Rc::pmb + m)) + Gam * (unm - utn) * dpF_b;
        ut_b[KN] -= Gam * pm * dpF_b;
        ut_b[0] += M0 * um_b;
        ut_b[1] += M1 * um_b;
        ut_b[2] += M2 * um_b;
        const R rinv_b = mn * un_bt;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            R v = ut[k] * um_b;
            if (k == KN) v += R(rec.get(Rc::Mnb + m)) + rinv * un_bt;
            out.u(IM + k, m, double(v));
        }
        const R sp = R(rec.get(Rc::rhb + m)) - rinv * rinv * rinv_b;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            chi_b[s] += R(st.u(s, m)) * sc_b;
            out.u(s, m, double(chi[s] * sc_b + sp));
        }
        out.u(IE, m, double(E_b));
        out.p(0, m, double(pm_bt));
    }

    XF_FENCE();
    // ================= Roe state: c^2, Gamma, chi_s, thermo at T~, averages
    ct_b += R(0.5) * ic2 * cih_b;
    ic2_b += R(0.5) * ct * cih_b;
    const R c2_b = -ic2 * ic2 * ic2_b + ct_b / (R(2) * ct);
    Gam_b += (Ht - q2) * c2_b - iGam * iGam * iGam_b;
    Ht_b += Gam * c2_b;
    q2_b -= Gam * c2_b;
    R Tt_b = R(0);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        Yt_b[s] += chi[s] * c2_b;
        chi_b[s] += Yt[s] * c2_b;
        const R es = e_species(th, s, Tt);
        Gam_b += (R(0.5) * q2 - es) * chi_b[s];
        q2_b += R(0.5) * Gam * chi_b[s];
        Tt_b += th.Rs[s] * chi_b[s] - cv_species(th, s, Tt) * Gam * chi_b[s];
    }
    const R Rb_b = Gam_b / cvb;
    const R cvb_b = -Gam / cvb * Gam_b;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        Yt_b[s] += th.Rs[s] * Rb_b + cv_species(th, s, Tt) * cvb_b;
        Tt_b += Yt[s] * dcv_species(th, s, Tt) * cvb_b;
    }
#pragma unroll
    for (int k = 0; k < 3; ++k) ut_b[k] += R(2) * ut[k] * q2_b;

    R aL_b = (R(st.u(IE, 2)) + R(st.p(1, 2))) * Ht_b, aR_b = (R(st.u(IE, 3)) + R(st.p(1, 3))) * Ht_b;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        aL_b += R(st.u(IM + k, 2)) * ut_b[k];
        aR_b += R(st.u(IM + k, 3)) * ut_b[k];
        out.u(IM + k, 2, double(aL * ut_b[k]));
        out.u(IM + k, 3, double(aR * ut_b[k]));
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        aL_b += R(st.u(s, 2)) * Yt_b[s];
        aR_b += R(st.u(s, 3)) * Yt_b[s];
    }
    out.u(IE, 2, double(aL * Ht_b));
    out.u(IE, 3, double(aR * Ht_b));
    out.p(0, 2, double(aL * Ht_b));
    out.p(0, 3, double(aR * Ht_b));
    out.p(1, 2, double(wL * Tt_b));
    out.p(1, 3, double(wR * Tt_b));
    R wL_b = R(st.p(0, 2)) * Tt_b + r2 * aL_b;
    const R wR_b = R(st.p(0, 3)) * Tt_b + r3 * aR_b;
    const R r2_b = wL * aL_b, r3_b = wR * aR_b;
    wL_b -= wR_b;
    const R iS2 = R(1) / (Ssum * Ssum);
    const R rL_b = wL_b * sR * iS2 / (R(2) * sL);
    const R rR_b = -wL_b * sL * iS2 / (R(2) * sR);
    const R x2 = rL_b - r2 * r2 * r2_b, x3 = rR_b - r3 * r3 * r3_b;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        out.u(s, 2, double(aL * Yt_b[s] + x2));
        out.u(s, 3, double(aR * Yt_b[s] + x3));
    }
}

// ---------------------------------------------------------------------------
// The face VJP runs as two kernels per group of faces (HALF 0: face_vjp_a,
// HALF 1: face_vjp_b) so that neither keeps the other's live state; the
// record between them is indexed by the thread's linear index in the launch
// (both halves use the same grid), with stride nrec.
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
// those of w and w + 2 cannot; launch `grp` takes the waves w = grp mod 6.
// ---------------------------------------------------------------------------
template <int NS, typename R, int HALF, bool CU6>
__global__ __launch_bounds__(256) void k_face_vjp_x(const double *__restrict__ U, const double *__restrict__ P,
                                                    const double *__restrict__ rbar, double *__restrict__ Ubar,
                                                    double *__restrict__ Pbar, double *__restrict__ rec,
                                                    long long nrec, Geo g, ThermoK<R> th, int W, int grp,
                                                    Dissip ds) {
    constexpr int NV = NS + 4;
    extern __shared__ double xf_win[];
    const int wpb = blockDim.x >> 6, wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const long long rowf = (long long)g.nx + 1;          // faces per row
    const long long nfp = rowf * g.ny;                   // faces per plane
    const long long wpp = (nfp + 63) / 64;               // waves per plane
    const long long wid = 6 * ((long long)blockIdx.x * wpb + wv) + grp;
    const long long C = g.cells;
    const long long zb = (long long)(g.gz + blockIdx.y) * g.sz + (long long)g.gy * g.sy;   // plane's first row
    double *w = xf_win + (size_t)wv * (NV + 2) * W;
    for (int i = lane; i < (NV + 2) * W; i += 64) w[i] = 0.0;
    __syncthreads();
    const long long f0 = wid * 64, f = f0 + lane;
    const long long r0 = f0 / rowf;
    const long long base0 = zb + r0 * g.sy + (f0 - r0 * rowf);   // stencil cell 0 of the wave's first face
    if (wid < wpp && f < nfp) {
        const long long r = f / rowf;
        const int i = (int)(f - r * rowf);
        const long long row = zb + r * g.sy + g.gx;             // interior cell 0 of the row
        R Fb[NV];
        bool any = false;
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            const double rr = i < g.nx ? rbar[q * C + row + i] : 0.0;
            const double rl = i > 0 ? rbar[q * C + row + i - 1] : 0.0;
            Fb[q] = R((rr - rl) * g.idx);
            any = any || (Fb[q] != R(0));
        }
        if (any) {
            const long long base = row + i - 3;
            Stencil st{U, P, base, 1, C};
            SinkLds sk{(volatile lds_double *)w, W, (int)(base - base0), 1, NV * W};
            const VjpRec<NS> rc{rec, nrec, ((long long)blockIdx.y * gridDim.x + blockIdx.x) * blockDim.x + threadIdx.x};
            if constexpr (HALF == 0)
                face_vjp_a<NS, R, 0, CU6>(st, th, Fb, sk, rc, ds);
            else
                face_vjp_b<NS, R, 0>(st, th, sk, rc);
        }
    }
    __syncthreads();
    if (wid < wpp) {
        const long long fl = min(f0 + 63, nfp - 1);
        const long long rl = fl / rowf;
        const int span = (int)(zb + rl * g.sy + (fl - rl * rowf) - base0) + 6;
        for (int c = lane; c < span; c += 64) {
#pragma unroll
            for (int q = 0; q < NV; ++q) Ubar[q * C + base0 + c] += w[q * W + c];
            Pbar[base0 + c] += w[NV * W + c];
            Pbar[C + base0 + c] += w[(NV + 1) * W + c];
        }
    }
}

// ---------------------------------------------------------------------------
// y and z directions, blocked: a block takes 16 x-columns by 16 consecutive
// faces j0..j0+15 of the sweep axis (j0 = 16 b) in one plane of the third
// axis; wave w of the block takes faces j0+4w..j0+4w+3 (lane = 16 ts + tx),
// so each stencil load of a wave reads four whole 128-byte rows.  Wave w
// accumulates in a private LDS window of sweep rows j0+4w-3..j0+4w+5 (within
// one instruction its lanes address distinct cells); the block then adds,
// for each of its 21 x 16 cells, the windows that cover it in wave order to
// Ubar / Pbar (one coalesced read-modify-write per cell and field).  Blocks
// b and b + 1 share six rows, blocks b and b + 6 none: launch `phase` takes
// the blocks b = phase mod 6.
// ---------------------------------------------------------------------------
constexpr int kVjpTX = 16, kVjpFB = 16, kVjpWin = kVjpTX * 9;

template <int NS, typename R, int DIR, int HALF, bool CU6>
__global__ __launch_bounds__(256) void k_face_vjp_yz(const double *__restrict__ U, const double *__restrict__ P,
                                                     const double *__restrict__ rbar, double *__restrict__ Ubar,
                                                     double *__restrict__ Pbar, double *__restrict__ rec,
                                                     long long nrec, Geo g, ThermoK<R> th, int phase, Dissip ds) {
    constexpr int NV = NS + 4;
    __shared__ double xf_wyz[4][(NV + 2) * kVjpWin];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int tx = lane & (kVjpTX - 1), ts = lane / kVjpTX;
    const int nsw = DIR == 1 ? g.ny : g.nz;
    const long long ss = DIR == 1 ? g.sy : g.sz;
    const int gs = DIR == 1 ? g.gy : g.gz;
    const int xt = (g.nx + kVjpTX - 1) / kVjpTX;                   // x tiles
    const int nfb = (nsw + 1 + kVjpFB - 1) / kVjpFB;               // face blocks along the sweep axis
    const int nb = (nfb - phase + kVjpGroups - 1) / kVjpGroups;    // face blocks of this phase
    const int xi = blockIdx.x % xt;
    const int b = phase + kVjpGroups * (int)(blockIdx.x / xt);     // this block's face block (< nfb)
    const int tr = blockIdx.y;                                     // plane of the third axis
    const int j0 = b * kVjpFB;
    const int x = xi * kVjpTX + tx;
    const int j = j0 + 4 * wv + ts;
    const long long C = g.cells;
    // padded index of the cell at x = x0 + tx, interior sweep index 0, in this plane
    const long long col0 = (long long)g.gx + (DIR == 1 ? (long long)(g.gz + tr) * g.sz : (long long)(g.gy + tr) * g.sy) +
                           (long long)gs * ss;
    volatile double *w = xf_wyz[wv];
    for (int i = lane; i < (NV + 2) * kVjpWin; i += 64) w[i] = 0.0;
    __syncthreads();
    (void)nb;
    if (x < g.nx && j <= nsw) {
        const long long col = col0 + x;
        const double id = DIR == 1 ? g.idy : g.idz;
        R Fb[NV];
        bool any = false;
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            const double rr = j < nsw ? rbar[q * C + col + (long long)j * ss] : 0.0;
            const double rl = j > 0 ? rbar[q * C + col + (long long)(j - 1) * ss] : 0.0;
            Fb[q] = R((rr - rl) * id);
            any = any || (Fb[q] != R(0));
        }
        if (any) {
            const long long base = col + (long long)(j - 3) * ss;
            Stencil st{U, P, base, ss, C};
            // window row r of wave w = sweep row j0 + 4w - 3 + r; stencil cell m is row ts + m
            SinkLds sk{(volatile lds_double *)xf_wyz[wv], kVjpWin, ts * kVjpTX + tx, kVjpTX, NV * kVjpWin};
            const VjpRec<NS> rc{rec, nrec, (long long)(blockIdx.y * gridDim.x + blockIdx.x) * 256 + threadIdx.x};
            if constexpr (HALF == 0)
                face_vjp_a<NS, R, DIR, CU6>(st, th, Fb, sk, rc, ds);
            else
                face_vjp_b<NS, R, DIR>(st, th, sk, rc);
        }
    }
    __syncthreads();
    // block rows r = 0..20 (sweep rows j0-3 .. j0+17); wave w covers r in [4w, 4w+9)
    for (int c = threadIdx.x; c < kVjpTX * (kVjpFB + 5); c += 256) {
        const int r = c / kVjpTX, cx = xi * kVjpTX + (c % kVjpTX);
        const int row = j0 - 3 + r;                       // interior index along the sweep axis
        if (cx >= g.nx || row > nsw + 2) continue;
        const int wlo = r >= 8 ? (r - 8 + 3) / 4 : 0, whi = min(3, r / 4);
        const long long cell = col0 + cx + (long long)row * ss;
#pragma unroll
        for (int q = 0; q < NV + 2; ++q) {
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

// Per-cell backward of (p, T)(U): p = T sum_s rho_s R_s, and T from
// rho e(T) = E - |m|^2 / (2 rho) by the implicit-function rule
//   dT = (dE - u.dm + |u|^2/2 sum_s drho_s - sum_s e_s(T) drho_s) / (rho C_v).
// u: the cell's conservative values (stride `stride`), T and 1/rho from the
// primitive pass, (pb, Tb) the cotangents of p and T; adds into ub.
template <int NS>
XF_HD void prims_vjp_cell(const ThermoK<double> &th, const double *u, long long stride, double T, double rinv,
                          double pb, double Tb, double *ub) {
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
    for (int s = 0; s < NS; ++s) ub[s * stride] += pb * T * th.Rs[s] + gT * (k2 - e_species(th, s, T));
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
    const double pb = Pbar[idx], Tb = Pbar[C + idx];
    if (pb == 0.0 && Tb == 0.0) return;
    prims_vjp_cell<NS>(th, U + idx, C, P[idx], P[3 * C + idx], pb, Tb, Ubar + idx);
}

}  // namespace xf
