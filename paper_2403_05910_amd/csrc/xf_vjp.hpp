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
    const R i0 = R(1) / (R(1e-6) + (R(13.0 / 12.0) * t0 * t0 + R(0.25) * u0 * u0));
    const R i1 = R(1) / (R(1e-6) + (R(13.0 / 12.0) * t1 * t1 + R(0.25) * u1 * u1));
    const R i2 = R(1) / (R(1e-6) + (R(13.0 / 12.0) * t2 * t2 + R(0.25) * u2 * u2));
    const R al0 = R(0.1) * i0 * i0, al1 = R(0.6) * i1 * i1, al2 = R(0.3) * i2 * i2;
    const R iS = R(1) / (al0 + al1 + al2);
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

template <int NS, typename R, int DIR>
XF_HD void face_vjp(const Stencil &st, const ThermoK<R> &th, const R *Fb, const Sink &out) {
    constexpr int IM = NS;
    constexpr int IE = NS + 3;
    constexpr int KN = Axes<DIR>::n, K1 = Axes<DIR>::t1, K2 = Axes<DIR>::t2;
    constexpr int IN = NS + KN, I1 = NS + K1, I2 = NS + K2;

    // ================= forward: Roe state and per-cell scalars =================
    R rL = R(0), rR = R(0);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        rL += R(st.u(s, 2));
        rR += R(st.u(s, 3));
    }
    const R sL = xsqrt(rL), sR = xsqrt(rR);
    const R Ssum = sL + sR;
    const R wL = sL / Ssum;
    const R wR = R(1) - wL;
    const R r2 = R(st.p(3, 2)), r3 = R(st.p(3, 3));
    const R aL = wL * r2, aR = wR * r3;
    R ut[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) ut[k] = aL * R(st.u(IM + k, 2)) + aR * R(st.u(IM + k, 3));
    const R Ht = aL * (R(st.u(IE, 2)) + R(st.p(1, 2))) + aR * (R(st.u(IE, 3)) + R(st.p(1, 3)));
    const R Tt = wL * R(st.p(0, 2)) + wR * R(st.p(0, 3));
    R Yt[NS], chi[NS];
    R Rb = R(0), cvb = R(0);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        Yt[s] = aL * R(st.u(s, 2)) + aR * R(st.u(s, 3));
        Rb += Yt[s] * th.Rs[s];
        cvb += Yt[s] * cv_species(th, s, Tt);
        chi[s] = e_species(th, s, Tt);
    }
    const R Gam = Rb / cvb;
    const R q2 = ut[0] * ut[0] + ut[1] * ut[1] + ut[2] * ut[2];
    R c2 = Gam * (Ht - q2);
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        chi[s] = Gam * (R(0.5) * q2 - chi[s]) + th.Rs[s] * Tt;
        c2 += Yt[s] * chi[s];
    }
    const R ct = xsqrt(c2);
    const R ic2 = R(1) / c2;
    const R cih = R(0.5) * ct * ic2;
    const R iGam = R(1) / Gam;
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
        const R hm = split_weno_fb(gMp, gMm, aM, Asum_b - Dif_b, wFmb, wUmb);
        const R hp = split_weno_fb(gPp, gPm, aP, Asum_b + Dif_b, wFpb, wUpb);
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
        const R ha = split_weno_fb(gp, gm, a0, hb, wFb, wUb);
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
        const R hs = split_weno_fb(gp, gm, a0, hsb, wFb, wUb);
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
        const R um = ut[0] * M0 + ut[1] * M1 + ut[2] * M2;
        const R dpU = sc - Gam * um + Gam * E;
        const R dpF = un[m] * sc - Gam * (un[m] * um + pm * utn) + Gam * ((E + pm) * un[m]);
        const R dpU_b = ic2 * DU_b[m], dpF_b = ic2 * DF_b[m];
        ic2_b += dpU * DU_b[m] + dpF * DF_b[m];
        const R sc_b = dpU_b + un[m] * dpF_b;
        const R um_b = -Gam * (dpU_b + un[m] * dpF_b);
        const R E_b = Gam * (dpU_b + un[m] * dpF_b);
        Gam_b += (E - um) * dpU_b + ((E + pm) * un[m] - un[m] * um - pm * utn) * dpF_b;
        const R un_bt = un_b[m] + (sc - Gam * um + Gam * (E + pm)) * dpF_b;
        const R pm_bt = pm_b[m] + Gam * (un[m] - utn) * dpF_b;
        ut_b[KN] -= Gam * pm * dpF_b;
        ut_b[0] += M0 * um_b;
        ut_b[1] += M1 * um_b;
        ut_b[2] += M2 * um_b;
        const R rinv_b = mn * un_bt;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            R v = ut[k] * um_b;
            if (k == KN) v += Mn_b[m] + rinv * un_bt;
            out.u(IM + k, m, double(v));
        }
        const R sp = rh_b[m] - rinv * rinv * rinv_b;
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
// Marching VJP sweep.  Memory axes are given by strides, so the same kernel
// serves x (lanes along y), y and z (lanes along x).  A thread owns one column
// and one segment of its faces; faces j-1/2 scatter into cells j-3..j+2 of
// their own column, so two segments of a column are in flight together only if
// they are at least one segment apart: launch 0 takes the even segments,
// launch 1 the odd ones.  No atomics; the summation order is fixed.
// ---------------------------------------------------------------------------
struct MarchGeo {
    long long origin;         // padded index of interior cell (0, 0, 0)
    long long sl, st, ss;     // strides of the lane, transverse and sweep axes
    int nl, nt, nsw;          // interior extents of those axes
};

template <int NS, typename R, int DIR>
__global__ __launch_bounds__(256) void k_sweep_vjp(const double *__restrict__ U, const double *__restrict__ P,
                                                   const double *__restrict__ rbar, double *__restrict__ Ubar,
                                                   double *__restrict__ Pbar, long long cells, MarchGeo mg,
                                                   ThermoK<R> th, double id, int seglen, int parity) {
    constexpr int NV = NS + 4;
    unsigned bx, by, bz;
    xcd_block(bx, by, bz);
    const int l = bx * 64 + threadIdx.x;
    const int tr = by * 4 + threadIdx.y;
    if (l >= mg.nl || tr >= mg.nt) return;
    const int seg = 2 * bz + parity;
    const int j0 = seg * seglen;
    const int nfaces = mg.nsw + 1;
    if (j0 >= nfaces) return;
    const int j1 = min(j0 + seglen, nfaces);
    const long long col = mg.origin + l * mg.sl + tr * mg.st;
    for (int j = j0; j < j1; ++j) {
        // face j-1/2 between interior cells j-1 and j: dF = (rbar_j - rbar_{j-1}) / dx
        R Fb[NV];
        bool any = false;
#pragma unroll
        for (int q = 0; q < NV; ++q) {
            const double rr = (j < mg.nsw) ? rbar[q * cells + col + (long long)j * mg.ss] : 0.0;
            const double rl = (j > 0) ? rbar[q * cells + col + (long long)(j - 1) * mg.ss] : 0.0;
            Fb[q] = R((rr - rl) * id);
            any = any || (Fb[q] != R(0));
        }
        if (!any) continue;
        const long long base = col + (long long)(j - 3) * mg.ss;
        Stencil st{U, P, base, mg.ss, cells};
        Sink sk{Ubar, Pbar, base, mg.ss, cells};
        face_vjp<NS, R, DIR>(st, th, Fb, sk);
    }
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
