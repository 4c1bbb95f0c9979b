// Reverse-mode derivatives of the point-pair terms of the Galerkin assembly with respect to
// the pair's geometry (host and device code).
//
// An ordered point pair (observation point o, source point s) of an element pair adds, to
// a real loss, the real part of
//   smooth rule:   wD Dk + wDt Dt + wS St + (wN1 - k^2 nn wN2) gk
//   log-split rule (touching elements, Sec. II eq. (4) with the logarithm integrated by
//   moments): sum over the four kernels of w_w B + w_m A with K = A log|s - s'| + B
// where the w are the loss weights of the matrix entries the pair feeds times its
// quadrature and hat weights, R = |r_o - r_s|, nu = (r_o - r_s).n_s / R, nn = n_o.n_s,
// kt = k + i beta, and the kernels are those of the assembly:
//   gk = (i/4) H0(kR), Dk = (ik/4) H1(kR) nu, St = (i/4) H0(kt R), Dt = (ikt/4) H1(kt R) nu.
// The derivatives use H0' = -H1, (z H1)' = z H0 and H1' = H0 - H1/z.
#pragma once
#include "bessel.h"
#include "cplx.h"

namespace cfie {

// partial derivatives of one pair's loss term
struct PairD {
    double R, nu, nn;      // d/dR, d/dnu, d/dnn
    double beta;           // d/d(Im kt)
    double vh2;            // value of the terms that scale with h^2 (their d/dh is 2 vh2 / h)
    double h;              // explicit d/dh beyond the h^2 scaling (coincident points)
    double curv;           // d/d(curvature) (coincident points)
};

// weights of the smooth rule (the h^2 w_g w_h hat products are folded into wD, wDt, wS,
// wN2; wN1 carries w_g w_h s_a s_b of the Maue derivative term and does not scale with h)
struct SmoothW {
    zd wD, wDt, wS, wN1, wN2;
};

// g0 = (i/4) H0(kR), g1 = (ik/4) H1(kR), t0 = (i/4) H0(kt R), t1 = (ikt/4) H1(kt R)
CFIE_HD PairD smooth_pair_adjoint(double k, zd kt, double R, double nu, double nn, zd g0,
                                  zd g1, zd t0, zd t1, const SmoothW &w) {
    const double k2 = k * k;
    const double iR = 1.0 / R;
    const zd kt2 = kt * kt;
    const zd wN = w.wN1 - w.wN2 * (k2 * nn);
    // d/dR of g1 and t1: kappa^2 (i/4) H0 - (i kappa / 4) H1 / R
    const zd dg1 = g0 * k2 - g1 * iR;
    const zd dt1 = kt2 * t0 - t1 * iR;
    PairD d;
    d.R = (w.wD * dg1 * nu + w.wDt * dt1 * nu - w.wS * t1 - wN * g1).x;
    d.nu = (w.wD * g1 + w.wDt * t1).x;
    d.nn = -(w.wN2 * g0).x * k2;
    // d/dkt: St -> -(R/kt) t1, Dt -> kt R t0 nu; d kt = i d beta
    const zd dkt = w.wS * (t1 * cinv(kt)) * (-R) + w.wDt * (kt * t0) * (R * nu);
    d.beta = -dkt.y;
    d.vh2 = (w.wD * g1 * nu + w.wDt * t1 * nu + w.wS * t0 - w.wN2 * g0 * (k2 * nn)).x;
    d.h = 0.0;
    d.curv = 0.0;
    return d;
}

// weights of the log-split rule: *_w multiply the smooth parts B (h^2 w_g w_h hat products),
// *_m the log parts A (h^2 times the product-integration moment with the hats); wN_s and
// wN_sm0 carry the Maue derivative term (w_g w_h s_a s_b and s_a s_b times the moment
// without hats) and do not scale with h
struct SplitW {
    zd wD_w, wD_m, wDt_w, wDt_m, wS_w, wS_m, wN_s, wN_w, wN_sm0, wN_m;
};

// pieces of one kernel in the log-split form and their derivatives
struct SplitK {
    zd A, B, AR, BR, Anu, Bnu, Ak, Bk;   // value, d/dR, d/dnu, d/dkappa
};

// S^kappa: A = -J0/(2 pi), B = (i/4) H0 - A log(l), with l = |s - s'| / h the parametric
// distance of the pair (B then includes the log h of the assembly)
CFIE_HD SplitK split_single(zd kap, double R, double logl, zd J0, zd J1, zd H0, zd H1) {
    const double i2p = 1.0 / (2.0 * kPi);
    SplitK s;
    s.A = J0 * (-i2p);
    s.B = cmul_i(H0) * 0.25 - s.A * logl;
    s.AR = kap * J1 * i2p;
    s.BR = cmul_i(kap * H1) * (-0.25) - s.AR * logl;
    s.Anu = s.Bnu = mk(0.0, 0.0);
    s.Ak = J1 * (R * i2p);
    s.Bk = cmul_i(H1) * (-0.25 * R) - s.Ak * logl;
    return s;
}

// D^kappa: A = -(kappa/(2 pi)) J1 nu, B = (i kappa/4) H1 nu - A log(l)
CFIE_HD SplitK split_double(zd kap, double R, double nu, double logl, zd J0, zd J1, zd H0,
                            zd H1) {
    const double i2p = 1.0 / (2.0 * kPi);
    const zd kR = kap * R;
    const zd J1z = J1 * cinv(kR), H1z = H1 * cinv(kR);
    SplitK s;
    s.Anu = kap * J1 * (-i2p);
    s.A = s.Anu * nu;
    s.Bnu = cmul_i(kap * H1) * 0.25 - s.Anu * logl;
    s.B = s.Bnu * nu;
    s.AR = kap * kap * (J0 - J1z) * (-i2p * nu);
    s.BR = cmul_i(kap * kap * (H0 - H1z)) * (0.25 * nu) - s.AR * logl;
    s.Ak = kR * J0 * (-i2p * nu);
    s.Bk = cmul_i(kR * H0) * (0.25 * nu) - s.Ak * logl;
    return s;
}

// log-split rule at distinct points; jk, jt: Bessel split at k R and kt R with the Hankel
// values H0, H1 formed from them
CFIE_HD PairD split_pair_adjoint(double k, zd kt, double R, double nu, double nn, double logl,
                                 const zd (&jk)[4], const zd (&jt)[4], const SplitW &w) {
    const double k2 = k * k;
    const zd kk = mk(k, 0.0);
    const SplitK sg = split_single(kk, R, logl, jk[0], jk[1], jk[2], jk[3]);
    const SplitK ss = split_single(kt, R, logl, jt[0], jt[1], jt[2], jt[3]);
    const SplitK sd = split_double(kk, R, nu, logl, jk[0], jk[1], jk[2], jk[3]);
    const SplitK st = split_double(kt, R, nu, logl, jt[0], jt[1], jt[2], jt[3]);
    const zd wNb = w.wN_s - w.wN_w * (k2 * nn);
    const zd wNa = w.wN_sm0 - w.wN_m * (k2 * nn);
    PairD d;
    d.R = (w.wD_w * sd.BR + w.wD_m * sd.AR + w.wDt_w * st.BR + w.wDt_m * st.AR +
           w.wS_w * ss.BR + w.wS_m * ss.AR + wNb * sg.BR + wNa * sg.AR).x;
    d.nu = (w.wD_w * sd.Bnu + w.wD_m * sd.Anu + w.wDt_w * st.Bnu + w.wDt_m * st.Anu).x;
    d.nn = -(w.wN_w * sg.B + w.wN_m * sg.A).x * k2;
    const zd dkt = w.wDt_w * st.Bk + w.wDt_m * st.Ak + w.wS_w * ss.Bk + w.wS_m * ss.Ak;
    d.beta = -dkt.y;
    d.vh2 = (w.wD_w * sd.B + w.wD_m * sd.A + w.wDt_w * st.B + w.wDt_m * st.A + w.wS_w * ss.B +
             w.wS_m * ss.A - (w.wN_w * sg.B + w.wN_m * sg.A) * (k2 * nn)).x;
    d.h = 0.0;
    d.curv = 0.0;
    return d;
}

// log-split rule at coincident points (R = 0): the limits of the assembly,
//   A_S = -1/(2 pi), B_S = i/4 - (log(kappa h / 2) + gamma)/(2 pi), A_D = 0,
//   B_D = -curv/(4 pi), nn = 1
CFIE_HD PairD coincident_adjoint(double k, zd kt, double h, double curv, const SplitW &w) {
    const double k2 = k * k;
    const double i2p = 1.0 / (2.0 * kPi);
    const zd lk = mk(std::log(k * 0.5 * h) + kEulerGamma, 0.0);
    const zd lt = clog(kt * (0.5 * h)) + mk(kEulerGamma, 0.0);
    const zd BSk = mk(0.0, 0.25) - lk * i2p;
    const zd BSt = mk(0.0, 0.25) - lt * i2p;
    const zd AS = mk(-i2p, 0.0);
    const double BD = -curv / (4.0 * kPi);
    const zd wNb = w.wN_s - w.wN_w * k2;
    PairD d;
    d.R = d.nu = d.nn = 0.0;
    d.curv = -(w.wD_w + w.wDt_w).x / (4.0 * kPi);
    // dB_S/dkappa = -1/(2 pi kappa)
    const zd dkt = w.wS_w * cinv(kt) * (-i2p);
    d.beta = -dkt.y;
    // dB_S/dh = -1/(2 pi h)
    d.h = (w.wS_w + wNb).x * (-i2p / h);
    d.vh2 = ((w.wD_w + w.wDt_w) * BD + w.wS_w * BSt + w.wS_m * AS -
             (w.wN_w * BSk + w.wN_m * AS) * k2).x;
    return d;
}

// chain rule from (R, nu, nn) to the coordinates and unit tangents of both points:
// o[0..3], s[0..3] += d/d(x, y, tx, ty)
CFIE_HD void pair_geom_adjoint(double dx, double dy, double R, double nu, double txo,
                               double tyo, double txs, double tys, const PairD &d, double *o,
                               double *s) {
    const double iR = 1.0 / R;
    const double gx = d.R * dx * iR + d.nu * (tys - nu * dx * iR) * iR;
    const double gy = d.R * dy * iR + d.nu * (-txs - nu * dy * iR) * iR;
    if (o) {
        o[0] += gx;
        o[1] += gy;
        o[2] += d.nn * txs;
        o[3] += d.nn * tys;
    }
    if (s) {
        s[0] -= gx;
        s[1] -= gy;
        s[2] += d.nn * txo - d.nu * dy * iR;
        s[3] += d.nn * tyo + d.nu * dx * iR;
    }
}

}  // namespace cfie
