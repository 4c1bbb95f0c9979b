// Host build of the point-pair derivative formulas of the shape gradient, for CPU tests.
// Each entry evaluates one pair's loss term the way the assembly kernels form it (Hankel
// values from the same header routines) and the analytic partial derivatives, so that the
// test can compare them with central differences.
#include "../paper_2203_13283_amd/csrc/shape_grad.h"
using namespace cfie;

namespace {

// geometry: p[0..3] = observation x, y, tx, ty; p[4..7] = source x, y, tx, ty; p[8] = h;
// p[9] = beta; p[10] = curvature (coincident rule)
struct Geo {
    double dx, dy, R, nu, nn;
};
Geo geo(const double *p) {
    Geo g;
    g.dx = p[0] - p[4];
    g.dy = p[1] - p[5];
    g.R = std::sqrt(g.dx * g.dx + g.dy * g.dy);
    g.nu = (g.dx * p[7] - g.dy * p[6]) / g.R;
    g.nn = p[2] * p[6] + p[3] * p[7];
    return g;
}
zd wz(const double *w, int i) { return mk(w[2 * i], w[2 * i + 1]); }

}  // namespace

// smooth rule: loss value and gradient (out[0..9]) for raw weights w (5 complex:
// D, Dt, S, N1, N2); the h^2 factor is applied here
extern "C" double sg_smooth(double k, const double *p, const double *w, double *grad) {
    Geo g = geo(p);
    double h = p[8];
    zd kt = mk(k, p[9]);
    zd H0, H1;
    hankel01(mk(k * g.R, 0.0), H0, H1);
    zd g0 = cmul_i(H0) * 0.25, g1 = cmul_i(H1) * (0.25 * k);
    hankel01(kt * g.R, H0, H1);
    zd t0 = cmul_i(H0) * 0.25, t1 = cmul_i(kt * H1) * 0.25;
    SmoothW W;
    double h2 = h * h;
    W.wD = wz(w, 0) * h2;
    W.wDt = wz(w, 1) * h2;
    W.wS = wz(w, 2) * h2;
    W.wN1 = wz(w, 3);
    W.wN2 = wz(w, 4) * h2;
    double val = (W.wD * g1 * g.nu + W.wDt * t1 * g.nu + W.wS * t0 +
                  (W.wN1 - W.wN2 * (k * k * g.nn)) * g0).x;
    if (grad) {
        PairD d = smooth_pair_adjoint(k, kt, g.R, g.nu, g.nn, g0, g1, t0, t1, W);
        for (int i = 0; i < 10; ++i) grad[i] = 0.0;
        pair_geom_adjoint(g.dx, g.dy, g.R, g.nu, p[2], p[3], p[6], p[7], d, grad, grad + 4);
        grad[8] = 2.0 * d.vh2 / h + d.h;
        grad[9] = d.beta;
    }
    return val;
}

// log-split rule at distinct points, written as the near-field assembly forms it:
//   S^kappa: A = -J0/(2 pi), B = (i/4) J0 - (log(kappa/2) + log(R/sig)) J0/(2 pi) - Yh0/4
//   D^kappa: A = -(kappa/(2 pi)) J1 nu,
//            B = [(i kappa/4) J1 - (kappa/(2 pi))(log(kappa/2) + log(R/sig)) J1
//                 - (kappa/4) Yh1] nu + nu/(2 pi R)
//   then B += A log h, sig = h l.  w: 10 raw complex weights (D_w, D_m, Dt_w, Dt_m, S_w,
//   S_m, N_s, N_w, N_sm0, N_m); the h^2 factor is applied to all but N_s, N_sm0.
extern "C" double sg_split(double k, double logl, const double *p, const double *w,
                           double *grad) {
    Geo g = geo(p);
    double h = p[8];
    zd kt = mk(k, p[9]);
    double sig = h * std::exp(logl);
    double lr = std::log(g.R / sig);
    const double i2p = 1.0 / (2.0 * kPi);
    auto parts = [&](zd kap, zd &AS, zd &BS, zd &AD, zd &BD, zd (&j)[4]) {
        BesselSplit b = bessel_split(kap * g.R);
        zd lk2 = clog(kap * 0.5);
        AS = b.J0 * (-i2p);
        BS = cmul_i(b.J0) * 0.25 - (lk2 + mk(lr, 0.0)) * b.J0 * i2p - b.Yh0 * 0.25;
        AD = kap * b.J1 * (-i2p * g.nu);
        BD = (cmul_i(kap) * b.J1 * 0.25 - kap * (lk2 + mk(lr, 0.0)) * b.J1 * i2p -
              kap * b.Yh1 * 0.25) * g.nu + mk(g.nu / (2.0 * kPi * g.R), 0.0);
        BS = BS + AS * std::log(h);
        BD = BD + AD * std::log(h);
        zd H0, H1;
        hankel_from_split(kap * g.R, b, H0, H1);
        j[0] = b.J0; j[1] = b.J1; j[2] = H0; j[3] = H1;
    };
    zd ASk, BSk, ADk, BDk, ASt, BSt, ADt, BDt, jk[4], jt[4];
    parts(mk(k, 0.0), ASk, BSk, ADk, BDk, jk);
    parts(kt, ASt, BSt, ADt, BDt, jt);
    double h2 = h * h;
    SplitW W;
    W.wD_w = wz(w, 0) * h2; W.wD_m = wz(w, 1) * h2;
    W.wDt_w = wz(w, 2) * h2; W.wDt_m = wz(w, 3) * h2;
    W.wS_w = wz(w, 4) * h2; W.wS_m = wz(w, 5) * h2;
    W.wN_s = wz(w, 6); W.wN_w = wz(w, 7) * h2;
    W.wN_sm0 = wz(w, 8); W.wN_m = wz(w, 9) * h2;
    double k2 = k * k;
    double val = (W.wD_w * BDk + W.wD_m * ADk + W.wDt_w * BDt + W.wDt_m * ADt + W.wS_w * BSt +
                  W.wS_m * ASt + (W.wN_s - W.wN_w * (k2 * g.nn)) * BSk +
                  (W.wN_sm0 - W.wN_m * (k2 * g.nn)) * ASk).x;
    if (grad) {
        PairD d = split_pair_adjoint(k, kt, g.R, g.nu, g.nn, logl, jk, jt, W);
        for (int i = 0; i < 10; ++i) grad[i] = 0.0;
        pair_geom_adjoint(g.dx, g.dy, g.R, g.nu, p[2], p[3], p[6], p[7], d, grad, grad + 4);
        grad[8] = 2.0 * d.vh2 / h + d.h;
        grad[9] = d.beta;
    }
    return val;
}

// coincident points, as the near-field assembly forms them; gradient out[0] = d/dh,
// out[1] = d/dbeta, out[2] = d/dcurv
extern "C" double sg_coincident(double k, const double *p, const double *w, double *grad) {
    double h = p[8];
    zd kt = mk(k, p[9]);
    double curv = p[10];
    const double i2p = 1.0 / (2.0 * kPi);
    zd AS = mk(-i2p, 0.0);
    zd BSk = mk(0.0, 0.25) - (clog(mk(k * 0.5, 0.0)) + mk(kEulerGamma, 0.0)) * i2p;
    zd BSt = mk(0.0, 0.25) - (clog(kt * 0.5) + mk(kEulerGamma, 0.0)) * i2p;
    zd BD = mk(-curv / (4.0 * kPi), 0.0);
    BSk = BSk + AS * std::log(h);
    BSt = BSt + AS * std::log(h);
    double h2 = h * h;
    SplitW W;
    W.wD_w = wz(w, 0) * h2; W.wD_m = wz(w, 1) * h2;
    W.wDt_w = wz(w, 2) * h2; W.wDt_m = wz(w, 3) * h2;
    W.wS_w = wz(w, 4) * h2; W.wS_m = wz(w, 5) * h2;
    W.wN_s = wz(w, 6); W.wN_w = wz(w, 7) * h2;
    W.wN_sm0 = wz(w, 8); W.wN_m = wz(w, 9) * h2;
    double k2 = k * k;
    double val = (W.wD_w * BD + W.wDt_w * BD + W.wS_w * BSt + W.wS_m * AS +
                  (W.wN_s - W.wN_w * k2) * BSk + (W.wN_sm0 - W.wN_m * k2) * AS).x;
    if (grad) {
        PairD d = coincident_adjoint(k, kt, h, curv, W);
        grad[0] = 2.0 * d.vh2 / h + d.h;
        grad[1] = d.beta;
        grad[2] = d.curv;
    }
    return val;
}
