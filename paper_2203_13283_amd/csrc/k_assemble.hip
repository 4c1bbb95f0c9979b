// Galerkin assembly of D^k, N^k, D^kt, S^kt on the contour (Sec. II eqs. (2)-(4),
// Sec. III eq. (5)): [A]_ij = int int lambda_i(s) K(r(s), r(s')) lambda_j(s') ds ds' with
//   S^kappa : (i/4) H0(kappa R)
//   D^kappa : (i kappa/4) H1(kappa R) (r - r').n' / R
//   N^k     : (i/4) H0(k R) [lambda_i' lambda_j' - k^2 n.n' lambda_i lambda_j]  (Maue form)
// Hats are linear in arc length on N equal elements.  Every output entry is written by
// exactly one thread (no atomics), so the assembly is deterministic.
//
// Far kernel: one wavefront owns 63 output rows and a strip of columns.  Lane l holds the
// Gauss points of element e = i0 - 1 + l and walks the element columns; each element pair
// gives a 2x2 block per matrix.  The column (b) direction is combined in registers through
// a carry, the row (a) direction by a lane shuffle: entry (i, j) = block(i-1, .)[1][.] +
// block(i, .)[0][.].  The four Hankel values per point pair share one sincos and one exp:
// Re kt = k, so e^{i kt R} = e^{i k R} e^{-beta R}.
//
// Near kernel: one thread per entry in the band |i - j| <= nb + 1 sums its four element
// pairs.  Element pairs that share a point use the split K = A log|s - s'| + B with A, B
// smooth: B by Gauss-Legendre on the q x q grid, A by product integration with the
// precomputed moments int int l_g l_h phi_a phi_b log(sigma).
#include "internal.h"

namespace cfie {

// ------------------------------------------------------------------ Gauss points ----------
__global__ void k_points(int N, int q, double h, double L, double c0, int Ms, const zd *cm,
                         int M, const zd *zhat, const double *xi, double *X, double *Y,
                         double *TX, double *TY, double *CV) {
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= N * q) return;
    int e = idx / q, g = idx - e * q;
    double s = ((double)e + xi[g]) * h;
    double t = 2.0 * kPi * s / L;
    int extra = 2;
    for (int it = 0; it < 60; ++it) {
        double sn, cs;
        sincos(t, &sn, &cs);
        zd E1 = mk(cs, sn), E = E1;
        double st = c0 * t, sp = c0;
        for (int m = 1; m <= Ms; ++m) {
            zd c = cm[m - 1];
            zd cE = c * E;
            sp += 2.0 * cE.x;
            st += 2.0 * (cE.y - c.y) / (double)m;     // 2 Re(c (E - 1) / (i m))
            E = E * E1;
        }
        double dt = (st - s) / sp;
        t -= dt;
        if (fabs(dt) < 1e-14) {
            if (--extra == 0) break;
        }
    }
    double sn, cs;
    sincos(t, &sn, &cs);
    zd E1 = mk(cs, sn);
    sincos(-(double)M * t, &sn, &cs);
    zd E = mk(cs, sn);
    zd z = mk(0.0, 0.0), d1 = mk(0.0, 0.0), d2 = mk(0.0, 0.0);
    for (int m = -M; m <= M; ++m) {
        zd v = zhat[m + M] * E;
        z = z + v;
        d1 = d1 + cmul_i(v) * (double)m;
        d2 = d2 - v * ((double)m * (double)m);
        E = E * E1;
    }
    double sp = sqrt(d1.x * d1.x + d1.y * d1.y);
    X[idx] = z.x;
    Y[idx] = z.y;
    TX[idx] = d1.x / sp;
    TY[idx] = d1.y / sp;
    CV[idx] = (d1.x * d2.y - d1.y * d2.x) / (sp * sp * sp);
}

void launch_points(const GeomDev &g, const double *xi, PointTable &pt, hipStream_t s) {
    int n = g.N * pt.q;
    int bs = 256;
    hipLaunchKernelGGL(k_points, dim3((n + bs - 1) / bs), dim3(bs), 0, s, g.N, pt.q, g.h, g.L,
                       g.c0, g.Ms, g.cm, g.M, g.zhat, xi, pt.x, pt.y, pt.tx, pt.ty, pt.curv);
}

// ------------------------------------------------------------------ kernel values ---------
struct PairConsts {
    double k, beta;                  // kt = k + i beta
    zd kt;
    zd Cg, CD, CS, CDt;              // prefactors of the large-argument forms
    zd ik4, ikt4;                    // i k / 4, i kt / 4
};

// Point-pair kernels: gk = (i/4) H0(kR), Dk = (ik/4) H1(kR) nu, St = (i/4) H0(ktR),
// Dt = (ikt/4) H1(ktR) nu, with nu = (r - r').n' / R.
__device__ __forceinline__ void pair_kernels(const PairConsts &c, double R, double nu,
                                             zd &gk, zd &Dk, zd &St, zd &Dt) {
    double kR = c.k * R;
    if (kR >= kAsymMin) {
        double invR = 1.0 / R;
        double sn, cs;
        sincos(kR, &sn, &cs);
        double rs = sqrt(invR);
        zd E = mk(cs * rs, sn * rs);                    // e^{ikR} R^{-1/2}
        zd Et = E * exp(-c.beta * R);
        // real-argument series: w1 = i q1, q1 = 1 / (kR)
        double q1 = invR / c.k;
        zd w2 = cmul_i(cinv(c.kt)) * invR;              // i / (kt R)
        zd t0 = mk(1.0, 0.0), t1 = t0, p0 = t0, p1 = t0;
        zd u0 = t0, u1 = t0, s0 = t0, s1 = t0;
        for (int n = 1; n < 64; ++n) {
            double m = (double)(2 * n - 1);
            double r0 = -m * m / (8.0 * n), r1 = (4.0 - m * m) / (8.0 * n);
            t0 = mk(-t0.y, t0.x) * (r0 * q1);
            t1 = mk(-t1.y, t1.x) * (r1 * q1);
            u0 = u0 * w2 * r0;
            u1 = u1 * w2 * r1;
            p0 = p0 + t0;
            p1 = p1 + t1;
            s0 = s0 + u0;
            s1 = s1 + u1;
            if (abs2(t0) + abs2(t1) + abs2(u0) + abs2(u1) < 1e-34) break;
        }
        gk = c.Cg * E * p0;
        Dk = c.CD * E * p1 * nu;
        St = c.CS * Et * s0;
        Dt = c.CDt * Et * s1 * nu;
    } else {
        zd H0, H1;
        hankel01(mk(kR, 0.0), H0, H1);
        gk = cmul_i(H0) * 0.25;
        Dk = c.ik4 * H1 * nu;
        hankel01(c.kt * R, H0, H1);
        St = cmul_i(H0) * 0.25;
        Dt = c.ikt4 * H1 * nu;
    }
}

static PairConsts make_consts(const KernelConsts &kc) {
    PairConsts c;
    c.k = kc.k;
    c.kt = kc.kt;
    c.beta = kc.kt.y;
    const double r2 = 0.70710678118654752440;
    zd em1 = mk(r2, -r2);                                // e^{-i pi/4}
    zd em3 = mk(-r2, -r2);                               // e^{-3 i pi/4}
    zd pk = mk(std::sqrt(2.0 / (kPi * kc.k)), 0.0);      // sqrt(2/(pi k))
    zd pt = csqrt(cinv(kc.kt) * (2.0 / kPi));             // sqrt(2/(pi kt))
    zd i4 = mk(0.0, 0.25);
    c.ik4 = mk(0.0, 0.25 * kc.k);
    c.ikt4 = cmul_i(kc.kt) * 0.25;
    c.Cg = i4 * pk * em1;
    c.CD = c.ik4 * pk * em3;
    c.CS = i4 * pt * em1;
    c.CDt = c.ikt4 * pt * em3;
    return c;
}

// ------------------------------------------------------------------ far kernel -----------
constexpr int kFarCols = 64;          // node columns per wavefront

template <int Q>
struct QuadConsts {
    double xi[Q], w[Q];
};

template <int Q>
__global__ __launch_bounds__(256) void k_far(int N, double h, PairConsts c, int nb, int r0,
                                             int r1, int64_t ld, zd *o0, zd *o1, zd *o2,
                                             zd *o3, const double *__restrict__ PX,
                                             const double *__restrict__ PY,
                                             const double *__restrict__ PTX,
                                             const double *__restrict__ PTY, QuadConsts<Q> qc,
                                             int n_row_tiles) {
    const int lane = threadIdx.x & 63;
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int n_col_tiles = (N + kFarCols - 1) / kFarCols;
    if (wave >= n_row_tiles * n_col_tiles) return;
    const int rt = wave % n_row_tiles;
    const int ct = wave / n_row_tiles;
    const int i0 = r0 + rt * 63;                     // first output row of this wave
    const int j0 = ct * kFarCols;                    // first output column
    const int jend = min(N, j0 + kFarCols);
    int e = i0 - 1 + lane;
    e = (e % N + N) % N;
    double xo[Q], yo[Q], txo[Q], tyo[Q];
#pragma unroll
    for (int g = 0; g < Q; ++g) {
        xo[g] = PX[e * Q + g];
        yo[g] = PY[e * Q + g];
        txo[g] = PTX[e * Q + g];
        tyo[g] = PTY[e * Q + g];
    }
    double Wa[2][Q];                                  // h w_g phi_a(xi_g)
#pragma unroll
    for (int g = 0; g < Q; ++g) {
        Wa[0][g] = h * qc.w[g] * (1.0 - qc.xi[g]);
        Wa[1][g] = h * qc.w[g] * qc.xi[g];
    }
    const double k2 = c.k * c.k;
    // carry[m][a]: contribution of element column f-1 (b = 1) to node column f
    zd carry[4][2];
#pragma unroll
    for (int m = 0; m < 4; ++m) carry[m][0] = carry[m][1] = mk(0.0, 0.0);
    const int out_row = i0 + lane;                    // row produced by this lane (a = 1 part)
    const bool row_ok = lane < 63 && out_row < r1 && out_row < N;
    for (int f = j0 - 1; f < jend; ++f) {
        int fe = (f % N + N) % N;
        int off = fe - e;
        off = ((off % N) + N) % N;
        int dist = min(off, N - off);
        zd B[4][2][2];
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int a = 0; a < 2; ++a) B[m][a][0] = B[m][a][1] = mk(0.0, 0.0);
        if (dist > nb) {
            double xs[Q], ys[Q], txs[Q], tys[Q];
#pragma unroll
            for (int hh = 0; hh < Q; ++hh) {
                xs[hh] = PX[fe * Q + hh];
                ys[hh] = PY[fe * Q + hh];
                txs[hh] = PTX[fe * Q + hh];
                tys[hh] = PTY[fe * Q + hh];
            }
            for (int g = 0; g < Q; ++g) {
                zd TS[2], TD[2], TT[2], TN1[2], TN0;
                TS[0] = TS[1] = TD[0] = TD[1] = TT[0] = TT[1] = TN1[0] = TN1[1] = TN0 =
                    mk(0.0, 0.0);
#pragma unroll
                for (int hh = 0; hh < Q; ++hh) {
                    double dx = xo[g] - xs[hh], dy = yo[g] - ys[hh];
                    double R = sqrt(dx * dx + dy * dy);
                    double nu = (dx * tys[hh] - dy * txs[hh]) / R;
                    double nn = tyo[g] * tys[hh] + txo[g] * txs[hh];
                    zd gk, Dk, St, Dt;
                    pair_kernels(c, R, nu, gk, Dk, St, Dt);
                    double wb0 = Wa[0][hh], wb1 = Wa[1][hh];
                    TS[0] = TS[0] + St * wb0;
                    TS[1] = TS[1] + St * wb1;
                    TD[0] = TD[0] + Dk * wb0;
                    TD[1] = TD[1] + Dk * wb1;
                    TT[0] = TT[0] + Dt * wb0;
                    TT[1] = TT[1] + Dt * wb1;
                    TN0 = TN0 + gk * qc.w[hh];
                    zd gn = gk * nn;
                    TN1[0] = TN1[0] + gn * wb0;
                    TN1[1] = TN1[1] + gn * wb1;
                }
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    double wa = Wa[a][g];
                    double sa = a ? 1.0 : -1.0;
#pragma unroll
                    for (int b = 0; b < 2; ++b) {
                        double sb = b ? 1.0 : -1.0;
                        B[0][a][b] = B[0][a][b] + TD[b] * wa;
                        B[2][a][b] = B[2][a][b] + TT[b] * wa;
                        B[3][a][b] = B[3][a][b] + TS[b] * wa;
                        B[1][a][b] = B[1][a][b] + TN0 * (sa * sb * qc.w[g]) -
                                     TN1[b] * (k2 * wa);
                    }
                }
            }
        }
        // node column f: carry (b = 1 of column f-1) + b = 0 of column f
        zd col[4][2];
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            col[m][0] = carry[m][0] + B[m][0][0];
            col[m][1] = carry[m][1] + B[m][1][0];
            carry[m][0] = B[m][0][1];
            carry[m][1] = B[m][1][1];
        }
        if (f >= j0) {
            int j = f;
            int dij = out_row - j;
            dij = ((dij % N) + N) % N;
            int dd = min(dij, N - dij);
            zd *outs[4] = {o0, o1, o2, o3};
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                // row out_row = e + 1: own a = 1 part + a = 0 part of lane + 1
                double nx = __shfl_down(col[m][0].x, 1);
                double ny = __shfl_down(col[m][0].y, 1);
                zd v = col[m][1] + mk(nx, ny);
                if (row_ok && dd >= nb + 2) outs[m][(int64_t)out_row + (int64_t)j * ld] = v;
            }
        }
    }
}

void launch_assemble_far(const AsmParams &p, const PointTable &far, const double *xi,
                         const double *w, hipStream_t s) {
    PairConsts c = make_consts(p.kc);
    int nrows = p.r1 - p.r0;
    int n_row_tiles = (nrows + 62) / 63;
    int n_col_tiles = (p.N + kFarCols - 1) / kFarCols;
    long waves = (long)n_row_tiles * n_col_tiles;
    int blocks = (int)((waves + 3) / 4);
    // algorithmic work: Gauss point pairs of the well-separated element pairs of the rows
    double far_pairs = (double)nrows * (double)(p.N - std::min(p.N, 2 * p.nb + 1)) *
                       (double)far.q * far.q;
    ProfScope prof(PROF_FAR, far_pairs, s);
#define CFIE_FAR_CASE(QQ)                                                                   \
    case QQ: {                                                                             \
        QuadConsts<QQ> qc;                                                                 \
        for (int i = 0; i < QQ; ++i) { qc.xi[i] = xi[i]; qc.w[i] = w[i]; }                 \
        hipLaunchKernelGGL(k_far<QQ>, dim3(blocks), dim3(256), 0, s, p.N, p.h, c, p.nb,    \
                           p.r0, p.r1, p.ld, p.out[0], p.out[1], p.out[2], p.out[3], far.x,  \
                           far.y, far.tx, far.ty, qc, n_row_tiles);                        \
        break;                                                                             \
    }
    switch (far.q) {
        CFIE_FAR_CASE(3)
        CFIE_FAR_CASE(4)
        CFIE_FAR_CASE(5)
        CFIE_FAR_CASE(6)
        CFIE_FAR_CASE(8)
        default: break;
    }
#undef CFIE_FAR_CASE
}

// ------------------------------------------------------------------ near kernel ----------
constexpr int kMaxQNear = 16;

struct NearConsts {
    PairConsts pc;
    double h, logh;
    zd logk2, logkt2;                 // log(k/2), log(kt/2)
    double xi[kMaxQNear], w[kMaxQNear];
};

// contribution of element pair (e, f) (kind: -1 regular, 0 same, 1 f = e+1, 2 f = e-1) to
// the entry with local hats (a, b); adds to acc[4] (Dk, Nk, Dkt, Skt)
__device__ void near_pair(const NearConsts &nc, int q, int e, int f, int kind, int a, int b,
                          const double *__restrict__ PX, const double *__restrict__ PY,
                          const double *__restrict__ PTX, const double *__restrict__ PTY,
                          const double *__restrict__ PCV, const double *__restrict__ mom,
                          zd acc[4]) {
    const PairConsts &c = nc.pc;
    const double h = nc.h;
    const double k = c.k;
    const double k2 = k * k;
    const double sab = (a ? 1.0 : -1.0) * (b ? 1.0 : -1.0);
    const double *Mab = mom + ((size_t)(kind < 0 ? 0 : kind) * 5 + (2 * a + b)) * q * q;
    const double *M0 = mom + ((size_t)(kind < 0 ? 0 : kind) * 5 + 4) * q * q;
    const double inv2pi = 1.0 / (2.0 * kPi);
    for (int g = 0; g < q; ++g) {
        double xg = nc.xi[g];
        double pa = a ? xg : 1.0 - xg;
        double xo = PX[e * q + g], yo = PY[e * q + g];
        double txo = PTX[e * q + g], tyo = PTY[e * q + g];
        for (int hh = 0; hh < q; ++hh) {
            double xh = nc.xi[hh];
            double pb = b ? xh : 1.0 - xh;
            double wgt = nc.w[g] * nc.w[hh];
            double xs = PX[f * q + hh], ys = PY[f * q + hh];
            double txs = PTX[f * q + hh], tys = PTY[f * q + hh];
            if (kind < 0) {
                double dx = xo - xs, dy = yo - ys;
                double R = sqrt(dx * dx + dy * dy);
                double nu = (dx * tys - dy * txs) / R;
                double nn = tyo * tys + txo * txs;
                zd gk, Dk, St, Dt;
                pair_kernels(c, R, nu, gk, Dk, St, Dt);
                double hw = h * h * wgt * pa * pb;
                acc[0] = acc[0] + Dk * hw;
                acc[2] = acc[2] + Dt * hw;
                acc[3] = acc[3] + St * hw;
                acc[1] = acc[1] + gk * (wgt * sab - k2 * nn * hw);
                continue;
            }
            double mab = Mab[g * q + hh], m0 = M0[g * q + hh];
            zd Ag, As, Ad, At, Bg, Bs, Bd, Bt;
            double nn;
            if (kind == 0 && g == hh) {
                // coincident points: limits of the smooth parts as R -> 0
                double kc_ = PCV[e * q + g];
                Ag = mk(-inv2pi, 0.0);
                As = Ag;
                Ad = At = mk(0.0, 0.0);
                Bg = mk(0.0, 0.25) - (nc.logk2 + mk(kEulerGamma, 0.0)) * inv2pi;
                Bs = mk(0.0, 0.25) - (nc.logkt2 + mk(kEulerGamma, 0.0)) * inv2pi;
                Bd = Bt = mk(-kc_ / (4.0 * kPi), 0.0);
                nn = 1.0;
            } else {
                double dx = xo - xs, dy = yo - ys;
                double R = sqrt(dx * dx + dy * dy);
                double nu = (dx * tys - dy * txs) / R;
                nn = tyo * tys + txo * txs;
                double sig;
                if (kind == 0) sig = h * fabs(xg - xh);
                else if (kind == 1) sig = h * (1.0 - xg + xh);
                else sig = h * (1.0 + xg - xh);
                double lr = log(R / sig);
                BesselSplit b1 = bessel_split(mk(k * R, 0.0));
                BesselSplit b2 = bessel_split(c.kt * R);
                // S^kappa: A = -J0/(2 pi), B = (i/4) J0 - (log(kappa/2) + lr) J0/(2 pi) - Yh0/4
                Ag = b1.J0 * (-inv2pi);
                As = b2.J0 * (-inv2pi);
                Bg = cmul_i(b1.J0) * 0.25 - (nc.logk2 + mk(lr, 0.0)) * b1.J0 * inv2pi -
                     b1.Yh0 * 0.25;
                Bs = cmul_i(b2.J0) * 0.25 - (nc.logkt2 + mk(lr, 0.0)) * b2.J0 * inv2pi -
                     b2.Yh0 * 0.25;
                // D^kappa: A = -(kappa/(2 pi)) J1 nu,
                // B = [(i kappa/4) J1 - (kappa/(2 pi))(log(kappa/2) + lr) J1 - (kappa/4) Yh1] nu
                //     + nu / (2 pi R)
                zd kk = mk(k, 0.0);
                Ad = kk * b1.J1 * (-inv2pi * nu);
                At = c.kt * b2.J1 * (-inv2pi * nu);
                Bd = (cmul_i(kk) * b1.J1 * 0.25 - kk * (nc.logk2 + mk(lr, 0.0)) * b1.J1 * inv2pi -
                      kk * b1.Yh1 * 0.25) * nu + mk(nu / (2.0 * kPi * R), 0.0);
                Bt = (cmul_i(c.kt) * b2.J1 * 0.25 -
                      c.kt * (nc.logkt2 + mk(lr, 0.0)) * b2.J1 * inv2pi - c.kt * b2.Yh1 * 0.25) *
                         nu + mk(nu / (2.0 * kPi * R), 0.0);
            }
            // log h goes with the smooth part
            Bg = Bg + Ag * nc.logh;
            Bs = Bs + As * nc.logh;
            Bd = Bd + Ad * nc.logh;
            Bt = Bt + At * nc.logh;
            double hw = h * h * wgt * pa * pb;
            double hm = h * h * mab;
            acc[0] = acc[0] + Bd * hw + Ad * hm;
            acc[2] = acc[2] + Bt * hw + At * hm;
            acc[3] = acc[3] + Bs * hw + As * hm;
            acc[1] = acc[1] + Bg * (wgt * sab - k2 * nn * hw) + Ag * (sab * m0 - k2 * nn * hm);
        }
    }
}

__global__ __launch_bounds__(256) void k_near(int N, NearConsts nc, int q, int nb, int r0,
                                              int r1, int64_t ld, zd *o0, zd *o1, zd *o2,
                                              zd *o3, const double *__restrict__ PX,
                                              const double *__restrict__ PY,
                                              const double *__restrict__ PTX,
                                              const double *__restrict__ PTY,
                                              const double *__restrict__ PCV,
                                              const double *__restrict__ mom) {
    int nrows = r1 - r0;
    int ndiag = 2 * nb + 3;
    long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= (long)nrows * ndiag) return;
    int i = r0 + (int)(tid % nrows);
    int delta = (int)(tid / nrows) - (nb + 1);
    // skip duplicate diagonals when the band wraps around a small mesh
    if (2 * (nb + 1) + 1 > N) {
        int dd = ((delta % N) + N) % N;
        // keep the representative delta in [-(N-1)/2, N/2]
        int rep = dd > N / 2 ? dd - N : dd;
        if (rep != delta) return;
    }
    int j = ((i + delta) % N + N) % N;
    zd acc[4] = {mk(0.0, 0.0), mk(0.0, 0.0), mk(0.0, 0.0), mk(0.0, 0.0)};
    for (int p = 0; p < 4; ++p) {
        int a = (p >> 1) ? 0 : 1;                       // p = 0,1: element i-1 (a = 1)
        int b = (p & 1) ? 0 : 1;                        // p = 0,2: element j-1 (b = 1)
        int e = a ? i - 1 : i;
        int f = b ? j - 1 : j;
        e = (e + N) % N;
        f = (f + N) % N;
        int off = ((f - e) % N + N) % N;
        int kind;
        if (off == 0) kind = 0;
        else if (off == 1) kind = 1;
        else if (off == N - 1) kind = 2;
        else kind = -1;
        near_pair(nc, q, e, f, kind, a, b, PX, PY, PTX, PTY, PCV, mom, acc);
    }
    int64_t idx = (int64_t)i + (int64_t)j * ld;
    o0[idx] = acc[0];
    o1[idx] = acc[1];
    o2[idx] = acc[2];
    o3[idx] = acc[3];
}

void launch_assemble_near(const AsmParams &p, const PointTable &near, const double *xi,
                          const double *w, const double *moments, hipStream_t s) {
    NearConsts nc;
    nc.pc = make_consts(p.kc);
    nc.h = p.h;
    nc.logh = std::log(p.h);
    nc.logk2 = clog(mk(p.kc.k * 0.5, 0.0));
    nc.logkt2 = clog(p.kc.kt * 0.5);
    for (int i = 0; i < near.q && i < kMaxQNear; ++i) {
        nc.xi[i] = xi[i];
        nc.w[i] = w[i];
    }
    int nrows = p.r1 - p.r0;
    long n = (long)nrows * (2 * p.nb + 3);
    int bs = 64;
    ProfScope prof(PROF_NEAR, 4.0 * n * near.q * near.q, s);
    hipLaunchKernelGGL(k_near, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, s, p.N, nc,
                       near.q, p.nb, p.r0, p.r1, p.ld, p.out[0], p.out[1], p.out[2], p.out[3],
                       near.x, near.y, near.tx, near.ty, near.curv, moments);
}

// ------------------------------------------------------------------ excitation -----------
// e'_i = int lambda_i (d.n) e^{ik d.r} ds,  h_i = int lambda_i e^{ik d.r} ds  (Sec. II)
__global__ void k_excitation(int N, int q, double h, double k, const double *__restrict__ PX,
                             const double *__restrict__ PY, const double *__restrict__ PTX,
                             const double *__restrict__ PTY, const double *xi, const double *w,
                             const double *angles, int64_t m, zd *E, zd *H, int64_t ld) {
    long tid = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= (long)N * m) return;
    int i = (int)(tid % N);
    int64_t jc = tid / N;
    double sa, ca;
    sincos(angles[jc], &sa, &ca);
    zd ev = mk(0.0, 0.0), hv = mk(0.0, 0.0);
    for (int side = 0; side < 2; ++side) {
        int e = side == 0 ? (i - 1 + N) % N : i;        // element i-1 (a = 1) or i (a = 0)
        for (int g = 0; g < q; ++g) {
            int idx = e * q + g;
            double phi = side == 0 ? xi[g] : 1.0 - xi[g];
            double wt = h * w[g] * phi;
            double ph = k * (ca * PX[idx] + sa * PY[idx]);
            double sn, cs;
            sincos(ph, &sn, &cs);
            double dn = ca * PTY[idx] - sa * PTX[idx];  // d.n with n = (ty, -tx)
            hv = hv + mk(cs, sn) * wt;
            ev = ev + mk(cs, sn) * (wt * dn);
        }
    }
    E[i + jc * ld] = ev;
    H[i + jc * ld] = hv;
}

void launch_excitation(const GeomDev &g, const PointTable &pt, const double *xi,
                       const double *w, double k, const double *angles, int64_t m, zd *e,
                       zd *hvec, int64_t ld, hipStream_t s) {
    long n = (long)g.N * m;
    int bs = 256;
    hipLaunchKernelGGL(k_excitation, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, s, g.N,
                       pt.q, g.h, k, pt.x, pt.y, pt.tx, pt.ty, xi, w, angles, m, e, hvec, ld);
}

}  // namespace cfie
