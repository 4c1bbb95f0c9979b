// Device-side pieces shared by the assembly and its reverse-mode derivative: the
// parameter t(s) of arc length s on the contour, the contour and its derivatives, and the
// point-pair Hankel kernels of the Galerkin integrals (Sec. II eqs. (2)-(4)).
#pragma once
#include <hip/hip_runtime.h>

#include "internal.h"

namespace cfie {

// t with s(t) = s, s(t) = c0 t + 2 Re sum_{m=1..Ms} c_m (e^{imt} - 1) / (im) (the arc length
// of the Fourier series of the speed |z'(t)|), by Newton's method from t = 2 pi s / L.
__device__ __forceinline__ double arc_param(double s, double L, double c0, int Ms,
                                            const zd *cm) {
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
    return t;
}

// z(t) = sum_{m=-M..M} zhat_m e^{imt} and its first three derivatives
__device__ __forceinline__ void contour_derivs(double t, int M, const zd *zhat, zd &z, zd &d1,
                                               zd &d2, zd &d3) {
    double sn, cs;
    sincos(t, &sn, &cs);
    zd E1 = mk(cs, sn);
    sincos(-(double)M * t, &sn, &cs);
    zd E = mk(cs, sn);
    z = d1 = d2 = d3 = mk(0.0, 0.0);
    for (int m = -M; m <= M; ++m) {
        zd v = zhat[m + M] * E;
        double dm = (double)m;
        z = z + v;
        d1 = d1 + cmul_i(v) * dm;
        d2 = d2 - v * (dm * dm);
        d3 = d3 - cmul_i(v) * (dm * dm * dm);
        E = E * E1;
    }
}

// ------------------------------------------------------------------ kernel values ---------
// Large-argument Hankel expansion (DLMF 10.17.5): H_nu(z) = sqrt(2/(pi z)) e^{i(z - nu pi/2 -
// pi/4)} F_nu(z), F_nu(z) = sum_n a_n(nu) (i/z)^n, a_n(nu) = prod_{j<=n} (4nu^2 - (2j-1)^2)/(8j).
// Truncated after T terms: T = 8, 12, 22 keep the first omitted term below 3e-17 relative for
// |z| >= 200, 50, 22.  For the real argument x = k R the even and odd terms give F = P + i Q
// with P, Q polynomials in 1/x^2; for kt R the series is a complex Horner in w = i/(kt R).
// The coefficients are compile-time constants.
constexpr int kSerMax = 22;
struct SerCoef {
    double a[2][kSerMax];            // a_n(nu)
    double p[2][kSerMax / 2];        // (-1)^j a_2j(nu)
    double q[2][kSerMax / 2];        // (-1)^j a_2j+1(nu)
};
constexpr SerCoef make_ser() {
    SerCoef c{};
    for (int nu = 0; nu < 2; ++nu) {
        double an = 1.0;
        for (int n = 0; n < kSerMax; ++n) {
            if (n > 0) {
                double m = (double)(2 * n - 1);
                an *= (4.0 * nu * nu - m * m) / (8.0 * n);
            }
            c.a[nu][n] = an;
            double sg = ((n / 2) % 2) ? -1.0 : 1.0;
            if (n % 2 == 0) c.p[nu][n / 2] = sg * an;
            else c.q[nu][n / 2] = sg * an;
        }
    }
    return c;
}
constexpr SerCoef kSer = make_ser();

struct PairConsts {
    double k, beta, invk;            // kt = k + i beta
    zd kt, iwk;                      // iwk = i / kt
    zd Cg, CD, CS, CDt;              // prefactors of the large-argument forms
    zd ik4, ikt4;                    // i k / 4, i kt / 4
};

// p x + c for a Horner step whose coefficient c is a loop-invariant value: one three-address
// FMA (the coefficient stays in its register; the two-address form would first copy it into
// the destination)
__device__ __forceinline__ double horner(double p, double x, double c) {
    double r;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(p), "v"(x), "v"(c));
    return r;
}

// sin and cos of a phase x with |x| < 2^20 (the far kernels' k R: a contour of N <= 32768
// nodes at 0.8 or more nodes per wavelength spans less than 2^17 radians): Cody and Waite's
// reduction r = x - n pi/2 with n = rint(2 x / pi) and pi/2 split into three parts, the first
// two with 33 significant bits so that n times them is exact, then the Taylor series of sin
// (through r^15) and cos (through r^16) on |r| <= pi/4, whose first omitted terms are below
// 5e-17 and 2e-18, and the quadrant n mod 4.
__device__ __forceinline__ void sincos_phase(double x, double &s, double &c) {
    constexpr double kP1 = 0x1.921fb544p+0, kP2 = 0x1.0b4611a6p-34,
                     kP3 = 0x1.3198a2e037073p-69;
    const double n = rint(x * 0.63661977236758134308);
    double r = fma(-n, kP1, x);
    r = fma(-n, kP2, r);
    r = fma(-n, kP3, r);
    const double r2 = r * r;
    double ps = -1.0 / 1307674368000.0;
    ps = horner(ps, r2, 1.0 / 6227020800.0);
    ps = horner(ps, r2, -1.0 / 39916800.0);
    ps = horner(ps, r2, 1.0 / 362880.0);
    ps = horner(ps, r2, -1.0 / 5040.0);
    ps = horner(ps, r2, 1.0 / 120.0);
    ps = horner(ps, r2, -1.0 / 6.0);
    const double sr = fma(ps * r2, r, r);
    double pc = 1.0 / 20922789888000.0;
    pc = horner(pc, r2, -1.0 / 87178291200.0);
    pc = horner(pc, r2, 1.0 / 479001600.0);
    pc = horner(pc, r2, -1.0 / 3628800.0);
    pc = horner(pc, r2, 1.0 / 40320.0);
    pc = horner(pc, r2, -1.0 / 720.0);
    pc = horner(pc, r2, 1.0 / 24.0);
    pc = fma(pc, r2, -0.5);
    const double cr = fma(pc, r2, 1.0);
    const int q = (int)n & 3;
    const double a = (q & 1) ? cr : sr, b = (q & 1) ? sr : cr;
    s = (q & 2) ? -a : a;
    c = ((q + 1) & 2) ? -b : b;
}

// 1/sqrt(x) for positive, finite, normal x: the hardware estimate y refined by one step of
// the second-order iteration y (1 + e/2 + 3 e^2/8), e = 1 - x y^2, whose error is about the
// cube of the estimate's; the checks for zero, infinity and denormals are left out.
__device__ __forceinline__ double rsqrt_pos(double x) {
    const double y = __builtin_amdgcn_rsq(x);
    const double e = fma(-x * y, y, 1.0);
    return fma(y * e, fma(e, 0.375, 0.5), y);
}

// e^x for x <= 0 (the decay e^{-beta R} of the complex wavenumber's kernels): Cody and
// Waite's reduction x = n ln 2 + r, |r| <= ln 2 / 2, with ln 2 split so that n times its
// leading part (28 significant bits) is exact, then e^r by its Taylor series to r^13 (the
// remainder is below 1e-17 relative) and the scaling by 2^n.  x <= 0 needs no overflow
// handling, and the scaling flushes x below about -745 to zero.
__device__ __forceinline__ double exp_decay(double x) {
    constexpr double kL2E = 0x1.71547652b82fep+0, kLn2Hi = 0x1.62e42ff000000p-1,
                     kLn2Lo = -0x1.718432a1b0e26p-35;
    const double n = rint(x * kL2E);
    double r = fma(-n, kLn2Hi, x);
    r = fma(-n, kLn2Lo, r);
    double p = 1.0 / 6227020800.0;
    p = horner(p, r, 1.0 / 479001600.0);
    p = horner(p, r, 1.0 / 39916800.0);
    p = horner(p, r, 1.0 / 3628800.0);
    p = horner(p, r, 1.0 / 362880.0);
    p = horner(p, r, 1.0 / 40320.0);
    p = horner(p, r, 1.0 / 5040.0);
    p = horner(p, r, 1.0 / 720.0);
    p = horner(p, r, 1.0 / 120.0);
    p = horner(p, r, 1.0 / 24.0);
    p = horner(p, r, 1.0 / 6.0);
    p = fma(p, r, 0.5);
    p = fma(p, r, 1.0);
    p = fma(p, r, 1.0);
    return ldexp(p, (int)n);
}

// Large-argument kernels (k R >= 22 for this lane) with a T-term series, given R and 1/R,
// without their constant prefactors: gk / Cg, Dk / CD, St / CS, Dt / CDt (a sum of such
// values over point pairs is multiplied by the prefactor once).
template <int T>
__device__ __forceinline__ void pair_kernels_asym_unscaled(const PairConsts &c, double R,
                                                           double invR, double nu, zd &gk,
                                                           zd &Dk, zd &St, zd &Dt) {
    double sn, cs;
    sincos_phase(c.k * R, sn, cs);
    const double rs = rsqrt_pos(R);
    const zd E = mk(cs * rs, sn * rs);                   // e^{ikR} R^{-1/2}
    const zd Et = E * exp_decay(-c.beta * R);
    const double y = invR * c.invk, y2 = y * y;
    double P0 = kSer.p[0][T / 2 - 1], Q0 = kSer.q[0][T / 2 - 1];
    double P1 = kSer.p[1][T / 2 - 1], Q1 = kSer.q[1][T / 2 - 1];
#pragma unroll
    for (int j = T / 2 - 2; j >= 0; --j) {
        P0 = fma(P0, y2, kSer.p[0][j]);
        Q0 = fma(Q0, y2, kSer.q[0][j]);
        P1 = fma(P1, y2, kSer.p[1][j]);
        Q1 = fma(Q1, y2, kSer.q[1][j]);
    }
    const zd w = c.iwk * invR;                           // i / (kt R)
    // s0, s1 = sum_n a_n w^n with real a_n, by the second-order recurrence for a real
    // polynomial at a complex point (Knuth, TAOCP vol. 2, sec. 4.6.4): w is a root of
    // t^2 - r t + q with r = 2 Re w, q = |w|^2; b_k = a_k + r b_{k+1} - q b_{k+2} gives the
    // remainder b_1 t + a_0 - q b_2 of the division by that quadratic, so
    // p(w) = (Re w) b_1 + a_0 - q b_2 + i (Im w) b_1: two real operations per term instead
    // of the four of a complex Horner step.
    static_assert(T >= 3, "series too short for the recurrence");
    const double rr = 2.0 * w.x, mq = -fma(w.x, w.x, w.y * w.y);
    // (u2, u1) = (b_k, b_{k+1}), from k = T - 2 down to k = 1 (b_{T-1} = a_{T-1}, b_T = 0)
    double u1 = kSer.a[0][T - 1], v1 = kSer.a[1][T - 1];
    double u2 = fma(rr, u1, kSer.a[0][T - 2]), v2 = fma(rr, v1, kSer.a[1][T - 2]);
#pragma unroll
    for (int n = T - 3; n >= 1; --n) {
        const double u = fma(rr, u2, fma(mq, u1, kSer.a[0][n]));
        const double v = fma(rr, v2, fma(mq, v1, kSer.a[1][n]));
        u1 = u2;
        u2 = u;
        v1 = v2;
        v2 = v;
    }
    // u2 = b_1, u1 = b_2
    const zd s0 = mk(fma(w.x, u2, fma(mq, u1, kSer.a[0][0])), w.y * u2);
    const zd s1 = mk(fma(w.x, v2, fma(mq, v1, kSer.a[1][0])), w.y * v2);
    gk = E * mk(P0, Q0 * y);
    Dk = E * mk(P1 * nu, Q1 * y * nu);
    St = Et * s0;
    Dt = Et * (s1 * nu);
}
// the same with the prefactors
template <int T>
__device__ __forceinline__ void pair_kernels_asym(const PairConsts &c, double R, double invR,
                                                  double nu, zd &gk, zd &Dk, zd &St, zd &Dt) {
    pair_kernels_asym_unscaled<T>(c, R, invR, nu, gk, Dk, St, Dt);
    gk = c.Cg * gk;
    Dk = c.CD * Dk;
    St = c.CS * St;
    Dt = c.CDt * Dt;
}
template <int T>
__device__ __forceinline__ void pair_kernels_asym(const PairConsts &c, double R, double nu,
                                                  zd &gk, zd &Dk, zd &St, zd &Dt) {
    pair_kernels_asym<T>(c, R, 1.0 / R, nu, gk, Dk, St, Dt);
}

// Any argument: ascending series / Miller recurrence below k R = 22 (kept out of line so
// that the register allocation of the far kernel's main loop is not sized for it).
static __device__ __attribute__((noinline)) void pair_kernels_small(const PairConsts &c, double R,
                                                             double nu, zd &gk, zd &Dk,
                                                             zd &St, zd &Dt) {
    zd H0, H1;
    hankel01(mk(c.k * R, 0.0), H0, H1);
    gk = cmul_i(H0) * 0.25;
    Dk = c.ik4 * H1 * nu;
    hankel01(c.kt * R, H0, H1);
    St = cmul_i(H0) * 0.25;
    Dt = c.ikt4 * H1 * nu;
}

// Point-pair kernels: gk = (i/4) H0(kR), Dk = (ik/4) H1(kR) nu, St = (i/4) H0(ktR),
// Dt = (ikt/4) H1(ktR) nu, with nu = (r - r').n' / R.  Per-thread choice of the form.
__device__ __forceinline__ void pair_kernels(const PairConsts &c, double R, double nu,
                                             zd &gk, zd &Dk, zd &St, zd &Dt) {
    const double kR = c.k * R;
    if (kR >= 200.0) pair_kernels_asym<8>(c, R, nu, gk, Dk, St, Dt);
    else if (kR >= 50.0) pair_kernels_asym<12>(c, R, nu, gk, Dk, St, Dt);
    else if (kR >= kAsymMin) pair_kernels_asym<kSerMax>(c, R, nu, gk, Dk, St, Dt);
    else pair_kernels_small(c, R, nu, gk, Dk, St, Dt);
}

static inline PairConsts make_consts(const KernelConsts &kc) {
    PairConsts c;
    c.k = kc.k;
    c.kt = kc.kt;
    c.beta = kc.kt.y;
    c.invk = 1.0 / kc.k;
    c.iwk = cmul_i(cinv(kc.kt));
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

// Lower bound of k R over the Gauss point pairs of two elements whose reference points
// (Gauss point Q/2, within arc length h of every Gauss point of its element) are dxr, dyr
// apart.  Rounded operations only, so that both far passes take the same decision.
__device__ __forceinline__ double far_kRmin(double k, double h, double dxr, double dyr) {
    return __dmul_rn(k, __dsub_rn(__dsqrt_rn(__dadd_rn(__dmul_rn(dxr, dxr), __dmul_rn(dyr, dyr))),
                                  __dmul_rn(2.0, h)));
}
constexpr double kFarFast = 200.0;    // k R above which the 8-term series is used

// Whether no element pair of a wavefront's tile can need the 22-term or small-argument
// passes: every lane holds one row element's reference point (xr, yr) and two column
// elements' (xa, ya), (xb, yb).  Bounding circles of the two sets (centroid, largest
// distance to it) bound every reference-point distance of the tile from below by D, and
// k (D - 2h) >= kFarFast (with a margin far above the rounding of D) means far_kRmin >=
// kFarFast for every pair of the tile.  The result is the same on all lanes.
__device__ __forceinline__ bool far_tile_all_fast(double k, double h, double xr, double yr,
                                                  double xa, double ya, double xb, double yb) {
    auto wsum = [](double v) {
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
        return v;
    };
    auto wmax = [](double v) {
        for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
        return v;
    };
    const double rcx = wsum(xr) * (1.0 / 64), rcy = wsum(yr) * (1.0 / 64);
    const double rr = wmax(sqrt((xr - rcx) * (xr - rcx) + (yr - rcy) * (yr - rcy)));
    const double ccx = wsum(xa + xb) * (1.0 / 128), ccy = wsum(ya + yb) * (1.0 / 128);
    const double rc = wmax(fmax(sqrt((xa - ccx) * (xa - ccx) + (ya - ccy) * (ya - ccy)),
                                sqrt((xb - ccx) * (xb - ccx) + (yb - ccy) * (yb - ccy))));
    const double D = sqrt((rcx - ccx) * (rcx - ccx) + (rcy - ccy) * (rcy - ccy)) - rr - rc;
    return k * (D - 2.0 * h) >= kFarFast + 1e-6;
}

}  // namespace cfie
