// Bessel and Hankel functions of order 0 and 1 for complex argument z with Re z > 0 and
// small Im z >= 0 (z = kappa R, kappa = k or k + i beta).  Host and device code.
//
// The Green's function of the paper is g_k(R) = (i/4) H0^(1)(k R) (Sec. II); its normal
// derivative brings in H1^(1).  Three regimes:
//   |z| <  SERIES_MAX : ascending series (DLMF 10.2.2, 10.8.1, 10.8.2)
//   |z| <  ASYM_MIN   : Miller's backward recurrence for J_n, normalised by
//                       J_0 + 2 sum J_2k = 1, with Neumann series for Y_0 and Y_1
//                       (expansions of log(z/2) J_0 in J_2k, see bessel_miller)
//   otherwise         : Hankel's large-argument expansion (DLMF 10.17.5), summed until the
//                       terms drop below 1e-17.
// The "split" form returns the pieces used for the singular Galerkin integrals:
//   Y0(z) = (2/pi) log(z/2) J0(z) + Yh0(z)
//   Y1(z) = (2/pi) log(z/2) J1(z) - 2/(pi z) + Yh1(z)
// with Yh0, Yh1 entire functions, so that the logarithm can be integrated exactly.
#pragma once
#include "cplx.h"

namespace cfie {

constexpr double kPi = 3.14159265358979323846;
constexpr double kEulerGamma = 0.57721566490153286061;
constexpr double kSeriesMax = 5.0;
constexpr double kAsymMin = 22.0;

struct BesselSplit {
    zd J0, J1, Yh0, Yh1;
};

// Ascending series.  t_k = (-z^2/4)^k / (k!)^2,  u_k = (-z^2/4)^k / (k!(k+1)!).
//   J0 = sum t_k,  J1 = (z/2) sum u_k
//   Yh0 = (2/pi) gamma J0 - (2/pi) sum_{k>=1} H_k t_k
//   Yh1 = -(z/(2 pi)) sum_{k>=0} (psi(k+1) + psi(k+2)) u_k,  psi(n+1) = -gamma + H_n
CFIE_HD BesselSplit bessel_series(zd z) {
    zd q = z * z * (-0.25);
    zd t = mk(1.0, 0.0), u = mk(1.0, 0.0);
    zd sJ0 = t, sJ1 = u, sY0 = mk(0.0, 0.0);
    double Hk = 0.0;                                     // H_k
    zd sY1 = u * (-2.0 * kEulerGamma + 1.0);             // k = 0: psi(1)+psi(2) = -2g+1
    for (int k = 1; k < 40; ++k) {
        double dk = (double)k;
        t = t * q * (1.0 / (dk * dk));
        u = u * q * (1.0 / (dk * (dk + 1.0)));
        Hk += 1.0 / dk;
        sJ0 = sJ0 + t;
        sJ1 = sJ1 + u;
        sY0 = sY0 + t * Hk;
        sY1 = sY1 + u * (-2.0 * kEulerGamma + 2.0 * Hk + 1.0 / (dk + 1.0));
        if (abs2(t) + abs2(u) < 1e-36 * (abs2(sJ0) + abs2(sJ1) + 1e-300)) break;
    }
    BesselSplit r;
    r.J0 = sJ0;
    r.J1 = sJ1 * z * 0.5;
    r.Yh0 = sJ0 * (2.0 / kPi * kEulerGamma) - sY0 * (2.0 / kPi);
    r.Yh1 = sY1 * z * (-0.5 / kPi);
    return r;
}

// Miller's backward recurrence f_{n-1} = (2n/z) f_n - f_{n+1} from an even start index
// well above |z|; f_n / S with S = f_0 + 2 sum f_{2k} gives J_n.  Neumann series
//   Y0 = (2/pi)(log(z/2) + gamma) J0 - (4/pi) sum_{k>=1} (-1)^k J_{2k} / k
//   Y1 = -Y0' = -(2/(pi z)) J0 + (2/pi)(log(z/2) + gamma) J1
//               + (2/pi) sum_{k>=1} (-1)^k (J_{2k-1} - J_{2k+1}) / k
CFIE_HD BesselSplit bessel_miller(zd z) {
    double az = cabs(z);
    int n0 = 2 * (int)((az + 26.0 + 4.0 * cbrt(az)) * 0.5);
    zd w = cinv(z) * 2.0;                                // 2 / z
    zd fp1 = mk(0.0, 0.0);                               // f_{n+1}
    zd f = mk(1e-200, 0.0);                              // f_n, n = n0
    zd S = mk(0.0, 0.0), Sy0 = mk(0.0, 0.0), Sy1 = mk(0.0, 0.0);
    // n runs from n0 down to 1; at each step produce f_{n-1}
    for (int n = n0; n >= 1; --n) {
        if ((n & 1) == 0) {
            // f currently holds f_n with n even >= 2
            int kk = n / 2;
            double sgn = (kk & 1) ? -1.0 : 1.0;
            S = S + f * 2.0;
            Sy0 = Sy0 + f * (sgn / (double)kk);
            // f_{2k+1} is fp1, f_{2k-1} arrives next step; store pieces
            Sy1 = Sy1 - fp1 * (sgn / (double)kk);
        } else {
            // f holds f_n with n odd = 2k-1 -> contributes to the term of k = (n+1)/2
            int kk = (n + 1) / 2;
            double sgn = (kk & 1) ? -1.0 : 1.0;
            Sy1 = Sy1 + f * (sgn / (double)kk);
        }
        zd fm1 = w * f * (double)n - fp1;
        fp1 = f;
        f = fm1;
        if (abs2(f) > 1e200) {                          // rescale to stay in range
            double s = 1e-100;
            f = f * s; fp1 = fp1 * s; S = S * s; Sy0 = Sy0 * s; Sy1 = Sy1 * s;
        }
    }
    // now f = f_0, fp1 = f_1
    S = S + f;
    zd inv = cinv(S);
    BesselSplit r;
    r.J0 = f * inv;
    r.J1 = fp1 * inv;
    // Yh0 = Y0 - (2/pi) log(z/2) J0 = (2/pi) gamma J0 - (4/pi) sum (-1)^k J_2k / k
    r.Yh0 = r.J0 * (2.0 / kPi * kEulerGamma) - Sy0 * inv * (4.0 / kPi);
    // Yh1 = Y1 - (2/pi) log(z/2) J1 + 2/(pi z)
    //     = (2/pi) gamma J1 + (2/(pi z)) (1 - J0) + (2/pi) sum (-1)^k (J_{2k-1}-J_{2k+1})/k
    zd one_m_J0 = mk(1.0, 0.0) - r.J0;
    r.Yh1 = r.J1 * (2.0 / kPi * kEulerGamma) + w * one_m_J0 * (1.0 / kPi) +
            Sy1 * inv * (2.0 / kPi);
    return r;
}

CFIE_HD BesselSplit bessel_split(zd z) {
    return cabs(z) < kSeriesMax ? bessel_series(z) : bessel_miller(z);
}

// H0 and H1 from the split form: H = J + i Y.
CFIE_HD void hankel_from_split(zd z, const BesselSplit &b, zd &H0, zd &H1) {
    zd lg = clog(z * 0.5) * (2.0 / kPi);
    zd Y0 = lg * b.J0 + b.Yh0;
    zd Y1 = lg * b.J1 - cinv(z) * (2.0 / kPi) + b.Yh1;
    H0 = b.J0 + cmul_i(Y0);
    H1 = b.J1 + cmul_i(Y1);
}

// Hankel's expansion: H_nu(z) = sqrt(2/(pi z)) e^{i(z - nu pi/2 - pi/4)} sum a_k(nu) (i/z)^k,
// a_0 = 1, a_k / a_{k-1} = (4 nu^2 - (2k-1)^2) / (8k).
CFIE_HD void hankel_asym(zd z, zd &H0, zd &H1) {
    zd w = cmul_i(cinv(z));
    zd t0 = mk(1.0, 0.0), t1 = mk(1.0, 0.0);
    zd s0 = t0, s1 = t1;
    for (int k = 1; k < 64; ++k) {
        double m = (double)(2 * k - 1);
        t0 = t0 * w * ((0.0 - m * m) / (8.0 * k));
        t1 = t1 * w * ((4.0 - m * m) / (8.0 * k));
        s0 = s0 + t0;
        s1 = s1 + t1;
        if (abs2(t0) + abs2(t1) < 1e-34) break;
    }
    zd pre = csqrt(cinv(z) * (2.0 / kPi));
    double ez = exp(-z.y);
    double sn, cs;
#if defined(__HIP_DEVICE_COMPILE__)
    sincos(z.x, &sn, &cs);
#else
    sn = std::sin(z.x);
    cs = std::cos(z.x);
#endif
    // e^{i(z - pi/4)} = e^{iz} (1 - i)/sqrt(2); the shift is applied after the sincos so
    // that it adds no rounding to a large argument
    const double r2 = 0.70710678118654752440;
    zd ph = mk((cs + sn) * r2 * ez, (sn - cs) * r2 * ez);
    zd p0 = pre * ph;
    H0 = p0 * s0;
    H1 = mk(p0.y, -p0.x) * s1;                          // times e^{-i pi/2} = -i
}

CFIE_HD void hankel01(zd z, zd &H0, zd &H1) {
    if (cabs(z) >= kAsymMin) {
        hankel_asym(z, H0, H1);
    } else {
        BesselSplit b = bessel_split(z);
        hankel_from_split(z, b, H0, H1);
    }
}

}  // namespace cfie
