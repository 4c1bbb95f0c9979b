// Host build of the device Bessel/Hankel routines, for CPU tests only.
#include "../paper_2203_13283_amd/csrc/bessel.h"
using namespace cfie;
extern "C" void hb_hankel01(int n, const double *z, double *out) {
    for (int i = 0; i < n; ++i) {
        zd H0, H1;
        hankel01(mk(z[2 * i], z[2 * i + 1]), H0, H1);
        out[4 * i] = H0.x; out[4 * i + 1] = H0.y; out[4 * i + 2] = H1.x; out[4 * i + 3] = H1.y;
    }
}
extern "C" void hb_split(int n, const double *z, double *out) {
    for (int i = 0; i < n; ++i) {
        BesselSplit b = bessel_split(mk(z[2 * i], z[2 * i + 1]));
        double *o = out + 8 * i;
        o[0] = b.J0.x; o[1] = b.J0.y; o[2] = b.J1.x; o[3] = b.J1.y;
        o[4] = b.Yh0.x; o[5] = b.Yh0.y; o[6] = b.Yh1.x; o[7] = b.Yh1.y;
    }
}
extern "C" void hb_asym(int n, const double *z, double *out) {
    for (int i = 0; i < n; ++i) {
        zd H0, H1;
        hankel_asym(mk(z[2 * i], z[2 * i + 1]), H0, H1);
        out[4 * i] = H0.x; out[4 * i + 1] = H0.y; out[4 * i + 2] = H1.x; out[4 * i + 3] = H1.y;
    }
}
extern "C" void hb_miller(int n, const double *z, double *out) {
    for (int i = 0; i < n; ++i) {
        BesselSplit b = bessel_miller(mk(z[2 * i], z[2 * i + 1]));
        zd H0, H1;
        hankel_from_split(mk(z[2 * i], z[2 * i + 1]), b, H0, H1);
        out[4 * i] = H0.x; out[4 * i + 1] = H0.y; out[4 * i + 2] = H1.x; out[4 * i + 3] = H1.y;
    }
}
