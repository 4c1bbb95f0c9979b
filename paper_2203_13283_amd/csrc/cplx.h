// Minimal complex arithmetic usable in host and device code.  Values are stored as
// interleaved (re, im) pairs, the layout of complex128 / complex64 arrays in memory.
#pragma once
#include <cmath>

#if defined(__HIPCC__) || defined(__HIP__)
#include <hip/hip_runtime.h>
#define CFIE_HD __host__ __device__ __forceinline__
#else
#define CFIE_HD inline
#endif

namespace cfie {

template <typename T>
struct cpx {
    T x, y;
};
using zd = cpx<double>;
using zf = cpx<float>;

template <typename T> CFIE_HD cpx<T> mk(T a, T b) { return cpx<T>{a, b}; }
template <typename T> CFIE_HD cpx<T> operator+(cpx<T> a, cpx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T> CFIE_HD cpx<T> operator-(cpx<T> a, cpx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T> CFIE_HD cpx<T> operator-(cpx<T> a) { return {-a.x, -a.y}; }
template <typename T> CFIE_HD cpx<T> operator*(cpx<T> a, cpx<T> b) {
    return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T> CFIE_HD cpx<T> operator*(cpx<T> a, T s) { return {a.x * s, a.y * s}; }
template <typename T> CFIE_HD cpx<T> operator*(T s, cpx<T> a) { return {a.x * s, a.y * s}; }
template <typename T> CFIE_HD cpx<T> conj(cpx<T> a) { return {a.x, -a.y}; }
template <typename T> CFIE_HD T abs2(cpx<T> a) { return a.x * a.x + a.y * a.y; }
template <typename T> CFIE_HD cpx<T> cmul_i(cpx<T> a) { return {-a.y, a.x}; }   // i * a
// a += b * c
template <typename T> CFIE_HD void cfma(cpx<T> &a, cpx<T> b, cpx<T> c) {
    a.x = std::fma(b.x, c.x, a.x);
    a.x = std::fma(-b.y, c.y, a.x);
    a.y = std::fma(b.x, c.y, a.y);
    a.y = std::fma(b.y, c.x, a.y);
}
template <typename T> CFIE_HD cpx<T> cinv(cpx<T> a) {
    // scaled to avoid overflow of |a|^2 for large entries
    T s = std::fabs(a.x) > std::fabs(a.y) ? std::fabs(a.x) : std::fabs(a.y);
    T ax = a.x / s, ay = a.y / s;
    T d = s * (ax * ax + ay * ay);
    return {ax / d, -ay / d};
}
template <typename T> CFIE_HD cpx<T> cdiv(cpx<T> a, cpx<T> b) { return a * cinv(b); }
CFIE_HD double cabs(zd a) { return std::hypot(a.x, a.y); }
// principal square root
CFIE_HD zd csqrt(zd a) {
    double r = std::hypot(a.x, a.y);
    if (r == 0.0) return {0.0, 0.0};
    if (a.x >= 0.0) {
        double t = std::sqrt(0.5 * (r + a.x));
        return {t, a.y / (2.0 * t)};
    }
    double t = std::sqrt(0.5 * (r - a.x));
    return {std::fabs(a.y) / (2.0 * t), a.y >= 0.0 ? t : -t};
}
// principal logarithm
CFIE_HD zd clog(zd a) { return {std::log(std::hypot(a.x, a.y)), std::atan2(a.y, a.x)}; }

}  // namespace cfie
