// Host-side geometry of the contour and constant quadrature tables.
//
// The paper discretises gamma and its equivalent circle gamma_c with hat functions that
// are piecewise linear in the curvilinear abscissa, on the same uniform arc-length mesh
// (Sec. V), so that the Gram matrices coincide.  Here the curve is a trigonometric
// polynomial; its arc-length density |z'(t)| is expanded in a Fourier series (sampled on a
// fine grid and transformed), which gives s(t) in closed form for the device-side Newton
// inversion t(s).
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <string>
#include <vector>

#include "internal.h"

namespace cfie {

namespace {

zd zeval(const std::vector<zd> &zh, int M, double t, int deriv) {
    zd acc = mk(0.0, 0.0);
    for (int m = -M; m <= M; ++m) {
        double s = std::sin(m * t), c = std::cos(m * t);
        zd e = mk(c, s);
        zd v = zh[m + M] * e;
        if (deriv == 1) v = cmul_i(v) * (double)m;
        if (deriv == 2) v = v * (-(double)m * (double)m);
        acc = acc + v;
    }
    return acc;
}

bool seg_intersect(zd a, zd b, zd c, zd d) {
    auto cross = [](zd u, zd v) { return u.x * v.y - u.y * v.x; };
    zd r = b - a, s = d - c, ca = c - a;
    double den = cross(r, s);
    if (den == 0.0) return false;
    double t = cross(ca, s) / den, u = cross(ca, r) / den;
    return t > 0.0 && t < 1.0 && u > 0.0 && u < 1.0;
}

// Whether two edges of the closed polygon p that do not share a vertex cross.  The edges are
// put into the cells of a uniform grid that their bounding boxes overlap (cells about two
// mean edge lengths wide, at most about 4 cells per edge), and only edges sharing a cell are
// tested against each other: linear work for a smooth curve instead of all pairs.
bool polygon_self_intersects(const std::vector<zd> &p) {
    const int64_t Q = (int64_t)p.size();
    if (Q < 4) return false;
    double x0 = p[0].x, x1 = p[0].x, y0 = p[0].y, y1 = p[0].y, len = 0.0;
    for (int64_t j = 0; j < Q; ++j) {
        x0 = std::fmin(x0, p[j].x);
        x1 = std::fmax(x1, p[j].x);
        y0 = std::fmin(y0, p[j].y);
        y1 = std::fmax(y1, p[j].y);
        len += cabs(p[(j + 1) % Q] - p[j]);
    }
    double cell = std::fmax(2.0 * len / (double)Q, 1e-300);
    while (((x1 - x0) / cell + 1.0) * ((y1 - y0) / cell + 1.0) > 4.0 * (double)Q) cell *= 2.0;
    const int64_t gx = (int64_t)((x1 - x0) / cell) + 1;
    std::vector<std::pair<int64_t, int64_t>> ce;      // (cell, edge)
    ce.reserve((size_t)Q * 4);
    for (int64_t e = 0; e < Q; ++e) {
        const zd a = p[e], b = p[(e + 1) % Q];
        const int64_t i0 = (int64_t)((std::fmin(a.x, b.x) - x0) / cell);
        const int64_t i1 = (int64_t)((std::fmax(a.x, b.x) - x0) / cell);
        const int64_t j0 = (int64_t)((std::fmin(a.y, b.y) - y0) / cell);
        const int64_t j1 = (int64_t)((std::fmax(a.y, b.y) - y0) / cell);
        for (int64_t j = j0; j <= j1; ++j)
            for (int64_t i = i0; i <= i1; ++i) ce.emplace_back(j * gx + i, e);
    }
    std::sort(ce.begin(), ce.end());
    for (size_t lo = 0; lo < ce.size();) {
        size_t hi = lo;
        while (hi < ce.size() && ce[hi].first == ce[lo].first) ++hi;
        for (size_t u = lo; u < hi; ++u)
            for (size_t v = u + 1; v < hi; ++v) {
                const int64_t a = ce[u].second, b = ce[v].second;
                const int64_t d = b > a ? b - a : a - b;
                if (d <= 1 || d == Q - 1) continue;          // edges sharing a vertex
                if (seg_intersect(p[a], p[(a + 1) % Q], p[b], p[(b + 1) % Q])) return true;
            }
        lo = hi;
    }
    return false;
}

}  // namespace

void gauss_legendre01(int n, std::vector<double> &x, std::vector<double> &w) {
    // Newton on the Legendre polynomial from the usual cosine guesses; nodes ascending
    x.assign(n, 0.0);
    w.assign(n, 0.0);
    for (int i = 0; i < n; ++i) {
        double z = std::cos(kPi * (i + 0.75) / (n + 0.5));
        double p0 = 1.0, p1 = z, dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            p0 = 1.0;
            p1 = z;
            for (int j = 2; j <= n; ++j) {
                double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
                p0 = p1;
                p1 = p2;
            }
            if (n == 1) p0 = 1.0;
            dp = n * (z * p1 - p0) / (z * z - 1.0);
            double dz = p1 / dp;
            z -= dz;
            if (std::fabs(dz) < 1e-17) break;
        }
        p0 = 1.0;
        p1 = z;
        for (int j = 2; j <= n; ++j) {
            double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
            p0 = p1;
            p1 = p2;
        }
        dp = n * (z * p1 - p0) / (z * z - 1.0);
        x[n - 1 - i] = 0.5 * (z + 1.0);
        w[n - 1 - i] = 1.0 / ((1.0 - z * z) * dp * dp);
    }
}

std::string build_geometry(const cfie_contour &c, HostGeometry &g) {
    if (c.n_modes < 1) return "n_modes must be >= 1";
    if (c.zhat == nullptr) return "zhat is NULL";
    g.M = c.n_modes;
    g.zhat.resize(2 * g.M + 1);
    for (int i = 0; i < 2 * g.M + 1; ++i) {
        double a = c.zhat[2 * i], b = c.zhat[2 * i + 1];
        if (!std::isfinite(a) || !std::isfinite(b)) return "non-finite contour coefficient";
        g.zhat[i] = mk(a, b);
    }
    int P = 4096;
    while (P < 64 * (2 * g.M + 1)) P *= 2;
    std::vector<double> speed(P), curv(P);
    double area = 0.0;
    double min_speed = 1e300;
    for (int j = 0; j < P; ++j) {
        double t = 2.0 * kPi * j / P;
        zd z = zeval(g.zhat, g.M, t, 0);
        zd d1 = zeval(g.zhat, g.M, t, 1);
        zd d2 = zeval(g.zhat, g.M, t, 2);
        double sp = cabs(d1);
        speed[j] = sp;
        min_speed = std::fmin(min_speed, sp);
        curv[j] = (d1.x * d2.y - d1.y * d2.x) / (sp * sp * sp);
        area += 0.5 * (z.x * d1.y - z.y * d1.x);
    }
    area *= 2.0 * kPi / P;
    if (!(min_speed > 0.0)) return "contour has a zero tangent (not a regular curve)";
    if (!(area > 0.0)) return "contour must be counter-clockwise (positive signed area)";
    // self-intersection of the polygon through 16 N points of the curve (at least 1024)
    {
        const int Q = std::max(1024, 16 * c.n_nodes);
        std::vector<zd> poly(Q);
        for (int j = 0; j < Q; ++j) {
            // z(t) = sum_m zhat_m w^m, w = e^{it}, by Horner in w and in 1/w = conj(w)
            const double t = 2.0 * kPi * j / Q;
            const zd w = mk(std::cos(t), std::sin(t)), wc = mk(w.x, -w.y);
            zd hi = mk(0.0, 0.0), lo = mk(0.0, 0.0);
            for (int m = g.M; m >= 1; --m) {
                hi = hi * w + g.zhat[g.M + m];
                lo = lo * wc + g.zhat[g.M - m];
            }
            poly[j] = g.zhat[g.M] + hi * w + lo * wc;
        }
        if (polygon_self_intersects(poly)) return "contour intersects itself";
    }
    // Fourier coefficients of the speed by direct summation with exact root indices
    std::vector<zd> roots(P);
    for (int j = 0; j < P; ++j) roots[j] = mk(std::cos(2.0 * kPi * j / P), -std::sin(2.0 * kPi * j / P));
    double c0 = 0.0;
    for (int j = 0; j < P; ++j) c0 += speed[j];
    c0 /= P;
    g.c0 = c0;
    g.cm.clear();
    int mmax = P / 4;
    std::vector<zd> coef(mmax + 1);
    for (int m = 1; m <= mmax; ++m) {
        zd acc = mk(0.0, 0.0);
        for (int j = 0; j < P; ++j) acc = acc + roots[(long)m * j % P] * speed[j];
        coef[m] = acc * (1.0 / P);
    }
    // rounding floor of the transform from its upper half, where an analytic speed has
    // decayed below it; keep modes clearly above that floor
    double noise = 0.0;
    for (int m = mmax / 2 + 1; m <= mmax; ++m) noise += abs2(coef[m]);
    noise = std::sqrt(noise / (mmax - mmax / 2));
    double thr = std::max(1e-17 * c0, 16.0 * noise);
    int last = 0;
    for (int m = 1; m <= mmax; ++m)
        if (cabs(coef[m]) > thr) last = m;
    if (last >= mmax / 2) return "arc-length density not resolved (contour too irregular)";
    g.cm.assign(coef.begin() + 1, coef.begin() + last + 1);
    g.L = 2.0 * kPi * c0;
    g.radius = g.L / (2.0 * kPi);
    g.min_curvature = 1e300;
    for (int j = 0; j < P; ++j) g.min_curvature = std::fmin(g.min_curvature, curv[j]);
    g.convex = g.min_curvature >= 0.0;
    return "";
}

// The speed coefficients are c0 = (1/P) sum_j |z'(tau_j)| and c_m = (1/P) sum_j |z'(tau_j)|
// e^{-i m tau_j} on the P-point grid tau_j = 2 pi j / P of build_geometry (m = 1..Ms, the
// retained modes), and d|z'| = Re(conj(T) dz') with the unit tangent T.  With the loss
// differential Re(conj(cbar_m) dc_m) + c0bar dc0, the sample adjoints are
//   spbar_j = (c0bar + sum_m Re(conj(cbar_m) e^{-i m tau_j})) / P
// and zbar_m += sum_j spbar_j T_j conj(i m e^{i m tau_j}).
void speed_coeffs_adjoint(const HostGeometry &g, double c0bar, const std::vector<zd> &cmbar,
                          std::vector<zd> &zbar) {
    int P = 4096;
    while (P < 64 * (2 * g.M + 1)) P *= 2;
    const int Ms = (int)g.cm.size();
    std::vector<zd> roots(P);
    for (int j = 0; j < P; ++j)
        roots[j] = mk(std::cos(2.0 * kPi * j / P), -std::sin(2.0 * kPi * j / P));
    for (int j = 0; j < P; ++j) {
        double sb = c0bar;
        for (int m = 1; m <= Ms && m <= (int)cmbar.size(); ++m) {
            zd E = roots[(long)m * j % P];
            sb += (conj(cmbar[m - 1]) * E).x;
        }
        sb /= P;
        if (sb == 0.0) continue;
        zd d1 = zeval(g.zhat, g.M, 2.0 * kPi * j / P, 1);
        double sp = cabs(d1);
        zd T = d1 * (1.0 / sp);
        for (int m = -g.M; m <= g.M; ++m) {
            // conj(i m e^{i m tau}) = -i m e^{-i m tau}
            zd E = roots[(long)(((m % P) + P) % P) * j % P];
            zd w = cmul_i(E) * (-(double)m);
            zbar[m + g.M] = zbar[m + g.M] + T * w * sb;
        }
    }
}

HostGeometry circle_geometry(double radius) {
    HostGeometry g;
    g.M = 1;
    g.zhat = {mk(0.0, 0.0), mk(0.0, 0.0), mk(radius, 0.0)};
    g.c0 = radius;
    g.cm.clear();
    g.L = 2.0 * kPi * radius;
    g.radius = radius;
    g.convex = true;
    g.min_curvature = 1.0 / radius;
    return g;
}

// ---------------------------------------------------------------- log moments -------------
namespace {

// tanh-sinh rule on [0,1], nodes accurate near 0
void tanh_sinh01(double step, std::vector<double> &u, std::vector<double> &w) {
    u.clear();
    w.clear();
    for (int k = -400; k <= 400; ++k) {
        double x = k * step;
        double y = 0.5 * kPi * std::sinh(x);
        double uu = 1.0 / (1.0 + std::exp(-2.0 * y));
        double ww = step * 0.25 * kPi * std::cosh(x) / (std::cosh(y) * std::cosh(y));
        if (uu < 1e-30 || 1.0 - uu < 1e-17 || ww < 1e-40) continue;
        u.push_back(uu);
        w.push_back(ww);
    }
}

// Lagrange basis polynomial l_g on the nodes xs, evaluated at x (barycentric form)
double lagrange(const std::vector<double> &xs, const std::vector<double> &bw, int g, double x) {
    double num = 0.0, den = 0.0;
    for (size_t j = 0; j < xs.size(); ++j) {
        double d = x - xs[j];
        if (d == 0.0) return (int)j == g ? 1.0 : 0.0;
        double t = bw[j] / d;
        den += t;
        if ((int)j == g) num = t;
    }
    return num / den;
}

}  // namespace

void log_moments(int q, std::vector<double> &mom) {
    std::vector<double> xs, wq;
    gauss_legendre01(q, xs, wq);
    std::vector<double> bw(q, 1.0);
    for (int j = 0; j < q; ++j)
        for (int i = 0; i < q; ++i)
            if (i != j) bw[j] /= (xs[j] - xs[i]);
    std::vector<double> tu, tw;
    tanh_sinh01(1.0 / 32.0, tu, tw);
    int nv = 40;
    std::vector<double> vx, vw;
    gauss_legendre01(nv, vx, vw);
    // the inner polynomial integrals (degree <= 2q+1) are exact with q+2 points
    int ni = q + 2;
    std::vector<double> ix, iw;
    gauss_legendre01(ni, ix, iw);
    mom.assign((size_t)3 * 5 * q * q, 0.0);
    auto P = [&](int g, int c, double x, bool obs) {
        double l = lagrange(xs, bw, g, x);
        if (c == 4) return l;
        int a = obs ? (c >> 1) : (c & 1);
        return l * (a == 0 ? 1.0 - x : x);
    };
    for (int c = 0; c < 5; ++c)
        for (int g = 0; g < q; ++g)
            for (int hh = 0; hh < q; ++hh) {
                // kind 0: coincident, int_0^1 log(u) F(u) du with
                // F(u) = int_u^1 P(xi) Q(xi-u) dxi + int_0^{1-u} P(xi) Q(xi+u) dxi
                double acc0 = 0.0;
                for (size_t t = 0; t < tu.size(); ++t) {
                    double u = tu[t];
                    double F = 0.0;
                    for (int i = 0; i < ni; ++i) {
                        double xa = u + (1.0 - u) * ix[i];
                        double xb = (1.0 - u) * ix[i];
                        F += (1.0 - u) * iw[i] *
                             (P(g, c, xa, true) * P(hh, c, xa - u, false) +
                              P(g, c, xb, true) * P(hh, c, xb + u, false));
                    }
                    acc0 += tw[t] * std::log(u) * F;
                }
                // kind 1: source element follows, sigma = a + b, a = 1 - xi, b = xi'
                // kind 2: source element precedes, sigma = a + b, a = xi, b = 1 - xi'
                double acc1 = 0.0, acc2 = 0.0;
                for (size_t t = 0; t < tu.size(); ++t) {
                    double rho = tu[t];
                    double s1 = 0.0, s2 = 0.0;
                    for (int i = 0; i < nv; ++i) {
                        double v = vx[i];
                        double lg = std::log(rho) + std::log1p(v);
                        // triangle a >= b: a = rho, b = rho v ; triangle a < b: b = rho, a = rho v
                        double a1 = rho, b1 = rho * v, a2 = rho * v, b2 = rho;
                        s1 += vw[i] * lg *
                              (P(g, c, 1.0 - a1, true) * P(hh, c, b1, false) +
                               P(g, c, 1.0 - a2, true) * P(hh, c, b2, false));
                        s2 += vw[i] * lg *
                              (P(g, c, a1, true) * P(hh, c, 1.0 - b1, false) +
                               P(g, c, a2, true) * P(hh, c, 1.0 - b2, false));
                    }
                    acc1 += tw[t] * rho * s1;
                    acc2 += tw[t] * rho * s2;
                }
                mom[((size_t)0 * 5 + c) * q * q + g * q + hh] = acc0;
                mom[((size_t)1 * 5 + c) * q * q + g * q + hh] = acc1;
                mom[((size_t)2 * 5 + c) * q * q + g * q + hh] = acc2;
            }
}

}  // namespace cfie
