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
#include <limits>
#include <string>
#include <vector>

#include "internal.h"

namespace cfie {

namespace {

// e^{-2 pi i j / P}, j = 0..P-1
std::vector<zd> unit_roots(int P) {
    std::vector<zd> r(P);
    for (int j = 0; j < P; ++j) r[j] = mk(std::cos(2.0 * kPi * j / P), -std::sin(2.0 * kPi * j / P));
    return r;
}

// z, z' and z'' at tau_j = 2 pi j / P, with e^{i m tau_j} taken from the root table of P
void zeval_grid(const std::vector<zd> &zh, int M, const std::vector<zd> &roots, int64_t j,
                zd &z, zd &d1, zd &d2) {
    const int64_t P = (int64_t)roots.size();
    z = d1 = d2 = mk(0.0, 0.0);
    for (int m = -M; m <= M; ++m) {
        const int64_t r = (((int64_t)m * j) % P + P) % P;
        const zd v = zh[m + M] * conj(roots[r]);
        z = z + v;
        d1 = d1 + cmul_i(v) * (double)m;
        d2 = d2 + v * (-(double)m * (double)m);
    }
}

// Whether segments ab and cd cross at interior points of both (parallel segments never do):
// a + t (b - a) = c + u (d - c) with 0 < t, u < 1, compared without dividing by the
// determinant.
bool seg_intersect(zd a, zd b, zd c, zd d) {
    auto cross = [](zd u, zd v) { return u.x * v.y - u.y * v.x; };
    const zd r = b - a, s = d - c, ca = c - a;
    const double den = cross(r, s);
    if (den == 0.0) return false;
    const double tn = cross(ca, s), un = cross(ca, r);
    if (den > 0.0) return tn > 0.0 && tn < den && un > 0.0 && un < den;
    return tn < 0.0 && tn > den && un < 0.0 && un > den;
}

// Whether two edges of the closed polygon p that do not share a vertex cross.  The edges, in
// their order along the curve, are grouped in leaves of four; a binary tree over the leaves
// holds the bounding box of each run of consecutive edges.  Two runs are compared only when
// their boxes overlap, and two leaves edge by edge; for a smooth curve only runs that meet
// end to end (or pass close to each other) overlap, so the work is about linear in the
// number of edges, with the boxes read in order.
bool polygon_self_intersects(const std::vector<zd> &p) {
    const int64_t Q = (int64_t)p.size();
    if (Q < 4) return false;
    constexpr int64_t kLeaf = 4;
    const int64_t nl = (Q + kLeaf - 1) / kLeaf;
    int64_t np = 1;
    while (np < nl) np <<= 1;
    struct Box { double x0, x1, y0, y1; };
    const double inf = std::numeric_limits<double>::infinity();
    std::vector<Box> bx((size_t)(2 * np), Box{inf, -inf, inf, -inf});   // empty boxes
    for (int64_t l = 0; l < nl; ++l) {
        Box bb{inf, -inf, inf, -inf};
        for (int64_t e = l * kLeaf; e <= std::min(Q, (l + 1) * kLeaf); ++e) {   // vertices
            const zd v = p[e % Q];
            bb = Box{std::fmin(bb.x0, v.x), std::fmax(bb.x1, v.x), std::fmin(bb.y0, v.y),
                     std::fmax(bb.y1, v.y)};
        }
        bx[(size_t)(np + l)] = bb;
    }
    for (int64_t i = np - 1; i >= 1; --i) {
        const Box &u = bx[(size_t)(2 * i)], &v = bx[(size_t)(2 * i + 1)];
        bx[(size_t)i] = Box{std::fmin(u.x0, v.x0), std::fmax(u.x1, v.x1), std::fmin(u.y0, v.y0),
                            std::fmax(u.y1, v.y1)};
    }
    auto overlap = [](const Box &u, const Box &v) {
        return u.x0 <= v.x1 && v.x0 <= u.x1 && u.y0 <= v.y1 && v.y0 <= u.y1;
    };
    auto leaves = [&](int64_t la, int64_t lb) {         // edges of leaf la against leaf lb
        const int64_t ea = std::min(Q, (la + 1) * kLeaf), eb = std::min(Q, (lb + 1) * kLeaf);
        for (int64_t a = la * kLeaf; a < ea; ++a)
            for (int64_t b = la == lb ? a + 2 : lb * kLeaf; b < eb; ++b) {
                const int64_t d = b > a ? b - a : a - b;
                if (d <= 1 || d == Q - 1) continue;          // edges sharing a vertex
                if (seg_intersect(p[a], p[(a + 1) % Q], p[b], p[(b + 1) % Q])) return true;
            }
        return false;
    };
    // pairs of nodes of one level: (i, i) = the pairs within node i, (i, j) = i against j
    std::vector<std::pair<int64_t, int64_t>> st{{1, 1}};
    while (!st.empty()) {
        const auto [a, b] = st.back();
        st.pop_back();
        if (!overlap(bx[(size_t)a], bx[(size_t)b])) continue;   // also skips empty nodes
        if (a >= np) {
            if (leaves(a - np, b - np)) return true;
            continue;
        }
        if (a == b) {
            st.push_back({2 * a, 2 * a});
            st.push_back({2 * a + 1, 2 * a + 1});
            st.push_back({2 * a, 2 * a + 1});
        } else {
            st.push_back({2 * a, 2 * b});
            st.push_back({2 * a, 2 * b + 1});
            st.push_back({2 * a + 1, 2 * b});
            st.push_back({2 * a + 1, 2 * b + 1});
        }
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
    const std::vector<zd> roots = unit_roots(P);
    std::vector<double> speed(P), curv(P);
    double area = 0.0;
    double min_speed = 1e300;
    for (int j = 0; j < P; ++j) {
        zd z, d1, d2;
        zeval_grid(g.zhat, g.M, roots, j, z, d1, d2);
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
        // w_j = e^{2 pi i j / Q} as the product of two table entries, j = 512 a + b
        const int nb = 512, na = (Q + nb - 1) / nb;
        std::vector<zd> wa(na), wb(nb);
        for (int a = 0; a < na; ++a)
            wa[a] = mk(std::cos(2.0 * kPi * ((double)a * nb) / Q), std::sin(2.0 * kPi * ((double)a * nb) / Q));
        for (int b = 0; b < nb; ++b) wb[b] = mk(std::cos(2.0 * kPi * b / Q), std::sin(2.0 * kPi * b / Q));
        std::vector<zd> poly(Q);
        // z(t) = sum_m zhat_m w^m, w = e^{it}, by Horner in w and in 1/w = conj(w); four
        // points at a time, so that their recurrences overlap
        constexpr int kU = 4;
        for (int j0 = 0; j0 < Q; j0 += kU) {
            zd w[kU], wc[kU], hi[kU], lo[kU];
            for (int u = 0; u < kU; ++u) {
                const int j = std::min(j0 + u, Q - 1);
                w[u] = wa[j / nb] * wb[j % nb];
                wc[u] = mk(w[u].x, -w[u].y);
                hi[u] = lo[u] = mk(0.0, 0.0);
            }
            for (int m = g.M; m >= 1; --m)
                for (int u = 0; u < kU; ++u) {
                    hi[u] = hi[u] * w[u] + g.zhat[g.M + m];
                    lo[u] = lo[u] * wc[u] + g.zhat[g.M - m];
                }
            for (int u = 0; u < kU && j0 + u < Q; ++u)
                poly[j0 + u] = g.zhat[g.M] + hi[u] * w[u] + lo[u] * wc[u];
        }
        if (polygon_self_intersects(poly)) return "contour intersects itself";
    }
    // Fourier coefficients of the speed by direct summation with exact root indices
    // the mean speed by compensated (Neumaier) summation: the perimeter 2 pi c0 sets the mesh
    double c0 = 0.0, comp = 0.0;
    for (int j = 0; j < P; ++j) {
        const double t = c0 + speed[j];
        comp += std::fabs(c0) >= std::fabs(speed[j]) ? (c0 - t) + speed[j] : (speed[j] - t) + c0;
        c0 = t;
    }
    c0 = (c0 + comp) / P;
    g.c0 = c0;
    g.cm.clear();
    int mmax = P / 4;
    std::vector<zd> coef(mmax + 1);
    for (int m = 1; m <= mmax; ++m) {
        zd acc = mk(0.0, 0.0);
        for (int j = 0, r = 0; j < P; ++j) {          // r = m j mod P
            acc = acc + roots[r] * speed[j];
            r += m;
            if (r >= P) r -= P;
        }
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
    const std::vector<zd> roots = unit_roots(P);
    for (int j = 0; j < P; ++j) {
        double sb = c0bar;
        for (int m = 1; m <= Ms && m <= (int)cmbar.size(); ++m) {
            zd E = roots[(long)m * j % P];
            sb += (conj(cmbar[m - 1]) * E).x;
        }
        sb /= P;
        if (sb == 0.0) continue;
        zd z, d1, d2;
        zeval_grid(g.zhat, g.M, roots, j, z, d1, d2);
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

// all Lagrange basis polynomials l_0..l_{q-1} on the nodes xs, evaluated at x (barycentric
// form), into l
void lagrange_all(const std::vector<double> &xs, const std::vector<double> &bw, double x,
                  double *l) {
    const int q = (int)xs.size();
    double den = 0.0;
    for (int j = 0; j < q; ++j) {
        const double d = x - xs[j];
        if (d == 0.0) {
            for (int i = 0; i < q; ++i) l[i] = i == j ? 1.0 : 0.0;
            return;
        }
        l[j] = bw[j] / d;
        den += l[j];
    }
    for (int j = 0; j < q; ++j) l[j] /= den;
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
    // Every moment of one kind is a sum over the same quadrature points (xi, xi') with weight
    // w of w P_g(xi) Q_h(xi'), where P and Q are a Lagrange polynomial times a linear hat
    // factor (1 - x or x, none for c = 4; the observation factor is chosen by bit 1 of c,
    // the source factor by bit 0).  The Lagrange values at a point serve all g, h and c.
    std::vector<double> lo(q), ls(q);
    auto point = [&](int kind, double w, double xo, double xsrc) {
        lagrange_all(xs, bw, xo, lo.data());
        lagrange_all(xs, bw, xsrc, ls.data());
        for (int c = 0; c < 5; ++c) {
            const double fo = c == 4 ? 1.0 : ((c >> 1) == 0 ? 1.0 - xo : xo);
            const double fs = c == 4 ? 1.0 : ((c & 1) == 0 ? 1.0 - xsrc : xsrc);
            const double f = w * fo * fs;
            double *m = &mom[((size_t)kind * 5 + c) * q * q];
            for (int g = 0; g < q; ++g) {
                const double a = f * lo[g];
                for (int h = 0; h < q; ++h) m[g * q + h] += a * ls[h];
            }
        }
    };
    // kind 0: coincident, int_0^1 log(u) F(u) du with
    // F(u) = int_u^1 P(xi) Q(xi-u) dxi + int_0^{1-u} P(xi) Q(xi+u) dxi
    for (size_t t = 0; t < tu.size(); ++t) {
        const double u = tu[t];
        const double wt = tw[t] * std::log(u) * (1.0 - u);
        for (int i = 0; i < ni; ++i) {
            const double xa = u + (1.0 - u) * ix[i];
            const double xb = (1.0 - u) * ix[i];
            point(0, wt * iw[i], xa, xa - u);
            point(0, wt * iw[i], xb, xb + u);
        }
    }
    // kind 1: source element follows, sigma = a + b, a = 1 - xi, b = xi'
    // kind 2: source element precedes, sigma = a + b, a = xi, b = 1 - xi'
    // each over the triangles a >= b (a = rho, b = rho v) and a < b (b = rho, a = rho v)
    for (size_t t = 0; t < tu.size(); ++t) {
        const double rho = tu[t];
        for (int i = 0; i < nv; ++i) {
            const double v = vx[i];
            const double w = tw[t] * rho * vw[i] * (std::log(rho) + std::log1p(v));
            const double a1 = rho, b1 = rho * v, a2 = rho * v, b2 = rho;
            point(1, w, 1.0 - a1, b1);
            point(1, w, 1.0 - a2, b2);
            point(2, w, a1, 1.0 - b1);
            point(2, w, a2, 1.0 - b2);
        }
    }
}

}  // namespace cfie
