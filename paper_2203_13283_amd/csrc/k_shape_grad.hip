// Reverse-mode derivative of the assembly, the plane-wave vectors and the contour's
// arc-length discretisation with respect to the contour's Fourier coefficients.
//
// The loss depends on the matrices D^k, N^k, D^kt, S^kt through real bilinear forms
//   Re sum_ij Omega_M[i, j] M_ij,
// with loss weights Omega_M (N x N, formed from the solution and adjoint vectors by GEMMs),
// and on the plane-wave vectors through Re sum_ij w_ij e'_ij (+ w'_ij h_ij).  Every matrix
// entry is the Galerkin sum of its element pairs (Sec. II eqs. (2)-(4)); each element pair is
// a sum over Gauss point pairs of the kernels at (r_o, r_s), with the weights that the
// forward kernels use.  The backward kernels differentiate those sums with respect to the
// point data (x, y, unit tangent, curvature) of every Gauss point, the element length h and
// beta = Im kt.  The chain to the Fourier coefficients runs through the points' parameters
// t(s) (the arc-length inversion) and the Fourier series of the speed.
//
//   k_grad_far:  lanes own row elements e, walk a strip of column elements f; both ordered
//                pairs (e, f) and (f, e) of an element pair share one Hankel evaluation
//                and the lane keeps only the derivative with respect to its own points, so
//                no two lanes write the same value (partial sums per strip are added in a
//                fixed order afterwards).
//   k_grad_near: one thread per Gauss point of the near table, over the element pairs of the
//                near band (the touching ones by the log-split rule with moments).
//   k_grad_exc:  one thread per Gauss point, over the plane-wave directions.
//   k_grad_prep, k_grad_modes: per-point chain to (t, z, z', z'') and reductions onto the
//                Fourier modes of z and of the speed.
#include "internal.h"
#include "pair_kernels.h"
#include "shape_grad.h"

namespace cfie {

namespace {

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// cyclic distance of node indices
__device__ __forceinline__ int cdist(int i, int j, int N) {
    int d = i - j;
    d = ((d % N) + N) % N;
    return min(d, N - d);
}

template <int Q>
struct QW {
    double xi[Q], w[Q];
};

}  // namespace

// ------------------------------------------------------------------ far pairs -------------
// Omega: the four loss-weight matrices (Dk, Nk, Dkt, Skt), column-major with leading
// dimension ld.  part: [strip][4][N Q] partial adjoints of (x, y, tx, ty) (MODE 0 writes,
// MODE 1 and 2 add); spart: per wave (d/dh, d/dbeta).  The passes split the element pairs
// as the forward assembly does, by the lower bound of k R (far_kRmin): MODE 0 the 8-term
// large-argument series, MODE 1 the 22-term series, MODE 2 the small arguments beyond
// dband elements from the diagonal (those within go to k_grad_far_band).
template <int Q, int MODE>
__global__ __launch_bounds__(256) void k_grad_far(int N, double h, PairConsts c, int nb,
                                                  int dband, int SL,
                                                  const zd *__restrict__ O0,
                                                  const zd *__restrict__ O1,
                                                  const zd *__restrict__ O2,
                                                  const zd *__restrict__ O3, int64_t ld,
                                                  const double *__restrict__ PX,
                                                  const double *__restrict__ PY,
                                                  const double *__restrict__ PTX,
                                                  const double *__restrict__ PTY, QW<Q> qc,
                                                  int n_eg, int n_strips, double *part,
                                                  double *spart) {
    const int lane = threadIdx.x & 63;
    const int wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    if (wave >= n_eg * n_strips) return;
    const int eg = wave % n_eg, strip = wave / n_eg;
    const int e_raw = eg * 64 + lane;
    const bool valid = e_raw < N;
    const int e = valid ? e_raw : N - 1;
    const int e1 = (e + 1) % N;
    const int f0 = strip * SL, f1 = min(N, f0 + SL);
    if constexpr (MODE != 0) {
        // most tiles hold no element pair for these passes (SL = 128 columns: two per lane,
        // clamped); such a wavefront adds nothing and reports zero scalar derivatives
        const int fa = min(f0 + lane, f1 - 1), fb = min(f0 + 64 + lane, f1 - 1);
        if (far_tile_all_fast(c.k, h, PX[e * Q + Q / 2], PY[e * Q + Q / 2], PX[fa * Q + Q / 2],
                              PY[fa * Q + Q / 2], PX[fb * Q + Q / 2], PY[fb * Q + Q / 2])) {
            if (lane == 0) {
                spart[2 * (size_t)wave] = 0.0;
                spart[2 * (size_t)wave + 1] = 0.0;
            }
            return;
        }
    }
    // own points and their adjoints in LDS (stride 256: one column per thread)
    __shared__ double lds[8 * Q * 256];
    double *own = lds + threadIdx.x;                    // [4][Q]: x, y, tx, ty
    double *adj = lds + 4 * Q * 256 + threadIdx.x;      // [4][Q]
    for (int g = 0; g < Q; ++g) {
        own[(0 * Q + g) * 256] = PX[e * Q + g];
        own[(1 * Q + g) * 256] = PY[e * Q + g];
        own[(2 * Q + g) * 256] = PTX[e * Q + g];
        own[(3 * Q + g) * 256] = PTY[e * Q + g];
        for (int v = 0; v < 4; ++v) adj[(v * Q + g) * 256] = 0.0;
    }
    const double k = c.k, h2 = h * h;
    const double rsafe = 1000.0 * c.invk;
    const zd *Om[4] = {O0, O1, O2, O3};
    const double xref = own[(0 * Q + Q / 2) * 256], yref = own[(1 * Q + Q / 2) * 256];
    double hbar = 0.0, bbar = 0.0;
    for (int f = f0; f < f1; ++f) {
        const int fn = (f + 1) % N;
        const int cd = cdist(e, f, N);
        const double kRmin = far_kRmin(c.k, h, xref - PX[f * Q + Q / 2],
                                       yref - PY[f * Q + Q / 2]);
        const bool fast = kRmin >= kFarFast;
        const bool mid = !fast && kRmin >= kAsymMin;
        const bool on = valid && cd > nb &&
                        (MODE == 0 ? fast : MODE == 1 ? mid : (!fast && !mid && cd > dband));
        if (!__any(on)) continue;
        // loss weights of the 2x2 node blocks, far entries only:
        //   Omega_m[e + a, f + b]   (own element observes)
        //   Omega_m[f + a, e + b]   (own element is the source)
        // read again for every partner point (they stay in the caches) so that only their
        // contractions with the partner's hats are live in the point loop
        const int ri[2] = {e, e1}, rf[2] = {f, fn};
        bool m1[2][2], m2[2][2];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b) {
                m1[a][b] = on && cdist(ri[a], rf[b], N) >= nb + 2;
                m2[a][b] = on && cdist(rf[a], ri[b], N) >= nb + 2;
            }
#pragma unroll 1
        for (int hh = 0; hh < Q; ++hh) {
            const double xs = PX[f * Q + hh], ys = PY[f * Q + hh];
            const double txs = PTX[f * Q + hh], tys = PTY[f * Q + hh];
            const double xh = qc.xi[hh], wh = qc.w[hh];
            const double ph[2] = {1.0 - xh, xh};
            // contract the partner's hat index: c1[m][a] = sum_b Omega_m[e+a, f+b] phi_b(xh),
            // c2[m][b] = sum_a Omega_m[f+a, e+b] phi_a(xh); for the Maue term the signs
            // s_0 = -1, s_1 = 1 of the hat derivatives: n1[a] = sum_b s_b Omega_N[e+a, f+b],
            // n2[b] = sum_a s_a Omega_N[f+a, e+b]
            zd c1[4][2], c2[4][2], n1[2], n2[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) {
                n1[a] = n2[a] = mk(0.0, 0.0);
#pragma unroll
                for (int m = 0; m < 4; ++m) c1[m][a] = c2[m][a] = mk(0.0, 0.0);
            }
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    const double sb = b ? 1.0 : -1.0, sa = a ? 1.0 : -1.0;
#pragma unroll
                    for (int m = 0; m < 4; ++m) {
                        const zd v1 = m1[a][b] ? Om[m][(int64_t)ri[a] + (int64_t)rf[b] * ld]
                                               : mk(0.0, 0.0);
                        const zd v2 = m2[a][b] ? Om[m][(int64_t)rf[a] + (int64_t)ri[b] * ld]
                                               : mk(0.0, 0.0);
                        c1[m][a] = c1[m][a] + v1 * ph[b];
                        c2[m][b] = c2[m][b] + v2 * ph[a];
                        if (m == 1) {
                            n1[a] = n1[a] + v1 * sb;
                            n2[b] = n2[b] + v2 * sa;
                        }
                    }
                }
#pragma unroll 1
            for (int g = 0; g < Q; ++g) {
                const double xo = own[(0 * Q + g) * 256], yo = own[(1 * Q + g) * 256];
                const double txo = own[(2 * Q + g) * 256], tyo = own[(3 * Q + g) * 256];
                double dx = xo - xs, dy = yo - ys;
                dx = on ? dx : rsafe;
                dy = on ? dy : 0.0;
                const double R = sqrt(dx * dx + dy * dy);
                const double nu1 = (dx * tys - dy * txs) / R;
                const double nu2 = (dy * txo - dx * tyo) / R;
                const double nn = txo * txs + tyo * tys;
                zd g0, g1, t0, t1;
                if constexpr (MODE == 0) pair_kernels_asym<8>(c, R, 1.0, g0, g1, t0, t1);
                else if constexpr (MODE == 1) pair_kernels_asym<kSerMax>(c, R, 1.0, g0, g1, t0, t1);
                else pair_kernels(c, R, 1.0, g0, g1, t0, t1);
                const double xg = qc.xi[g], wg = qc.w[g];
                const double pg[2] = {1.0 - xg, xg};
                const double ww = wg * wh, hw = h2 * ww;
                SmoothW W1, W2;
                W1.wD = (c1[0][0] * pg[0] + c1[0][1] * pg[1]) * hw;
                W1.wN2 = (c1[1][0] * pg[0] + c1[1][1] * pg[1]) * hw;
                W1.wDt = (c1[2][0] * pg[0] + c1[2][1] * pg[1]) * hw;
                W1.wS = (c1[3][0] * pg[0] + c1[3][1] * pg[1]) * hw;
                W1.wN1 = (n1[1] - n1[0]) * ww;
                W2.wD = (c2[0][0] * pg[0] + c2[0][1] * pg[1]) * hw;
                W2.wN2 = (c2[1][0] * pg[0] + c2[1][1] * pg[1]) * hw;
                W2.wDt = (c2[2][0] * pg[0] + c2[2][1] * pg[1]) * hw;
                W2.wS = (c2[3][0] * pg[0] + c2[3][1] * pg[1]) * hw;
                W2.wN1 = (n2[1] - n2[0]) * ww;
                double oa[4] = {0.0, 0.0, 0.0, 0.0}, sa[4] = {0.0, 0.0, 0.0, 0.0};
                const PairD d1 = smooth_pair_adjoint(k, c.kt, R, nu1, nn, g0, g1, t0, t1, W1);
                pair_geom_adjoint(dx, dy, R, nu1, txo, tyo, txs, tys, d1, oa, nullptr);
                const PairD d2 = smooth_pair_adjoint(k, c.kt, R, nu2, nn, g0, g1, t0, t1, W2);
                pair_geom_adjoint(-dx, -dy, R, nu2, txs, tys, txo, tyo, d2, nullptr, sa);
#pragma unroll
                for (int v = 0; v < 4; ++v) adj[(v * Q + g) * 256] += oa[v] + sa[v];
                // the ordered pair (own observes) carries the scalar derivatives once
                hbar += 2.0 * d1.vh2 / h;
                bbar += d1.beta;
            }
        }
    }
    if (valid) {
        const size_t np = (size_t)N * Q;
        for (int v = 0; v < 4; ++v)
            for (int g = 0; g < Q; ++g) {
                double *dst = part + ((size_t)strip * 4 + v) * np + (size_t)e * Q + g;
                *dst = (MODE == 0 ? 0.0 : *dst) + adj[(v * Q + g) * 256];
            }
    }
    hbar = wave_sum(hbar);
    bbar = wave_sum(bbar);
    if (lane == 0) {
        spart[2 * (size_t)wave] = hbar;
        spart[2 * (size_t)wave + 1] = bbar;
    }
}

// Ordered element pairs (e, f = e + d) with nb < |d| <= band and k R below kAsymMin (the
// forward's k_far_band pairs): one thread per pair, lanes sharing the offset d.  The
// derivatives of the pair's loss terms with respect to the observation element's points go
// to ob[v][didx][e Q + g], those with respect to the source element's points to
// sb[v][didx][e Q + hh] (zero for the other pairs); d = didx - dl.  spart: per block
// (d/dh, d/dbeta).
template <int Q>
__global__ __launch_bounds__(256) void k_grad_far_band(int N, double h, PairConsts c, int nb,
                                                       int dl, int dr,
                                                       const zd *__restrict__ O0,
                                                       const zd *__restrict__ O1,
                                                       const zd *__restrict__ O2,
                                                       const zd *__restrict__ O3, int64_t ld,
                                                       const double *__restrict__ PX,
                                                       const double *__restrict__ PY,
                                                       const double *__restrict__ PTX,
                                                       const double *__restrict__ PTY,
                                                       QW<Q> qc, double *ob, double *sb,
                                                       double *spart) {
    const int nd = dl + dr + 1;
    const size_t np = (size_t)N * Q;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double hbar = 0.0, bbar = 0.0;
    if (tid < (int64_t)N * nd) {
        const int e = (int)(tid % N), didx = (int)(tid / N);
        const int d = didx - dl;
        const int f = ((e + d) % N + N) % N;
        const int ad = d < 0 ? -d : d;
        double oa[Q][4], sa[Q][4];
        for (int g = 0; g < Q; ++g)
            for (int v = 0; v < 4; ++v) oa[g][v] = sa[g][v] = 0.0;
        const double kRmin = far_kRmin(c.k, h, PX[e * Q + Q / 2] - PX[f * Q + Q / 2],
                                       PY[e * Q + Q / 2] - PY[f * Q + Q / 2]);
        if (ad > nb && kRmin < kAsymMin) {
            const zd *Om[4] = {O0, O1, O2, O3};
            const int ri[2] = {e, (e + 1) % N}, rf[2] = {f, (f + 1) % N};
            zd o[4][2][2];
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b) {
                    const bool far_entry = cdist(ri[a], rf[b], N) >= nb + 2;
                    for (int m = 0; m < 4; ++m)
                        o[m][a][b] = far_entry ? Om[m][(int64_t)ri[a] + (int64_t)rf[b] * ld]
                                               : mk(0.0, 0.0);
                }
            const double k = c.k, h2 = h * h;
            for (int g = 0; g < Q; ++g) {
                const double xo = PX[e * Q + g], yo = PY[e * Q + g];
                const double txo = PTX[e * Q + g], tyo = PTY[e * Q + g];
                const double xg = qc.xi[g], wg = qc.w[g];
                const double pg[2] = {1.0 - xg, xg};
                for (int hh = 0; hh < Q; ++hh) {
                    const double xs = PX[f * Q + hh], ys = PY[f * Q + hh];
                    const double txs = PTX[f * Q + hh], tys = PTY[f * Q + hh];
                    const double xh = qc.xi[hh], wh = qc.w[hh];
                    const double ph[2] = {1.0 - xh, xh};
                    const double dx = xo - xs, dy = yo - ys;
                    const double R = sqrt(dx * dx + dy * dy);
                    const double nu = (dx * tys - dy * txs) / R;
                    const double nn = txo * txs + tyo * tys;
                    zd g0, g1, t0, t1;
                    pair_kernels(c, R, 1.0, g0, g1, t0, t1);
                    const double ww = wg * wh, hw = h2 * ww;
                    zd wm[4] = {mk(0.0, 0.0), mk(0.0, 0.0), mk(0.0, 0.0), mk(0.0, 0.0)};
                    zd wsg = mk(0.0, 0.0);
                    for (int a = 0; a < 2; ++a)
                        for (int b = 0; b < 2; ++b) {
                            for (int m = 0; m < 4; ++m) wm[m] = wm[m] + o[m][a][b] * (pg[a] * ph[b]);
                            wsg = wsg + o[1][a][b] * (a == b ? 1.0 : -1.0);
                        }
                    SmoothW W;
                    W.wD = wm[0] * hw;
                    W.wN2 = wm[1] * hw;
                    W.wDt = wm[2] * hw;
                    W.wS = wm[3] * hw;
                    W.wN1 = wsg * ww;
                    const PairD pd = smooth_pair_adjoint(k, c.kt, R, nu, nn, g0, g1, t0, t1, W);
                    pair_geom_adjoint(dx, dy, R, nu, txo, tyo, txs, tys, pd, oa[g], sa[hh]);
                    hbar += 2.0 * pd.vh2 / h;
                    bbar += pd.beta;
                }
            }
        }
        for (int g = 0; g < Q; ++g)
            for (int v = 0; v < 4; ++v) {
                const size_t at = ((size_t)v * nd + didx) * np + (size_t)e * Q + g;
                ob[at] = oa[g][v];
                sb[at] = sa[g][v];
            }
    }
    __shared__ double red[2][256];
    red[0][threadIdx.x] = hbar;
    red[1][threadIdx.x] = bbar;
    __syncthreads();
    for (int o = 128; o >= 1; o >>= 1) {
        if ((int)threadIdx.x < o) {
            red[0][threadIdx.x] += red[0][threadIdx.x + o];
            red[1][threadIdx.x] += red[1][threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        spart[2 * (size_t)blockIdx.x] = red[0][0];
        spart[2 * (size_t)blockIdx.x + 1] = red[1][0];
    }
}

// adj[v][x Q + g] += sum_d ob[v][d][x Q + g] + sum_d sb[v][d][(x - d) Q + g], in order of d
template <int Q>
__global__ void k_grad_band_sum(int N, int dl, int dr, const double *ob, const double *sb,
                                double *adj) {
    const int nd = dl + dr + 1;
    const int64_t np = (int64_t)N * Q;
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 4 * np) return;
    const int v = (int)(i / np);
    const int64_t p = i % np;
    const int x = (int)(p / Q), g = (int)(p % Q);
    double acc = 0.0;
    for (int didx = 0; didx < nd; ++didx) {
        const int d = didx - dl;
        const int e = ((x - d) % N + N) % N;
        acc += ob[((int64_t)v * nd + didx) * np + p];
        acc += sb[((int64_t)v * nd + didx) * np + (int64_t)e * Q + g];
    }
    adj[i] += acc;
}

// sum of the strip partials: adj[v][p] = sum_s part[s][v][p]
__global__ void k_sum_strips(int64_t np, int n_strips, const double *part, double *adj) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= 4 * np) return;
    double acc = 0.0;
    for (int s = 0; s < n_strips; ++s) acc += part[(int64_t)s * 4 * np + i];
    adj[i] = acc;
}

// work space of launch_grad_far in doubles: strip partials, then the band kernel's two
// partial arrays
size_t grad_far_ws_doubles(int N, int q, double k, double h, int nb) {
    const int n_strips = (N + 127) / 128;
    const int D = far_band_width(N, k, h, nb);
    const int dl = std::min(D, (N - 1) / 2), dr = std::min(D, N / 2);
    return (size_t)n_strips * 4 * N * q + (size_t)2 * 4 * (dl + dr + 1) * N * q;
}
// number of (d/dh, d/dbeta) pairs launch_grad_far writes to spart
int grad_far_spart_pairs(int N, double k, double h, int nb) {
    const int n_eg = (N + 63) / 64, n_strips = (N + 127) / 128;
    const int D = far_band_width(N, k, h, nb);
    const int dl = std::min(D, (N - 1) / 2), dr = std::min(D, N / 2);
    const int64_t nbt = (int64_t)N * (dl + dr + 1);
    return 3 * n_eg * n_strips + (int)((nbt + 255) / 256);
}

void launch_grad_far(int N, double h, const KernelConsts &kc, int nb, const zd *const Om[4],
                     int64_t ld, const PointTable &pt, const double *xi, const double *w,
                     double *ws, double *spart, double *adj, int &n_pairs, hipStream_t s) {
    PairConsts c = make_consts(kc);
    const int SL = 128;
    const int n_eg = (N + 63) / 64, n_strips = (N + SL - 1) / SL;
    const int n_waves = n_eg * n_strips;
    const int blocks = (n_waves + 3) / 4;
    const int D = far_band_width(N, kc.k, h, nb);
    const int dl = std::min(D, (N - 1) / 2), dr = std::min(D, N / 2);
    const int dband = std::min(D, N / 2);
    const int64_t np = (int64_t)N * pt.q;
    const int64_t nbt = (int64_t)N * (dl + dr + 1);
    const int bband = (int)((nbt + 255) / 256);
    n_pairs = 3 * n_waves + bband;
    double *part = ws;
    double *ob = ws + (size_t)n_strips * 4 * np;
    double *sb = ob + (size_t)4 * (dl + dr + 1) * np;
    ProfScope prof(PROF_FAR, 2.0 * (double)N * N * pt.q * pt.q, s);
#define CFIE_GFAR(QQ)                                                                        \
    case QQ: {                                                                              \
        QW<QQ> qc;                                                                          \
        for (int i = 0; i < QQ; ++i) { qc.xi[i] = xi[i]; qc.w[i] = w[i]; }                  \
        hipLaunchKernelGGL((k_grad_far<QQ, 0>), dim3(blocks), dim3(256), 0, s, N, h, c, nb,  \
                           dband, SL, Om[0], Om[1], Om[2], Om[3], ld, pt.x, pt.y, pt.tx,     \
                           pt.ty, qc, n_eg, n_strips, part, spart);                         \
        hipLaunchKernelGGL((k_grad_far<QQ, 1>), dim3(blocks), dim3(256), 0, s, N, h, c, nb,  \
                           dband, SL, Om[0], Om[1], Om[2], Om[3], ld, pt.x, pt.y, pt.tx,     \
                           pt.ty, qc, n_eg, n_strips, part, spart + 2 * (size_t)n_waves);   \
        hipLaunchKernelGGL((k_grad_far<QQ, 2>), dim3(blocks), dim3(256), 0, s, N, h, c, nb,  \
                           dband, SL, Om[0], Om[1], Om[2], Om[3], ld, pt.x, pt.y, pt.tx,     \
                           pt.ty, qc, n_eg, n_strips, part, spart + 4 * (size_t)n_waves);   \
        hipLaunchKernelGGL((k_grad_far_band<QQ>), dim3(bband), dim3(256), 0, s, N, h, c, nb, \
                           dl, dr, Om[0], Om[1], Om[2], Om[3], ld, pt.x, pt.y, pt.tx, pt.ty, \
                           qc, ob, sb, spart + 6 * (size_t)n_waves);                        \
        hipLaunchKernelGGL(k_sum_strips, dim3((unsigned)((4 * np + 255) / 256)), dim3(256),  \
                           0, s, np, n_strips, part, adj);                                  \
        hipLaunchKernelGGL((k_grad_band_sum<QQ>), dim3((unsigned)((4 * np + 255) / 256)),    \
                           dim3(256), 0, s, N, dl, dr, (const double *)ob,                  \
                           (const double *)sb, adj);                                        \
        break;                                                                              \
    }
    switch (pt.q) {
        CFIE_GFAR(3)
        CFIE_GFAR(4)
        CFIE_GFAR(5)
        CFIE_GFAR(6)
        CFIE_GFAR(8)
        default: break;
    }
#undef CFIE_GFAR
}

// ------------------------------------------------------------------ near pairs ------------
constexpr int kMaxQN = 16;
struct NearGradConsts {
    PairConsts pc;
    double h;
    double xi[kMaxQN], w[kMaxQN];
};

// element-pair kind as the near assembly classifies it: 0 same element, 1 source element
// follows, 2 source element precedes, -1 otherwise
__device__ __forceinline__ int pair_kind(int eo, int es, int N) {
    int off = ((es - eo) % N + N) % N;
    return off == 0 ? 0 : off == 1 ? 1 : off == N - 1 ? 2 : -1;
}

// parametric distance |s - s'| / h of touching elements (observation node xo, source xs)
__device__ __forceinline__ double touch_dist(int kind, double xo, double xs) {
    return kind == 0 ? fabs(xo - xs) : kind == 1 ? 1.0 - xo + xs : 1.0 + xo - xs;
}

// One thread per Gauss point P = (e, g) of the near table: derivative with respect to P's
// data of every near-entry term in which P takes part, as observation point (element pairs
// (e, f)) or as source point (element pairs (f, e)).  adj: [5][N q] (x, y, tx, ty, curvature),
// written; spart: per block (d/dh, d/dbeta).
__global__ __launch_bounds__(128) void k_grad_near(int N, NearGradConsts nc, int q, int nb,
                                                   const zd *__restrict__ O0,
                                                   const zd *__restrict__ O1,
                                                   const zd *__restrict__ O2,
                                                   const zd *__restrict__ O3, int64_t ld,
                                                   const double *__restrict__ PX,
                                                   const double *__restrict__ PY,
                                                   const double *__restrict__ PTX,
                                                   const double *__restrict__ PTY,
                                                   const double *__restrict__ PCV,
                                                   const double *__restrict__ mom,
                                                   double *adj, double *spart) {
    const int64_t np = (int64_t)N * q;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double hbar = 0.0, bbar = 0.0;
    if (idx < np) {
        const PairConsts &c = nc.pc;
        const double k = c.k, h = nc.h, h2 = h * h;
        const int e = (int)(idx / q), g = (int)(idx % q);
        const double xo = PX[idx], yo = PY[idx], txo = PTX[idx], tyo = PTY[idx];
        const double xg = nc.xi[g], wg = nc.w[g];
        const double pg[2] = {1.0 - xg, xg};
        const zd *Om[4] = {O0, O1, O2, O3};
        double A[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        const int span = nb + 2;
        const bool all = 2 * span + 1 >= N;
        const int nf = all ? N : 2 * span + 1;
        for (int it = 0; it < nf; ++it) {
            const int f = all ? it : ((e + it - span) % N + N) % N;
            const int fn = (f + 1) % N, en = (e + 1) % N;
            const int ri[2] = {e, en}, rf[2] = {f, fn};
            zd o1[4][2][2], o2[4][2][2];
            bool any = false;
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    const bool m1 = cdist(ri[a], rf[b], N) <= nb + 1;
                    const bool m2 = cdist(rf[a], ri[b], N) <= nb + 1;
                    any = any || m1 || m2;
#pragma unroll
                    for (int m = 0; m < 4; ++m) {
                        o1[m][a][b] = m1 ? Om[m][(int64_t)ri[a] + (int64_t)rf[b] * ld] : mk(0.0, 0.0);
                        o2[m][a][b] = m2 ? Om[m][(int64_t)rf[a] + (int64_t)ri[b] * ld] : mk(0.0, 0.0);
                    }
                }
            if (!any) continue;
            const int kind1 = pair_kind(e, f, N), kind2 = pair_kind(f, e, N);
            for (int hh = 0; hh < q; ++hh) {
                const int64_t pi = (int64_t)f * q + hh;
                const double xs = PX[pi], ys = PY[pi], txs = PTX[pi], tys = PTY[pi];
                const double xh = nc.xi[hh], wh = nc.w[hh];
                const double ph[2] = {1.0 - xh, xh};
                const double ww = wg * wh, hw = h2 * ww;
                const bool self = f == e && hh == g;
                for (int orient = 0; orient < 2; ++orient) {
                    if (orient == 1 && self) continue;
                    // orient 0: P observes (hats a on e at xg, b on f at xh);
                    // orient 1: P is the source (hats a on f at xh, b on e at xg)
                    const int kind = orient == 0 ? kind1 : kind2;
                    const double *pa = orient == 0 ? pg : ph;
                    const double *pb = orient == 0 ? ph : pg;
                    zd wm[4], wsg = mk(0.0, 0.0);
                    for (int m = 0; m < 4; ++m) {
                        zd acc = mk(0.0, 0.0);
                        for (int a = 0; a < 2; ++a)
                            for (int b = 0; b < 2; ++b) {
                                zd o = orient == 0 ? o1[m][a][b] : o2[m][a][b];
                                acc = acc + o * (pa[a] * pb[b]);
                                if (m == 1) wsg = wsg + o * ((a == b) ? 1.0 : -1.0);
                            }
                        wm[m] = acc * hw;
                    }
                    PairD d;
                    double dx = 0.0, dy = 0.0, R = 1.0, nu = 0.0, nn = 1.0;
                    if (kind >= 0) {
                        // moments of the log part: observation node first
                        const int go = orient == 0 ? g : hh, gs = orient == 0 ? hh : g;
                        const double *Mk = mom + (size_t)kind * 5 * q * q;
                        zd wmm[4], wsm = mk(0.0, 0.0);
                        const double m0 = Mk[(size_t)4 * q * q + go * q + gs];
                        for (int m = 0; m < 4; ++m) {
                            zd acc = mk(0.0, 0.0);
                            for (int a = 0; a < 2; ++a)
                                for (int b = 0; b < 2; ++b) {
                                    zd o = orient == 0 ? o1[m][a][b] : o2[m][a][b];
                                    acc = acc + o * Mk[(size_t)(2 * a + b) * q * q + go * q + gs];
                                }
                            wmm[m] = acc * h2;
                        }
                        wsm = wsg * m0;
                        SplitW W;
                        W.wD_w = wm[0]; W.wD_m = wmm[0];
                        W.wDt_w = wm[2]; W.wDt_m = wmm[2];
                        W.wS_w = wm[3]; W.wS_m = wmm[3];
                        W.wN_s = wsg * ww; W.wN_w = wm[1];
                        W.wN_sm0 = wsm; W.wN_m = wmm[1];
                        if (self) {
                            d = coincident_adjoint(k, c.kt, h, PCV[idx], W);
                        } else {
                            dx = orient == 0 ? xo - xs : xs - xo;
                            dy = orient == 0 ? yo - ys : ys - yo;
                            R = sqrt(dx * dx + dy * dy);
                            nu = orient == 0 ? (dx * tys - dy * txs) / R : (dx * tyo - dy * txo) / R;
                            nn = txo * txs + tyo * tys;
                            const double xob = orient == 0 ? xg : xh, xsb = orient == 0 ? xh : xg;
                            const double logl = log(touch_dist(kind, xob, xsb));
                            zd jk[4], jt[4];
                            {
                                const zd z = mk(k * R, 0.0);
                                BesselSplit b = bessel_split(z);
                                jk[0] = b.J0; jk[1] = b.J1;
                                hankel_from_split(z, b, jk[2], jk[3]);
                            }
                            {
                                const zd z = c.kt * R;
                                BesselSplit b = bessel_split(z);
                                jt[0] = b.J0; jt[1] = b.J1;
                                hankel_from_split(z, b, jt[2], jt[3]);
                            }
                            d = split_pair_adjoint(k, c.kt, R, nu, nn, logl, jk, jt, W);
                        }
                    } else {
                        dx = orient == 0 ? xo - xs : xs - xo;
                        dy = orient == 0 ? yo - ys : ys - yo;
                        R = sqrt(dx * dx + dy * dy);
                        nu = orient == 0 ? (dx * tys - dy * txs) / R : (dx * tyo - dy * txo) / R;
                        nn = txo * txs + tyo * tys;
                        zd g0, g1, t0, t1;
                        pair_kernels(c, R, 1.0, g0, g1, t0, t1);
                        SmoothW W;
                        W.wD = wm[0]; W.wN2 = wm[1]; W.wDt = wm[2]; W.wS = wm[3];
                        W.wN1 = wsg * ww;
                        d = smooth_pair_adjoint(k, c.kt, R, nu, nn, g0, g1, t0, t1, W);
                    }
                    if (self) {
                        A[4] += d.curv;
                    } else if (orient == 0) {
                        pair_geom_adjoint(dx, dy, R, nu, txo, tyo, txs, tys, d, A, nullptr);
                    } else {
                        pair_geom_adjoint(dx, dy, R, nu, txs, tys, txo, tyo, d, nullptr, A);
                    }
                    if (orient == 0) {
                        hbar += 2.0 * d.vh2 / h + d.h;
                        bbar += d.beta;
                    }
                }
            }
        }
        for (int v = 0; v < 5; ++v) adj[(size_t)v * np + idx] = A[v];
    }
    // per-block sums of the scalar derivatives
    __shared__ double red[2][128];
    red[0][threadIdx.x] = hbar;
    red[1][threadIdx.x] = bbar;
    __syncthreads();
    for (int o = 64; o >= 1; o >>= 1) {
        if ((int)threadIdx.x < o) {
            red[0][threadIdx.x] += red[0][threadIdx.x + o];
            red[1][threadIdx.x] += red[1][threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        spart[2 * (size_t)blockIdx.x] = red[0][0];
        spart[2 * (size_t)blockIdx.x + 1] = red[1][0];
    }
}

int launch_grad_near(int N, double h, const KernelConsts &kc, int nb, const zd *const Om[4],
                     int64_t ld, const PointTable &pt, const double *xi, const double *w,
                     const double *moments, double *adj, double *spart, hipStream_t s) {
    NearGradConsts nc;
    nc.pc = make_consts(kc);
    nc.h = h;
    for (int i = 0; i < pt.q && i < kMaxQN; ++i) {
        nc.xi[i] = xi[i];
        nc.w[i] = w[i];
    }
    const int64_t np = (int64_t)N * pt.q;
    const int bs = 128;
    const int blocks = (int)((np + bs - 1) / bs);
    ProfScope prof(PROF_NEAR, 2.0 * (double)np * (2 * nb + 5) * pt.q, s);
    hipLaunchKernelGGL(k_grad_near, dim3(blocks), dim3(bs), 0, s, N, nc, pt.q, nb, Om[0], Om[1],
                       Om[2], Om[3], ld, pt.x, pt.y, pt.tx, pt.ty, pt.curv, moments, adj, spart);
    return blocks;
}

// ------------------------------------------------------------------ plane-wave vectors ----
// e'_i(alpha) = int lambda_i (d.n) e^{ik d.r} ds, h_i(alpha) = int lambda_i e^{ik d.r} ds
// (Sec. II) with the loss Re sum_ij (WE_ij e'_ij + WH_ij h_ij), WE = aE (conj?) WEsrc, the
// same for WH (optional).  One thread per Gauss point; adds to adj[0..3] (x, y, tx, ty);
// spart: per block d/dh.
__global__ __launch_bounds__(256) void k_grad_exc(int N, int q, double h, double k,
                                                  const double *__restrict__ PX,
                                                  const double *__restrict__ PY,
                                                  const double *__restrict__ PTX,
                                                  const double *__restrict__ PTY,
                                                  const double *__restrict__ xi,
                                                  const double *__restrict__ w,
                                                  const double *__restrict__ angles, int64_t m,
                                                  const zd *__restrict__ WE, int64_t lde, zd aE,
                                                  int cE, const zd *__restrict__ WH, int64_t ldh,
                                                  zd aH, int cH, double *adj, double *spart) {
    const int64_t np = (int64_t)N * q;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double hb = 0.0;
    if (idx < np) {
        const int e = (int)(idx / q), g = (int)(idx % q);
        const int en = (e + 1) % N;
        const double x = PX[idx], y = PY[idx], tx = PTX[idx], ty = PTY[idx];
        const double p0 = 1.0 - xi[g], p1 = xi[g];
        const double wq = w[g];
        double ax = 0.0, ay = 0.0, atx = 0.0, aty = 0.0;
        for (int64_t j = 0; j < m; ++j) {
            double sa, ca;
            sincos(angles[j], &sa, &ca);
            zd we = WE[e + j * lde] * p0 + WE[en + j * lde] * p1;
            if (cE) we = conj(WE[e + j * lde]) * p0 + conj(WE[en + j * lde]) * p1;
            we = aE * we;
            zd wh = mk(0.0, 0.0);
            if (WH) {
                wh = cH ? conj(WH[e + j * ldh]) * p0 + conj(WH[en + j * ldh]) * p1
                        : WH[e + j * ldh] * p0 + WH[en + j * ldh] * p1;
                wh = aH * wh;
            }
            double sn, cs;
            sincos(k * (ca * x + sa * y), &sn, &cs);
            const zd E = mk(cs, sn);
            const double dn = ca * ty - sa * tx;
            const zd v = (we * dn + wh) * E;               // loss term / (h w_g)
            const zd ve = we * E;
            // d/dx of e^{ik d.r} = i k d_x e^{ik d.r}
            const double ik = -(v.y) * k;                  // Re(i k v) = -k Im v
            ax += ik * ca;
            ay += ik * sa;
            atx += -ve.x * sa;
            aty += ve.x * ca;
            hb += v.x;
        }
        const double hw = h * wq;
        adj[0 * np + idx] += hw * ax;
        adj[1 * np + idx] += hw * ay;
        adj[2 * np + idx] += hw * atx;
        adj[3 * np + idx] += hw * aty;
        hb *= wq;
    }
    __shared__ double red[256];
    red[threadIdx.x] = hb;
    __syncthreads();
    for (int o = 128; o >= 1; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) spart[blockIdx.x] = red[0];
}

int launch_grad_exc(int N, double h, double k, const PointTable &pt, const double *xi,
                    const double *w, const double *angles, int64_t m, const zd *WE,
                    int64_t lde, zd aE, bool cE, const zd *WH, int64_t ldh, zd aH, bool cH,
                    double *adj, double *spart, hipStream_t s) {
    const int64_t np = (int64_t)N * pt.q;
    const int blocks = (int)((np + 255) / 256);
    hipLaunchKernelGGL(k_grad_exc, dim3(blocks), dim3(256), 0, s, N, pt.q, h, k, pt.x, pt.y,
                       pt.tx, pt.ty, xi, w, angles, m, WE, lde, aE, cE ? 1 : 0, WH, ldh, aH,
                       cH ? 1 : 0, adj, spart);
    return blocks;
}

// ------------------------------------------------------------------ chain to the contour --
// Per Gauss point (parameter s = (e + xi_g) h): from the adjoints of (x, y, tx, ty, curv)
// to those of z, z', z'' at t(s) and of t itself; out[p] = {t, 2 pi sigma - t, b,
// Az, Ad1, Ad2} with b = (d loss / dt) / s'(t), 10 doubles per point.
__global__ void k_grad_prep(int N, int q, double h, double L, double c0, int Ms, const zd *cm,
                            int M, const zd *zhat, const double *xi, const double *adj,
                            int has_curv, double *out) {
    const int64_t np = (int64_t)N * q;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= np) return;
    const int e = (int)(idx / q), g = (int)(idx % q);
    const double s = ((double)e + xi[g]) * h;
    const double t = arc_param(s, L, c0, Ms, cm);
    zd z, d1, d2, d3;
    contour_derivs(t, M, zhat, z, d1, d2, d3);
    const double sp = sqrt(d1.x * d1.x + d1.y * d1.y);
    const zd T = d1 * (1.0 / sp);
    const zd az = mk(adj[0 * np + idx], adj[1 * np + idx]);
    const zd at = mk(adj[2 * np + idx], adj[3 * np + idx]);
    const double ak = has_curv ? adj[4 * np + idx] : 0.0;
    const double kap = (d1.x * d2.y - d1.y * d2.x) / (sp * sp * sp);
    // T = d1 / |d1|: d T = i T Im(conj(T) d d1) / |d1|
    const double alpha = (conj(at) * cmul_i(T)).x / sp;
    zd ad1 = cmul_i(T) * alpha;
    // curvature Im(conj(d1) d2) / |d1|^3
    const double isp3 = 1.0 / (sp * sp * sp);
    ad1 = ad1 + cmul_i(d2) * (-ak * isp3) + d1 * (-3.0 * ak * kap / (sp * sp));
    const zd ad2 = cmul_i(d1) * (ak * isp3);
    const double tbar = (conj(az) * d1 + conj(ad1) * d2 + conj(ad2) * d3).x;
    // s'(t) of the speed series (the derivative used by the arc-length inversion)
    double sdot = c0;
    {
        double sn, cs;
        sincos(t, &sn, &cs);
        const zd E1 = mk(cs, sn);
        zd E = E1;
        for (int m = 1; m <= Ms; ++m) {
            sdot += 2.0 * (cm[m - 1] * E).x;
            E = E * E1;
        }
    }
    double *o = out + 10 * idx;
    o[0] = t;
    o[1] = 2.0 * kPi * s / L - t;
    o[2] = tbar / sdot;
    o[3] = az.x; o[4] = az.y;
    o[5] = ad1.x; o[6] = ad1.y;
    o[7] = ad2.x; o[8] = ad2.y;
    o[9] = 0.0;
}

// One block per output: blocks [0, 2M] the modes m = -M..M of z (sum_p e^{-imt}(Az - i m Ad1
// - m^2 Ad2)); [2M+1, 2M+Ms] the speed modes m = 1..Ms (sum_p -2 b i (e^{-imt} - 1) / m);
// block 2M+Ms+1 the mean speed c0 (sum_p b (2 pi sigma - t)).  Points of up to two tables.
__global__ __launch_bounds__(256) void k_grad_modes(int M, int Ms, int64_t n1, const double *P1,
                                                    int64_t n2, const double *P2, zd *out) {
    const int bid = blockIdx.x;
    const int kind = bid <= 2 * M ? 0 : (bid <= 2 * M + Ms ? 1 : 2);
    const int m = kind == 0 ? bid - M : (kind == 1 ? bid - 2 * M : 0);
    const double dm = (double)m;
    zd acc = mk(0.0, 0.0);
    for (int tab = 0; tab < 2; ++tab) {
        const int64_t n = tab == 0 ? n1 : n2;
        const double *P = tab == 0 ? P1 : P2;
        for (int64_t p = threadIdx.x; p < n; p += blockDim.x) {
            const double *o = P + 10 * p;
            const double t = o[0];
            if (kind == 2) {
                acc.x += o[2] * o[1];
                continue;
            }
            double sn, cs;
            sincos(-dm * t, &sn, &cs);
            const zd Em = mk(cs, sn);                     // e^{-imt}
            if (kind == 0) {
                const zd az = mk(o[3], o[4]), ad1 = mk(o[5], o[6]), ad2 = mk(o[7], o[8]);
                acc = acc + Em * (az - cmul_i(ad1) * dm - ad2 * (dm * dm));
            } else {
                acc = acc + cmul_i(Em - mk(1.0, 0.0)) * (-2.0 * o[2] / dm);
            }
        }
    }
    __shared__ double rx[256], ry[256];
    rx[threadIdx.x] = acc.x;
    ry[threadIdx.x] = acc.y;
    __syncthreads();
    for (int o = 128; o >= 1; o >>= 1) {
        if ((int)threadIdx.x < o) {
            rx[threadIdx.x] += rx[threadIdx.x + o];
            ry[threadIdx.x] += ry[threadIdx.x + o];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) out[bid] = mk(rx[0], ry[0]);
}

void launch_grad_prep(const GeomDev &g, const PointTable &pt, const double *xi,
                      const double *adj, bool has_curv, double *out, hipStream_t s) {
    const int64_t np = (int64_t)g.N * pt.q;
    hipLaunchKernelGGL(k_grad_prep, dim3((unsigned)((np + 255) / 256)), dim3(256), 0, s, g.N,
                       pt.q, g.h, g.L, g.c0, g.Ms, g.cm, g.M, g.zhat, xi, adj, has_curv ? 1 : 0,
                       out);
}

void launch_grad_modes(int M, int Ms, int64_t n1, const double *P1, int64_t n2,
                       const double *P2, zd *out, hipStream_t s) {
    hipLaunchKernelGGL(k_grad_modes, dim3(2 * M + Ms + 2), dim3(256), 0, s, M, Ms, n1, P1, n2,
                       P2, out);
}

// ------------------------------------------------------------------ small helpers ---------
// Re sum_ij conj(A_ij) (G B)_ij, G = h circ(2/3, 1/6, ..., 1/6) (the Gram matrix); per-block
// partial sums
__global__ void k_gdot(int N, int64_t m, double h, const zd *A, int64_t lda, const zd *B,
                       int64_t ldb, zd coef, double *part) {
    const int64_t n = (int64_t)N * m;
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double v = 0.0;
    if (idx < n) {
        const int i = (int)(idx % N);
        const int64_t j = idx / N;
        const int im = i == 0 ? N - 1 : i - 1, ip = i == N - 1 ? 0 : i + 1;
        const zd *b = B + j * ldb;
        const zd gb = b[i] * (2.0 * h / 3.0) + (b[im] + b[ip]) * (h / 6.0);
        v = (coef * conj(A[i + j * lda]) * gb).x;
    }
    __shared__ double red[256];
    red[threadIdx.x] = v;
    __syncthreads();
    for (int o = 128; o >= 1; o >>= 1) {
        if ((int)threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

int launch_gdot(int N, int64_t m, double h, const zd *A, int64_t lda, const zd *B, int64_t ldb,
                zd coef, double *part, hipStream_t s) {
    const int64_t n = (int64_t)N * m;
    const int blocks = (int)((n + 255) / 256);
    hipLaunchKernelGGL(k_gdot, dim3(blocks), dim3(256), 0, s, N, m, h, A, lda, B, ldb, coef,
                       part);
    return blocks;
}

// dst[j + i ldd] = alpha op(src[i + j lds]) (op = conj when cj), src rows x cols
__global__ void k_transpose(int64_t rows, int64_t cols, const zd *src, int64_t lds, zd *dst,
                            int64_t ldd, zd alpha, int cj) {
    __shared__ zd tile[32][33];
    const int64_t i0 = (int64_t)blockIdx.x * 32, j0 = (int64_t)blockIdx.y * 32;
    const int tx = threadIdx.x, ty = threadIdx.y;       // 32 x 8
    for (int r = ty; r < 32; r += 8) {
        const int64_t i = i0 + tx, j = j0 + r;
        if (i < rows && j < cols) {
            zd v = src[i + j * lds];
            tile[r][tx] = cj ? conj(v) : v;
        }
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        const int64_t j = j0 + tx, i = i0 + r;
        if (i < rows && j < cols) dst[j + i * ldd] = alpha * tile[tx][r];
    }
}

void launch_transpose(int64_t rows, int64_t cols, const zd *src, int64_t lds, zd *dst,
                      int64_t ldd, zd alpha, bool cj, hipStream_t s) {
    if (rows <= 0 || cols <= 0) return;
    dim3 grid((unsigned)((rows + 31) / 32), (unsigned)((cols + 31) / 32));
    hipLaunchKernelGGL(k_transpose, grid, dim3(32, 8), 0, s, rows, cols, src, lds, dst, ldd,
                       alpha, cj ? 1 : 0);
}

// dst = alpha conj(src) elementwise (rows x cols)
__global__ void k_conj_scale(int64_t rows, int64_t cols, const zd *src, int64_t lds, zd *dst,
                             int64_t ldd, zd alpha) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= rows * cols) return;
    const int64_t i = idx % rows, j = idx / rows;
    dst[i + j * ldd] = alpha * conj(src[i + j * lds]);
}

void launch_conj_scale(int64_t rows, int64_t cols, const zd *src, int64_t lds, zd *dst,
                       int64_t ldd, zd alpha, hipStream_t s) {
    const int64_t n = rows * cols;
    if (n <= 0) return;
    hipLaunchKernelGGL(k_conj_scale, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, rows,
                       cols, src, lds, dst, ldd, alpha);
}

}  // namespace cfie
