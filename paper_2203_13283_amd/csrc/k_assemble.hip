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
#include "pair_kernels.h"

namespace cfie {

// ------------------------------------------------------------------ Gauss points ----------
__global__ void k_points(int N, int q, double h, double L, double c0, int Ms, const zd *cm,
                         int M, const zd *zhat, const double *xi, double *X, double *Y,
                         double *TX, double *TY, double *CV) {
    int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= N * q) return;
    int e = idx / q, g = idx - e * q;
    double s = ((double)e + xi[g]) * h;
    double t = arc_param(s, L, c0, Ms, cm);
    zd z, d1, d2, d3;
    contour_derivs(t, M, zhat, z, d1, d2, d3);
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

// ------------------------------------------------------------------ far kernel -----------
constexpr int kFarCols = 64;          // node columns per wavefront

template <int Q>
struct QuadConsts {
    double xi[Q], w[Q];
    double ha0[Q], ha1[Q];           // h w_g phi_0(xi_g), h w_g phi_1(xi_g) (far kernel)
};

// 2x2 block of element pair (e, f) for the four matrices: A_b[m][a] += sum_hh h w_hh
// phi_b(xi_hh) sum_g K_m(g, hh) h w_g phi_a(xi_g) (b = 0 into acc0, the node column f; b = 1
// into acc1, the node column f + 1), and for N^k the Maue term K (s_a s_b w_g w_hh -
// k^2 n.n' h^2 w_g w_hh phi_a phi_b) with s_a = +/-1 the sign of phi_a'.  SPLIT: the sums
// over the row element's points g come first, weighted by phi_a only, and the column
// weights phi_b once per column point hh (half the multiply-adds per point pair, for 36 more
// registers); otherwise every point pair adds into the accumulators with its full weight.
// Lanes with on = false add nothing (their kernel is evaluated at a harmless separation).
// KERNEL(R, 1/R, nu, gk, Dk, St, Dt) evaluates the point-pair kernels (in the large-argument
// passes without their constant prefactors, which the write-out applies).
template <int Q, bool SPLIT, typename KERNEL>
__device__ __forceinline__ void far_block(const double *rp, int fe, bool on, double rsafe,
                                          double h, double k2, const double *__restrict__ PX,
                                          const double *__restrict__ PY,
                                          const double *__restrict__ PTX,
                                          const double *__restrict__ PTY,
                                          const QuadConsts<Q> &qc, zd (&acc0)[4][2],
                                          zd (&acc1)[4][2], KERNEL kern) {
    // rp: this lane's row-element points in LDS, [4][Q] with stride 256 (x, y, tx, ty)
    const double msk = on ? 1.0 : 0.0;
    // lanes that add nothing get dx = rsafe, dy = 0 (multiplies instead of selects)
    const double dx_off = on ? 0.0 : rsafe;
#pragma unroll 1
    for (int hh = 0; hh < Q; ++hh) {
        const double xs = PX[fe * Q + hh], ys = PY[fe * Q + hh];
        const double txs = PTX[fe * Q + hh], tys = PTY[fe * Q + hh];
        const double xh = qc.xi[hh], wh = qc.w[hh];
        const double wb0 = msk * h * wh * (1.0 - xh), wb1 = msk * h * wh * xh;
        const double whm = msk * wh;
        zd sD[2], sDt[2], sS[2], sNn[2], sNw = mk(0.0, 0.0);
#pragma unroll
        for (int aa = 0; aa < 2; ++aa) sD[aa] = sDt[aa] = sS[aa] = sNn[aa] = mk(0.0, 0.0);
#pragma unroll 1
        for (int g = 0; g < Q; ++g) {
            const double dx = fma(rp[(0 * Q + g) * 256] - xs, msk, dx_off);
            const double dy = (rp[(1 * Q + g) * 256] - ys) * msk;
            // 1/R from one reciprocal square root; R and nu = (r - r').n' / R from it
            const double r2 = fma(dx, dx, dy * dy);
            const double invR = rsqrt_pos(r2);
            const double R = r2 * invR;
            const double nu = (dx * tys - dy * txs) * invR;
            const double nn = rp[(3 * Q + g) * 256] * tys + rp[(2 * Q + g) * 256] * txs;
            zd gk, Dk, St, Dt;
            kern(R, invR, nu, gk, Dk, St, Dt);
            const double wa[2] = {qc.ha0[g], qc.ha1[g]};
            if constexpr (SPLIT) {
                const zd gn = gk * nn;
                sNw = sNw + gk * qc.w[g];
#pragma unroll
                for (int aa = 0; aa < 2; ++aa) {
                    sD[aa] = sD[aa] + Dk * wa[aa];
                    sDt[aa] = sDt[aa] + Dt * wa[aa];
                    sS[aa] = sS[aa] + St * wa[aa];
                    sNn[aa] = sNn[aa] + gn * wa[aa];
                }
            } else {
                const double wgh = whm * qc.w[g];
#pragma unroll
                for (int aa = 0; aa < 2; ++aa) {
                    const double w0 = wa[aa] * wb0, w1 = wa[aa] * wb1;
                    acc0[0][aa] = acc0[0][aa] + Dk * w0;
                    acc1[0][aa] = acc1[0][aa] + Dk * w1;
                    acc0[2][aa] = acc0[2][aa] + Dt * w0;
                    acc1[2][aa] = acc1[2][aa] + Dt * w1;
                    acc0[3][aa] = acc0[3][aa] + St * w0;
                    acc1[3][aa] = acc1[3][aa] + St * w1;
                    // s_a s_b: + for a == b
                    acc0[1][aa] = acc0[1][aa] + gk * ((aa == 0 ? wgh : -wgh) - k2 * nn * w0);
                    acc1[1][aa] = acc1[1][aa] + gk * ((aa == 1 ? wgh : -wgh) - k2 * nn * w1);
                }
            }
        }
        if constexpr (SPLIT) {
            const zd nw = sNw * whm;
#pragma unroll
            for (int aa = 0; aa < 2; ++aa) {
                acc0[0][aa] = acc0[0][aa] + sD[aa] * wb0;
                acc1[0][aa] = acc1[0][aa] + sD[aa] * wb1;
                acc0[2][aa] = acc0[2][aa] + sDt[aa] * wb0;
                acc1[2][aa] = acc1[2][aa] + sDt[aa] * wb1;
                acc0[3][aa] = acc0[3][aa] + sS[aa] * wb0;
                acc1[3][aa] = acc1[3][aa] + sS[aa] * wb1;
                // s_a s_b: + for a == b
                acc0[1][aa] = acc0[1][aa] + (aa == 0 ? nw : -nw) - sNn[aa] * (k2 * wb0);
                acc1[1][aa] = acc1[1][aa] + (aa == 1 ? nw : -nw) - sNn[aa] * (k2 * wb1);
            }
        }
    }
}


// One wavefront: 63 output rows (lane l holds element i0 - 1 + l) and kFarCols node
// columns, walking the element columns f.  Three passes over the same tiles, by the lower
// bound of k R over the element pair's point pairs (far_kRmin):
//   MODE 0: k R >= kFarFast for every point pair: the 8-term large-argument series; writes
//           every entry of the tile;
//   MODE 1: kAsymMin <= k R < kFarFast: the 22-term series (one code path for the whole
//           wavefront, no divergence between lanes); adds to the entries it touches;
//   MODE 2: the remaining element pairs outside the near band (small arguments: ascending
//           series or Miller's recurrence, per-lane forms) further than dband elements from
//           the diagonal (none on a contour that does not fold back on itself); adds to the
//           entries it touches.
// Entry (i, j) is owned by one lane in each pass, so the sum is deterministic.  The small-
// argument element pairs within dband of the diagonal go to k_far_band / k_far_band_add: a
// long serial chain per wavefront there left most of the device idle.
template <int Q, int MODE>
__global__ __launch_bounds__(256, MODE == 2 ? 1 : 2) void k_far(int N, double h, PairConsts c,
                                                           int nb, int dband, int r0, int r1,
                                                           int64_t ld,
                                                           zd *o0, zd *o1, zd *o2, zd *o3,
                                                           const double *__restrict__ PX,
                                                           const double *__restrict__ PY,
                                                           const double *__restrict__ PTX,
                                                           const double *__restrict__ PTY,
                                                           QuadConsts<Q> qc, int n_row_tiles) {
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
    if constexpr (MODE != 0) {
        // most tiles hold no element pair for these passes (the column elements j0 - 1 ..
        // jend - 1, up to 65: two per lane, clamped)
        const int fa = min(j0 - 1 + lane, jend - 1), fb = min(j0 + lane, jend - 1);
        const int fea = (fa % N + N) % N, feb = (fb % N + N) % N;
        if (far_tile_all_fast(c.k, h, PX[e * Q + Q / 2], PY[e * Q + Q / 2],
                              PX[fea * Q + Q / 2], PY[fea * Q + Q / 2], PX[feb * Q + Q / 2],
                              PY[feb * Q + Q / 2]))
            return;
    }
    // the row element's Gauss points live in LDS (one column of 4 Q doubles per thread)
    __shared__ double rows_lds[4 * Q * 256];
    double *rp = rows_lds + threadIdx.x;
#pragma unroll
    for (int g = 0; g < Q; ++g) {
        rp[(0 * Q + g) * 256] = PX[e * Q + g];
        rp[(1 * Q + g) * 256] = PY[e * Q + g];
        rp[(2 * Q + g) * 256] = PTX[e * Q + g];
        rp[(3 * Q + g) * 256] = PTY[e * Q + g];
    }
    const double xref = rp[(0 * Q + Q / 2) * 256], yref = rp[(1 * Q + Q / 2) * 256];
    const double k2 = c.k * c.k;
    const double rsafe = 1000.0 * c.invk;             // k R = 1000 for lanes that add nothing
    const int out_row = i0 + lane;                    // row produced by this lane (a = 1 part)
    const bool row_ok = lane < 63 && out_row < r1 && out_row < N;
    // acc0[m][a]: node column f (b = 0 of element f plus b = 1 of element f - 1);
    // acc1[m][a]: node column f + 1 (b = 1 of element f)
    zd acc0[4][2], acc1[4][2];
#pragma unroll
    for (int m = 0; m < 4; ++m) acc0[m][0] = acc0[m][1] = acc1[m][0] = acc1[m][1] = mk(0.0, 0.0);
    bool used_prev = false;                           // MODE > 0: this lane added at f - 1
    for (int f = j0 - 1; f < jend; ++f) {
        int fe = (f % N + N) % N;
        int off = fe - e;
        off = ((off % N) + N) % N;
        const bool on = min(off, N - off) > nb;       // near-band pairs: near kernel
        const double kRmin = far_kRmin(c.k, h, xref - PX[fe * Q + Q / 2],
                                       yref - PY[fe * Q + Q / 2]);
        const bool fast = kRmin >= kFarFast;
        const bool mid = !fast && kRmin >= kAsymMin;
        // MODE 2 leaves the element pairs within dband of the diagonal to k_far_band
        const bool use = on && (MODE == 0 ? fast
                                : MODE == 1 ? mid
                                            : (!fast && !mid && min(off, N - off) > dband));
        if (__any(use)) {
            if constexpr (MODE == 1) {
                auto K22 = [&](double R, double invR, double nu, zd &g0, zd &g1, zd &g2,
                               zd &g3) {
                    pair_kernels_asym_unscaled<kSerMax>(c, R, invR, nu, g0, g1, g2, g3);
                };
                far_block<Q, false>(rp, fe, use, rsafe, h, k2, PX, PY, PTX, PTY, qc, acc0, acc1, K22);
            } else if constexpr (MODE == 2) {
                auto KG = [&](double R, double, double nu, zd &g0, zd &g1, zd &g2, zd &g3) {
                    pair_kernels(c, R, nu, g0, g1, g2, g3);
                };
                far_block<Q, true>(rp, fe, use, rsafe, h, k2, PX, PY, PTX, PTY, qc, acc0, acc1, KG);
            } else {
                auto K8 = [&](double R, double invR, double nu, zd &g0, zd &g1, zd &g2,
                              zd &g3) {
                    pair_kernels_asym_unscaled<8>(c, R, invR, nu, g0, g1, g2, g3);
                };
                far_block<Q, true>(rp, fe, use, rsafe, h, k2, PX, PY, PTX, PTY, qc, acc0, acc1, K8);
            }
        }
        if (f >= j0) {
            int j = f;
            int dij = out_row - j;
            dij = ((dij % N) + N) % N;
            int dd = min(dij, N - dij);
            // MODE > 0: the entry changes if any of its element pairs (e, f-1), (e, f),
            // (e+1, f-1), (e+1, f) was added in this pass
            const int mine = (use || used_prev) ? 1 : 0;
            const bool touched = MODE != 0 ? (mine | __shfl_down(mine, 1)) != 0 : true;
            zd *outs[4] = {o0, o1, o2, o3};
            // the large-argument passes sum kernels without their constant prefactors
            const zd scale[4] = {c.CD, c.Cg, c.CDt, c.CS};
#pragma unroll
            for (int m = 0; m < 4; ++m) {
                // row out_row = e + 1: own a = 1 part + a = 0 part of lane + 1
                double nx = __shfl_down(acc0[m][0].x, 1);
                double ny = __shfl_down(acc0[m][0].y, 1);
                zd v = acc0[m][1] + mk(nx, ny);
                if constexpr (MODE != 2) v = scale[m] * v;
                if (row_ok && dd >= nb + 2 && touched) {
                    zd *dst = outs[m] + (int64_t)out_row + (int64_t)j * ld;
                    if (MODE != 0) v = v + *dst;
                    *dst = v;
                }
            }
        }
        used_prev = use;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            acc0[m][0] = acc1[m][0];
            acc0[m][1] = acc1[m][1];
            acc1[m][0] = acc1[m][1] = mk(0.0, 0.0);
        }
    }
}

// Element pairs (e, f = e + d) with nb < |d| <= dband whose k R can be below kAsymMin (the
// MODE 2 condition of k_far): one thread per element pair, lanes of a wavefront share the
// offset d (similar arguments, coherent branches).  The 2x2 node block of each of the four
// matrices goes to Bk[((m 4 + 2a + b) nd + didx) ne + eidx] (zero for the other pairs);
// elements e = r0 - 1 + eidx, offsets d = didx - dl.
template <int Q>
__global__ __launch_bounds__(256) void k_far_band(int N, double h, PairConsts c, int nb, int dl,
                                                  int dr, int r0, int ne,
                                                  const double *__restrict__ PX,
                                                  const double *__restrict__ PY,
                                                  const double *__restrict__ PTX,
                                                  const double *__restrict__ PTY,
                                                  QuadConsts<Q> qc, zd *Bk) {
    const int nd = dl + dr + 1;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= (int64_t)ne * nd) return;
    const int eidx = (int)(tid % ne), didx = (int)(tid / ne);
    const int d = didx - dl;
    const int e = ((r0 - 1 + eidx) % N + N) % N;
    const int f = ((e + d) % N + N) % N;
    zd acc[4][2][2];
#pragma unroll
    for (int m = 0; m < 4; ++m)
        acc[m][0][0] = acc[m][0][1] = acc[m][1][0] = acc[m][1][1] = mk(0.0, 0.0);
    const double kRmin = far_kRmin(c.k, h, PX[e * Q + Q / 2] - PX[f * Q + Q / 2],
                                   PY[e * Q + Q / 2] - PY[f * Q + Q / 2]);
    const int ad = d < 0 ? -d : d;
    if (ad > nb && kRmin < kAsymMin) {
        const double k2 = c.k * c.k;
        for (int g = 0; g < Q; ++g) {
            const double xo = PX[e * Q + g], yo = PY[e * Q + g];
            const double txo = PTX[e * Q + g], tyo = PTY[e * Q + g];
            const double xg = qc.xi[g], wg = qc.w[g];
            const double wa[2] = {h * wg * (1.0 - xg), h * wg * xg};
            for (int hh = 0; hh < Q; ++hh) {
                const double xs = PX[f * Q + hh], ys = PY[f * Q + hh];
                const double txs = PTX[f * Q + hh], tys = PTY[f * Q + hh];
                const double xh = qc.xi[hh], wh = qc.w[hh];
                const double wb[2] = {h * wh * (1.0 - xh), h * wh * xh};
                const double dx = xo - xs, dy = yo - ys;
                const double R = sqrt(dx * dx + dy * dy);
                const double nu = (dx * tys - dy * txs) / R;
                const double nn = tyo * tys + txo * txs;
                zd gk, Dk, St, Dt;
                pair_kernels(c, R, nu, gk, Dk, St, Dt);
                const double wgh = wg * wh;
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int b = 0; b < 2; ++b) {
                        const double w = wa[a] * wb[b];
                        acc[0][a][b] = acc[0][a][b] + Dk * w;
                        acc[2][a][b] = acc[2][a][b] + Dt * w;
                        acc[3][a][b] = acc[3][a][b] + St * w;
                        acc[1][a][b] = acc[1][a][b] + gk * ((a == b ? wgh : -wgh) - k2 * nn * w);
                    }
            }
        }
    }
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
                Bk[((int64_t)(m * 4 + 2 * a + b) * nd + didx) * ne + eidx] = acc[m][a][b];
}

// entry (i, j), r0 <= i < r1, in the far region (cyclic |i - j| >= nb + 2) within dband + 1
// of the diagonal: adds the blocks of its element pairs (i - a, j - b) that k_far_band holds
template <int Q>
__global__ __launch_bounds__(256) void k_far_band_add(int N, int nb, int dl, int dr, int r0,
                                                      int r1, int ne, int64_t ld, zd *o0,
                                                      zd *o1, zd *o2, zd *o3,
                                                      const zd *__restrict__ Bk) {
    const int nd = dl + dr + 1;
    const int nrows = r1 - r0;
    const int no = dl + dr + 3;                      // entry offsets -(dl+1) .. dr+1
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= (int64_t)nrows * no) return;
    const int i = r0 + (int)(tid % nrows);
    const int o = (int)(tid / nrows) - (dl + 1);
    // one representative per entry: offsets in (-N/2, N/2]
    if (2 * o <= -N || 2 * o > N) return;
    const int ao = o < 0 ? -o : o;
    if (min(ao, N - ao) < nb + 2) return;
    const int j = ((i + o) % N + N) % N;
    zd v[4] = {mk(0.0, 0.0), mk(0.0, 0.0), mk(0.0, 0.0), mk(0.0, 0.0)};
    bool any = false;
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            // element pair (e = i - a, f = j - b), offset o - b + a in (-N/2, N/2]
            int d = o - b + a;
            d = ((d % N) + N) % N;
            if (2 * d > N) d -= N;
            if (d < -dl || d > dr) continue;
            const int eidx = i - a - (r0 - 1);
            if (eidx < 0 || eidx >= ne) continue;
            const int didx = d + dl;
            any = true;
            for (int m = 0; m < 4; ++m)
                v[m] = v[m] + Bk[((int64_t)(m * 4 + 2 * a + b) * nd + didx) * ne + eidx];
        }
    if (!any) return;
    zd *outs[4] = {o0, o1, o2, o3};
    const int64_t idx = (int64_t)i + (int64_t)j * ld;
    for (int m = 0; m < 4; ++m) outs[m][idx] = outs[m][idx] + v[m];
}

// half-widths (dl, dr) of the band of k_far_band: past it the chord between the elements'
// reference points exceeds kAsymMin / k + 2h on a contour that does not fold back (arc
// length and chord agree to second order), with a margin of a quarter and four elements
int far_band_width(int N, double k, double h, int nb) {
    const double w = 1.25 * kAsymMin / (k * h) + 4.0;
    int D = nb + (int)std::ceil(w);
    return D;
}
size_t far_band_ws_elems(const AsmParams &p) {
    const int D = far_band_width(p.N, p.kc.k, p.h, p.nb);
    const int dl = std::min(D, (p.N - 1) / 2), dr = std::min(D, p.N / 2);
    const int ne = std::min(p.r1 - p.r0 + 1, p.N + 1);
    return (size_t)16 * (size_t)(dl + dr + 1) * (size_t)ne;
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
    const int D = far_band_width(p.N, p.kc.k, p.h, p.nb);
    const int dl = std::min(D, (p.N - 1) / 2), dr = std::min(D, p.N / 2);
    const int dband = std::min(D, p.N / 2);
    const int ne = std::min(p.r1 - p.r0 + 1, p.N + 1);
    const int64_t nbe = (int64_t)ne * (dl + dr + 1);
    const int64_t nbadd = (int64_t)(p.r1 - p.r0) * (dl + dr + 3);
#define CFIE_FAR_CASE(QQ)                                                                   \
    case QQ: {                                                                             \
        QuadConsts<QQ> qc;                                                                 \
        for (int i = 0; i < QQ; ++i) {                                                     \
            qc.xi[i] = xi[i];                                                              \
            qc.w[i] = w[i];                                                                \
            qc.ha0[i] = p.h * w[i] * (1.0 - xi[i]);                                        \
            qc.ha1[i] = p.h * w[i] * xi[i];                                                \
        }                                                                                  \
        hipLaunchKernelGGL((k_far<QQ, 0>), dim3(blocks), dim3(256), 0, s, p.N, p.h, c,     \
                           p.nb, dband, p.r0, p.r1, p.ld, p.out[0], p.out[1], p.out[2],     \
                           p.out[3], far.x, far.y, far.tx, far.ty, qc, n_row_tiles);       \
        hipLaunchKernelGGL((k_far<QQ, 1>), dim3(blocks), dim3(256), 0, s, p.N, p.h, c,     \
                           p.nb, dband, p.r0, p.r1, p.ld, p.out[0], p.out[1], p.out[2],     \
                           p.out[3], far.x, far.y, far.tx, far.ty, qc, n_row_tiles);       \
        hipLaunchKernelGGL((k_far<QQ, 2>), dim3(blocks), dim3(256), 0, s, p.N, p.h, c,     \
                           p.nb, dband, p.r0, p.r1, p.ld, p.out[0], p.out[1], p.out[2],     \
                           p.out[3], far.x, far.y, far.tx, far.ty, qc, n_row_tiles);       \
        hipLaunchKernelGGL((k_far_band<QQ>), dim3((unsigned)((nbe + 255) / 256)), dim3(256), \
                           0, s, p.N, p.h, c, p.nb, dl, dr, p.r0, ne, far.x, far.y, far.tx, \
                           far.ty, qc, p.ws);                                              \
        hipLaunchKernelGGL((k_far_band_add<QQ>), dim3((unsigned)((nbadd + 255) / 256)),    \
                           dim3(256), 0, s, p.N, p.nb, dl, dr, p.r0, p.r1, ne, p.ld,        \
                           p.out[0], p.out[1], p.out[2], p.out[3], (const zd *)p.ws);      \
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

// The 2x2 node blocks acc[m][a][b] (m: Dk, Nk, Dkt, Skt; a, b: hats of the observation and
// source elements) of element pair (e, f) (kind: -1 regular, 0 same, 1 f = e+1,
// 2 f = e-1), all four hat combinations from one evaluation of the kernels per point pair.
__device__ void near_block(const NearConsts &nc, int q, int e, int f, int kind,
                           const double *__restrict__ PX, const double *__restrict__ PY,
                           const double *__restrict__ PTX, const double *__restrict__ PTY,
                           const double *__restrict__ PCV, const double *__restrict__ mom,
                           zd (&acc)[4][2][2]) {
    const PairConsts &c = nc.pc;
    const double h = nc.h;
    const double k = c.k;
    const double k2 = k * k;
    const double *Mk = mom + (size_t)(kind < 0 ? 0 : kind) * 5 * q * q;
    const double inv2pi = 1.0 / (2.0 * kPi);
    for (int g = 0; g < q; ++g) {
        const double xg = nc.xi[g];
        const double pa[2] = {1.0 - xg, xg};
        const double xo = PX[e * q + g], yo = PY[e * q + g];
        const double txo = PTX[e * q + g], tyo = PTY[e * q + g];
        for (int hh = 0; hh < q; ++hh) {
            const double xh = nc.xi[hh];
            const double pb[2] = {1.0 - xh, xh};
            const double wgt = nc.w[g] * nc.w[hh];
            const double xs = PX[f * q + hh], ys = PY[f * q + hh];
            const double txs = PTX[f * q + hh], tys = PTY[f * q + hh];
            if (kind < 0) {
                const double dx = xo - xs, dy = yo - ys;
                const double R = sqrt(dx * dx + dy * dy);
                const double nu = (dx * tys - dy * txs) / R;
                const double nn = tyo * tys + txo * txs;
                zd gk, Dk, St, Dt;
                pair_kernels(c, R, nu, gk, Dk, St, Dt);
                for (int a = 0; a < 2; ++a)
                    for (int b = 0; b < 2; ++b) {
                        const double hw = h * h * wgt * pa[a] * pb[b];
                        const double sab = (a == b) ? 1.0 : -1.0;
                        acc[0][a][b] = acc[0][a][b] + Dk * hw;
                        acc[2][a][b] = acc[2][a][b] + Dt * hw;
                        acc[3][a][b] = acc[3][a][b] + St * hw;
                        acc[1][a][b] = acc[1][a][b] + gk * (wgt * sab - k2 * nn * hw);
                    }
                continue;
            }
            const double m0 = Mk[(size_t)4 * q * q + g * q + hh];
            zd Ag, As, Ad, At, Bg, Bs, Bd, Bt;
            double nn;
            if (kind == 0 && g == hh) {
                // coincident points: limits of the smooth parts as R -> 0
                const double kc_ = PCV[e * q + g];
                Ag = mk(-inv2pi, 0.0);
                As = Ag;
                Ad = At = mk(0.0, 0.0);
                Bg = mk(0.0, 0.25) - (nc.logk2 + mk(kEulerGamma, 0.0)) * inv2pi;
                Bs = mk(0.0, 0.25) - (nc.logkt2 + mk(kEulerGamma, 0.0)) * inv2pi;
                Bd = Bt = mk(-kc_ / (4.0 * kPi), 0.0);
                nn = 1.0;
            } else {
                const double dx = xo - xs, dy = yo - ys;
                const double R = sqrt(dx * dx + dy * dy);
                const double nu = (dx * tys - dy * txs) / R;
                nn = tyo * tys + txo * txs;
                double sig;
                if (kind == 0) sig = h * fabs(xg - xh);
                else if (kind == 1) sig = h * (1.0 - xg + xh);
                else sig = h * (1.0 + xg - xh);
                const double lr = log(R / sig);
                const BesselSplit b1 = bessel_split(mk(k * R, 0.0));
                const BesselSplit b2 = bessel_split(c.kt * R);
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
                const zd kk = mk(k, 0.0);
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
            for (int a = 0; a < 2; ++a)
                for (int b = 0; b < 2; ++b) {
                    const double mab = Mk[(size_t)(2 * a + b) * q * q + g * q + hh];
                    const double hw = h * h * wgt * pa[a] * pb[b];
                    const double hm = h * h * mab;
                    const double sab = (a == b) ? 1.0 : -1.0;
                    acc[0][a][b] = acc[0][a][b] + Bd * hw + Ad * hm;
                    acc[2][a][b] = acc[2][a][b] + Bt * hw + At * hm;
                    acc[3][a][b] = acc[3][a][b] + Bs * hw + As * hm;
                    acc[1][a][b] = acc[1][a][b] + Bg * (wgt * sab - k2 * nn * hw) +
                                   Ag * (sab * m0 - k2 * nn * hm);
                }
        }
    }
}

// One thread per element pair (e = r0 - 1 + eidx, f = e + d) with |d| <= nb + 2 (the pairs
// that feed the near entries); lanes of a wavefront share d.  Blocks to
// Bk[((m 4 + 2a + b) nd + didx) ne + eidx], d = didx - dl.
__global__ __launch_bounds__(128) void k_near_pairs(int N, NearConsts nc, int q, int dl, int dr,
                                                    int r0, int ne,
                                                    const double *__restrict__ PX,
                                                    const double *__restrict__ PY,
                                                    const double *__restrict__ PTX,
                                                    const double *__restrict__ PTY,
                                                    const double *__restrict__ PCV,
                                                    const double *__restrict__ mom, zd *Bk) {
    const int nd = dl + dr + 1;
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= (int64_t)ne * nd) return;
    const int eidx = (int)(tid % ne), didx = (int)(tid / ne);
    const int d = didx - dl;
    const int e = ((r0 - 1 + eidx) % N + N) % N;
    const int f = ((e + d) % N + N) % N;
    const int off = ((f - e) % N + N) % N;
    const int kind = off == 0 ? 0 : off == 1 ? 1 : off == N - 1 ? 2 : -1;
    zd acc[4][2][2];
    for (int m = 0; m < 4; ++m)
        acc[m][0][0] = acc[m][0][1] = acc[m][1][0] = acc[m][1][1] = mk(0.0, 0.0);
    near_block(nc, q, e, f, kind, PX, PY, PTX, PTY, PCV, mom, acc);
    for (int m = 0; m < 4; ++m)
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b)
                Bk[((int64_t)(m * 4 + 2 * a + b) * nd + didx) * ne + eidx] = acc[m][a][b];
}

// Entry (i, j), r0 <= i < r1, cyclic |i - j| <= nb + 1: the sum of its four element pairs'
// blocks, in the order (i-1, j-1), (i-1, j), (i, j-1), (i, j).
__global__ __launch_bounds__(256) void k_near_write(int N, int nb, int dl, int dr, int r0, int r1,
                                                    int ne, int64_t ld, zd *o0, zd *o1,
                                                    zd *o2, zd *o3, const zd *__restrict__ Bk) {
    const int nd = dl + dr + 1;
    const int nrows = r1 - r0;
    const int no = 2 * nb + 3;                        // offsets -(nb+1) .. nb+1
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= (int64_t)nrows * no) return;
    const int i = r0 + (int)(tid % nrows);
    const int o = (int)(tid / nrows) - (nb + 1);
    // one representative per entry when the band wraps around a small mesh
    if (2 * (nb + 1) + 1 > N) {
        int dd = ((o % N) + N) % N;
        const int rep = 2 * dd > N ? dd - N : dd;
        if (rep != o) return;
    }
    const int j = ((i + o) % N + N) % N;
    zd v[4] = {mk(0.0, 0.0), mk(0.0, 0.0), mk(0.0, 0.0), mk(0.0, 0.0)};
    for (int p = 0; p < 4; ++p) {
        const int a = (p >> 1) ? 0 : 1, b = (p & 1) ? 0 : 1;
        int d = o - b + a;
        d = ((d % N) + N) % N;
        if (2 * d > N) d -= N;
        const int eidx = i - a - (r0 - 1);
        const int didx = d + dl;
        for (int m = 0; m < 4; ++m)
            v[m] = v[m] + Bk[((int64_t)(m * 4 + 2 * a + b) * nd + didx) * ne + eidx];
    }
    const int64_t idx = (int64_t)i + (int64_t)j * ld;
    o0[idx] = v[0];
    o1[idx] = v[1];
    o2[idx] = v[2];
    o3[idx] = v[3];
}

size_t near_ws_elems(const AsmParams &p) {
    const int D = p.nb + 2;
    const int dl = std::min(D, (p.N - 1) / 2), dr = std::min(D, p.N / 2);
    const int ne = std::min(p.r1 - p.r0 + 1, p.N + 1);
    return (size_t)16 * (size_t)(dl + dr + 1) * (size_t)ne;
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
    const int D = p.nb + 2;
    const int dl = std::min(D, (p.N - 1) / 2), dr = std::min(D, p.N / 2);
    const int ne = std::min(p.r1 - p.r0 + 1, p.N + 1);
    const int64_t npairs = (int64_t)ne * (dl + dr + 1);
    const int64_t nent = (int64_t)(p.r1 - p.r0) * (2 * p.nb + 3);
    ProfScope prof(PROF_NEAR, (double)npairs * near.q * near.q, s);
    hipLaunchKernelGGL(k_near_pairs, dim3((unsigned)((npairs + 127) / 128)), dim3(128), 0, s,
                       p.N, nc, near.q, dl, dr, p.r0, ne, near.x, near.y, near.tx, near.ty,
                       near.curv, moments, p.ws);
    hipLaunchKernelGGL(k_near_write, dim3((unsigned)((nent + 255) / 256)), dim3(256), 0, s, p.N,
                       p.nb, dl, dr, p.r0, p.r1, ne, p.ld, p.out[0], p.out[1], p.out[2], p.out[3],
                       (const zd *)p.ws);
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
    if (H) H[i + jc * ld] = hv;
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
