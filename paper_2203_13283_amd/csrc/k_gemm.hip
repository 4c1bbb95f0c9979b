// Complex GEMM on CDNA matrix cores: C = alpha * op(A) * B + beta * C with op(A) = A or A^H,
// column-major, complex interleaved.  Used for every dense product of the method: the
// sketch of the remainder C - C_c (Sec. V eq. (7)), the capacitance matrix of eq. (9) and
// the Woodbury correction, and the FP64 residual of the refinement.
//
// The complex product runs on split real/imaginary tiles held in LDS with the 16x16x4 MFMA
// (f64 or f32), either as four real products per k-step (Cr += Ar Br - Ai Bi,
// Ci += Ar Bi + Ai Br) or as three (the 3M form: P1 = Ar Br, P2 = Ai Bi,
// P3 = (Ar + Ai)(Br + Bi), Cr = P1 - P2, Ci = P3 - P1 - P2), which takes a quarter fewer
// matrix-core operations for a normwise error of the same order.
// Block tile BM x BN = 32 TI x 32 TJ with a K-slice of BKT, 256 threads = 4 wavefronts,
// each wavefront a (BM/2) x (BN/2) sub-tile of TI x TJ MFMA tiles of 16 x 16.  Global loads
// of the next K-slice are issued before the MFMAs of the current one.
//
// Shapes with few output tiles and a long K (Gram matrices Y^H Y, projections Q^H Y) are
// split along K over slices of the grid: each writes its partial product to a workspace and a
// second kernel sums the slices in a fixed order (deterministic) and applies alpha, beta.
#include "internal.h"

#include <atomic>
#include <condition_variable>
#include <map>
#include <mutex>
#include <type_traits>
#include <utility>

namespace cfie {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));

template <typename T> struct MfmaAcc;
template <> struct MfmaAcc<double> { typedef d4 type; };
template <> struct MfmaAcc<float> { typedef f4 type; };

// Output layout of the 16x16x4 MFMA (checked on gfx950): lane l, accumulator register r
// holds D[row][l % 16] with row = l/16 + 4 r for f64 and row = 4 (l/16) + r for f32.
template <typename T> __device__ __forceinline__ int acc_row(int lane, int r);
template <> __device__ __forceinline__ int acc_row<double>(int lane, int r) {
    return (lane >> 4) + 4 * r;
}
template <> __device__ __forceinline__ int acc_row<float>(int lane, int r) {
    return 4 * (lane >> 4) + r;
}

__device__ __forceinline__ d4 mfma(double a, double b, d4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4 mfma(float a, float b, f4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

template <typename T, int OPA, int TI, int TJ, int BKT, bool G3, int MINB = 1>
__global__ __launch_bounds__(256, MINB) void k_zgemm(int64_t m, int64_t n, int64_t kdim,
                                               int64_t kchunk, cpx<T> alpha,
                                               const cpx<T> *__restrict__ A, int64_t lda,
                                               const cpx<T> *__restrict__ B, int64_t ldb,
                                               cpx<T> beta, cpx<T> *C, int64_t ldc,
                                               cpx<T> *W) {
    constexpr bool CONJA = OPA == 1;
    constexpr bool BREAL = OPA == 3;          // op(A) = A, B real (its imaginary parts unread)
    constexpr bool P3 = G3 && !BREAL;         // the third product of the 3M form
    constexpr int BM = 32 * TI, BN = 32 * TJ;
    // LDS tiles split into real and imaginary parts.  The layout follows the order in which
    // the global loads arrive so that the stores are free of bank conflicts: A is [k][i]
    // (rows contiguous) for op(A) = A and [i][k] (k contiguous) for op(A) = A^H; B is
    // always [j][k].  The k-contiguous layouts are padded by one element per row so that
    // the 16 lanes reading one MFMA fragment hit distinct banks.
    constexpr int AK = CONJA ? BM : BKT, AI = CONJA ? BKT + 1 : BM + 2;
    __shared__ T As[2][AK * AI];
    __shared__ T Bs[2][BN * (BKT + 1)];
    auto aidx = [&](int kk, int i) { return CONJA ? i * AI + kk : kk * AI + i; };
    auto bidx = [&](int kk, int j) { return j * (BKT + 1) + kk; };
    typedef typename MfmaAcc<T>::type acc_t;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wv = tid >> 6;
    const int wrow = (wv & 1) * (BM / 2);
    const int wcol = (wv >> 1) * (BN / 2);
    // Tile of this workgroup.  The grid is one-dimensional over (K-slice, tile).  Workgroups
    // are dealt round-robin to the 8 XCDs (workgroup id mod 8), each with its own L2, so the
    // id is first mapped to a logical index that gives every XCD a contiguous run; logical
    // indices then walk groups of GROUP_M row panels column by column, so the workgroups
    // resident on one XCD share both their A row panels and their B column panels in L2.
    constexpr int NXCD = 8, GROUP_M = 8;
    const int64_t tiles_m = (m + BM - 1) / BM, tiles_n = (n + BN - 1) / BN;
    const int64_t ntile = tiles_m * tiles_n;
    const int64_t total = (int64_t)gridDim.x;
    int64_t lg;
    {
        const int64_t g = blockIdx.x, x = g % NXCD, loc = g / NXCD;
        const int64_t q = total / NXCD, r = total % NXCD;
        lg = x < r ? x * (q + 1) + loc : r * (q + 1) + (x - r) * q + loc;
    }
    const int64_t zslice = lg / ntile, t = lg % ntile;
    const int64_t gsz = (int64_t)GROUP_M * tiles_n;
    const int64_t fm = (t / gsz) * GROUP_M;
    const int64_t gm = min((int64_t)GROUP_M, tiles_m - fm);
    const int64_t tm = fm + (t % gsz) % gm, tn = (t % gsz) / gm;
    const int64_t row0 = tm * BM;
    const int64_t col0 = tn * BN;
    const int64_t kbeg = zslice * kchunk;
    const int64_t kend = min(kdim, kbeg + kchunk);

    // 4M and real B: accr, acci are the real and imaginary parts; 3M: accr = P1, acci = P2,
    // acc3 = P3
    acc_t accr[TI][TJ], acci[TI][TJ], acc3[P3 ? TI : 1][P3 ? TJ : 1];
#pragma unroll
    for (int a = 0; a < TI; ++a)
#pragma unroll
        for (int b = 0; b < TJ; ++b) {
            accr[a][b] = acc_t{0, 0, 0, 0};
            acci[a][b] = acc_t{0, 0, 0, 0};
            if constexpr (P3) acc3[a][b] = acc_t{0, 0, 0, 0};
        }

    constexpr int NA = BM * BKT / 256;
    constexpr int NB = BN * BKT / 256;
    cpx<T> ra[NA], rb[NB];

    // Global loads of one K-slice into registers.  Rows of op(A) and columns of B beyond the
    // matrix are clamped onto the last one: they only feed outputs that are never stored.
    // Only the ragged last slice (CHECKK) zeroes what lies beyond kend.  The full slices
    // run without control flow, which keeps the accumulators in the matrix-core registers.
    auto load_tiles = [&](int64_t k0, auto checkk) {
        constexpr bool CHECKK = decltype(checkk)::value;
#pragma unroll
        for (int r = 0; r < NA; ++r) {
            int e = tid + 256 * r;
            int i, kk;
            if (!CONJA) { i = e % BM; kk = e / BM; }      // contiguous along rows
            else { kk = e % BKT; i = e / BKT; }            // contiguous along k
            int64_t gi = min(row0 + i, m - 1), gk = k0 + kk;
            if constexpr (CHECKK) {
                const bool in = gk < kend;
                gk = min(gk, kend - 1);
                cpx<T> v = CONJA ? A[gk + gi * lda] : A[gi + gk * lda];
                ra[r] = in ? v : mk((T)0, (T)0);
            } else {
                ra[r] = CONJA ? A[gk + gi * lda] : A[gi + gk * lda];
            }
        }
#pragma unroll
        for (int r = 0; r < NB; ++r) {
            int e = tid + 256 * r;
            int kk = e % BKT, j = e / BKT;
            int64_t gj = min(col0 + j, n - 1), gk = k0 + kk;
            if constexpr (CHECKK) {
                const bool in = gk < kend;
                gk = min(gk, kend - 1);
                cpx<T> v = B[gk + gj * ldb];
                rb[r] = in ? v : mk((T)0, (T)0);
            } else {
                rb[r] = B[gk + gj * ldb];
            }
        }
    };
    auto store_tiles = [&]() {
#pragma unroll
        for (int r = 0; r < NA; ++r) {
            int e = tid + 256 * r;
            int i, kk;
            if (!CONJA) { i = e % BM; kk = e / BM; }
            else { kk = e % BKT; i = e / BKT; }
            As[0][aidx(kk, i)] = ra[r].x;
            As[1][aidx(kk, i)] = ra[r].y;
        }
#pragma unroll
        for (int r = 0; r < NB; ++r) {
            int e = tid + 256 * r;
            int kk = e % BKT, j = e / BKT;
            Bs[0][bidx(kk, j)] = rb[r].x;
            if constexpr (!BREAL) Bs[1][bidx(kk, j)] = rb[r].y;
        }
    };
    auto mma_slice = [&]() {
        __builtin_amdgcn_s_setprio(1);
#pragma unroll
        for (int k4 = 0; k4 < BKT; k4 += 4) {
            const int kk = k4 + (lane >> 4);
            T ar[TI], ai[TI], br[TJ], bi[TJ];
#pragma unroll
            for (int a = 0; a < TI; ++a) {
                ar[a] = As[0][aidx(kk, wrow + a * 16 + (lane & 15))];
                ai[a] = As[1][aidx(kk, wrow + a * 16 + (lane & 15))];
            }
#pragma unroll
            for (int b = 0; b < TJ; ++b) {
                br[b] = Bs[0][bidx(kk, wcol + b * 16 + (lane & 15))];
                bi[b] = BREAL ? (T)0 : Bs[1][bidx(kk, wcol + b * 16 + (lane & 15))];
            }
            if constexpr (BREAL) {
                // a complex matrix times a real one: two real products
#pragma unroll
                for (int a = 0; a < TI; ++a)
#pragma unroll
                    for (int b = 0; b < TJ; ++b) {
                        accr[a][b] = mfma(ar[a], br[b], accr[a][b]);
                        acci[a][b] = mfma(ai[a], br[b], acci[a][b]);
                    }
            } else if constexpr (G3) {
                // conj(A) (op A^H and op conj(A)): P3 takes Ar - Ai and the signs of P2 flip
                // in the epilogue, so no operand is negated
                T sb[TJ];
#pragma unroll
                for (int b = 0; b < TJ; ++b) sb[b] = br[b] + bi[b];
#pragma unroll
                for (int a = 0; a < TI; ++a) {
                    T sa = OPA != 0 ? ar[a] - ai[a] : ar[a] + ai[a];
#pragma unroll
                    for (int b = 0; b < TJ; ++b) {
                        accr[a][b] = mfma(ar[a], br[b], accr[a][b]);
                        acci[a][b] = mfma(ai[a], bi[b], acci[a][b]);
                        acc3[a][b] = mfma(sa, sb[b], acc3[a][b]);
                    }
                }
            } else {
#pragma unroll
                for (int a = 0; a < TI; ++a) {
                    // conj(A) flips the sign of the Ai products; the sign is applied here
                    // rather than on the loaded values (measured faster)
                    T nai = -ai[a];
                    T s_r = OPA != 0 ? ai[a] : nai;   // coefficient of Bi in the real part
                    T s_i = OPA != 0 ? nai : ai[a];   // coefficient of Br in the imaginary part
#pragma unroll
                    for (int b = 0; b < TJ; ++b) {
                        accr[a][b] = mfma(ar[a], br[b], accr[a][b]);
                        accr[a][b] = mfma(s_r, bi[b], accr[a][b]);
                        acci[a][b] = mfma(ar[a], bi[b], acci[a][b]);
                        acci[a][b] = mfma(s_i, br[b], acci[a][b]);
                    }
                }
            }
        }
        __builtin_amdgcn_s_setprio(0);
    };

    typedef std::integral_constant<bool, false> no_t;
    typedef std::integral_constant<bool, true> yes_t;
    const int64_t nfull = kend > kbeg ? (kend - kbeg) / BKT : 0;
    const bool tail = kend > kbeg && (kend - kbeg) % BKT != 0;
    if (nfull > 0) load_tiles(kbeg, no_t{});
    for (int64_t s = 0; s + 1 < nfull; ++s) {
        __syncthreads();
        store_tiles();
        __syncthreads();
        load_tiles(kbeg + (s + 1) * BKT, no_t{});
        mma_slice();
    }
    if (nfull > 0) {
        __syncthreads();
        store_tiles();
        __syncthreads();
        if (tail) load_tiles(kbeg + nfull * BKT, yes_t{});
        mma_slice();
    } else if (tail) {
        load_tiles(kbeg, yes_t{});
    }
    if (tail) {
        __syncthreads();
        store_tiles();
        __syncthreads();
        mma_slice();
    }
    const bool beta_zero = (beta.x == (T)0 && beta.y == (T)0);
    cpx<T> *Wz = W ? W + zslice * m * n : nullptr;
#pragma unroll
    for (int a = 0; a < TI; ++a)
#pragma unroll
        for (int b = 0; b < TJ; ++b) {
            int64_t gj = col0 + wcol + b * 16 + (lane & 15);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                int64_t gi = row0 + wrow + a * 16 + acc_row<T>(lane, r);
                if (gi < m && gj < n) {
                    cpx<T> v;
                    if constexpr (P3) {
                        T p1 = accr[a][b][r], p2 = acci[a][b][r], p3 = acc3[a][b][r];
                        v = OPA != 0 ? mk(p1 + p2, p3 - p1 + p2) : mk(p1 - p2, p3 - p1 - p2);
                    } else {
                        v = mk((T)accr[a][b][r], (T)acci[a][b][r]);
                    }
                    if (Wz) {
                        Wz[gi + gj * m] = v;                     // partial of this K-slice
                    } else {
                        v = alpha * v;
                        cpx<T> *p = C + gi + gj * ldc;
                        if (!beta_zero) v = v + beta * (*p);
                        *p = v;
                    }
                }
            }
        }
}

// ---------------------------------------------------------------- wide complex128 tile ---
// The large FP64 products of the solver (the sketch's N x N x b products and their adjoints,
// the capacitance matrix V^T U~, the solve's W Y) with a 128 x 128 output tile per workgroup
// of 8 wavefronts (each 64 x 32), which halves the operand traffic per flop of the 64 x 64
// tile.  Every output element sees the same MFMA sequence (k ascending in steps of 4, 3M
// form) as in k_zgemm, so the two kernels give bitwise identical results.
//
// Operands go from global memory straight into LDS (gfx950's 16-byte global_load_lds: each
// lane's element lands at the wave's LDS base + 16 x lane, with no staging registers and no
// LDS store instructions), laid out as "fragments": the 16 x 4 block of op(A) (rows x k) or
// of B (k x columns) that one 16x16x4 MFMA consumes, in the MFMA's own lane order
// (lane = (k % 4) * 16 + row % 16).  Reading an operand is one contiguous, conflict-free
// ds_read_b128 per lane that brings its real and imaginary parts together.
//
// Schedule, measured on the N x N x 256 products (executed-flop fraction of the FP64 matrix
// peak 0.78-0.85 before, 0.82-0.89 after):
// * two LDS buffers used in turn, the slice loop unrolled in pairs so that each buffer is a
//   compile-time array (the wait-count pass then keeps LDS reads of one buffer independent
//   of the direct loads in flight into the other);
// * the fragments of the next k-quad are read while the MFMAs of the current one run (A
//   fragments slot by slot after their MFMAs, B fragments double-buffered), and the slice's
//   barrier sits before its last k-quad, whose fragments are then already in registers, so
//   that the next slice's first k-quad is read during it;
// * the direct loads are spread over the slice in the middle of k-quads (two fragment pairs
//   after the barrier, one in each of the next two k-quads): issued together they cost about
//   8% of the matrix-core time;
// * edge tiles are shifted to end inside the matrix (their rows and columns below the
//   nominal start are computed and not written), so that each lane addresses its fragments
//   as one 32-bit offset from a uniform base: this needs m, n >= 128 and leading dimensions
//   below 2^24.
typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) void glb_void_t;
constexpr int kWideTile = 128;
constexpr int64_t kWideMaxLd = int64_t(1) << 24;

template <int OPA>
__global__ __launch_bounds__(512, 1) void k_zgemm_wide(int64_t m, int64_t n, int64_t kdim,
                                                     int64_t kchunk, zd alpha,
                                                     const zd *__restrict__ A, int64_t lda,
                                                     const zd *__restrict__ B, int64_t ldb,
                                                     zd beta, zd *C, int64_t ldc, zd *W) {
    constexpr bool BREAL = OPA == 3;
    constexpr int BM = kWideTile, BN = kWideTile, BK = 16;
    // fragment f = kq * 8 + t: MFMA tile t (of 8 along the rows of op(A), or along the
    // columns of B) at k-quad kq of the slice
    __shared__ zd As0[32][64], As1[32][64], Bs0[32][64], Bs1[32][64];
    const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
    // XCD-aware tile order as in k_zgemm, groups of 4 row panels
    constexpr int NXCD = 8, GROUP_M = 4;
    const int64_t tiles_m = (m + BM - 1) / BM, tiles_n = (n + BN - 1) / BN;
    const int64_t ntile = tiles_m * tiles_n;
    const int64_t total = (int64_t)gridDim.x;
    int64_t lg;
    {
        const int64_t g = blockIdx.x, x = g % NXCD, loc = g / NXCD;
        const int64_t q = total / NXCD, r = total % NXCD;
        lg = x < r ? x * (q + 1) + loc : r * (q + 1) + (x - r) * q + loc;
    }
    const int64_t zslice = lg / ntile, t = lg % ntile;
    const int64_t gsz = (int64_t)GROUP_M * tiles_n;
    const int64_t fm = (t / gsz) * GROUP_M;
    const int64_t gm = min((int64_t)GROUP_M, tiles_m - fm);
    const int64_t tm = fm + (t % gsz) % gm, tn = (t % gsz) / gm;
    // nominal start of the tile (the first row and column it writes) and the computed tile
    const int64_t rlo = tm * BM, clo = tn * BN;
    const int64_t row0 = min(rlo, m - BM), col0 = min(clo, n - BN);
    const int64_t kbeg = zslice * kchunk;
    const int64_t kend = min(kdim, kbeg + kchunk);
    const int64_t nslice = kend > kbeg ? (kend - kbeg + BK - 1) / BK : 0;
    // wave w fills fragments w*4 + q (q = 0..3) of each operand: k-quad w/2, tiles
    // (w%2)*4 + q; its lane's element of fragment q sits at (slice base + q x stride +
    // lane offset), with the lane's k row kk in the slice
    const int kl = 4 * (w >> 1) + (lane >> 4), t0 = (w & 1) * 4, il = lane & 15;
    auto lane_off = [&](int kk, uint32_t &oa, uint32_t &ob) {
        const int64_t r = 16 * t0 + il;
        oa = (uint32_t)(16 * (OPA == 1 ? kk + r * lda : r + kk * lda));
        ob = (uint32_t)(16 * (kk + r * ldb));
    };
    uint32_t oa, ob;
    lane_off(kl, oa, ob);
    const int64_t qa = 16 * (OPA == 1 ? 16 * lda : 16), qb = 16 * 16 * ldb;
    const char *abase = (const char *)(OPA == 1 ? A + row0 * lda : A + row0);
    const char *bbase = (const char *)(B + col0 * ldb);
    // the last slice's k rows beyond kend are clamped onto kend - 1 (in bounds); B is
    // zeroed there after they land
    const int64_t klast = kend - 1 - (kbeg + (nslice - 1) * BK);
    // direct loads of fragments qlo..qhi-1 of slice s into buffer BUF
    auto issue = [&](int64_t s, auto bufc, int qlo, int qhi) {
        constexpr int BUF = decltype(bufc)::value;
        const int64_t k0 = kbeg + s * BK;
        const char *sa = abase + 16 * (OPA == 1 ? k0 : k0 * lda);
        const char *sb = bbase + 16 * k0;
        uint32_t xa = oa, xb = ob;
        if (s + 1 == nslice && kl > klast) lane_off((int)klast, xa, xb);
        // keeps the offsets 32-bit lane values (no 64-bit address per fragment kept live)
        asm volatile("" : "+v"(xa), "+v"(xb));
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (q < qlo || q >= qhi) continue;
            __builtin_amdgcn_global_load_lds((glb_void_t *)(sa + q * qa + xa),
                (lds_void_t *)(BUF ? &As1[w * 4 + q][0] : &As0[w * 4 + q][0]), 16, 0, 0);
            __builtin_amdgcn_global_load_lds((glb_void_t *)(sb + q * qb + xb),
                (lds_void_t *)(BUF ? &Bs1[w * 4 + q][0] : &Bs0[w * 4 + q][0]), 16, 0, 0);
        }
    };
    auto clear_tail = [&](int64_t s, auto bufc) {
        constexpr int BUF = decltype(bufc)::value;
        if (kbeg + s * BK + kl >= kend) {
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (BUF) Bs1[w * 4 + q][lane] = mk(0.0, 0.0);
                else Bs0[w * 4 + q][lane] = mk(0.0, 0.0);
            }
        }
    };
    // 3M: acc1 = Ar Br, acc2 = Ai Bi, acc3 = (Ar +- Ai)(Br + Bi); real B: acc1, acc2 = Ar, Ai B
    d4 acc1[4][2], acc2[4][2], acc3[BREAL ? 1 : 4][BREAL ? 1 : 2];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            acc1[a][b] = d4{0, 0, 0, 0};
            acc2[a][b] = d4{0, 0, 0, 0};
            if constexpr (!BREAL) acc3[a][b] = d4{0, 0, 0, 0};
        }
    const int ta = (w & 1) * 4, tb = (w >> 1) * 2;    // this wave's 4 x 2 MFMA tiles
    zd av[4], bv[2], bn[2];
    // one k-quad on the fragments in registers, reading those of k-quad NKQ of buffer NBUF
    // meanwhile; hook() runs after the second A fragment's MFMAs
    auto kquad = [&](auto nbufc, auto nkqc, auto hook) {
        constexpr int NBUF = decltype(nbufc)::value, NKQ = decltype(nkqc)::value;
#pragma unroll
        for (int b = 0; b < 2; ++b) bn[b] = NBUF ? Bs1[NKQ * 8 + tb + b][lane] : Bs0[NKQ * 8 + tb + b][lane];
        double sb[2];
        if constexpr (!BREAL) {
#pragma unroll
            for (int b = 0; b < 2; ++b) sb[b] = bv[b].x + bv[b].y;
        }
        __builtin_amdgcn_s_setprio(1);
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            if constexpr (BREAL) {
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    acc1[a][b] = mfma(av[a].x, bv[b].x, acc1[a][b]);
                    acc2[a][b] = mfma(av[a].y, bv[b].x, acc2[a][b]);
                }
            } else {
                const double sa = OPA != 0 ? av[a].x - av[a].y : av[a].x + av[a].y;
#pragma unroll
                for (int b = 0; b < 2; ++b) {
                    acc1[a][b] = mfma(av[a].x, bv[b].x, acc1[a][b]);
                    acc2[a][b] = mfma(av[a].y, bv[b].y, acc2[a][b]);
                    acc3[a][b] = mfma(sa, sb[b], acc3[a][b]);
                }
            }
            av[a] = NBUF ? As1[NKQ * 8 + ta + a][lane] : As0[NKQ * 8 + ta + a][lane];
            if (a == 1) hook();
        }
        __builtin_amdgcn_s_setprio(0);
#pragma unroll
        for (int b = 0; b < 2; ++b) bv[b] = bn[b];
    };
    typedef std::integral_constant<int, 0> I0;
    typedef std::integral_constant<int, 1> I1;
    typedef std::integral_constant<int, 2> I2;
    typedef std::integral_constant<int, 3> I3;
    // slice s in buffer CUR, its first k-quad's fragments in registers
    auto slice = [&](int64_t s, auto curc) {
        constexpr int CUR = decltype(curc)::value;
        typedef std::integral_constant<int, CUR> IC;
        typedef std::integral_constant<int, 1 - CUR> IN;
        const bool more = s + 1 < nslice;
        // fragments 2 and 3 of the next slice into buffer IN, free since the last barrier
        kquad(IC{}, I1{}, [&] { if (more) issue(s + 1, IN{}, 2, 3); });
        kquad(IC{}, I2{}, [&] { if (more) issue(s + 1, IN{}, 3, 4); });
        kquad(IC{}, I3{}, [] {});
        // k-quad 3's fragments are in registers, the next slice's operands have landed (the
        // direct loads count on vmcnt; no other vector memory operation is in flight)
        asm volatile("s_waitcnt vmcnt(0) lgkmcnt(0)" ::: "memory");
        if (more) clear_tail(s + 1, IN{});
        __syncthreads();
        // buffer CUR is read by nobody now: fragments 0 and 1 of slice s + 2.  After the last
        // slice the fragments read here are not used (in-bounds LDS reads).
        kquad(IN{}, I0{}, [&] { if (s + 2 < nslice) issue(s + 2, IC{}, 0, 2); });
    };
    if (nslice > 0) {
        issue(0, I0{}, 0, 4);
        asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
        clear_tail(0, I0{});
        __syncthreads();
        if (nslice > 1) issue(1, I1{}, 0, 2);
#pragma unroll
        for (int b = 0; b < 2; ++b) bv[b] = Bs0[tb + b][lane];
#pragma unroll
        for (int a = 0; a < 4; ++a) av[a] = As0[ta + a][lane];
        for (int64_t s = 0; s < nslice; s += 2) {
            slice(s, I0{});
            if (s + 1 < nslice) slice(s + 1, I1{});
        }
    }
    const bool beta_zero = (beta.x == 0.0 && beta.y == 0.0);
    zd *Wz = W ? W + zslice * m * n : nullptr;
    const int wrow = ta * 16, wcol = tb * 16;
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) {
            const int64_t gj = col0 + wcol + b * 16 + (lane & 15);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int64_t gi = row0 + wrow + a * 16 + acc_row<double>(lane, r);
                if (gi >= rlo && gj >= clo) {
                    zd v;
                    if constexpr (BREAL) {
                        v = mk((double)acc1[a][b][r], (double)acc2[a][b][r]);
                    } else {
                        const double p1 = acc1[a][b][r], p2 = acc2[a][b][r], p3 = acc3[a][b][r];
                        v = OPA != 0 ? mk(p1 + p2, p3 - p1 + p2) : mk(p1 - p2, p3 - p1 - p2);
                    }
                    if (Wz) {
                        Wz[gi + gj * m] = v;                     // partial of this K-slice
                    } else {
                        v = alpha * v;
                        zd *p = C + gi + gj * ldc;
                        if (!beta_zero) v = v + beta * (*p);
                        *p = v;
                    }
                }
            }
        }
}

// C = alpha * sum_z W[z] + beta * C, slices summed in order
template <typename T>
__global__ void k_splitk_reduce(int64_t m, int64_t n, int S, const cpx<T> *__restrict__ W,
                                cpx<T> alpha, cpx<T> beta, cpx<T> *C, int64_t ldc) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= m * n) return;
    int64_t i = t % m, j = t / m;
    cpx<T> acc = W[t];
    for (int z = 1; z < S; ++z) acc = acc + W[(int64_t)z * m * n + t];
    cpx<T> v = alpha * acc;
    cpx<T> *p = C + i + j * ldc;
    if (!(beta.x == (T)0 && beta.y == (T)0)) v = v + beta * (*p);
    *p = v;
}

// ---------------------------------------------------------------- skinny products -------
// C = alpha A B + beta C when B has at most 16 columns (op(A) = A, the Woodbury solve of a few
// right-hand sides): the product streams A once from HBM and does 8 n flops per element of A,
// so it is bound by memory, and a 64 x 64 matrix-core tile would spend its time on columns
// that do not exist.  A workgroup of 256 threads takes 256 rows of A (one per thread, the
// loads of a wavefront contiguous) and a range of K; the range's rows of B pass through LDS in
// tiles and every thread forms NB complex dot products in registers, k in increasing order.
// Ranges of K are summed by the split-K reduction in a fixed order.
constexpr int kSkinnyMaxN = 16, kSkinnyRows = 256;

// K-tiles of KT rows of B, loads of A issued LB at a time: 32 and 8 for up to 8 columns, 64
// and 16 for up to 16 (measured at N = 16384)
template <int NB> struct SkinnyTile { static constexpr int KT = NB <= 8 ? 32 : 64, LB = NB <= 8 ? 8 : 16; };

template <typename T, int NB>
__global__ __launch_bounds__(256, 2) void k_zgemm_skinny(int64_t m, int n, int64_t k,
                                                      int64_t kchunk, cpx<T> alpha,
                                                      const cpx<T> *__restrict__ A, int64_t lda,
                                                      const cpx<T> *__restrict__ B, int64_t ldb,
                                                      cpx<T> beta, cpx<T> *C, int64_t ldc,
                                                      cpx<T> *W) {
    constexpr int kSkinnyKT = SkinnyTile<NB>::KT, kSkinnyLB = SkinnyTile<NB>::LB;
    __shared__ cpx<T> Bs[kSkinnyKT][NB];
    const int tid = threadIdx.x;
    const int64_t nrb = (m + kSkinnyRows - 1) / kSkinnyRows;
    const int64_t rb = blockIdx.x % nrb, z = blockIdx.x / nrb;
    const int64_t row = rb * kSkinnyRows + tid;
    const int64_t rowc = row < m ? row : m - 1;     // loads in bounds; the store is skipped
    const int64_t kb = z * kchunk, ke = min(k, kb + kchunk);
    cpx<T> acc[NB];
#pragma unroll
    for (int j = 0; j < NB; ++j) acc[j] = mk((T)0, (T)0);
    for (int64_t k0 = kb; k0 < ke; k0 += kSkinnyKT) {
        const int kt = (int)min((int64_t)kSkinnyKT, ke - k0);
        __syncthreads();
        for (int e = tid; e < kSkinnyKT * NB; e += 256) {
            const int kk = e % kSkinnyKT, j = e / kSkinnyKT;
            Bs[kk][j] = (kk < kt && j < n) ? B[k0 + kk + (int64_t)j * ldb] : mk((T)0, (T)0);
        }
        __syncthreads();
        const cpx<T> *a0 = A + rowc + k0 * lda;
        if (kt == kSkinnyKT) {
            for (int k8 = 0; k8 < kSkinnyKT; k8 += kSkinnyLB) {
                cpx<T> a[kSkinnyLB];
#pragma unroll
                for (int u = 0; u < kSkinnyLB; ++u) a[u] = a0[(int64_t)(k8 + u) * lda];
#pragma unroll
                for (int u = 0; u < kSkinnyLB; ++u)
#pragma unroll
                    for (int j = 0; j < NB; ++j) acc[j] = acc[j] + a[u] * Bs[k8 + u][j];
            }
        } else {
            for (int kk = 0; kk < kt; ++kk) {
                const cpx<T> a = a0[(int64_t)kk * lda];
#pragma unroll
                for (int j = 0; j < NB; ++j) acc[j] = acc[j] + a * Bs[kk][j];
            }
        }
    }
    if (row >= m) return;
    // fully unrolled over the register array (a loop over it would move it to scratch)
    if (W) {
        cpx<T> *w = W + z * m * n + row;
#pragma unroll
        for (int j = 0; j < NB; ++j)
            if (j < n) w[(int64_t)j * m] = acc[j];
    } else {
        const bool beta_zero = (beta.x == (T)0 && beta.y == (T)0);
        cpx<T> *c = C + row;
#pragma unroll
        for (int j = 0; j < NB; ++j) {
            if (j < n) {
                cpx<T> v = alpha * acc[j];
                if (!beta_zero) v = v + beta * c[(int64_t)j * ldc];
                c[(int64_t)j * ldc] = v;
            }
        }
    }
}

// grow-only device workspaces for split-K partial products, one per (device, stream) so that
// contexts on different streams can run from different host threads.  Stream-ordered
// allocation and release: hipMalloc / hipFree may wait for the whole device, which on a
// device shared by several streams (batched problems) stalls one stream behind the others'
// queued work.
namespace {
std::mutex g_ws_mu;
std::map<std::pair<int, hipStream_t>, std::pair<void *, size_t>> g_ws;

// a caller-owned workspace used instead of the shared one (HIP graph capture: the recorded
// kernels must keep pointing at memory that no later call frees)
thread_local void *t_ws_override = nullptr;
thread_local size_t t_ws_override_bytes = 0;

void *splitk_ws(size_t need, hipStream_t s) {
    if (t_ws_override && need <= t_ws_override_bytes) return t_ws_override;
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lock(g_ws_mu);
    auto &e = g_ws[{dev, s}];
    if (e.second < need) {
        if (e.first) (void)hipFreeAsync(e.first, s);
        e.first = nullptr;
        e.second = 0;
        size_t nb = need + need / 2;
        if (hipMallocAsync(&e.first, nb, s) != hipSuccess) {
            (void)hipGetLastError();
            e.first = nullptr;
            return nullptr;
        }
        e.second = nb;
    }
    return e.first;
}
}  // namespace

void splitk_release(int device, hipStream_t s) {
    std::lock_guard<std::mutex> lock(g_ws_mu);
    auto it = g_ws.find({device, s});
    if (it == g_ws.end()) return;
    if (it->second.first) (void)hipFreeAsync(it->second.first, s);
    g_ws.erase(it);
}

namespace {
template <typename T, int OPA, int TI, int TJ, int BKT, bool G3 = true, int MINB = 1>
void launch(int64_t m, int64_t n, int64_t k, int S, cpx<T> alpha, const cpx<T> *A, int64_t lda,
            const cpx<T> *B, int64_t ldb, cpx<T> beta, cpx<T> *C, int64_t ldc, hipStream_t s) {
    constexpr int BM = 32 * TI, BN = 32 * TJ;
    int64_t kchunk = k;
    cpx<T> *W = nullptr;
    if (S > 1) {
        kchunk = ((k + S - 1) / S + BKT - 1) / BKT * BKT;
        S = (int)((k + kchunk - 1) / kchunk);
        W = (cpx<T> *)splitk_ws((size_t)S * m * n * sizeof(cpx<T>), s);
        if (!W) { S = 1; kchunk = k; }
    }
    const int64_t ntile = ((m + BM - 1) / BM) * ((n + BN - 1) / BN);
    dim3 grid((unsigned)(ntile * S));
    hipLaunchKernelGGL((k_zgemm<T, OPA, TI, TJ, BKT, G3, MINB>), grid, dim3(256), 0, s, m, n, k, kchunk,
                       alpha, A, lda, B, ldb, beta, C, ldc, S > 1 ? W : nullptr);
    if (S > 1) {
        int64_t t = m * n;
        hipLaunchKernelGGL(k_splitk_reduce<T>, dim3((unsigned)((t + 255) / 256)), dim3(256), 0, s,
                           m, n, S, (const cpx<T> *)W, alpha, beta, C, ldc);
    }
}
}  // namespace

namespace {
// the wide tile for a complex128 product (split along K exactly as for k_zgemm)
template <int OPA>
void launch_wide(int64_t m, int64_t n, int64_t k, int S, zd alpha, const zd *A, int64_t lda,
                 const zd *B, int64_t ldb, zd beta, zd *C, int64_t ldc, hipStream_t s) {
    int64_t kchunk = k;
    zd *W = nullptr;
    if (S > 1) {
        kchunk = ((k + S - 1) / S + 15) / 16 * 16;
        S = (int)((k + kchunk - 1) / kchunk);
        W = (zd *)splitk_ws((size_t)S * m * n * sizeof(zd), s);
        if (!W) { S = 1; kchunk = k; }
    }
    const int64_t ntile = ((m + kWideTile - 1) / kWideTile) * ((n + kWideTile - 1) / kWideTile);
    hipLaunchKernelGGL((k_zgemm_wide<OPA>), dim3((unsigned)(ntile * S)), dim3(512), 0, s, m, n,
                       k, kchunk, alpha, A, lda, B, ldb, beta, C, ldc, S > 1 ? W : nullptr);
    if (S > 1) {
        const int64_t t = m * n;
        hipLaunchKernelGGL(k_splitk_reduce<double>, dim3((unsigned)((t + 255) / 256)), dim3(256),
                           0, s, m, n, S, (const zd *)W, alpha, beta, C, ldc);
    }
}
}  // namespace

// ---------------------------------------------------------------- tile autotuner --------
// Output tiles of 64 x 64, 32 x 64, 64 x 32 or 32 x 32 per workgroup.  Every variant runs the
// same K loop for every output element (the same K-slices in the same order, the same MFMA
// sequence per slice), so the variants give bitwise identical results and the choice only
// changes speed: smaller tiles put more workgroups on the 256 CUs when the output is small.
// The split along K is fixed beforehand by the 64 x 64 tile count, so it does not depend on
// the variant either.  The first product of each shape class (op, precision, and the binary
// orders of m, n, k and the split) whose 64 x 64 grid is too small to fill the device runs
// every variant once into a scratch output, timed with HIP events on the caller's stream,
// and the fastest is kept for the rest of the process; other threads that need the same
// class meanwhile wait for that decision.
namespace {
template <typename T>
using LaunchFn = void (*)(int64_t, int64_t, int64_t, int, cpx<T>, const cpx<T> *, int64_t,
                          const cpx<T> *, int64_t, cpx<T>, cpx<T> *, int64_t, hipStream_t);
constexpr int kVariants = 4;
template <typename T, int OPA>
LaunchFn<T> variant(int v) {
    switch (v) {
        case 1: return launch<T, OPA, 1, 2, 16, true, 2>;
        case 2: return launch<T, OPA, 2, 1, 16, true, 2>;
        case 3: return launch<T, OPA, 1, 1, 16, true, 2>;
        default: return launch<T, OPA, 2, 2, 16, true, 2>;
    }
}
template <typename T>
LaunchFn<T> variant_op(int op, int v) {
    return op == GEMM_C       ? variant<T, 1>(v)
           : op == GEMM_R     ? variant<T, 2>(v)
           : op == GEMM_NREAL ? variant<T, 3>(v)
                              : variant<T, 0>(v);
}

struct TuneKey {
    int op, bytes, lm, ln, lk, S;
    bool operator<(const TuneKey &o) const {
        const int a[6] = {op, bytes, lm, ln, lk, S}, b[6] = {o.op, o.bytes, o.lm, o.ln, o.lk, o.S};
        for (int i = 0; i < 6; ++i)
            if (a[i] != b[i]) return a[i] < b[i];
        return false;
    }
};
std::mutex g_tune_mu;
std::condition_variable g_tune_cv;
std::map<TuneKey, int> g_tune;            // variant, or -1 while being measured
std::atomic<int> g_tune_mode{1};
std::atomic<int> g_tuned{0};
thread_local bool t_tune_off = false;     // this thread's products take the 64 x 64 tile

int ilog2c(int64_t x) {
    int l = 0;
    while ((int64_t(1) << l) < x) ++l;
    return l;
}

template <typename T>
int tuned_variant(int op, int64_t m, int64_t n, int64_t k, int S, cpx<T> alpha,
                  const cpx<T> *A, int64_t lda, const cpx<T> *B, int64_t ldb, hipStream_t s) {
    const int64_t tiles = ((m + 63) / 64) * ((n + 63) / 64);
    if (g_tune_mode.load() == 0 || t_tune_off || tiles * S >= 512) return 0;
    if (8.0 * (double)m * (double)n * (double)k > 3.5e10) return 0;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(s, &cap) != hipSuccess || cap != hipStreamCaptureStatusNone) {
        (void)hipGetLastError();
        return 0;
    }
    const TuneKey key{op, (int)sizeof(T), ilog2c(m), ilog2c(n), ilog2c(k), S};
    {
        std::unique_lock<std::mutex> lock(g_tune_mu);
        for (;;) {
            auto it = g_tune.find(key);
            if (it == g_tune.end()) {
                g_tune[key] = -1;
                break;
            }
            if (it->second >= 0) return it->second;
            g_tune_cv.wait(lock);
        }
    }
    // measure every variant once (after one warm-up launch) into a scratch output
    int best = 0;
    cpx<T> *Ct = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    bool ok = hipMallocAsync((void **)&Ct, (size_t)m * n * sizeof(cpx<T>), s) == hipSuccess &&
              hipEventCreate(&e0) == hipSuccess && hipEventCreate(&e1) == hipSuccess;
    if (ok) {
        float tbest = 1e30f;
        variant_op<T>(op, 0)(m, n, k, S, alpha, A, lda, B, ldb, mk((T)0, (T)0), Ct, m, s);
        for (int v = 0; v < kVariants && ok; ++v) {
            ok = hipEventRecord(e0, s) == hipSuccess;
            variant_op<T>(op, v)(m, n, k, S, alpha, A, lda, B, ldb, mk((T)0, (T)0), Ct, m, s);
            ok = ok && hipEventRecord(e1, s) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
            float ms = 0.0f;
            ok = ok && hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
            if (ok && ms < tbest) {
                tbest = ms;
                best = v;
            }
        }
    }
    if (Ct) (void)hipFreeAsync(Ct, s);
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (!ok) {
        (void)hipGetLastError();
        best = 0;
    }
    {
        std::lock_guard<std::mutex> lock(g_tune_mu);
        g_tune[key] = best;
        ++g_tuned;
    }
    g_tune_cv.notify_all();
    return best;
}
}  // namespace

int set_gemm_autotune(int mode) { return g_tune_mode.exchange(mode ? 1 : 0); }

bool set_gemm_tune_thread(bool on) {
    const bool was = !t_tune_off;
    t_tune_off = !on;
    return was;
}

void set_splitk_override(void *p, size_t bytes) {
    t_ws_override = p;
    t_ws_override_bytes = p ? bytes : 0;
}

namespace {
int splitk_factor(int op, int64_t m, int64_t n, int64_t k) {
    const int64_t tiles = ((m + 63) / 64) * ((n + 63) / 64);
    int S = 1;
    if (tiles < 192 && k >= 4096) {
        S = (int)std::min<int64_t>((512 + tiles - 1) / tiles, k / 512);
        // A^H products whose 128 x 128 grid is short of one wave (the sketch's projections
        // Q^H Y against the directions found so far): enough K slices for one wave of wide
        // tiles.  The split depends on the shape only, not on the tile that runs it, so the
        // tile choice stays bitwise-neutral.
        if (op == GEMM_C && m >= kWideTile && n >= kWideTile) {
            const int64_t tw =
                ((m + kWideTile - 1) / kWideTile) * ((n + kWideTile - 1) / kWideTile);
            S = (int)std::max<int64_t>(S, std::min<int64_t>((256 + tw - 1) / tw, k / 512));
        }
        S = std::max(1, std::min(S, 64));
    }
    return S;
}
}  // namespace

namespace {
// the skinny product for op(A) = A, at most 16 columns, and enough rows and K to matter
bool skinny(int op, int64_t m, int64_t n, int64_t k) {
    return op == GEMM_N && n <= kSkinnyMaxN && m >= 1024 && k >= 1024;
}
// K split of the skinny product: about four workgroups per compute unit; K-ranges that are
// whole tiles of 32 (all but the last)
void skinny_split(int64_t m, int64_t n, int64_t k, int &S, int64_t &kchunk) {
    const int kt = n <= 4 ? SkinnyTile<4>::KT : n <= 8 ? SkinnyTile<8>::KT : SkinnyTile<16>::KT;
    const int64_t nrb = (m + kSkinnyRows - 1) / kSkinnyRows;
    S = (int)std::max<int64_t>(1, std::min<int64_t>((1024 + nrb - 1) / nrb, k / 256));
    kchunk = ((k + S - 1) / S + kt - 1) / kt * kt;
    S = (int)((k + kchunk - 1) / kchunk);
}
template <typename T, int NB>
void launch_skinny_nb(int64_t m, int64_t n, int64_t k, cpx<T> alpha, const cpx<T> *A,
                      int64_t lda, const cpx<T> *B, int64_t ldb, cpx<T> beta, cpx<T> *C,
                      int64_t ldc, hipStream_t s) {
    int S;
    int64_t kchunk;
    skinny_split(m, n, k, S, kchunk);
    cpx<T> *W = nullptr;
    if (S > 1) {
        W = (cpx<T> *)splitk_ws((size_t)S * m * n * sizeof(cpx<T>), s);
        if (!W) { S = 1; kchunk = k; }
    }
    const int64_t nrb = (m + kSkinnyRows - 1) / kSkinnyRows;
    hipLaunchKernelGGL((k_zgemm_skinny<T, NB>), dim3((unsigned)(nrb * S)), dim3(kSkinnyRows), 0,
                       s, m, (int)n, k, kchunk, alpha, A, lda, B, ldb, beta, C, ldc,
                       S > 1 ? W : nullptr);
    if (S > 1) {
        const int64_t t = m * n;
        hipLaunchKernelGGL(k_splitk_reduce<T>, dim3((unsigned)((t + 255) / 256)), dim3(256), 0, s,
                           m, n, S, (const cpx<T> *)W, alpha, beta, C, ldc);
    }
}
template <typename T>
void launch_skinny(int64_t m, int64_t n, int64_t k, cpx<T> alpha, const cpx<T> *A, int64_t lda,
                   const cpx<T> *B, int64_t ldb, cpx<T> beta, cpx<T> *C, int64_t ldc,
                   hipStream_t s) {
    if (n <= 4) launch_skinny_nb<T, 4>(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, s);
    else if (n <= 8) launch_skinny_nb<T, 8>(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, s);
    else launch_skinny_nb<T, 16>(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, s);
}
}  // namespace

namespace {
std::atomic<int> g_wide_mode{1};
// The wide tile for complex128 products whose 128 x 128 grid fills the device (about one
// workgroup of 8 wavefronts per compute unit or more) and whose K is not short: measured
// 5-15% faster than the 64 x 64 tile there (at N = 16384: the sketch's N x N x 256 products
// and their adjoints, V^T U~, the solve's W Y and U~ Z with K = 3943, the Gram-Schmidt
// updates; 7% at K = 2048); with fewer tiles than compute units its one workgroup per
// compute unit loses against the 64 x 64 tile's two.  From K = 256 to 2048 only for a grid of
// one wave (240-256 tiles, one per compute unit): N x 256 x K Gram-Schmidt updates and
// Newton-Schulz products, 256 x N x K superblock products of the triangular solves, 5-10%
// faster; with several waves of such short-K tiles the 64 x 64 tile's two workgroups per
// compute unit hide each other's epilogues, and it wins.  The two kernels give bitwise equal
// results.  The shifted edge tiles need m, n >= 128, the 32-bit lane offsets leading
// dimensions below 2^24.
bool use_wide(int64_t m, int64_t n, int64_t k, int S, int64_t lda, int64_t ldb) {
    const int64_t t = ((m + kWideTile - 1) / kWideTile) * ((n + kWideTile - 1) / kWideTile);
    const int64_t g = t * S;
    const bool fit = k >= 2048 ? g >= 240 : (k >= 256 && g >= 240 && g <= 256);
    return g_wide_mode.load() != 0 && fit && m >= kWideTile && n >= kWideTile &&
           lda < kWideMaxLd && ldb < kWideMaxLd;
}
}  // namespace

int set_gemm_wide(int mode) { return g_wide_mode.exchange(mode ? 1 : 0); }

size_t gemm_splitk_bytes(int op, int64_t m, int64_t n, int64_t k, size_t elem) {
    if (m <= 0 || n <= 0) return 0;
    if (skinny(op, m, n, k)) {
        int S;
        int64_t kchunk;
        skinny_split(m, n, k, S, kchunk);
        return S > 1 ? (size_t)S * (size_t)m * (size_t)n * elem : 0;
    }
    int S = splitk_factor(op, m, n, k);
    if (S <= 1) return 0;
    const int64_t kchunk = ((k + S - 1) / S + 15) / 16 * 16;
    S = (int)((k + kchunk - 1) / kchunk);
    return (size_t)S * (size_t)m * (size_t)n * elem;
}
int gemm_tuned_classes() { return g_tuned.load(); }

template <typename T>
void gemm(int op, int64_t m, int64_t n, int64_t k, cpx<T> alpha, const cpx<T> *A, int64_t lda,
          const cpx<T> *B, int64_t ldb, cpx<T> beta, cpx<T> *C, int64_t ldc, hipStream_t s) {
    if (m <= 0 || n <= 0) return;
    if (skinny(op, m, n, k)) {
        // bound by HBM, not counted with the matrix-core products
        launch_skinny<T>(m, n, k, alpha, A, lda, B, ldb, beta, C, ldc, s);
        return;
    }
    // K is split when the output has too few 64 x 64 tiles to fill 256 CUs
    const int S = splitk_factor(op, m, n, k);
    const bool wide = sizeof(T) == sizeof(double) && use_wide(m, n, k, S, lda, ldb);
    const int v = wide ? 0 : tuned_variant<T>(op, m, n, k, S, alpha, A, lda, B, ldb, s);
    // work: the real flops the kernel executes -- 6 m n k for a complex product in the 3M
    // form (three real products), 4 m n k with a real B (two real products).  The classical
    // complex product counts 8 m n k; the 3M form reaches the same result with 3/4 of it.
    ProfScope prof(sizeof(T) == sizeof(double) ? PROF_GEMM64 : PROF_GEMM32,
                   (op == GEMM_NREAL ? 4.0 : 6.0) * (double)m * (double)n *
                       (double)std::max<int64_t>(k, 0),
                   s);
    // 64 x 64 tiles in the 3M form measured fastest on gfx950 for every large shape of the
    // solver; two workgroups (two wavefronts per SIMD) per CU: the register budget of 256
    // per lane that this imposes measured 15-20% faster than one wavefront with more
    // registers
    if constexpr (sizeof(T) == sizeof(double)) {
        if (wide) {
            const zd *Ad = (const zd *)A, *Bd = (const zd *)B;
            zd al = mk((double)alpha.x, (double)alpha.y), be = mk((double)beta.x, (double)beta.y);
            zd *Cd = (zd *)C;
            switch (op) {
            case GEMM_C: launch_wide<1>(m, n, k, S, al, Ad, lda, Bd, ldb, be, Cd, ldc, s); break;
            case GEMM_R: launch_wide<2>(m, n, k, S, al, Ad, lda, Bd, ldb, be, Cd, ldc, s); break;
            case GEMM_NREAL: launch_wide<3>(m, n, k, S, al, Ad, lda, Bd, ldb, be, Cd, ldc, s); break;
            default: launch_wide<0>(m, n, k, S, al, Ad, lda, Bd, ldb, be, Cd, ldc, s); break;
            }
            return;
        }
    }
    variant_op<T>(op, v)(m, n, k, S, alpha, A, lda, B, ldb, beta, C, ldc, s);
}

template void gemm<double>(int, int64_t, int64_t, int64_t, zd, const zd *, int64_t,
                           const zd *, int64_t, zd, zd *, int64_t, hipStream_t);
template void gemm<float>(int, int64_t, int64_t, int64_t, zf, const zf *, int64_t,
                          const zf *, int64_t, zf, zf *, int64_t, hipStream_t);

}  // namespace cfie
