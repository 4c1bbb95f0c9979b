// Complex GEMM on CDNA matrix cores: C = alpha * op(A) * B + beta * C with op(A) = A or A^H,
// column-major, complex interleaved.  Used for every dense product of the method: the
// sketch of the remainder C - C_c (Sec. V eq. (7)), the capacitance matrix of eq. (9) and
// the Woodbury correction, and the FP64 residual of the refinement.
//
// The complex product is four real products per k-step on split real/imaginary tiles held
// in LDS: Cr += Ar Br - Ai Bi, Ci += Ar Bi + Ai Br, with the 16x16x4 MFMA (f64 or f32).
// Block tile BM x BN with BK = 16, 256 threads = 4 wavefronts, each wavefront a
// (BM/2) x (BN/2) sub-tile made of 16x16 MFMA tiles.  Global loads for the next K-slice are
// issued before the MFMAs of the current one (register double buffering).
#include "internal.h"

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

constexpr int BK = 16;

// BM = 32 * TI, BN = 32 * TJ (each wavefront: TI x TJ MFMA tiles of 16 x 16)
template <typename T, bool CONJA, int TI, int TJ>
__global__ __launch_bounds__(256) void k_zgemm(int64_t m, int64_t n, int64_t kdim,
                                               cpx<T> alpha, const cpx<T> *__restrict__ A,
                                               int64_t lda, const cpx<T> *__restrict__ B,
                                               int64_t ldb, cpx<T> beta, cpx<T> *C,
                                               int64_t ldc) {
    constexpr int BM = 32 * TI, BN = 32 * TJ;
    constexpr int PAD = 2;
    __shared__ T As[2][BK][BM + PAD];     // [re/im][k][i]
    __shared__ T Bs[2][BK][BN + PAD];     // [re/im][k][j]
    typedef typename MfmaAcc<T>::type acc_t;

    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wv = tid >> 6;
    const int wrow = (wv & 1) * (BM / 2);
    const int wcol = (wv >> 1) * (BN / 2);
    const int64_t row0 = (int64_t)blockIdx.x * BM;
    const int64_t col0 = (int64_t)blockIdx.y * BN;

    acc_t accr[TI][TJ], acci[TI][TJ];
#pragma unroll
    for (int a = 0; a < TI; ++a)
#pragma unroll
        for (int b = 0; b < TJ; ++b) {
            accr[a][b] = acc_t{0, 0, 0, 0};
            acci[a][b] = acc_t{0, 0, 0, 0};
        }

    // per-thread staging registers: A tile BM*BK elements, B tile BK*BN, over 256 threads
    constexpr int NA = BM * BK / 256;
    constexpr int NB = BN * BK / 256;
    cpx<T> ra[NA], rb[NB];

    auto load_tiles = [&](int64_t k0) {
#pragma unroll
        for (int r = 0; r < NA; ++r) {
            int e = tid + 256 * r;
            int i, kk;
            if (!CONJA) { i = e % BM; kk = e / BM; }      // contiguous along rows
            else { kk = e % BK; i = e / BK; }              // contiguous along k
            int64_t gi = row0 + i, gk = k0 + kk;
            cpx<T> v = mk((T)0, (T)0);
            if (gi < m && gk < kdim) {
                v = CONJA ? A[gk + gi * lda] : A[gi + gk * lda];
                if (CONJA) v.y = -v.y;
            }
            ra[r] = v;
        }
#pragma unroll
        for (int r = 0; r < NB; ++r) {
            int e = tid + 256 * r;
            int kk = e % BK, j = e / BK;
            int64_t gj = col0 + j, gk = k0 + kk;
            cpx<T> v = mk((T)0, (T)0);
            if (gj < n && gk < kdim) v = B[gk + gj * ldb];
            rb[r] = v;
        }
    };
    auto store_tiles = [&]() {
#pragma unroll
        for (int r = 0; r < NA; ++r) {
            int e = tid + 256 * r;
            int i, kk;
            if (!CONJA) { i = e % BM; kk = e / BM; }
            else { kk = e % BK; i = e / BK; }
            As[0][kk][i] = ra[r].x;
            As[1][kk][i] = ra[r].y;
        }
#pragma unroll
        for (int r = 0; r < NB; ++r) {
            int e = tid + 256 * r;
            int kk = e % BK, j = e / BK;
            Bs[0][kk][j] = rb[r].x;
            Bs[1][kk][j] = rb[r].y;
        }
    };

    load_tiles(0);
    for (int64_t k0 = 0; k0 < kdim; k0 += BK) {
        __syncthreads();
        store_tiles();
        __syncthreads();
        if (k0 + BK < kdim) load_tiles(k0 + BK);
#pragma unroll
        for (int k4 = 0; k4 < BK; k4 += 4) {
            const int kk = k4 + (lane >> 4);
            T ar[TI], ai[TI], br[TJ], bi[TJ];
#pragma unroll
            for (int a = 0; a < TI; ++a) {
                ar[a] = As[0][kk][wrow + a * 16 + (lane & 15)];
                ai[a] = As[1][kk][wrow + a * 16 + (lane & 15)];
            }
#pragma unroll
            for (int b = 0; b < TJ; ++b) {
                br[b] = Bs[0][kk][wcol + b * 16 + (lane & 15)];
                bi[b] = Bs[1][kk][wcol + b * 16 + (lane & 15)];
            }
#pragma unroll
            for (int a = 0; a < TI; ++a)
#pragma unroll
                for (int b = 0; b < TJ; ++b) {
                    accr[a][b] = mfma(ar[a], br[b], accr[a][b]);
                    accr[a][b] = mfma(-ai[a], bi[b], accr[a][b]);
                    acci[a][b] = mfma(ar[a], bi[b], acci[a][b]);
                    acci[a][b] = mfma(ai[a], br[b], acci[a][b]);
                }
        }
    }
    // epilogue: column lane%16 of each 16x16 tile, rows from acc_row
    const bool beta_zero = (beta.x == (T)0 && beta.y == (T)0);
#pragma unroll
    for (int a = 0; a < TI; ++a)
#pragma unroll
        for (int b = 0; b < TJ; ++b) {
            int64_t gj = col0 + wcol + b * 16 + (lane & 15);
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                int64_t gi = row0 + wrow + a * 16 + acc_row<T>(lane, r);
                if (gi < m && gj < n) {
                    cpx<T> v = mk((T)accr[a][b][r], (T)acci[a][b][r]);
                    v = alpha * v;
                    cpx<T> *p = C + gi + gj * ldc;
                    if (!beta_zero) v = v + beta * (*p);
                    *p = v;
                }
            }
        }
}

template <typename T>
void gemm(bool conjA, int64_t m, int64_t n, int64_t k, cpx<T> alpha, const cpx<T> *A,
          int64_t lda, const cpx<T> *B, int64_t ldb, cpx<T> beta, cpx<T> *C, int64_t ldc,
          hipStream_t s) {
    if (m <= 0 || n <= 0) return;
    if (k <= 0) {
        // C = beta C : run the kernel with an empty K loop
    }
    constexpr int TI = 2, TJ = 2;
    ProfScope prof(sizeof(T) == sizeof(double) ? PROF_GEMM64 : PROF_GEMM32,
                   8.0 * (double)m * (double)n * (double)k, s);
    dim3 grid((unsigned)((m + 32 * TI - 1) / (32 * TI)), (unsigned)((n + 32 * TJ - 1) / (32 * TJ)));
    if (conjA)
        hipLaunchKernelGGL((k_zgemm<T, true, TI, TJ>), grid, dim3(256), 0, s, m, n, k, alpha, A,
                           lda, B, ldb, beta, C, ldc);
    else
        hipLaunchKernelGGL((k_zgemm<T, false, TI, TJ>), grid, dim3(256), 0, s, m, n, k, alpha,
                           A, lda, B, ldb, beta, C, ldc);
}

template void gemm<double>(bool, int64_t, int64_t, int64_t, zd, const zd *, int64_t,
                           const zd *, int64_t, zd, zd *, int64_t, hipStream_t);
template void gemm<float>(bool, int64_t, int64_t, int64_t, zf, const zf *, int64_t,
                          const zf *, int64_t, zf, zf *, int64_t, hipStream_t);

}  // namespace cfie
