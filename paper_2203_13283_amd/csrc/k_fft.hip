// Circulant algebra on the equivalent circle (Sec. V): C_c and every Galerkin matrix on
// gamma_c are circulant, so they are diagonal in the discrete Fourier basis, and products
// with C_c, C_c^H or C_c^{-1} are y = IFFT(d .* FFT(x)) for an eigenvalue vector d.
//
// Length N = N1 * N2 (powers of two, N1 <= 4096) by the four-step splitting
//   step A : y[n1 + N1 k2] = W_N^{n1 k2} sum_{n2} x[n1 + N1 n2] W_{N2}^{n2 k2}
//   step B : for each k2, a length-N1 FFT of the contiguous chunk y[N1 k2 .. N1 k2 + N1)
// which leaves X[k2 + N2 k1] at position k1 + N1 k2.  The diagonal is stored in that
// order, so the middle kernel does FFT_N1 -> multiply -> inverse FFT_N1 while the chunk is
// in LDS, and the inverse of step A restores natural order.  Three passes over memory for
// N > 4096, one for N <= 4096.  Radix-4 Stockham stages in LDS (one radix-2 stage for odd
// powers of two), twiddles from tables, all index arithmetic by shifts and masks; N1 = 4096
// has a middle kernel of its own (radix 16, mostly in registers).
#include "internal.h"

namespace cfie {

__device__ __forceinline__ int ilog2(int n) { return 31 - __clz(n); }

// One Stockham stage of radix R (2 or 4) over the n points held in LDS (split re / im):
// for butterfly j < n/R with k = j mod L, inputs x[j + r n/R] times w^{r k},
// w = e^{-/+ 2 pi i / (R L)}, an R-point DFT, outputs at (j - k) R + k + s L.
// Results go through registers (read all, barrier, write all, barrier).  256 threads.
template <typename T, int R>
__device__ __forceinline__ void lds_stage(T *re, T *im, int lgn, int lgL,
                                          const cpx<T> *__restrict__ tw, bool inverse) {
    constexpr int MAXB = 4096 / R / 256;         // butterflies per thread (n <= 4096, 256 thr)
    const int n = 1 << lgn;
    const int nq = n / R;
    const int L = 1 << lgL;
    const int twsh = lgn - lgL - (R == 4 ? 2 : 1);   // table step n / (R L)
    cpx<T> y[MAXB][R];
#pragma unroll
    for (int nb = 0; nb < MAXB; ++nb) {
        const int j = threadIdx.x + nb * 256;
        if (j >= nq) break;
        const int k = j & (L - 1);
        cpx<T> a[R];
#pragma unroll
        for (int r = 0; r < R; ++r) a[r] = mk(re[j + r * nq], im[j + r * nq]);
#pragma unroll
        for (int r = 1; r < R; ++r) {
            cpx<T> w = tw[(r * k) << twsh];
            if (inverse) w.y = -w.y;
            a[r] = a[r] * w;
        }
        if constexpr (R == 2) {
            y[nb][0] = a[0] + a[1];
            y[nb][1] = a[0] - a[1];
        } else {
            // 4-point DFT; forward uses -i, inverse +i
            cpx<T> s02 = a[0] + a[2], d02 = a[0] - a[2];
            cpx<T> s13 = a[1] + a[3], d13 = a[1] - a[3];
            cpx<T> jd13 = inverse ? mk(-d13.y, d13.x) : mk(d13.y, -d13.x);   // -/+ i d13
            y[nb][0] = s02 + s13;
            y[nb][1] = d02 + jd13;
            y[nb][2] = s02 - s13;
            y[nb][3] = d02 - jd13;
        }
    }
    __syncthreads();
#pragma unroll
    for (int nb = 0; nb < MAXB; ++nb) {
        const int j = threadIdx.x + nb * 256;
        if (j >= nq) break;
        const int k = j & (L - 1);
        const int base = ((j >> lgL) << (lgL + (R == 4 ? 2 : 1))) + k;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            re[base + r * L] = y[nb][r].x;
            im[base + r * L] = y[nb][r].y;
        }
    }
    __syncthreads();
}

// In-place FFT of n = 2^lgn points in LDS: one radix-2 stage when lgn is odd, then radix-4
// stages.  tw: e^{-2 pi i j / n}, j < n.  No scaling.
template <typename T>
__device__ __forceinline__ void lds_fft(T *re, T *im, int lgn, const cpx<T> *__restrict__ tw,
                                        bool inverse) {
    int lgL = 0;
    if (lgn & 1) {
        lds_stage<T, 2>(re, im, lgn, 0, tw, inverse);
        lgL = 1;
    }
    for (; lgL < lgn; lgL += 2) lds_stage<T, 4>(re, im, lgn, lgL, tw, inverse);
}

// middle step: chunk k2 = blockIdx.x mod N2 of column blockIdx.x / N2
template <typename T>
__global__ __launch_bounds__(256) void k_fft_mid(int N1, int N2, const cpx<T> *__restrict__ tw1,
                                                 const cpx<T> *__restrict__ d, cpx<T> *x,
                                                 int64_t ldx) {
    extern __shared__ unsigned char smem_raw[];
    T *re = reinterpret_cast<T *>(smem_raw);
    T *im = re + N1;
    const int k2 = (int)(blockIdx.x % N2);
    cpx<T> *col = x + (int64_t)(blockIdx.x / N2) * ldx + (int64_t)k2 * N1;
    const cpx<T> *dc = d + (int64_t)k2 * N1;
    for (int i = threadIdx.x; i < N1; i += blockDim.x) {
        cpx<T> v = col[i];
        re[i] = v.x;
        im[i] = v.y;
    }
    __syncthreads();
    const int lg = ilog2(N1);
    lds_fft(re, im, lg, tw1, false);
    for (int i = threadIdx.x; i < N1; i += blockDim.x) {
        cpx<T> v = mk(re[i], im[i]) * dc[i];
        re[i] = v.x;
        im[i] = v.y;
    }
    __syncthreads();
    lds_fft(re, im, lg, tw1, true);
    for (int i = threadIdx.x; i < N1; i += blockDim.x) col[i] = mk(re[i], im[i]);
}

// ---- middle step for N1 = 4096 = 16^3: three radix-16 Stockham stages each way ----------
// Thread j (256 per workgroup) owns the 16 points j + 256 r of every stage's input.  A
// radix-16 butterfly is two layers of 4-point DFTs with the sixteenth roots of unity between
// them; the first stage (L = 1) needs no twiddles, and the last (L = 256) leaves point
// j + 256 q in the thread that computed it, so the chunk enters from global memory straight
// into registers, is multiplied by the diagonal and starts the inverse transform without an
// exchange, and leaves from registers.  Four exchanges through LDS in all, real and
// imaginary parts in turn through 35 KB (FP64), with one pad element per 16 so that the
// stride-16 writes of the first stage hit distinct banks.  The twiddles w^{r k} of the
// second and third stages come from the table of e^{-2 pi i m / 4096} (conjugated for the
// inverse).
template <typename T, bool INV>
__device__ __forceinline__ void dft4(cpx<T> &x0, cpx<T> &x1, cpx<T> &x2, cpx<T> &x3) {
    const cpx<T> s02 = x0 + x2, d02 = x0 - x2, s13 = x1 + x3, d13 = x1 - x3;
    const cpx<T> jd = INV ? mk(-d13.y, d13.x) : mk(d13.y, -d13.x);     // +/- i d13
    x0 = s02 + s13;
    x1 = d02 + jd;
    x2 = s02 - s13;
    x3 = d02 - jd;
}

// 16-point DFT of a[0..15]; output q = q1 + 4 q0 is left in a[4 q1 + q0]
template <typename T, bool INV>
__device__ __forceinline__ void dft16(cpx<T> (&a)[16]) {
    // cos and sin of 2 pi e / 16, e = 0..9
    constexpr double C1 = 0.92387953251128675613, S1 = 0.38268343236508977173;
    constexpr double R2 = 0.70710678118654752440;
    constexpr double cs[10][2] = {{1, 0},  {C1, S1},  {R2, R2},  {S1, C1},  {0, 1},
                                  {-S1, C1}, {-R2, R2}, {-C1, S1}, {-1, 0}, {-C1, -S1}};
#pragma unroll
    for (int r0 = 0; r0 < 4; ++r0) dft4<T, INV>(a[r0], a[r0 + 4], a[r0 + 8], a[r0 + 12]);
#pragma unroll
    for (int r0 = 1; r0 < 4; ++r0) {
#pragma unroll
        for (int q1 = 1; q1 < 4; ++q1) {
            const int e = r0 * q1;
            const cpx<T> w = mk((T)cs[e][0], (T)(INV ? cs[e][1] : -cs[e][1]));
            a[r0 + 4 * q1] = a[r0 + 4 * q1] * w;
        }
    }
#pragma unroll
    for (int q1 = 0; q1 < 4; ++q1)
        dft4<T, INV>(a[4 * q1], a[4 * q1 + 1], a[4 * q1 + 2], a[4 * q1 + 3]);
}

__device__ __forceinline__ int pad16(int p) { return p + (p >> 4); }

// write the 16 outputs of a butterfly to positions base + q L, then read the next stage's
// inputs j + 256 r; real and imaginary parts pass one after the other through the same
// 4096 + 256 words of LDS
template <typename T>
__device__ __forceinline__ void exchange16(T *buf, cpx<T> (&a)[16], int base, int L) {
    const int j = threadIdx.x;
#pragma unroll
    for (int part = 0; part < 2; ++part) {
#pragma unroll
        for (int q = 0; q < 16; ++q) {
            const cpx<T> v = a[4 * (q & 3) + (q >> 2)];
            buf[pad16(base + q * L)] = part ? v.y : v.x;
        }
        __syncthreads();
        T t[16];
#pragma unroll
        for (int r = 0; r < 16; ++r) t[r] = buf[pad16(j + 256 * r)];
        __syncthreads();
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            if (part) a[r].y = t[r];
            else a[r].x = t[r];
        }
    }
}

// multiply a[1..15] by the stage twiddles w^{r k} (conjugated for the inverse); the stage
// with L = 16 has w = e^{-2 pi i / 256}, k = j mod 16, the stage with L = 256 has
// w = e^{-2 pi i / 4096}, k = j.  w^k and w^{4k} come from the table, the other powers
// from at most two products of table values (w^{(4a + b) k} = w^{4ak} w^{bk}), which keeps
// 6 twiddles live instead of 15.
template <typename T, bool INV>
__device__ __forceinline__ void twiddle16(cpx<T> (&a)[16], const cpx<T> *__restrict__ tw1,
                                          int L) {
    const int j = threadIdx.x;
    const int k = L == 16 ? (j & 15) : j;
    const int sh = L == 16 ? 4 : 0;
    cpx<T> w1 = tw1[k << sh], w4 = tw1[(4 * k) << sh];
    if (INV) {
        w1 = conj(w1);
        w4 = conj(w4);
    }
    const cpx<T> w2 = w1 * w1, w3 = w2 * w1;
    const cpx<T> w8 = w4 * w4, w12 = w8 * w4;
    a[1] = a[1] * w1;
    a[2] = a[2] * w2;
    a[3] = a[3] * w3;
    a[4] = a[4] * w4;
    a[8] = a[8] * w8;
    a[12] = a[12] * w12;
#pragma unroll
    for (int b = 1; b < 4; ++b) {
        const cpx<T> wb = b == 1 ? w1 : (b == 2 ? w2 : w3);
        a[4 + b] = a[4 + b] * (w4 * wb);
        a[8 + b] = a[8 + b] * (w8 * wb);
        a[12 + b] = a[12 + b] * (w12 * wb);
    }
}

template <typename T, bool INV>
__device__ __forceinline__ void fft4096_regs(T *buf, cpx<T> (&a)[16],
                                             const cpx<T> *__restrict__ tw1) {
    const int j = threadIdx.x;
    dft16<T, INV>(a);
    exchange16<T>(buf, a, 16 * j, 1);
    twiddle16<T, INV>(a, tw1, 16);
    dft16<T, INV>(a);
    exchange16<T>(buf, a, (j >> 4) * 256 + (j & 15), 16);
    twiddle16<T, INV>(a, tw1, 256);
    dft16<T, INV>(a);
}

// chunk k2 = blockIdx.x mod N2 of column blockIdx.x / N2; registers budgeted for three
// workgroups per compute unit in FP64 and four in FP32 (the LDS would allow four in FP64)
template <typename T>
__global__ __launch_bounds__(256, sizeof(T) == 8 ? 3 : 4) void k_fft_mid4096(
    int N2, const cpx<T> *__restrict__ tw1, const cpx<T> *__restrict__ d, cpx<T> *x,
    int64_t ldx) {
    __shared__ T buf[4096 + 4096 / 16];
    const int j = threadIdx.x;
    const int k2 = (int)(blockIdx.x % N2);
    cpx<T> *col = x + (int64_t)(blockIdx.x / N2) * ldx + (int64_t)k2 * 4096;
    const cpx<T> *dc = d + (int64_t)k2 * 4096;
    cpx<T> a[16], b[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) a[r] = col[j + 256 * r];
    fft4096_regs<T, false>(buf, a, tw1);
    // spectrum point j + 256 q times the diagonal: the inverse's first-stage inputs
#pragma unroll
    for (int q = 0; q < 16; ++q) b[q] = a[4 * (q & 3) + (q >> 2)] * dc[j + 256 * q];
    fft4096_regs<T, true>(buf, b, tw1);
#pragma unroll
    for (int q = 0; q < 16; ++q) col[j + 256 * q] = b[4 * (q & 3) + (q >> 2)];
}

// step A (forward or inverse) for one (n1, column) per thread; N1, N2 powers of two.
// N2 is a template parameter so the per-thread vectors stay in registers.
// The input is read from src (leading dimension lds), which may be x itself.
template <typename T, int N2>
__global__ __launch_bounds__(256) void k_fft_stepA(int N1, const cpx<T> *__restrict__ twN,
                                                   const cpx<T> *src, int64_t lds, cpx<T> *x,
                                                   int64_t ldx, int64_t ncol, bool inverse) {
    int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= (int64_t)N1 * ncol) return;
    const int lg1 = ilog2(N1);
    const int mN = N1 * N2 - 1;
    const int n1 = (int)(tid & (N1 - 1));
    const int64_t c = tid >> lg1;
    cpx<T> *col = x + c * ldx;
    const cpx<T> *scol = src + c * lds;
    cpx<T> v[N2], o[N2];
#pragma unroll
    for (int a = 0; a < N2; ++a) v[a] = scol[n1 + (int64_t)N1 * a];
    if (!inverse) {
#pragma unroll
        for (int k2 = 0; k2 < N2; ++k2) {
            cpx<T> s = v[0];
#pragma unroll
            for (int n2 = 1; n2 < N2; ++n2) s = s + v[n2] * twN[((n2 * k2) & (N2 - 1)) << lg1];
            o[k2] = s * twN[(n1 * k2) & mN];
        }
    } else {
#pragma unroll
        for (int k2 = 1; k2 < N2; ++k2) v[k2] = v[k2] * conj(twN[(n1 * k2) & mN]);
#pragma unroll
        for (int n2 = 0; n2 < N2; ++n2) {
            cpx<T> s = v[0];
#pragma unroll
            for (int k2 = 1; k2 < N2; ++k2)
                s = s + v[k2] * conj(twN[((n2 * k2) & (N2 - 1)) << lg1]);
            o[n2] = s;
        }
    }
#pragma unroll
    for (int a = 0; a < N2; ++a) col[n1 + (int64_t)N1 * a] = o[a];
}

template <typename T>
void launch_stepA(const FFTPlan &p, const cpx<T> *twN, const cpx<T> *src, int64_t lds,
                  cpx<T> *x, int64_t ldx, int64_t nb, bool inverse, hipStream_t s) {
    const int bs = 256;
    int64_t n = (int64_t)p.N1 * nb;
    dim3 g((unsigned)((n + bs - 1) / bs));
    switch (p.N2) {
    case 2: hipLaunchKernelGGL((k_fft_stepA<T, 2>), g, dim3(bs), 0, s, p.N1, twN, src, lds, x, ldx, nb, inverse); break;
    case 4: hipLaunchKernelGGL((k_fft_stepA<T, 4>), g, dim3(bs), 0, s, p.N1, twN, src, lds, x, ldx, nb, inverse); break;
    case 8: hipLaunchKernelGGL((k_fft_stepA<T, 8>), g, dim3(bs), 0, s, p.N1, twN, src, lds, x, ldx, nb, inverse); break;
    default: hipLaunchKernelGGL((k_fft_stepA<T, 16>), g, dim3(bs), 0, s, p.N1, twN, src, lds, x, ldx, nb, inverse); break;
    }
}

// x[:, j] = src[:, j] for the n x nb block (the input copy of a circulant product whose
// first pass works in place)
template <typename T>
__global__ void k_copy_cols(int64_t n, int64_t nb, const cpx<T> *__restrict__ src, int64_t lds,
                            cpx<T> *x, int64_t ldx) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n * nb) return;
    const int64_t i = t % n, j = t / n;
    x[i + j * ldx] = src[i + j * lds];
}

template <typename T> const cpx<T> *tw1_of(const FFTPlan &p);
template <> const zd *tw1_of<double>(const FFTPlan &p) { return (const zd *)p.tw1; }
template <> const zf *tw1_of<float>(const FFTPlan &p) { return (const zf *)p.tw1f; }
template <typename T> const cpx<T> *twN_of(const FFTPlan &p);
template <> const zd *twN_of<double>(const FFTPlan &p) { return (const zd *)p.twM; }
template <> const zf *twN_of<float>(const FFTPlan &p) { return (const zf *)p.twMf; }

template <typename T>
void launch_circ_apply(const FFTPlan &p, const cpx<T> *d, cpx<T> *x, int64_t ldx, int64_t nb,
                       hipStream_t s, const cpx<T> *src, int64_t lds) {
    if (nb <= 0) return;
    const int bs = 256;
    if (!src) {
        src = x;
        lds = ldx;
    }
    if (src != x && p.N2 == 1) {
        // one pass, in place: copy the input first
        const int64_t n = (int64_t)p.M * nb;
        hipLaunchKernelGGL(k_copy_cols<T>, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, s,
                           (int64_t)p.M, nb, src, lds, x, ldx);
    }
    // algorithmic work: bytes of one read and one write of the batch
    ProfScope prof(PROF_FFT, 2.0 * sizeof(cpx<T>) * (double)p.M * (double)nb, s);
    if (p.N2 > 1) launch_stepA<T>(p, twN_of<T>(p), src, lds, x, ldx, nb, false, s);
    if (p.N1 == 4096) {
        hipLaunchKernelGGL(k_fft_mid4096<T>, dim3((unsigned)(p.N2 * nb)), dim3(256), 0, s,
                           p.N2, tw1_of<T>(p), d, x, ldx);
    } else {
        size_t sh = 2 * sizeof(T) * (size_t)p.N1;
        hipLaunchKernelGGL(k_fft_mid<T>, dim3((unsigned)(p.N2 * nb)), dim3(bs), sh, s, p.N1,
                           p.N2, tw1_of<T>(p), d, x, ldx);
    }
    if (p.N2 > 1) launch_stepA<T>(p, twN_of<T>(p), x, ldx, x, ldx, nb, true, s);
}

template void launch_circ_apply<double>(const FFTPlan &, const zd *, zd *, int64_t, int64_t,
                                        hipStream_t, const zd *, int64_t);
template void launch_circ_apply<float>(const FFTPlan &, const zf *, zf *, int64_t, int64_t,
                                       hipStream_t, const zf *, int64_t);

template <typename T>
__global__ void k_pad(int N, int M, int64_t nb, const cpx<T> *__restrict__ x, int64_t ldx,
                      cpx<T> *P) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)M * nb) return;
    int64_t i = t % M, j = t / M;
    P[t] = i < N ? x[i + j * ldx] : mk((T)0, (T)0);
}
template <typename T>
__global__ void k_unpad(int N, int M, int64_t nb, const cpx<T> *__restrict__ P, cpx<T> *x,
                        int64_t ldx) {
    int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)N * nb) return;
    int64_t i = t % N, j = t / N;
    x[i + j * ldx] = P[i + j * M];
}

template <typename T>
void launch_circ_apply_padded(const FFTPlan &p, const cpx<T> *d, cpx<T> *x, int64_t ldx,
                              int64_t nb, cpx<T> *P, hipStream_t s, const cpx<T> *src,
                              int64_t lds) {
    if (nb <= 0) return;
    const int bs = 256;
    if (!src) {
        src = x;
        lds = ldx;
    }
    int64_t nM = (int64_t)p.M * nb, nN = (int64_t)p.N * nb;
    hipLaunchKernelGGL(k_pad<T>, dim3((unsigned)((nM + bs - 1) / bs)), dim3(bs), 0, s, p.N, p.M,
                       nb, src, lds, P);
    launch_circ_apply<T>(p, d, P, p.M, nb, s, (const cpx<T> *)nullptr, 0);
    hipLaunchKernelGGL(k_unpad<T>, dim3((unsigned)((nN + bs - 1) / bs)), dim3(bs), 0, s, p.N,
                       p.M, nb, (const cpx<T> *)P, x, ldx);
}
template void launch_circ_apply_padded<double>(const FFTPlan &, const zd *, zd *, int64_t,
                                               int64_t, zd *, hipStream_t, const zd *, int64_t);
template void launch_circ_apply_padded<float>(const FFTPlan &, const zf *, zf *, int64_t,
                                              int64_t, zf *, hipStream_t, const zf *, int64_t);

// DFT by direct summation: y_m = scale sum_q x_q w^{m q} with w = tw[1] (tw: the n-th roots
// of unity, e^{-2 pi i j / n}), conjugated for inverse.  One wavefront per output m (so that
// a transform of a few thousand points still spreads over the whole device): lane l sums the
// terms q = l, l + 64, ..., its table index advancing by 64 m modulo n without division, for
// up to four columns at once (one table read serves them all); the 64 partial sums are
// combined by a butterfly, the same order on every run.
constexpr int kDftCols = 4;
__global__ __launch_bounds__(256) void k_dft_direct(int n, int ncol, const zd *__restrict__ x,
                                                    int64_t ldx, zd *y, int64_t ldy,
                                                    const zd *__restrict__ tw, bool inverse,
                                                    double scale) {
    const int lane = threadIdx.x & 63;
    const int64_t m = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (m >= n) return;                          // whole wavefronts only; no block barrier
    const int step = (int)((64 * m) % n);
    const int idx0 = (int)(((int64_t)lane * m) % n);
    for (int c0 = 0; c0 < ncol; c0 += kDftCols) {
        const int nc = min(kDftCols, ncol - c0);
        zd acc[kDftCols];
#pragma unroll
        for (int c = 0; c < kDftCols; ++c) acc[c] = mk(0.0, 0.0);
        int idx = idx0;
#pragma unroll 4
        for (int q = lane; q < n; q += 64) {
            zd w = tw[idx];
            if (inverse) w.y = -w.y;
#pragma unroll
            for (int c = 0; c < kDftCols; ++c)
                if (c < nc) acc[c] = acc[c] + x[q + (int64_t)(c0 + c) * ldx] * w;
            idx += step;
            if (idx >= n) idx -= n;
        }
#pragma unroll
        for (int c = 0; c < kDftCols; ++c) {
            double re = acc[c].x, im = acc[c].y;
#pragma unroll
            for (int o = 32; o >= 1; o >>= 1) {
                re += __shfl_xor(re, o, 64);
                im += __shfl_xor(im, o, 64);
            }
            if (lane == 0 && c < nc) y[m + (int64_t)(c0 + c) * ldy] = mk(re * scale, im * scale);
        }
    }
}

void launch_dft(int n, int ncol, const zd *x, int64_t ldx, zd *y, int64_t ldy, const zd *tw,
                bool inverse, double scale, hipStream_t s) {
    if (n <= 0 || ncol <= 0) return;
    hipLaunchKernelGGL(k_dft_direct, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, n, ncol, x,
                       ldx, y, ldy, tw, inverse, scale);
}

void launch_dft_direct_tw(int N, const zd *x, int64_t ldx, zd *y, int64_t ldy, int ncol,
                          const zd *twN, hipStream_t s) {
    launch_dft(N, ncol, x, ldx, y, ldy, twN, false, 1.0, s);
}

// kappa of length N (first column) -> wrapped kernel of length M: [0, N) and [M - N + 1, M)
__global__ void k_wrap(int N, int M, const zd *__restrict__ kap, zd *out) {
    int u = blockIdx.x * blockDim.x + threadIdx.x;
    if (u >= M) return;
    out[u] = u < N ? kap[u] : (u > M - N ? kap[u - M + N] : mk(0.0, 0.0));
}
// natural order (length M) -> transposed layout of the four-step FFT, FP64 and FP32
__global__ void k_diag_transpose(int M, int N1, int N2, const zd *__restrict__ nat, zd *dT,
                                 zf *fT) {
    int q = blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= M) return;
    int k2 = q % N2, k1 = q / N2;
    int pos = k1 + N1 * k2;
    zd v = nat[q];
    dT[pos] = v;
    fT[pos] = mk((float)v.x, (float)v.y);
}

void launch_padded_diagonal(const FFTPlan &p, const zd *eig_over_N, zd *work, zd *dT, zf *fT,
                            hipStream_t s) {
    // work: 3 M entries (kappa, wrapped kernel, its transform)
    const int bs = 256;
    zd *kap = work, *wrp = work + p.M, *hat = work + 2 * (size_t)p.M;
    launch_dft(p.N, 1, eig_over_N, p.N, kap, p.N, (const zd *)p.twN, true, 1.0, s);
    hipLaunchKernelGGL(k_wrap, dim3((p.M + bs - 1) / bs), dim3(bs), 0, s, p.N, p.M,
                       (const zd *)kap, wrp);
    launch_dft(p.M, 1, wrp, p.M, hat, p.M, (const zd *)p.twM, false, 1.0 / p.M, s);
    hipLaunchKernelGGL(k_diag_transpose, dim3((p.M + bs - 1) / bs), dim3(bs), 0, s, p.M, p.N1,
                       p.N2, (const zd *)hat, dT, fT);
}


// ------------------------------------------------------------------ SRFT row transform ---
// A D F for the sketch's structured test matrix (the SrftPlan passes over the transform
// length M, a power of two >= the N columns of A; columns N..M-1 of A count as zero): pass l
// of radix R = 2^bits[l] splits sub-arrays of L columns (L = M for the first pass, then
// L / R for the next) with stride S = L / R.  Butterfly group g (blockIdx.y, so uniform
// over the workgroup) takes the columns c_b = B + a + S b, b < R (B = (g / S) L,
// a = g mod S), forms the R-point DFT y_e = sum_b x_b w_R^{b e}, scales y_e by w_L^{a e} and
// writes it to column B + a + S e: the same columns, so every pass after the first runs in
// place.  After all passes column j of A D F sits at the position whose pass digits are
// those of j in reverse order (srft_freq).  Lanes run along the rows: every load and store
// is a row segment of 64 consecutive entries (1 KiB in FP64), and the table reads are
// uniform over the workgroup.  tw holds e^{-2 pi i j / (M tws)}: w_M^j = tw[j tws].
constexpr int bitrev_const(int q, int bits) {
    int r = 0;
    for (int i = 0; i < bits; ++i) r |= ((q >> i) & 1) << (bits - 1 - i);
    return r;
}
constexpr int log2_const(int r) { return r <= 1 ? 0 : 1 + log2_const(r / 2); }

template <typename T, int R, bool FIRST>
__global__ __launch_bounds__(256) void k_srft_pass(int64_t m, int N, int M, int L,
                                                   const cpx<T> *__restrict__ A, int64_t lda,
                                                   const cpx<T> *__restrict__ d,
                                                   const cpx<T> *__restrict__ tw, int tws,
                                                   cpx<T> *out, int64_t ldo) {
    constexpr int RB = log2_const(R);
    const int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= m) return;
    const int S = L / R;
    const int g = blockIdx.y;
    const int a = g & (S - 1);
    const int B = (g / S) * L;
    cpx<T> x[R];
#pragma unroll
    for (int b = 0; b < R; ++b) {
        const int col = B + a + S * b;
        if constexpr (FIRST)
            x[b] = col < N ? A[r + (int64_t)col * lda] * d[col] : mk((T)0, (T)0);
        else
            x[b] = out[r + (int64_t)col * ldo];
    }
    // R-point DFT by radix-2 decimation in frequency in registers: x[q] ends as y_{rev(q)}
    const int wst = (M / 2) * tws;                   // table step of w_2
#pragma unroll
    for (int h = R / 2; h >= 1; h >>= 1) {
#pragma unroll
        for (int b0 = 0; b0 < R; b0 += 2 * h) {
#pragma unroll
            for (int k = 0; k < h; ++k) {
                const cpx<T> u = x[b0 + k], v = x[b0 + k + h];
                x[b0 + k] = u + v;
                cpx<T> t = u - v;
                if (k != 0) {
                    if (2 * k == h) t = mk(t.y, -t.x);               // w_{2h}^{h/2} = -i
                    else t = t * tw[k * (wst / h)];                // w_{2h}^k
                }
                x[b0 + k + h] = t;
            }
        }
    }
    const int tsc = (M / L) * tws;
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int e = bitrev_const(q, RB);
        cpx<T> y = x[q];
        if (e != 0) y = y * tw[(a * e) * tsc];                     // w_L^{a e}, a e < L
        out[r + (int64_t)(B + a + S * e) * ldo] = y;
    }
}

template <typename T>
void launch_srft_rows(int64_t m, int N, int M, const cpx<T> *A, int64_t lda, const cpx<T> *d,
                      const cpx<T> *tw, int tws, cpx<T> *out, int64_t ldo, hipStream_t s) {
    if (m <= 0) return;
    int lgM = 0;
    while ((1 << lgM) < M) ++lgM;
    if ((1 << lgM) != M || N > M || N < 1 || tws < 1)
        throw std::invalid_argument("SRFT length must be a power of two >= N");
    const SrftPlan p = srft_plan(lgM);
    int L = M;
    for (int l = 0; l < p.npass; ++l) {
        const int R = 1 << p.bits[l];
        const dim3 grid((unsigned)((m + 255) / 256), (unsigned)(M / R));
#define CFIE_SRFT_CASE(RR)                                                                    \
    case RR:                                                                                  \
        if (l == 0)                                                                           \
            hipLaunchKernelGGL((k_srft_pass<T, RR, true>), grid, dim3(256), 0, s, m, N, M, L,  \
                               A, lda, d, tw, tws, out, ldo);                                 \
        else                                                                                  \
            hipLaunchKernelGGL((k_srft_pass<T, RR, false>), grid, dim3(256), 0, s, m, N, M, L, \
                               (const cpx<T> *)nullptr, (int64_t)0, d, tw, tws, out, ldo);    \
        break;
        switch (R) {
            CFIE_SRFT_CASE(2)
            CFIE_SRFT_CASE(4)
            CFIE_SRFT_CASE(8)
            CFIE_SRFT_CASE(16)
            CFIE_SRFT_CASE(32)
            default: throw std::logic_error("SRFT radix");
        }
#undef CFIE_SRFT_CASE
        L /= R;
    }
}
template void launch_srft_rows<double>(int64_t, int, int, const zd *, int64_t, const zd *,
                                       const zd *, int, zd *, int64_t, hipStream_t);
template void launch_srft_rows<float>(int64_t, int, int, const zf *, int64_t, const zf *,
                                      const zf *, int, zf *, int64_t, hipStream_t);

// Om[i, t] = d_i w_M^{i j} (i < N), j the frequency at position perm(off + t)
template <typename T>
__global__ void k_srft_omega(int N, int M, SrftPlan p, SrftPerm q, int64_t off, int nb,
                             const cpx<T> *__restrict__ d, const cpx<T> *__restrict__ tw,
                             int tws, cpx<T> *Om, int64_t ldo) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= (int64_t)N * nb) return;
    const int i = (int)(tid % N), t = (int)(tid / N);
    const int j = srft_freq(p, (int)srft_perm_apply(q, (uint32_t)(off + t)));
    const int64_t idx = (((int64_t)i * j) & (M - 1)) * tws;
    Om[i + (int64_t)t * ldo] = d[i] * tw[idx];
}

template <typename T>
void launch_srft_omega(int N, const SrftPerm &q, int64_t off, int nb, const cpx<T> *d,
                       const cpx<T> *tw, int tws, cpx<T> *Om, int64_t ldo, hipStream_t s) {
    const int64_t t = (int64_t)N * nb;
    if (t <= 0) return;
    const int M = 1 << q.lgN;
    if (N > M || off < 0 || off + nb > M) throw std::invalid_argument("SRFT columns exhausted");
    const SrftPlan p = srft_plan(q.lgN);
    hipLaunchKernelGGL(k_srft_omega<T>, dim3((unsigned)((t + 255) / 256)), dim3(256), 0, s, N,
                       M, p, q, off, nb, d, tw, tws, Om, ldo);
}
template void launch_srft_omega<double>(int, const SrftPerm &, int64_t, int, const zd *,
                                        const zd *, int, zd *, int64_t, hipStream_t);
template void launch_srft_omega<float>(int, const SrftPerm &, int64_t, int, const zf *,
                                       const zf *, int, zf *, int64_t, hipStream_t);

template <typename T>
__global__ void k_srft_gather(int64_t m, SrftPerm q, int64_t off, int nb,
                              const cpx<T> *__restrict__ AF, int64_t ldaf, cpx<T> *out,
                              int64_t ldo) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= m * nb) return;
    const int64_t i = tid % m;
    const int t = (int)(tid / m);
    const int64_t col = srft_perm_apply(q, (uint32_t)(off + t));
    out[i + (int64_t)t * ldo] = AF[i + col * ldaf];
}

template <typename T>
void launch_srft_gather(int64_t m, const SrftPerm &q, int64_t off, int nb, const cpx<T> *AF,
                        int64_t ldaf, cpx<T> *out, int64_t ldo, hipStream_t s) {
    const int64_t t = m * nb;
    if (t <= 0) return;
    if (off < 0 || off + nb > ((int64_t)1 << q.lgN))
        throw std::invalid_argument("SRFT columns exhausted");
    hipLaunchKernelGGL(k_srft_gather<T>, dim3((unsigned)((t + 255) / 256)), dim3(256), 0, s, m,
                       q, off, nb, AF, ldaf, out, ldo);
}
template void launch_srft_gather<double>(int64_t, const SrftPerm &, int64_t, int, const zd *,
                                         int64_t, zd *, int64_t, hipStream_t);
template void launch_srft_gather<float>(int64_t, const SrftPerm &, int64_t, int, const zf *,
                                        int64_t, zf *, int64_t, hipStream_t);

// splitmix64 (Steele, Lea and Flood, OOPSLA 2014) keys the permutation's rounds
SrftPerm srft_perm(uint64_t seed, int lgN) {
    SrftPerm q;
    q.lgN = lgN;
    uint64_t z = seed ^ 0x3c6ef372fe94f82bull;
    auto next = [&z]() {
        z += 0x9e3779b97f4a7c15ull;
        uint64_t x = z;
        x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
        x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
        return x ^ (x >> 31);
    };
    for (int r = 0; r < 3; ++r) {
        q.mul[r] = (uint32_t)next() | 1u;
        q.add[r] = (uint32_t)next();
    }
    return q;
}

}  // namespace cfie
