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
// N > 4096, one for N <= 4096.  Radix-2 Stockham passes in LDS, twiddles from tables.
#include "internal.h"

namespace cfie {

template <typename T>
__device__ __forceinline__ void lds_fft(T *re, T *im, int n, const cpx<T> *__restrict__ tw,
                                        bool inverse) {
    const int T_ = blockDim.x;
    const int half = n >> 1;
    for (int Ns = 1; Ns < n; Ns <<= 1) {
        // each thread: butterflies j = tid, tid + T, ...
        constexpr int MAXB = 8;                  // n / 2 / blockDim <= 8 (n <= 4096, 256 thr)
        cpx<T> b0[MAXB], b1[MAXB];
        int nb = 0;
        for (int j = threadIdx.x; j < half; j += T_) {
            cpx<T> a0 = mk(re[j], im[j]);
            cpx<T> a1 = mk(re[j + half], im[j + half]);
            cpx<T> w = tw[(j & (Ns - 1)) * (n / (2 * Ns))];
            if (inverse) w.y = -w.y;
            a1 = a1 * w;
            b0[nb] = a0 + a1;
            b1[nb] = a0 - a1;
            ++nb;
        }
        __syncthreads();
        nb = 0;
        for (int j = threadIdx.x; j < half; j += T_) {
            int idx = (j / Ns) * 2 * Ns + (j & (Ns - 1));
            re[idx] = b0[nb].x;
            im[idx] = b0[nb].y;
            re[idx + Ns] = b1[nb].x;
            im[idx + Ns] = b1[nb].y;
            ++nb;
        }
        __syncthreads();
    }
}

// middle step: chunk k2 = blockIdx.x of column blockIdx.y
template <typename T>
__global__ __launch_bounds__(256) void k_fft_mid(int N1, const cpx<T> *__restrict__ tw1,
                                                 const cpx<T> *__restrict__ d, cpx<T> *x,
                                                 int64_t ldx) {
    extern __shared__ unsigned char smem_raw[];
    T *re = reinterpret_cast<T *>(smem_raw);
    T *im = re + N1;
    const int k2 = blockIdx.x;
    cpx<T> *col = x + (int64_t)blockIdx.y * ldx + (int64_t)k2 * N1;
    const cpx<T> *dc = d + (int64_t)k2 * N1;
    for (int i = threadIdx.x; i < N1; i += blockDim.x) {
        cpx<T> v = col[i];
        re[i] = v.x;
        im[i] = v.y;
    }
    __syncthreads();
    lds_fft(re, im, N1, tw1, false);
    for (int i = threadIdx.x; i < N1; i += blockDim.x) {
        cpx<T> v = mk(re[i], im[i]) * dc[i];
        re[i] = v.x;
        im[i] = v.y;
    }
    __syncthreads();
    lds_fft(re, im, N1, tw1, true);
    for (int i = threadIdx.x; i < N1; i += blockDim.x) col[i] = mk(re[i], im[i]);
}

// step A (forward or inverse) for one (n1, column) per thread
template <typename T>
__global__ void k_fft_stepA(int N1, int N2, const cpx<T> *__restrict__ twN, cpx<T> *x,
                            int64_t ldx, int64_t ncol, bool inverse) {
    int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= (int64_t)N1 * ncol) return;
    const int N = N1 * N2;
    int n1 = (int)(tid % N1);
    int64_t c = tid / N1;
    cpx<T> *col = x + c * ldx;
    constexpr int MAXN2 = 16;
    cpx<T> v[MAXN2], o[MAXN2];
    for (int a = 0; a < N2; ++a) v[a] = col[n1 + (int64_t)N1 * a];
    if (!inverse) {
        for (int k2 = 0; k2 < N2; ++k2) {
            cpx<T> s = mk((T)0, (T)0);
            for (int n2 = 0; n2 < N2; ++n2) s = s + v[n2] * twN[(int64_t)((n2 * k2) % N2) * N1];
            o[k2] = s * twN[((int64_t)n1 * k2) % N];
        }
    } else {
        for (int k2 = 0; k2 < N2; ++k2) v[k2] = v[k2] * conj(twN[((int64_t)n1 * k2) % N]);
        for (int n2 = 0; n2 < N2; ++n2) {
            cpx<T> s = mk((T)0, (T)0);
            for (int k2 = 0; k2 < N2; ++k2)
                s = s + v[k2] * conj(twN[(int64_t)((n2 * k2) % N2) * N1]);
            o[n2] = s;
        }
    }
    for (int a = 0; a < N2; ++a) col[n1 + (int64_t)N1 * a] = o[a];
}

template <typename T> const cpx<T> *tw1_of(const FFTPlan &p);
template <> const zd *tw1_of<double>(const FFTPlan &p) { return (const zd *)p.tw1; }
template <> const zf *tw1_of<float>(const FFTPlan &p) { return (const zf *)p.tw1f; }
template <typename T> const cpx<T> *twN_of(const FFTPlan &p);
template <> const zd *twN_of<double>(const FFTPlan &p) { return (const zd *)p.twN; }
template <> const zf *twN_of<float>(const FFTPlan &p) { return (const zf *)p.twNf; }

template <typename T>
void launch_circ_apply(const FFTPlan &p, const cpx<T> *d, cpx<T> *x, int64_t ldx, int64_t nb,
                       hipStream_t s) {
    if (nb <= 0) return;
    const int bs = 256;
    // algorithmic work: bytes of one read and one write of the batch
    ProfScope prof(PROF_FFT, 2.0 * sizeof(cpx<T>) * (double)p.N * (double)nb, s);
    if (p.N2 > 1) {
        int64_t n = (int64_t)p.N1 * nb;
        hipLaunchKernelGGL(k_fft_stepA<T>, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, s,
                           p.N1, p.N2, twN_of<T>(p), x, ldx, nb, false);
    }
    size_t sh = 2 * sizeof(T) * (size_t)p.N1;
    hipLaunchKernelGGL(k_fft_mid<T>, dim3(p.N2, (unsigned)nb), dim3(bs), sh, s, p.N1,
                       tw1_of<T>(p), d, x, ldx);
    if (p.N2 > 1) {
        int64_t n = (int64_t)p.N1 * nb;
        hipLaunchKernelGGL(k_fft_stepA<T>, dim3((unsigned)((n + bs - 1) / bs)), dim3(bs), 0, s,
                           p.N1, p.N2, twN_of<T>(p), x, ldx, nb, true);
    }
}

template void launch_circ_apply<double>(const FFTPlan &, const zd *, zd *, int64_t, int64_t,
                                        hipStream_t);
template void launch_circ_apply<float>(const FFTPlan &, const zf *, zf *, int64_t, int64_t,
                                       hipStream_t);

// natural-order DFT by direct summation (a handful of length-N vectors, once per assembly)
__global__ void k_dft_direct(int N, const zd *__restrict__ x, int64_t ldx, zd *y, int64_t ldy,
                             const zd *__restrict__ twN) {
    int m = blockIdx.x * blockDim.x + threadIdx.x;
    int c = blockIdx.y;
    if (m >= N) return;
    const zd *xc = x + (int64_t)c * ldx;
    zd acc = mk(0.0, 0.0);
    for (int p = 0; p < N; ++p) acc = acc + xc[p] * twN[((int64_t)m * p) % N];
    y[m + (int64_t)c * ldy] = acc;
}

void launch_dft_direct_tw(int N, const zd *x, int64_t ldx, zd *y, int64_t ldy, int ncol,
                          const zd *twN, hipStream_t s) {
    int bs = 256;
    hipLaunchKernelGGL(k_dft_direct, dim3((N + bs - 1) / bs, ncol), dim3(bs), 0, s, N, x, ldx, y,
                       ldy, twN);
}

}  // namespace cfie
