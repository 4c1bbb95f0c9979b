// Dense helper kernels of the factor and solve phases: Gram-matrix products (G is the
// circulant h [1/6, 2/3, 1/6], its inverse a banded circulant), elementwise updates,
// the Gaussian sketch generator, column norms, small Cholesky/triangular inverses for the
// orthonormalisation of sketch blocks, and the blocked LU with partial pivoting of the
// capacitance matrix I + V^T C_c^{-1} U (Sec. V eq. (9)).
#include "internal.h"

namespace cfie {

// ------------------------------------------------------------------ G and G^{-1} ---------
// out = a X + b G^{-1} Y ; G^{-1} has first column ginv[n]; taps u = 0..ntap-1 at offset
// t = t0 + u: (G^{-1} Y)_i = sum_u coef[u] Y_{(i - t) mod N}
template <typename T>
__global__ void k_ginv(int N, int ntap, int t0, const double *__restrict__ coef, cpx<T> a,
                       const cpx<T> *X, int64_t ldx, cpx<T> b, const cpx<T> *__restrict__ Y,
                       int64_t ldy, cpx<T> *out, int64_t ldo, int64_t ncol) {
    int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= (int64_t)N * ncol) return;
    int i = (int)(tid % N);
    int64_t c = tid / N;
    const cpx<T> *y = Y + c * ldy;
    T sr = 0, si = 0;
    for (int u = 0; u < ntap; ++u) {
        int idx = i - (t0 + u);
        idx %= N;
        if (idx < 0) idx += N;
        cpx<T> v = y[idx];
        T w = (T)coef[u];
        sr += w * v.x;
        si += w * v.y;
    }
    cpx<T> r = b * mk(sr, si);
    if (X) r = r + a * X[i + c * ldx];
    out[i + c * ldo] = r;
}

// The same for the 61-tap band (N >= 61).  A workgroup takes 2048 consecutive rows of one
// column: the 2048 + 60 inputs they need enter LDS by coalesced loads (wrapping around the
// column), each thread forms 8 consecutive outputs from its window of 68 inputs (read once
// from LDS, one pad word per 8 so that the stride-8 windows of a wavefront hit distinct
// banks), and the outputs return through LDS so that the stores are coalesced too.  The taps
// of every output are summed in the same order as above.
constexpr int kGinvTaps = 61;
constexpr int kGinvSeg = 2048;
__device__ __forceinline__ int pad8(int e) { return e + (e >> 3); }

template <typename T>
__global__ __launch_bounds__(256) void k_ginv_seg(int N, int t0, const double *__restrict__ coef,
                                                  cpx<T> a, const cpx<T> *X, int64_t ldx,
                                                  cpx<T> b, const cpx<T> *__restrict__ Y,
                                                  int64_t ldy, cpx<T> *out, int64_t ldo) {
    constexpr int R = 8;
    constexpr int W = kGinvSeg + kGinvTaps - 1;
    constexpr int PW = W + W / 8 + 1;
    __shared__ T sre[PW], sim[PW];
    const int t = threadIdx.x;
    const int nseg = (N + kGinvSeg - 1) / kGinvSeg;
    const int i0 = (int)(blockIdx.x % nseg) * kGinvSeg;
    const int64_t c = blockIdx.x / nseg;
    const cpx<T> *y = Y + c * ldy;
    // window element e holds y[(i0 - t0 - (taps - 1) + e) mod N]
    const int first = i0 - t0 - (kGinvTaps - 1);
    for (int e = t; e < W; e += 256) {
        int idx = (first + e) % N;
        if (idx < 0) idx += N;
        const cpx<T> v = y[idx];
        sre[pad8(e)] = v.x;
        sim[pad8(e)] = v.y;
    }
    __syncthreads();
    // outputs o = 8 t + r use window elements 8 t + m, m = 0..67, with tap u = 60 + r - m;
    // m runs downwards so that each output takes its taps in increasing u
    T ar[R], ai[R];
#pragma unroll
    for (int r = 0; r < R; ++r) ar[r] = ai[r] = (T)0;
#pragma unroll
    for (int m = R + kGinvTaps - 2; m >= 0; --m) {
        const int p = 9 * t + m + (m >> 3);
        const T vr = sre[p], vi = sim[p];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int u = kGinvTaps - 1 + r - m;
            if (u >= 0 && u < kGinvTaps) {
                const T w = (T)coef[u];
                ar[r] += w * vr;
                ai[r] += w * vi;
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < R; ++r) {
        sre[pad8(R * t + r)] = ar[r];
        sim[pad8(R * t + r)] = ai[r];
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < R; ++q) {
        const int o = t + 256 * q;
        const int i = i0 + o;
        if (i < N) {
            cpx<T> res = b * mk(sre[pad8(o)], sim[pad8(o)]);
            if (X) res = res + a * X[i + c * ldx];
            out[i + c * ldo] = res;
        }
    }
}

// out = a X + b G Y, G = h circ(2/3; 1/6, 1/6)
template <typename T>
__global__ void k_gmul(int N, double h, cpx<T> a, const cpx<T> *X, int64_t ldx, cpx<T> b,
                       const cpx<T> *__restrict__ Y, int64_t ldy, cpx<T> *out, int64_t ldo,
                       int64_t ncol) {
    int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= (int64_t)N * ncol) return;
    int i = (int)(tid % N);
    int64_t c = tid / N;
    const cpx<T> *y = Y + c * ldy;
    int im = i == 0 ? N - 1 : i - 1, ip = i == N - 1 ? 0 : i + 1;
    T c0 = (T)(2.0 * h / 3.0), c1 = (T)(h / 6.0);
    cpx<T> g = y[i] * c0 + (y[im] + y[ip]) * c1;
    cpx<T> r = b * g;
    if (X) r = r + a * X[i + c * ldx];
    out[i + c * ldo] = r;
}

void ginv_taps(int N, double h, std::vector<double> &coef, int &t0) {
    // first column of G^{-1}: (6/h) (rho^n + rho^(N-n)) / (2 sqrt 3 (1 - rho^N)), rho = sqrt3-2
    const double rho = std::sqrt(3.0) - 2.0;
    auto g = [&](int n) {
        n = ((n % N) + N) % N;
        double rn = std::pow(rho, n), rNn = std::pow(rho, N - n), rN = std::pow(rho, N);
        return (6.0 / h) * (rn + rNn) / (2.0 * std::sqrt(3.0) * (1.0 - rN));
    };
    coef.clear();
    if (N >= 61) {
        t0 = -30;
        for (int t = -30; t <= 30; ++t) coef.push_back(g(t));
    } else {
        t0 = 0;
        for (int t = 0; t < N; ++t) coef.push_back(g(t));
    }
}

template <typename T>
void launch_ginv_ex(int N, int ntap, int t0, const double *coef, cpx<T> a, const cpx<T> *X,
                    int64_t ldx, cpx<T> b, const cpx<T> *Y, int64_t ldy, cpx<T> *out,
                    int64_t ldo, int64_t ncol, hipStream_t s) {
    int64_t n = (int64_t)N * ncol;
    if (n <= 0) return;
    if (ntap == kGinvTaps) {
        const int64_t nwg = (int64_t)((N + kGinvSeg - 1) / kGinvSeg) * ncol;
        hipLaunchKernelGGL(k_ginv_seg<T>, dim3((unsigned)nwg), dim3(256), 0, s, N, t0, coef, a,
                           X, ldx, b, Y, ldy, out, ldo);
        return;
    }
    hipLaunchKernelGGL(k_ginv<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, N, ntap,
                       t0, coef, a, X, ldx, b, Y, ldy, out, ldo, ncol);
}
template <typename T>
void launch_gmul(int N, double h, cpx<T> a, const cpx<T> *X, int64_t ldx, cpx<T> b,
                 const cpx<T> *Y, int64_t ldy, cpx<T> *out, int64_t ldo, int64_t ncol,
                 hipStream_t s) {
    int64_t n = (int64_t)N * ncol;
    if (n <= 0) return;
    hipLaunchKernelGGL(k_gmul<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, N, h, a,
                       X, ldx, b, Y, ldy, out, ldo, ncol);
}
template void launch_ginv_ex<double>(int, int, int, const double *, zd, const zd *, int64_t, zd,
                                     const zd *, int64_t, zd *, int64_t, int64_t, hipStream_t);
template void launch_ginv_ex<float>(int, int, int, const double *, zf, const zf *, int64_t, zf,
                                    const zf *, int64_t, zf *, int64_t, int64_t, hipStream_t);
template void launch_gmul<double>(int, double, zd, const zd *, int64_t, zd, const zd *, int64_t,
                                  zd *, int64_t, int64_t, hipStream_t);
template void launch_gmul<float>(int, double, zf, const zf *, int64_t, zf, const zf *, int64_t,
                                 zf *, int64_t, int64_t, hipStream_t);

// ------------------------------------------------------------------ elementwise ----------
// A = a I (set) or A += a I (add), n x n
template <typename T>
__global__ void k_diag(int64_t n, cpx<T> a, int set, cpx<T> *A, int64_t lda) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (set) {
        if (t >= n * n) return;
        const int64_t i = t % n, j = t / n;
        A[i + j * lda] = i == j ? a : mk((T)0, (T)0);
    } else {
        if (t >= n) return;
        A[t + t * lda] = A[t + t * lda] + a;
    }
}
template <typename T>
void launch_diag(int64_t n, cpx<T> a, bool set, cpx<T> *A, int64_t lda, hipStream_t s) {
    const int64_t cnt = set ? n * n : n;
    if (cnt <= 0) return;
    hipLaunchKernelGGL(k_diag<T>, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, n, a,
                       set ? 1 : 0, A, lda);
}
template void launch_diag<double>(int64_t, zd, bool, zd *, int64_t, hipStream_t);
template void launch_diag<float>(int64_t, zf, bool, zf *, int64_t, hipStream_t);

// Y = a X + b Y   (m rows, n cols)
template <typename T>
__global__ void k_axpby(int64_t m, int64_t n, cpx<T> a, const cpx<T> *X, int64_t ldx, cpx<T> b,
                        cpx<T> *Y, int64_t ldy) {
    int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= m * n) return;
    int64_t i = tid % m, c = tid / m;
    cpx<T> y = (b.x == (T)0 && b.y == (T)0) ? mk((T)0, (T)0) : b * Y[i + c * ldy];
    Y[i + c * ldy] = y + a * X[i + c * ldx];
}
template <typename T>
void axpby(int64_t m, int64_t n, cpx<T> a, const cpx<T> *X, int64_t ldx, cpx<T> b, cpx<T> *Y,
           int64_t ldy, hipStream_t s) {
    int64_t t = m * n;
    if (t <= 0) return;
    hipLaunchKernelGGL(k_axpby<T>, dim3((unsigned)((t + 255) / 256)), dim3(256), 0, s, m, n, a, X,
                       ldx, b, Y, ldy);
}
template void axpby<double>(int64_t, int64_t, zd, const zd *, int64_t, zd, zd *, int64_t,
                            hipStream_t);
template void axpby<float>(int64_t, int64_t, zf, const zf *, int64_t, zf, zf *, int64_t,
                           hipStream_t);

template <typename TO, typename TI>
__global__ void k_convert(int64_t m, int64_t n, const cpx<TI> *X, int64_t ldx, cpx<TO> *Y,
                          int64_t ldy) {
    int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= m * n) return;
    int64_t i = tid % m, c = tid / m;
    cpx<TI> v = X[i + c * ldx];
    Y[i + c * ldy] = mk((TO)v.x, (TO)v.y);
}
template <typename TO, typename TI>
void convert(int64_t m, int64_t n, const cpx<TI> *X, int64_t ldx, cpx<TO> *Y, int64_t ldy,
             hipStream_t s) {
    int64_t t = m * n;
    if (t <= 0) return;
    hipLaunchKernelGGL((k_convert<TO, TI>), dim3((unsigned)((t + 255) / 256)), dim3(256), 0, s, m,
                       n, X, ldx, Y, ldy);
}
template void convert<float, double>(int64_t, int64_t, const zd *, int64_t, zf *, int64_t,
                                     hipStream_t);
template void convert<double, float>(int64_t, int64_t, const zf *, int64_t, zd *, int64_t,
                                     hipStream_t);
template void convert<double, double>(int64_t, int64_t, const zd *, int64_t, zd *, int64_t,
                                      hipStream_t);
template void convert<float, float>(int64_t, int64_t, const zf *, int64_t, zf *, int64_t,
                                    hipStream_t);

// Y (n x m) = X^H (CONJ) or X^T (X is m x n)
template <typename T, bool CONJ>
__global__ void k_conj_transpose(int64_t m, int64_t n, const cpx<T> *X, int64_t ldx, cpx<T> *Y,
                                 int64_t ldy) {
    __shared__ cpx<T> tile[32][33];
    int64_t bx = (int64_t)blockIdx.x * 32, by = (int64_t)blockIdx.y * 32;
    int tx = threadIdx.x, ty = threadIdx.y;
    for (int r = ty; r < 32; r += 8) {
        int64_t i = bx + tx, j = by + r;
        if (i < m && j < n) tile[r][tx] = X[i + j * ldx];
    }
    __syncthreads();
    for (int r = ty; r < 32; r += 8) {
        int64_t i = by + tx, j = bx + r;         // Y(i, j) = conj X(j, i)
        if (i < n && j < m) Y[i + j * ldy] = CONJ ? conj(tile[tx][r]) : tile[tx][r];
    }
}
template <typename T>
void conj_transpose(bool conj_, int64_t m, int64_t n, const cpx<T> *X, int64_t ldx, cpx<T> *Y,
                    int64_t ldy, hipStream_t s) {
    if (m <= 0 || n <= 0) return;
    dim3 grid((unsigned)((m + 31) / 32), (unsigned)((n + 31) / 32));
    if (conj_)
        hipLaunchKernelGGL((k_conj_transpose<T, true>), grid, dim3(32, 8), 0, s, m, n, X, ldx, Y, ldy);
    else
        hipLaunchKernelGGL((k_conj_transpose<T, false>), grid, dim3(32, 8), 0, s, m, n, X, ldx, Y, ldy);
}
template void conj_transpose<double>(bool, int64_t, int64_t, const zd *, int64_t, zd *, int64_t,
                                     hipStream_t);
template void conj_transpose<float>(bool, int64_t, int64_t, const zf *, int64_t, zf *, int64_t,
                                    hipStream_t);

// ------------------------------------------------------------------ Gaussian sketch ------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): counter = (element index lo/hi,
// stream, 0), key = seed.  Its four 32-bit outputs make one pair of 53-bit uniforms ->
// Box-Muller -> one real standard normal per element.  The test matrix of the sketch is
// real: the range of a complex matrix is sampled as well by real Gaussian columns, and the
// products with the assembled complex matrices then need two real products instead of the
// three of the 3M form (GEMM_NREAL).
__device__ __forceinline__ void philox_round(uint32_t &c0, uint32_t &c1, uint32_t &c2,
                                             uint32_t &c3, uint32_t k0, uint32_t k1) {
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    uint32_t hi0 = __umulhi(M0, c0), lo0 = M0 * c0;
    uint32_t hi1 = __umulhi(M1, c2), lo1 = M1 * c2;
    uint32_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
}
__device__ __forceinline__ void philox4x32_10(uint32_t ctr[4], uint32_t k0, uint32_t k1) {
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        philox_round(ctr[0], ctr[1], ctr[2], ctr[3], k0, k1);
        k0 += W0;
        k1 += W1;
    }
}
template <typename T>
__global__ void k_randn(int64_t m, int64_t n, uint64_t seed, uint64_t stream, cpx<T> *X,
                        int64_t ldx) {
    int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= m * n) return;
    int64_t i = tid % m, c = tid / m;
    uint32_t ctr[4] = {(uint32_t)tid, (uint32_t)(tid >> 32), (uint32_t)stream,
                       (uint32_t)(stream >> 32)};
    philox4x32_10(ctr, (uint32_t)seed, (uint32_t)(seed >> 32));
    // 53-bit uniforms in (0, 1]
    double u1 = ((double)(((uint64_t)ctr[0] << 21) ^ (ctr[1] >> 11)) + 1.0) * (1.0 / 9007199254740993.0);
    double u2 = ((double)(((uint64_t)ctr[2] << 21) ^ (ctr[3] >> 11)) + 0.5) * (1.0 / 9007199254740992.0);
    double r = sqrt(-2.0 * log(u1));
    X[i + c * ldx] = mk((T)(r * cospi(2.0 * u2)), (T)0);
}
template <typename T>
void randn(int64_t m, int64_t n, uint64_t seed, uint64_t stream, cpx<T> *X, int64_t ldx,
           hipStream_t s) {
    int64_t t = m * n;
    if (t <= 0) return;
    hipLaunchKernelGGL(k_randn<T>, dim3((unsigned)((t + 255) / 256)), dim3(256), 0, s, m, n, seed,
                       stream, X, ldx);
}
template void randn<double>(int64_t, int64_t, uint64_t, uint64_t, zd *, int64_t, hipStream_t);
template void randn<float>(int64_t, int64_t, uint64_t, uint64_t, zf *, int64_t, hipStream_t);

// Unit-modulus entries of uniform random phase (the diagonal D of the SRFT test matrix):
// one 53-bit uniform u per entry from the same Philox stream layout, d = e^{2 pi i u}.
template <typename T>
__global__ void k_steinhaus(int64_t n, uint64_t seed, uint64_t stream, cpx<T> *d) {
    const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (tid >= n) return;
    uint32_t ctr[4] = {(uint32_t)tid, (uint32_t)(tid >> 32), (uint32_t)stream,
                       (uint32_t)(stream >> 32)};
    philox4x32_10(ctr, (uint32_t)seed, (uint32_t)(seed >> 32));
    const double u = (double)(((uint64_t)ctr[0] << 21) ^ (ctr[1] >> 11)) *
                     (1.0 / 9007199254740992.0);
    double sn, cs;
    sincospi(2.0 * u, &sn, &cs);
    d[tid] = mk((T)cs, (T)sn);
}
template <typename T>
void launch_steinhaus(int64_t n, uint64_t seed, uint64_t stream, cpx<T> *d, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_steinhaus<T>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n,
                       seed, stream, d);
}
template void launch_steinhaus<double>(int64_t, uint64_t, uint64_t, zd *, hipStream_t);
template void launch_steinhaus<float>(int64_t, uint64_t, uint64_t, zf *, hipStream_t);

// ------------------------------------------------------------------ column norms ---------
// out[c] = sum_i |X_ic|^2 (double), one block per column
template <typename T>
__global__ void k_colnorm2(int64_t m, const cpx<T> *X, int64_t ldx, double *out) {
    __shared__ double red[256];
    int64_t c = blockIdx.x;
    const cpx<T> *x = X + c * ldx;
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < m; i += blockDim.x) {
        cpx<T> v = x[i];
        s += (double)v.x * v.x + (double)v.y * v.y;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[c] = red[0];
}
template <typename T>
void colnorm2(int64_t m, int64_t n, const cpx<T> *X, int64_t ldx, double *out, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_colnorm2<T>, dim3((unsigned)n), dim3(256), 0, s, m, X, ldx, out);
}
template void colnorm2<double>(int64_t, int64_t, const zd *, int64_t, double *, hipStream_t);
template void colnorm2<float>(int64_t, int64_t, const zf *, int64_t, double *, hipStream_t);

// ------------------------------------------------------------------ circulant eigenvalues
// mu: 4 natural-order DFT vectors (Dk, Nk, Dkt, Skt rows of the circle); G has eigenvalue
// h (2 + cos(2 pi m / N)) / 3.  c_m = (g/2 + dt)(g/2 - d)/g + s n / g  (Sec. V eq. (6)).
// Writes c (natural) and the diagonals for the FFT layout: dC = c/N, dCH = conj(c)/N,
// dCinv = 1/(N c), in double and float.
__global__ void k_circ_eigs(int N, int N1, int N2, double h, const zd *__restrict__ mu,
                            zd *c, zd *dC, zd *dCH, zd *dCinv, zd *dCinvH, zf *fC, zf *fCH,
                            zf *fCinv, zf *fCinvH, double *absc) {
    int m = blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= N) return;
    zd md = mu[m], mn = mu[m + N], mdt = mu[m + 2 * N], ms = mu[m + 3 * N];
    double g = h * (2.0 + cospi(2.0 * m / (double)N)) / 3.0;
    zd hg = mk(0.5 * g, 0.0);
    zd cm = (hg + mdt) * (hg - md) * (1.0 / g) + ms * mn * (1.0 / g);
    c[m] = cm;
    absc[m] = cabs(cm);
    // position in the transposed layout of the four-step FFT: m = k2 + N2 k1 -> k1 + N1 k2
    int k2 = m % N2, k1 = m / N2;
    int p = k1 + N1 * k2;
    double invN = 1.0 / N;
    zd a = cm * invN, b = conj(cm) * invN, ci = cinv(cm) * invN;
    const zd cih = conj(ci);
    dC[p] = a;
    dCH[p] = b;
    dCinv[p] = ci;
    dCinvH[p] = cih;
    fC[p] = mk((float)a.x, (float)a.y);
    fCH[p] = mk((float)b.x, (float)b.y);
    fCinv[p] = mk((float)ci.x, (float)ci.y);
    fCinvH[p] = mk((float)cih.x, (float)cih.y);
}
void launch_circ_eigs(int N, int N1, int N2, double h, const zd *mu, zd *c, zd *dC, zd *dCH,
                      zd *dCinv, zd *dCinvH, zf *fC, zf *fCH, zf *fCinv, zf *fCinvH,
                      double *absc, hipStream_t s) {
    hipLaunchKernelGGL(k_circ_eigs, dim3((N + 255) / 256), dim3(256), 0, s, N, N1, N2, h, mu, c,
                       dC, dCH, dCinv, dCinvH, fC, fCH, fCinv, fCinvH, absc);
}

// max over n doubles (single block)
__global__ void k_maxmin(int64_t n, const double *x, double *out) {
    __shared__ double mx[256], mn[256];
    double a = -1e308, b = 1e308;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        a = fmax(a, x[i]);
        b = fmin(b, x[i]);
    }
    mx[threadIdx.x] = a;
    mn[threadIdx.x] = b;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            mx[threadIdx.x] = fmax(mx[threadIdx.x], mx[threadIdx.x + w]);
            mn[threadIdx.x] = fmin(mn[threadIdx.x], mn[threadIdx.x + w]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        out[0] = mx[0];
        out[1] = mn[0];
    }
}
void launch_maxmin(int64_t n, const double *x, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_maxmin, dim3(1), dim3(256), 0, s, n, x, out);
}

// ------------------------------------------------------------------ small dense ----------
// Hermitian positive definite W (b x b, in place, lower part used) -> upper Cholesky
// factor R with W = R^H R, then Rinv = R^{-1} (upper).  One workgroup.  A shift s is added
// to the diagonal first (shifted Cholesky QR).  info[0] = 1 on a non-positive pivot.
__global__ void k_chol_inv(int b, zd *W, int ldw, double shift, zd *Rinv, int ldr, int *info) {
    const int tid = threadIdx.x, nt = blockDim.x;
    for (int i = tid; i < b; i += nt) W[i + i * ldw].x += shift;
    __syncthreads();
    // right-looking Cholesky on the upper triangle: R(j, j:) row by row
    __shared__ double piv;
    for (int j = 0; j < b; ++j) {
        if (tid == 0) {
            double d = W[j + j * ldw].x;
            if (!(d > 0.0)) { info[0] = 1; d = 1e-300; }
            piv = sqrt(d);
        }
        __syncthreads();
        double p = piv;
        // row j of R: R(j, c) = W(j, c) / p for c > j ; R(j, j) = p
        for (int c = j + tid; c < b; c += nt) {
            zd v = W[j + c * ldw];
            W[j + c * ldw] = (c == j) ? mk(p, 0.0) : v * (1.0 / p);
        }
        __syncthreads();
        // trailing update: W(r, c) -= conj(R(j, r)) R(j, c) for j < r <= c
        int rem = b - j - 1;
        for (int64_t t = tid; t < (int64_t)rem * rem; t += nt) {
            int r = j + 1 + (int)(t % rem), c = j + 1 + (int)(t / rem);
            if (r <= c) W[r + c * ldw] = W[r + c * ldw] - conj(W[j + r * ldw]) * W[j + c * ldw];
        }
        __syncthreads();
    }
    // Rinv by back substitution, one column per thread: R X = I, X upper
    for (int c = tid; c < b; c += nt) {
        for (int r = b - 1; r >= 0; --r) {
            zd s = mk(r == c ? 1.0 : 0.0, 0.0);
            if (r > c) { Rinv[r + c * ldr] = mk(0.0, 0.0); continue; }
            for (int q = r + 1; q <= c; ++q) s = s - W[r + q * ldw] * Rinv[q + c * ldr];
            Rinv[r + c * ldr] = s * cinv(W[r + r * ldw]);
        }
    }
}
void launch_chol_inv(int b, zd *W, int ldw, double shift, zd *Rinv, int ldr, int *info,
                     hipStream_t s) {
    hipLaunchKernelGGL(k_chol_inv, dim3(1), dim3(1024), 0, s, b, W, ldw, shift, Rinv, ldr, info);
}

// Rank-revealing orthonormaliser for a sketch block: pivoted Cholesky of the Gram matrix
// W = Y^H Y (b x b, Hermitian, full storage, overwritten).  Pivots are taken while the
// largest remaining Schur-complement diagonal (squared norm of what a column adds to the
// span of the columns already taken) exceeds max(thr_abs, thr_rel * max diag).  With k
// pivots kept and R the k x k factor of the permuted Gram, Z (b x b, ld ldz) receives
// Z[perm[r], c] = (R^{-1})[r, c] for r, c < k and zeros elsewhere, so that Y Z[:, :k] has
// orthonormal columns (up to rounding; two plain Cholesky passes follow).  *kout = k.
__global__ void k_pchol(int b, zd *W, int ldw, double thr_abs, double thr_rel, zd *Z, int ldz,
                        int *kout) {
    const int tid = threadIdx.x, nt = blockDim.x;
    __shared__ int perm[512];
    __shared__ double bestv[1024];
    __shared__ int besti[1024];
    __shared__ int kk;
    __shared__ double thr;
    for (int i = tid; i < b; i += nt) perm[i] = i;
    // threshold from the largest diagonal
    double mx = 0.0;
    for (int i = tid; i < b; i += nt) mx = fmax(mx, W[i + i * ldw].x);
    bestv[tid] = mx;
    __syncthreads();
    for (int w = nt / 2; w > 0; w >>= 1) {
        if (tid < w) bestv[tid] = fmax(bestv[tid], bestv[tid + w]);
        __syncthreads();
    }
    if (tid == 0) {
        thr = fmax(thr_abs, thr_rel * bestv[0]);
        kk = b;
    }
    __syncthreads();
    for (int j = 0; j < b; ++j) {
        double bv = -1.0;
        int bi = j;
        for (int i = j + tid; i < b; i += nt) {
            double v = W[i + i * ldw].x;
            if (v > bv) { bv = v; bi = i; }
        }
        bestv[tid] = bv;
        besti[tid] = bi;
        __syncthreads();
        for (int w = nt / 2; w > 0; w >>= 1) {
            if (tid < w && (bestv[tid + w] > bestv[tid] ||
                            (bestv[tid + w] == bestv[tid] && besti[tid + w] < besti[tid]))) {
                bestv[tid] = bestv[tid + w];
                besti[tid] = besti[tid + w];
            }
            __syncthreads();
        }
        int p = besti[0];
        bool stop = !(bestv[0] > thr);
        __syncthreads();
        if (stop) {
            if (tid == 0) kk = j;
            break;
        }
        if (p != j) {
            // symmetric swap of rows and columns j <-> p
            for (int i = tid; i < b; i += nt) {
                zd t = W[j + i * ldw];
                W[j + i * ldw] = W[p + i * ldw];
                W[p + i * ldw] = t;
            }
            __syncthreads();
            for (int i = tid; i < b; i += nt) {
                zd t = W[i + j * ldw];
                W[i + j * ldw] = W[i + p * ldw];
                W[i + p * ldw] = t;
            }
            if (tid == 0) {
                int t = perm[j];
                perm[j] = perm[p];
                perm[p] = t;
            }
            __syncthreads();
        }
        double r = sqrt(W[j + j * ldw].x);
        __syncthreads();
        for (int c = j + tid; c < b; c += nt)
            W[j + c * ldw] = (c == j) ? mk(r, 0.0) : W[j + c * ldw] * (1.0 / r);
        __syncthreads();
        int rem = b - j - 1;
        for (int64_t t = tid; t < (int64_t)rem * rem; t += nt) {
            int rr = j + 1 + (int)(t % rem), cc = j + 1 + (int)(t / rem);
            W[rr + cc * ldw] = W[rr + cc * ldw] - conj(W[j + rr * ldw]) * W[j + cc * ldw];
        }
        __syncthreads();
    }
    __syncthreads();
    const int k = kk;
    for (int64_t t = tid; t < (int64_t)b * b; t += nt) Z[(t % b) + (t / b) * ldz] = mk(0.0, 0.0);
    __syncthreads();
    // R^{-1} by back substitution (one column per thread), scattered to rows perm[r]
    for (int c = tid; c < k; c += nt) {
        // temporary column stored directly into Z at permuted rows
        for (int r = c; r >= 0; --r) {
            zd s = mk(r == c ? 1.0 : 0.0, 0.0);
            for (int q = r + 1; q <= c; ++q) s = s - W[r + q * ldw] * Z[perm[q] + c * ldz];
            Z[perm[r] + c * ldz] = s * (1.0 / W[r + r * ldw].x);
        }
    }
    if (tid == 0) kout[0] = k;
}
// Panel-blocked form of the same factorisation (b <= 512).  No rows or columns are moved:
// with p_j the j-th pivot (largest remaining Schur-complement diagonal d), the pivot row is
// r^(j)_c = (W_j[p_j, c]) / sqrt(d_p) where W_j is W minus the rank-one terms of the earlier
// pivots, and the columns of Z are built alongside by
// z_j = (e_p - sum_{i<j} z_i r^(i)_p) / sqrt(d_p) (Gram-Schmidt in the coefficients of Y), so
// that Y z_j is the j-th orthonormal direction.  Pivots come in panels of NB: a single
// wavefront finds the panel's pivots (no workgroup barriers on that sequential path; rows and
// z vectors of the panel in LDS), and a grid-wide kernel then applies the panel's rank-NB
// terms to W and to M = -sum z_i r^(i) (b x b).  The state between launches (d, taken, the
// pivot count, the stop flag) lives in a small device workspace, so no host round trip is
// needed between panels; panels after a stop return at once.
constexpr int kPcholNB = 16;
// pivots per panel: 16, or 8 above b = 256 (the panel's rows and z vectors stay in LDS)
__host__ __device__ inline int pchol_nb(int b) { return b <= 256 ? kPcholNB : kPcholNB / 2; }
struct PcholWs {
    zd *Rg, *Zg;            // the current panel's pivot rows and z vectors (NB x b each)
    double *d, *thr;        // remaining diagonal; threshold
    int *taken, *st;        // st[0] pivots so far, st[1] pivots of the last panel, st[2] stop
};
__host__ __device__ inline size_t pchol_ws_bytes(int b) {
    auto up = [](size_t x) { return (x + 255) / 256 * 256; };
    return up((size_t)2 * kPcholNB * b * sizeof(zd)) + up((size_t)(b + 1) * sizeof(double)) +
           up((size_t)(b + 4) * sizeof(int));
}
__host__ __device__ inline PcholWs pchol_ws(void *base, int b) {
    auto up = [](size_t x) { return (x + 255) / 256 * 256; };
    char *p = (char *)base;
    PcholWs w;
    w.Rg = (zd *)p;
    w.Zg = w.Rg + (size_t)kPcholNB * b;
    p += up((size_t)2 * kPcholNB * b * sizeof(zd));
    w.d = (double *)p;
    w.thr = w.d + b;
    p += up((size_t)(b + 1) * sizeof(double));
    w.taken = (int *)p;
    w.st = w.taken + b;
    return w;
}

// M = 0, d = diag(W), taken = 0, threshold from the largest diagonal, counters cleared
__global__ __launch_bounds__(1024) void k_pchol_init(int b, const zd *W, int ldw, double thr_abs,
                                                     double thr_rel, zd *M, void *wsb) {
    const int tid = threadIdx.x;
    PcholWs ws = pchol_ws(wsb, b);
    __shared__ double wv[16];
    for (int t = tid; t < b * b; t += 1024) M[t] = mk(0.0, 0.0);
    double mx = 0.0;
    if (tid < b) {
        ws.d[tid] = W[tid + (int64_t)tid * ldw].x;
        ws.taken[tid] = 0;
        mx = ws.d[tid];
    }
    for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o));
    if ((tid & 63) == 0) wv[tid >> 6] = mx;
    __syncthreads();
    if (tid == 0) {
        double m = 0.0;
        for (int w = 0; w < 16; ++w) m = fmax(m, wv[w]);
        ws.thr[0] = fmax(thr_abs, thr_rel * m);
        ws.st[0] = ws.st[1] = ws.st[2] = 0;
    }
}

// the next panel's pivots, one wavefront (lane l handles columns / rows l, l + 64, ...)
__global__ __launch_bounds__(64) void k_pchol_pivots(int b, const zd *W, int ldw, zd *Z, int ldz,
                                                     const zd *M, void *wsb) {
    constexpr int PER = 8;                       // b <= 512 = 64 x 8
    const int lane = threadIdx.x;
    PcholWs ws = pchol_ws(wsb, b);
    if (ws.st[2] || ws.st[0] >= b) {
        if (lane == 0) ws.st[1] = 0;
        return;
    }
    __shared__ zd Rp[kPcholNB * 256];            // Rp[i * b + c], NB b <= 4096
    __shared__ zd Zp[kPcholNB * 256];            // Zp[i * b + r]
    const int NB = pchol_nb(b);
    double dl[PER];
    int tk[PER];
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int c = lane + 64 * q;
        dl[q] = c < b ? ws.d[c] : -1.0;
        tk[q] = c < b ? ws.taken[c] : 1;
    }
    const double thr = ws.thr[0];
    int k = ws.st[0];
    int jp = 0;
    bool stop = false;
    for (; jp < NB && k < b; ++jp) {
        // pivot: largest untaken d (ties: smallest index)
        double bv = -1.0;
        int bi = 0x7fffffff;
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int c = lane + 64 * q;
            if (c < b && !tk[q] && (dl[q] > bv || (dl[q] == bv && c < bi))) {
                bv = dl[q];
                bi = c;
            }
        }
        for (int o = 32; o > 0; o >>= 1) {
            const double ov = __shfl_xor(bv, o);
            const int oi = __shfl_xor(bi, o);
            if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
        }
        if (!(bv > thr)) {
            stop = true;
            break;
        }
        const int p = bi;
        const double sd = sqrt(bv), isd = 1.0 / sd;
        // column p of W (at the panel start) and of M for every lane, all loads issued before
        // the stores to Z below (which the compiler could not otherwise move them past)
        zd wp[PER], mp[PER];
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int cc = lane + 64 * q;
            if (cc < b) {
                wp[q] = W[cc + (int64_t)p * ldw];
                mp[q] = M[cc + (int64_t)p * b];
            }
        }
        // the pivot's entries of the earlier rows of this panel (the same for every lane),
        // read once; the sums over them below need neither W nor M, so they run while the
        // loads of column p are in flight (unrolled over the panel width so that the lanes'
        // LDS reads are issued ahead of the complex multiply-adds)
        zd rpv[kPcholNB];
#pragma unroll
        for (int i = 0; i < kPcholNB; ++i) rpv[i] = i < jp ? Rp[i * b + p] : mk(0.0, 0.0);
        zd sr[PER], sz[PER];
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int cc = lane + 64 * q;
            sr[q] = sz[q] = mk(0.0, 0.0);
            if (cc >= b) continue;
#pragma unroll
            for (int i = 0; i < kPcholNB; ++i) {
                if (i < jp) {
                    sr[q] = sr[q] + conj(rpv[i]) * Rp[i * b + cc];
                    sz[q] = sz[q] + Zp[i * b + cc] * rpv[i];
                }
            }
        }
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int cc = lane + 64 * q;
            if (cc >= b) break;
            // pivot row from column p of W at the panel start: W[p, c] = conj(W[c, p])
            zd r = mk(0.0, 0.0);
            if (cc == p) {
                r = mk(sd, 0.0);
            } else if (!tk[q]) {
                r = (conj(wp[q]) - sr[q]) * isd;
            }
            zd z = mp[q];
            if (cc == p) z = z + mk(1.0, 0.0);
            z = z - sz[q];
            z = z * isd;
            Zp[jp * b + cc] = z;
            Z[cc + (int64_t)k * ldz] = z;
            Rp[jp * b + cc] = r;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int c = lane + 64 * q;
            if (c >= b) break;
            if (c == p) tk[q] = 1;
            else if (!tk[q]) dl[q] -= abs2(Rp[jp * b + c]);
        }
        ++k;
    }
    // hand the panel to the update kernel and the state to the next panel
    for (int t = lane; t < jp * b; t += 64) {
        ws.Rg[t] = Rp[t];
        ws.Zg[t] = Zp[t];
    }
#pragma unroll
    for (int q = 0; q < PER; ++q) {
        const int c = lane + 64 * q;
        if (c < b) {
            ws.d[c] = dl[q];
            ws.taken[c] = tk[q];
        }
    }
    if (lane == 0) {
        ws.st[0] = k;
        ws.st[1] = jp;
        ws.st[2] = stop ? 1 : 0;
    }
}

// The same panel for b <= 256 by one workgroup of 256 threads, thread c owning column and row
// c: the same arithmetic in the same order per column as k_pchol_pivots (so the same pivots
// and values), with the sums of a column in one thread instead of four per lane.  The pivot
// search combines the four wavefronts' candidates through LDS slots that alternate between
// two sets (a set is rewritten two pivots later, after another barrier), so one barrier per
// pivot orders both the search and the panel rows read by the next pivot.
__global__ __launch_bounds__(256) void k_pchol_pivots_wg(int b, const zd *W, int ldw, zd *Z,
                                                         int ldz, const zd *M, void *wsb) {
    const int c = threadIdx.x, lane = c & 63, wv = c >> 6;
    PcholWs ws = pchol_ws(wsb, b);
    if (ws.st[2] || ws.st[0] >= b) {
        if (c == 0) ws.st[1] = 0;
        return;
    }
    __shared__ zd Rp[kPcholNB * 256];            // Rp[i * b + c]
    __shared__ zd Zp[kPcholNB * 256];            // Zp[i * b + r]
    __shared__ double slot_v[2][4];
    __shared__ int slot_i[2][4];
    const bool own = c < b;
    double dl = own ? ws.d[c] : -1.0;
    int tk = own ? ws.taken[c] : 1;
    const double thr = ws.thr[0];
    int k = ws.st[0];
    int jp = 0;
    bool stop = false;
    for (; jp < kPcholNB && k < b; ++jp) {
        // pivot: largest untaken d (ties: smallest index)
        double bv = -1.0;
        int bi = 0x7fffffff;
        if (own && !tk && dl >= bv) {
            bv = dl;
            bi = c;
        }
        for (int o = 32; o > 0; o >>= 1) {
            const double ov = __shfl_xor(bv, o);
            const int oi = __shfl_xor(bi, o);
            if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
        }
        const int par = jp & 1;
        if (lane == 0) {
            slot_v[par][wv] = bv;
            slot_i[par][wv] = bi;
        }
        __syncthreads();
        bv = slot_v[par][0];
        bi = slot_i[par][0];
#pragma unroll
        for (int x = 1; x < 4; ++x) {
            const double ov = slot_v[par][x];
            const int oi = slot_i[par][x];
            if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
        }
        if (!(bv > thr)) {
            stop = true;
            break;
        }
        const int p = bi;
        const double sd = sqrt(bv), isd = 1.0 / sd;
        zd wp = mk(0.0, 0.0), mp = mk(0.0, 0.0);
        if (own) {
            wp = W[c + (int64_t)p * ldw];
            mp = M[c + (int64_t)p * b];
        }
        // sums over the earlier rows of this panel (written before the barrier above)
        zd sr = mk(0.0, 0.0), sz = mk(0.0, 0.0);
#pragma unroll
        for (int i = 0; i < kPcholNB; ++i) {
            if (i < jp) {
                const zd rpv = Rp[i * b + p];
                if (own) {
                    sr = sr + conj(rpv) * Rp[i * b + c];
                    sz = sz + Zp[i * b + c] * rpv;
                }
            }
        }
        if (own) {
            // pivot row from column p of W at the panel start: W[p, c] = conj(W[c, p])
            zd r = mk(0.0, 0.0);
            if (c == p) {
                r = mk(sd, 0.0);
            } else if (!tk) {
                r = (conj(wp) - sr) * isd;
            }
            zd z = mp;
            if (c == p) z = z + mk(1.0, 0.0);
            z = z - sz;
            z = z * isd;
            Zp[jp * b + c] = z;
            Z[c + (int64_t)k * ldz] = z;
            Rp[jp * b + c] = r;
            if (c == p) tk = 1;
            else if (!tk) dl -= abs2(r);
        }
        ++k;
    }
    // hand the panel to the update kernel (each thread its own column) and the state to the
    // next panel
    if (own) {
        for (int i = 0; i < jp; ++i) {
            ws.Rg[i * b + c] = Rp[i * b + c];
            ws.Zg[i * b + c] = Zp[i * b + c];
        }
        ws.d[c] = dl;
        ws.taken[c] = tk;
    }
    if (c == 0) {
        ws.st[0] = k;
        ws.st[1] = jp;
        ws.st[2] = stop ? 1 : 0;
    }
}

// W -= Rp^H Rp and M -= Zp Rp over the whole b x b for the panel just found (nothing after
// the last panel: no pivots follow)
__global__ void k_pchol_update(int b, zd *W, int ldw, zd *M, const void *wsb) {
    const PcholWs ws = pchol_ws((void *)wsb, b);
    const int np = ws.st[1];
    if (np == 0 || ws.st[2] || ws.st[0] >= b) return;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= (int64_t)b * b) return;
    const int rr = (int)(t % b), cc = (int)(t / b);
    zd w = W[rr + (int64_t)cc * ldw], m = M[t];
    for (int i = 0; i < np; ++i) {
        const zd rc = ws.Rg[i * b + cc];
        w = w - conj(ws.Rg[i * b + rr]) * rc;
        m = m - ws.Zg[i * b + rr] * rc;
    }
    W[rr + (int64_t)cc * ldw] = w;
    M[t] = m;
}

// unused columns of Z are zero; kout = the number of pivots
__global__ void k_pchol_finish(int b, zd *Z, int ldz, const void *wsb, int *kout) {
    const PcholWs ws = pchol_ws((void *)wsb, b);
    const int k = ws.st[0];
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < (int64_t)b * (b - k)) Z[(t % b) + (int64_t)(k + t / b) * ldz] = mk(0.0, 0.0);
    if (t == 0) kout[0] = k;
}

size_t pchol_workspace_elems(int b) {
    return (size_t)b * b + (pchol_ws_bytes(b) + sizeof(zd) - 1) / sizeof(zd);
}

void launch_pchol(int b, zd *W, int ldw, double thr_abs, double thr_rel, zd *Z, int ldz, zd *M,
                  int *kout, hipStream_t s) {
    if (b <= 512 && M) {
        void *ws = M + (size_t)b * b;
        hipLaunchKernelGGL(k_pchol_init, dim3(1), dim3(1024), 0, s, b, (const zd *)W, ldw,
                           thr_abs, thr_rel, M, ws);
        const int npanel = (b + pchol_nb(b) - 1) / pchol_nb(b);
        const unsigned ub = (unsigned)(((int64_t)b * b + 255) / 256);
        for (int pnl = 0; pnl < npanel; ++pnl) {
            if (b <= 256)
                hipLaunchKernelGGL(k_pchol_pivots_wg, dim3(1), dim3(256), 0, s, b, (const zd *)W,
                                   ldw, Z, ldz, (const zd *)M, ws);
            else
                hipLaunchKernelGGL(k_pchol_pivots, dim3(1), dim3(64), 0, s, b, (const zd *)W,
                                   ldw, Z, ldz, (const zd *)M, ws);
            hipLaunchKernelGGL(k_pchol_update, dim3(ub), dim3(256), 0, s, b, W, ldw, M,
                               (const void *)ws);
        }
        const unsigned fb = (unsigned)(((int64_t)b * b + 255) / 256);
        hipLaunchKernelGGL(k_pchol_finish, dim3(fb), dim3(256), 0, s, b, Z, ldz,
                           (const void *)ws, kout);
    } else {
        hipLaunchKernelGGL(k_pchol, dim3(1), dim3(1024), 0, s, b, W, ldw, thr_abs, thr_rel, Z,
                           ldz, kout);
    }
}

// M = (3 I - G) / 2 in precision T (one Newton-Schulz step towards the polar factor)
template <typename T>
__global__ void k_polar_coef(int k, const zd *G, int ldg, cpx<T> *M, int ldm) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= k * k) return;
    int i = t % k, j = t / k;
    zd g = G[i + (int64_t)j * ldg];
    zd v = mk((i == j ? 1.5 : 0.0) - 0.5 * g.x, -0.5 * g.y);
    M[i + (int64_t)j * ldm] = mk((T)v.x, (T)v.y);
}
template <typename T>
void launch_polar_coef(int k, const zd *G, int ldg, cpx<T> *M, int ldm, hipStream_t s) {
    hipLaunchKernelGGL(k_polar_coef<T>, dim3((k * k + 255) / 256), dim3(256), 0, s, k, G, ldg, M, ldm);
}
template void launch_polar_coef<double>(int, const zd *, int, zd *, int, hipStream_t);
template void launch_polar_coef<float>(int, const zd *, int, zf *, int, hipStream_t);

// ---- LU with partial pivoting: panel of columns [k0, k0 + nb) of the n x n matrix A
// (rows k0..n-1), one workgroup of 1024 threads; piv[j] = global row swapped with row j.
// Pivot search by wavefront shuffles and one exchange through LDS (ties: smallest row).
__global__ __launch_bounds__(1024) void k_lu_panel(int n, int k0, int nb, zd *A, int64_t lda,
                                                   int *piv, int *info) {
    // nb <= 16 columns, rows k0 .. n-1, one workgroup.  Per column j: argmax of |a|^2 over
    // rows >= j (ties: smallest row), exchange of rows j and p inside the panel with the new
    // row j kept in LDS, then one pass over the rows below j that scales column j and
    // applies the rank-one update to the panel's later columns (all loads of a row issued
    // together) while it finds the largest entry of column j + 1 for the next step.
    const int tid = threadIdx.x;
    __shared__ double wv[16];
    __shared__ int wi[16];
    __shared__ zd rowj[16];
    double bv = -1.0;
    int bi = 0x7fffffff;
    for (int r = k0 + tid; r < n; r += 1024) {
        const double v = abs2(A[r + (int64_t)k0 * lda]);
        if (v > bv) { bv = v; bi = r; }
    }
    for (int jj = 0; jj < nb; ++jj) {
        const int j = k0 + jj;
        for (int o = 32; o > 0; o >>= 1) {
            const double ov = __shfl_xor(bv, o);
            const int oi = __shfl_xor(bi, o);
            if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
        }
        if ((tid & 63) == 0) { wv[tid >> 6] = bv; wi[tid >> 6] = bi; }
        __syncthreads();
        bv = wv[0];
        bi = wi[0];
        for (int w = 1; w < 16; ++w)
            if (wv[w] > bv || (wv[w] == bv && wi[w] < bi)) { bv = wv[w]; bi = wi[w]; }
        const int p = bi < n ? bi : j;
        if (tid == 0) {
            piv[j] = p;
            if (!(bv > 0.0)) info[0] = 1;
        }
        if (tid < nb) {
            const int64_t c = (int64_t)(k0 + tid) * lda;
            const zd aj = A[j + c], ap = A[p + c];
            if (p != j) {
                A[j + c] = ap;
                A[p + c] = aj;
            }
            rowj[tid] = p != j ? ap : aj;
        }
        __syncthreads();
        const zd d = rowj[jj];
        const zd dinv = (abs2(d) > 0.0) ? cinv(d) : mk(0.0, 0.0);
        bv = -1.0;
        bi = 0x7fffffff;
        for (int r = j + 1 + tid; r < n; r += 1024) {
            const zd l = A[r + (int64_t)j * lda] * dinv;
            A[r + (int64_t)j * lda] = l;
#pragma unroll
            for (int cc = 1; cc < 16; ++cc) {
                if (cc > jj && cc < nb) {
                    zd *ac = A + r + (int64_t)(k0 + cc) * lda;
                    const zd v = *ac - l * rowj[cc];
                    *ac = v;
                    if (cc == jj + 1) {
                        const double m2 = abs2(v);
                        if (m2 > bv) { bv = m2; bi = r; }
                    }
                }
            }
        }
        __syncthreads();
    }
}
// The same panel factorisation with the panel held in registers (row r of the panel,
// r = k0 + tid + 1024 q, in thread tid, q < RPT; panels of up to NBMAX columns, n - k0 <=
// 1024 RPT; RPT NBMAX <= 16 keeps it within the 128 registers of a 1024-thread workgroup):
// the panel is read and written once instead of once per column.  Used for the last
// panels of an LU (at most 1024 rows left).  Per column: argmax
// of |a|^2 over the rows (ties: smallest row), exchange of rows j and p through LDS, the
// pivot row broadcast through LDS, and the scaling and rank-one update in registers, in the
// same arithmetic order as k_lu_panel.
template <int RPT, int NBMAX>
__global__ __launch_bounds__(1024) void k_lu_panel_reg(int n, int k0, int nb, zd *A, int64_t lda,
                                                       int *piv, int *info) {
    const int tid = threadIdx.x;
    __shared__ double wv[16];
    __shared__ int wi[16];
    __shared__ zd rowj[NBMAX], rowp[NBMAX];
    zd a[RPT][NBMAX];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int r = k0 + tid + 1024 * q;
#pragma unroll
        for (int c = 0; c < NBMAX; ++c)
            a[q][c] = (r < n && c < nb) ? A[r + (int64_t)(k0 + c) * lda] : mk(0.0, 0.0);
    }
    for (int jj = 0; jj < nb; ++jj) {
        const int j = k0 + jj;
        double bv = -1.0;
        int bi = 0x7fffffff;
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int r = k0 + tid + 1024 * q;
            if (r >= j && r < n) {
                double v = 0.0;
#pragma unroll
                for (int c = 0; c < NBMAX; ++c)
                    if (c == jj) v = abs2(a[q][c]);
                if (v > bv) { bv = v; bi = r; }
            }
        }
        for (int o = 32; o > 0; o >>= 1) {
            const double ov = __shfl_xor(bv, o);
            const int oi = __shfl_xor(bi, o);
            if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
        }
        if ((tid & 63) == 0) { wv[tid >> 6] = bv; wi[tid >> 6] = bi; }
        __syncthreads();
        bv = wv[0];
        bi = wi[0];
        for (int w = 1; w < 16; ++w)
            if (wv[w] > bv || (wv[w] == bv && wi[w] < bi)) { bv = wv[w]; bi = wi[w]; }
        const int p = bi < n ? bi : j;
        if (tid == 0) {
            piv[j] = p;
            if (!(bv > 0.0)) info[0] = 1;
        }
        // rows j and p to LDS, then swapped back into registers
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int r = k0 + tid + 1024 * q;
            if (r == j)
#pragma unroll
                for (int c = 0; c < NBMAX; ++c) rowj[c] = a[q][c];
            if (r == p)
#pragma unroll
                for (int c = 0; c < NBMAX; ++c) rowp[c] = a[q][c];
        }
        __syncthreads();
        if (p != j) {
#pragma unroll
            for (int q = 0; q < RPT; ++q) {
                const int r = k0 + tid + 1024 * q;
                if (r == j)
#pragma unroll
                    for (int c = 0; c < NBMAX; ++c) a[q][c] = rowp[c];
                if (r == p)
#pragma unroll
                    for (int c = 0; c < NBMAX; ++c) a[q][c] = rowj[c];
            }
        }
        // the pivot row after the swap is rowp (rowj when p == j: the same row)
        const zd d = rowp[jj];
        const zd dinv = (abs2(d) > 0.0) ? cinv(d) : mk(0.0, 0.0);
#pragma unroll
        for (int q = 0; q < RPT; ++q) {
            const int r = k0 + tid + 1024 * q;
            if (r > j && r < n) {
                zd l = mk(0.0, 0.0);
#pragma unroll
                for (int c = 0; c < NBMAX; ++c)
                    if (c == jj) { l = a[q][c] * dinv; a[q][c] = l; }
#pragma unroll
                for (int c = 0; c < NBMAX; ++c)
                    if (c > jj && c < nb) a[q][c] = a[q][c] - l * rowp[c];
            }
        }
        __syncthreads();
    }
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int r = k0 + tid + 1024 * q;
        if (r < n)
#pragma unroll
            for (int c = 0; c < NBMAX; ++c)
                if (c < nb) A[r + (int64_t)(k0 + c) * lda] = a[q][c];
    }
}

// panel width of the LU (16 columns: narrower panels with two or four rows per thread in
// registers measured slower overall, by the extra panels and trailing updates)
// ---- tall panels (more than 1024 rows) by tournament pivoting: partial pivoting inside
// chunks of 256 rows picks 16 candidate rows per chunk (many workgroups at once), partial
// pivoting over all candidates picks the panel's pivots, and the panel is then the LU of
// its top block after the row exchanges with L21 = A21 U11^-1.  This is the
// communication-avoiding form of the panel factorisation (Grigori, Demmel and Xiang, 2011):
// the pivots can differ from those of partial pivoting over the whole column, the
// factorisation is P A = L U all the same, and no workgroup waits for another inside a
// column step (a single workgroup over the whole panel is held to one compute unit's
// bandwidth for every column).
constexpr int kTsluChunk = 256;
constexpr int kTsluMaxCand = 1024;           // chunks x 16 candidates held by one workgroup

// the entry jj of a register array (unrolled selection, no dynamic register indexing)
__device__ __forceinline__ zd pick16(const zd (&a)[16], int jj) {
    // value selects (a select of addresses would keep the array in scratch memory)
    double xr = 0.0, xi = 0.0;
#pragma unroll
    for (int c = 0; c < 16; ++c) {
        xr = c == jj ? a[c].x : xr;
        xi = c == jj ? a[c].y : xi;
    }
    return mk(xr, xi);
}

// partial pivoting over the rows held by the workgroup (one row per thread, values in a,
// rows already chosen or absent have taken = true); the chosen row ids go to out[0..nb)
// (-1 when no row is left).  NW wavefronts.  One barrier per pivot: each wavefront's best
// row (largest |a_jj|, ties to the smaller row id) publishes its value, id and its whole row
// in LDS slots of the pivot's parity, so that after the barrier every thread finds the
// winner and reads its row without a second barrier (the slots of pivot jj are rewritten at
// pivot jj + 2, after everyone has passed the barrier of pivot jj + 1).
template <int NW>
__device__ __forceinline__ void tournament(zd (&a)[16], bool taken, int row, int nb,
                                           int *out) {
    const int tid = threadIdx.x, w = tid >> 6;
    __shared__ double wv[2][NW];
    __shared__ int wi[2][NW];
    __shared__ zd wrow[2][NW][16];
    for (int jj = 0; jj < nb; ++jj) {
        const int par = jj & 1;
        double bv = taken ? -1.0 : abs2(pick16(a, jj));
        int bi = taken ? 0x7fffffff : row;
        for (int o = 32; o > 0; o >>= 1) {
            const double ov = __shfl_xor(bv, o);
            const int oi = __shfl_xor(bi, o);
            if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
        }
        if ((tid & 63) == 0) { wv[par][w] = bv; wi[par][w] = bi; }
        if (bv >= 0.0 && !taken && row == bi) {
#pragma unroll
            for (int c = 0; c < 16; ++c) wrow[par][w][c] = a[c];
        }
        __syncthreads();
        bv = wv[par][0];
        bi = wi[par][0];
        int bw = 0;
        for (int v = 1; v < NW; ++v)
            if (wv[par][v] > bv || (wv[par][v] == bv && wi[par][v] < bi)) {
                bv = wv[par][v];
                bi = wi[par][v];
                bw = v;
            }
        if (tid == 0) out[jj] = bv < 0.0 ? -1 : bi;
        if (bv >= 0.0 && !taken && row == bi) {
            taken = true;
        } else if (bv >= 0.0 && !taken) {
            const zd d = wrow[par][bw][jj];
            const zd dinv = (abs2(d) > 0.0) ? cinv(d) : mk(0.0, 0.0);
            const zd l = pick16(a, jj) * dinv;
#pragma unroll
            for (int c = 1; c < 16; ++c)
                if (c > jj && c < nb) a[c] = a[c] - l * wrow[par][bw][c];
        }
    }
    __syncthreads();
}

// candidates of chunk blockIdx.x (rows k0 + 256 blockIdx.x + tid) -> cand[16 blockIdx.x ..]
__global__ __launch_bounds__(256) void k_tslu_local(int n, int k0, int nb, const zd *A,
                                                    int64_t lda, int *cand) {
    const int row = k0 + blockIdx.x * kTsluChunk + threadIdx.x;
    const bool valid = row < n;
    zd a[16];
#pragma unroll
    for (int c = 0; c < 16; ++c)
        a[c] = (valid && c < nb) ? A[row + (int64_t)(k0 + c) * lda] : mk(0.0, 0.0);
    __shared__ int out[16];
    tournament<kTsluChunk / 64>(a, !valid, row, nb, out);
    if (threadIdx.x < 16)
        cand[blockIdx.x * 16 + threadIdx.x] = (int)threadIdx.x < nb ? out[threadIdx.x] : -1;
}

// the panel's pivots from all candidates, the row exchanges inside the panel (piv in the
// sequential-exchange form of partial pivoting), and the unpivoted LU of the top block
template <int NW>              // wavefronts: 64 NW >= max(candidates, 256)
__global__ __launch_bounds__(64 * NW) void k_tslu_final(int n, int k0, int nb, zd *A,
                                                        int64_t lda, const int *cand, int ncand,
                                                        int *piv, int *info) {
    const int tid = threadIdx.x;
    const int row = tid < ncand ? cand[tid] : -1;
    const bool valid = row >= 0;
    zd a[16];
#pragma unroll
    for (int c = 0; c < 16; ++c)
        a[c] = (valid && c < nb) ? A[row + (int64_t)(k0 + c) * lda] : mk(0.0, 0.0);
    __shared__ int P[16], pv[16];
    tournament<NW>(a, !valid, row, nb, P);
    if (tid == 0) {
        // pivot jj is original row P[jj]; its current position after the earlier exchanges
        // (rows displaced from the top block are tracked in a short list)
        int orig[32], pos[32], nd = 0;                 // at most two new entries per pivot
        for (int jj = 0; jj < nb; ++jj) {
            const int j = k0 + jj, t = P[jj];
            int q = t;
            for (int d = 0; d < nd; ++d)
                if (orig[d] == t) q = pos[d];
            pv[jj] = q < 0 ? j : q;
            piv[j] = pv[jj];
            if (q < 0) {                                  // fewer candidates than columns
                info[0] = 1;
                continue;
            }
            if (q != j) {
                int oj = j;                          // the original row now at position j
                for (int d = 0; d < nd; ++d)
                    if (pos[d] == j) oj = orig[d];
                bool f1 = false, f2 = false;
                for (int d = 0; d < nd; ++d) {
                    if (orig[d] == oj) { pos[d] = q; f1 = true; }
                    else if (orig[d] == t) { pos[d] = j; f2 = true; }
                }
                if (!f1) { orig[nd] = oj; pos[nd] = q; ++nd; }
                if (!f2) { orig[nd] = t; pos[nd] = j; ++nd; }
            }
        }
    }
    __syncthreads();
    // the exchanges, in order, on the panel's columns: thread tid < nb owns column k0 + tid,
    // so the sequence needs no barrier between exchanges
    if (tid < nb) {
        const int64_t c = (int64_t)(k0 + tid) * lda;
        for (int jj = 0; jj < nb; ++jj) {
            const int j = k0 + jj, q = pv[jj];
            if (q != j) {
                const zd t = A[j + c];
                A[j + c] = A[q + c];
                A[q + c] = t;
            }
        }
    }
    __syncthreads();
    // unpivoted LU of the nb x nb top block in LDS (thread (i, c) = (tid / 16, tid % 16))
    __shared__ zd T[16][16];
    const int i = tid >> 4, c = tid & 15;
    if (tid < 256 && i < nb && c < nb) T[i][c] = A[k0 + i + (int64_t)(k0 + c) * lda];
    __syncthreads();
    for (int jj = 0; jj < nb; ++jj) {
        if (tid < 256 && i > jj && i < nb && c == jj) {
            const zd d = T[jj][jj];
            T[i][jj] = T[i][jj] * ((abs2(d) > 0.0) ? cinv(d) : mk(0.0, 0.0));
        }
        __syncthreads();
        if (tid < 256 && i > jj && i < nb && c > jj && c < nb) T[i][c] = T[i][c] - T[i][jj] * T[jj][c];
        __syncthreads();
    }
    if (tid < 256 && i < nb && c < nb) {
        if (i == c && !(abs2(T[i][i]) > 0.0)) info[0] = 1;
        A[k0 + i + (int64_t)(k0 + c) * lda] = T[i][c];
    }
}

// L21 = A21 U11^-1 for the rows below the top block, one row per thread
__global__ __launch_bounds__(256) void k_tslu_l21(int n, int k0, int nb, zd *A, int64_t lda) {
    __shared__ zd U[16][16];
    const int tid = threadIdx.x;
    {
        const int i = tid >> 4, c = tid & 15;
        if (i < nb && c < nb) U[i][c] = A[k0 + i + (int64_t)(k0 + c) * lda];
    }
    __syncthreads();
    const int row = k0 + nb + blockIdx.x * 256 + tid;
    if (row >= n) return;
    zd a[16], l[16];
#pragma unroll
    for (int c = 0; c < 16; ++c)
        a[c] = c < nb ? A[row + (int64_t)(k0 + c) * lda] : mk(0.0, 0.0);
#pragma unroll
    for (int c = 0; c < 16; ++c) {
        zd x = a[c];
#pragma unroll
        for (int m = 0; m < c; ++m) x = x - l[m] * U[m][c];
        const zd d = U[c][c];
        l[c] = (c < nb && abs2(d) > 0.0) ? x * cinv(d) : mk(0.0, 0.0);
    }
#pragma unroll
    for (int c = 0; c < 16; ++c)
        if (c < nb) A[row + (int64_t)(k0 + c) * lda] = l[c];
}

size_t lu_panel_ws_ints() { return kTsluMaxCand; }

int lu_panel_width(int) { return 16; }

void launch_lu_panel(int n, int k0, int nb, zd *A, int64_t lda, int *piv, int *info, int *ws,
                     hipStream_t s) {
    if (nb < 1 || nb > 16) throw std::runtime_error("LU panel width must be in [1, 16]");
    const int rows = n - k0;
    const int nchunk = (rows + kTsluChunk - 1) / kTsluChunk;
    if (rows <= 1024) {
        hipLaunchKernelGGL((k_lu_panel_reg<1, 16>), dim3(1), dim3(1024), 0, s, n, k0, nb, A, lda,
                           piv, info);
    } else if (ws && nchunk * 16 <= kTsluMaxCand) {
        hipLaunchKernelGGL(k_tslu_local, dim3(nchunk), dim3(kTsluChunk), 0, s, n, k0, nb,
                           (const zd *)A, lda, ws);
        const int ncand = nchunk * 16;
        auto final_kernel = ncand <= 256 ? k_tslu_final<4>
                          : ncand <= 512 ? k_tslu_final<8> : k_tslu_final<16>;
        const int nthr = ncand <= 256 ? 256 : ncand <= 512 ? 512 : 1024;
        hipLaunchKernelGGL(final_kernel, dim3(1), dim3(nthr), 0, s, n, k0, nb, A, lda,
                           (const int *)ws, ncand, piv, info);
        const int below = rows - nb;
        hipLaunchKernelGGL(k_tslu_l21, dim3((below + 255) / 256), dim3(256), 0, s, n, k0, nb, A,
                           lda);
    } else {
        hipLaunchKernelGGL(k_lu_panel, dim3(1), dim3(1024), 0, s, n, k0, nb, A, lda, piv, info);
    }
}

// apply the row swaps piv[k0 .. k1) to columns [c0, c1) of A (one thread per column)
template <typename T>
__global__ void k_swaps(int k0, int k1, const int *piv, cpx<T> *A, int64_t lda, int64_t c0,
                        int64_t c1, bool reverse) {
    int64_t c = c0 + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= c1) return;
    cpx<T> *col = A + c * lda;
    if (!reverse) {
        for (int j = k0; j < k1; ++j) {
            int p = piv[j];
            if (p != j) { cpx<T> t = col[j]; col[j] = col[p]; col[p] = t; }
        }
    } else {
        for (int j = k1 - 1; j >= k0; --j) {
            int p = piv[j];
            if (p != j) { cpx<T> t = col[j]; col[j] = col[p]; col[p] = t; }
        }
    }
}
template <typename T>
void launch_swaps(int k0, int k1, const int *piv, cpx<T> *A, int64_t lda, int64_t c0, int64_t c1,
                  hipStream_t s) {
    if (c1 <= c0 || k1 <= k0) return;
    int64_t n = c1 - c0;
    hipLaunchKernelGGL(k_swaps<T>, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, s, k0, k1, piv, A,
                       lda, c0, c1, false);
}
// the swaps of piv[k0 .. k1) on two column ranges [a0, a1) and [b0, b1) in one launch (the
// columns left and right of an LU panel)
template <typename T>
__global__ void k_swaps2(int k0, int k1, const int *piv, cpx<T> *A, int64_t lda, int64_t a0,
                         int64_t na, int64_t b0, int64_t nb) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= na + nb) return;
    const int64_t c = t < na ? a0 + t : b0 + (t - na);
    cpx<T> *col = A + c * lda;
    for (int j = k0; j < k1; ++j) {
        const int p = piv[j];
        if (p != j) { cpx<T> v = col[j]; col[j] = col[p]; col[p] = v; }
    }
}
template <typename T>
void launch_swaps2(int k0, int k1, const int *piv, cpx<T> *A, int64_t lda, int64_t a0,
                   int64_t a1, int64_t b0, int64_t b1, hipStream_t s) {
    const int64_t na = a1 > a0 ? a1 - a0 : 0, nb = b1 > b0 ? b1 - b0 : 0;
    if (na + nb == 0 || k1 <= k0) return;
    hipLaunchKernelGGL(k_swaps2<T>, dim3((unsigned)((na + nb + 127) / 128)), dim3(128), 0, s, k0,
                       k1, piv, A, lda, a0, na, b0, nb);
}
template void launch_swaps2<double>(int, int, const int *, zd *, int64_t, int64_t, int64_t,
                                    int64_t, int64_t, hipStream_t);

// the inverse permutation: the swaps of piv[k0 .. k1) in reverse order
template <typename T>
void launch_swaps_reverse(int k0, int k1, const int *piv, cpx<T> *A, int64_t lda, int64_t c0,
                          int64_t c1, hipStream_t s) {
    if (c1 <= c0 || k1 <= k0) return;
    int64_t n = c1 - c0;
    hipLaunchKernelGGL(k_swaps<T>, dim3((unsigned)((n + 127) / 128)), dim3(128), 0, s, k0, k1,
                       piv, A, lda, c0, c1, true);
}
template void launch_swaps_reverse<double>(int, int, const int *, zd *, int64_t, int64_t,
                                           int64_t, hipStream_t);
template void launch_swaps<double>(int, int, const int *, zd *, int64_t, int64_t, int64_t,
                                   hipStream_t);

// inverse of the nb x nb (nb <= 64) diagonal block at A: unit lower (lower = true) or upper.
// The block is staged in LDS; one thread per column of the inverse (element (r, c) of the
// inverse at X[c + 65 r], so that the threads of a step touch consecutive words).
__device__ __forceinline__ void tri_inv_body(int nb, const zd *A, int64_t lda, bool lower,
                                             zd *Inv, int ldi, zd *Ab, zd *X) {
    const int c = threadIdx.x;
    for (int q = 0; q < nb; ++q)
        if (c < nb) Ab[c + q * 65] = A[c + (int64_t)q * lda];
    __syncthreads();
    if (c < nb) {
        if (lower) {
            for (int r = 0; r < nb; ++r) {
                zd sum = mk(r == c ? 1.0 : 0.0, 0.0);
                if (r > c)
                    for (int q = c; q < r; ++q) sum = sum - Ab[r + q * 65] * X[c + q * 65];
                X[c + r * 65] = r < c ? mk(0.0, 0.0) : sum;
            }
        } else {
            for (int r = nb - 1; r >= 0; --r) {
                zd sum = mk(r == c ? 1.0 : 0.0, 0.0);
                if (r <= c)
                    for (int q = r + 1; q <= c; ++q) sum = sum - Ab[r + q * 65] * X[c + q * 65];
                X[c + r * 65] = r > c ? mk(0.0, 0.0) : sum * cinv(Ab[r + r * 65]);
            }
        }
    }
    __syncthreads();
    // Inv[r, q] = X[q + 65 r]: thread c writes row c
    for (int q = 0; q < nb; ++q)
        if (c < nb) Inv[c + q * ldi] = X[q + c * 65];
}
// all diagonal blocks of an n x n LU at once: workgroup (bi, 0) inverts the unit lower
// triangle of block bi into Linv + bi blk^2, (bi, 1) the upper one into Uinv + bi blk^2
__global__ __launch_bounds__(64) void k_tri_inv_blocks(int n, int blk, const zd *A,
                                                       int64_t lda, zd *Linv, zd *Uinv) {
    __shared__ zd Ab[64 * 65];
    __shared__ zd X[64 * 65];
    const int bi = blockIdx.x;
    const bool lower = blockIdx.y == 0;
    const int k0 = bi * blk, kb = min(blk, n - k0);
    const zd *Ad = A + k0 + (int64_t)k0 * lda;
    zd *Inv = (lower ? Linv : Uinv) + (size_t)bi * blk * blk;
    tri_inv_body(kb, Ad, lda, lower, Inv, blk, Ab, X);
}
void launch_tri_inv_blocks(int n, int blk, const zd *A, int64_t lda, zd *Linv, zd *Uinv,
                           hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_tri_inv_blocks, dim3((n + blk - 1) / blk, 2), dim3(64), 0, s, n, blk, A,
                       lda, Linv, Uinv);
}

// U12 <- L11^-1 A12 in place for the kb x ncols block A12 of an LU panel (kb <= 16), L11 the
// unit lower triangle of the panel's diagonal block.  With Lin == nullptr the inverse is
// formed from L11 (forward substitution, one column per thread, as tri_inv_body) and workgroup
// 0 stores it to Lout (ld ldl) for later blocks; otherwise Lin (ld ldl) is used.  One thread
// per column of A12: y_r = x_r + sum_{q < r} Linv[r, q] x_q.  This replaces a tiny GEMM into a
// temporary, the copy back and the separate inverse.
__global__ __launch_bounds__(256) void k_panel_u12(int kb, const zd *L11, int64_t lda,
                                                   zd *A12, int64_t ncols, const zd *Lin,
                                                   zd *Lout, int ldl) {
    __shared__ zd Li[16 * 17];                    // Li[r + 17 q] = Linv[r, q]
    const int tid = threadIdx.x;
    if (Lin == nullptr) {
        __shared__ zd Ab[16 * 17];
        if (tid < kb * kb) {
            const int r = tid % kb, q = tid / kb;
            Ab[r + 17 * q] = L11[r + (int64_t)q * lda];
        }
        __syncthreads();
        if (tid < kb) {
            const int c = tid;                    // column c of the inverse
            for (int r = 0; r < kb; ++r) {
                zd sum = mk(r == c ? 1.0 : 0.0, 0.0);
                if (r > c)
                    for (int q = c; q < r; ++q) sum = sum - Ab[r + 17 * q] * Li[q + 17 * c];
                Li[r + 17 * c] = r < c ? mk(0.0, 0.0) : sum;
            }
        }
        __syncthreads();
        if (blockIdx.x == 0 && tid < kb * kb) {
            const int r = tid % kb, q = tid / kb;
            Lout[r + (int64_t)q * ldl] = Li[r + 17 * q];
        }
    } else {
        if (tid < kb * kb) {
            const int r = tid % kb, q = tid / kb;
            Li[r + 17 * q] = Lin[r + (int64_t)q * ldl];
        }
        __syncthreads();
    }
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + tid;
    if (c >= ncols) return;
    zd *col = A12 + c * lda;
    zd x[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) x[r] = r < kb ? col[r] : mk(0.0, 0.0);
#pragma unroll
    for (int r = 15; r >= 1; --r) {               // rows from the bottom: x_q, q < r, unchanged
        if (r >= kb) continue;
        zd y = x[r];
#pragma unroll
        for (int q = 0; q < 15; ++q)
            if (q < r) y = y + Li[r + 17 * q] * x[q];
        x[r] = y;
    }
#pragma unroll
    for (int r = 0; r < 16; ++r)
        if (r < kb) col[r] = x[r];
}
void launch_panel_u12(int kb, const zd *L11, int64_t lda, zd *A12, int64_t ncols,
                      const zd *Lin, zd *Lout, int ldl, hipStream_t s) {
    if (kb <= 0 || kb > 16 || (Lin != nullptr && ncols <= 0)) return;
    const unsigned nblk = (unsigned)std::max<int64_t>(1, (ncols + 255) / 256);
    hipLaunchKernelGGL(k_panel_u12, dim3(nblk), dim3(256), 0, s, kb, L11, lda, A12,
                       ncols < 0 ? 0 : ncols, Lin, Lout, ldl);
}

// identity added to the diagonal: A += I
__global__ void k_add_identity(int n, zd *A, int64_t lda) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) A[i + (int64_t)i * lda].x += 1.0;
}
void launch_add_identity(int n, zd *A, int64_t lda, hipStream_t s) {
    hipLaunchKernelGGL(k_add_identity, dim3((n + 255) / 256), dim3(256), 0, s, n, A, lda);
}

// per-column relative residual: out[c] = sqrt(r2[c] / b2[c]); max written to out[n]
__global__ void k_ratio_max(int64_t n, const double *r2, const double *b2, double *out) {
    __shared__ double mx[256];
    double a = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        double v = b2[i] > 0.0 ? sqrt(r2[i] / b2[i]) : sqrt(r2[i]);
        a = fmax(a, v);
    }
    mx[threadIdx.x] = a;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) mx[threadIdx.x] = fmax(mx[threadIdx.x], mx[threadIdx.x + w]);
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = mx[0];
}
void launch_ratio_max(int64_t n, const double *r2, const double *b2, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_ratio_max, dim3(1), dim3(256), 0, s, n, r2, b2, out);
}

// p[0..n) = v (a kernel rather than a memset node, for work that may be recorded in a graph)
__global__ void k_fill_int(int n, int v, int *p) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}
void launch_fill_int(int n, int v, int *p, hipStream_t s) {
    hipLaunchKernelGGL(k_fill_int, dim3((n + 255) / 256), dim3(256), 0, s, n, v, p);
}

// Check of one sketch block of a replayed factorisation against its recorded schedule:
// probe != 0 -- the block's squared column norms (n of them) must all be <= tau2 (the
// recorded run stopped at this block); otherwise the pivoted Cholesky must have kept exactly
// `planned` directions (*kdev).  A failed check sets `bit` in *flag.  One workgroup.
__global__ void k_replay_check(int n, const double *norms2, double tau2, int probe,
                               const int *kdev, int planned, int bit, int *flag) {
    __shared__ int bad;
    if (threadIdx.x == 0) bad = 0;
    __syncthreads();
    if (probe) {
        for (int i = threadIdx.x; i < n; i += blockDim.x)
            if (!(norms2[i] <= tau2)) bad = 1;
    } else if (threadIdx.x == 0) {
        bad = *kdev != planned;
    }
    __syncthreads();
    if (threadIdx.x == 0 && bad) *flag |= bit;
}
void launch_replay_check(int n, const double *norms2, double tau2, int probe, const int *kdev,
                         int planned, int bit, int *flag, hipStream_t s) {
    hipLaunchKernelGGL(k_replay_check, dim3(1), dim3(256), 0, s, n, norms2, tau2, probe, kdev,
                       planned, bit, flag);
}

}  // namespace cfie
