// Internal declarations shared by the HIP translation units of libcfie.
#pragma once
#include <hip/hip_runtime.h>

#include <cstdint>
#include <stdexcept>
#include <string>
#include <vector>

#include "../../include/cfie.h"
#include "bessel.h"
#include "cplx.h"

namespace cfie {

// ------------------------------------------------------------------ launch profiling ------
// When a context is created with profile != 0, every API call installs a Profiler for the
// calling thread; the hot kernels then bracket their launches with HIP events on their
// stream and record the algorithmic work of the launch (flops for GEMMs, point pairs for
// the assembly).  Totals are read back with cfie_query.
struct LaunchRec {
    int kind;                        // PROF_* below
    double work;
    hipEvent_t a, b;
};
enum { PROF_GEMM64 = 0, PROF_GEMM32 = 1, PROF_FAR = 2, PROF_NEAR = 3, PROF_FFT = 4, PROF_KINDS = 5 };
struct Profiler {
    std::vector<LaunchRec> recs;
    std::vector<hipEvent_t> pool;
    hipEvent_t get();
};
extern thread_local Profiler *g_prof;
struct ProfScope {                   // brackets one launch when profiling is on
    Profiler *p;
    LaunchRec r;
    hipStream_t s;
    ProfScope(int kind, double work, hipStream_t st) : p(g_prof), s(st) {
        if (p) {
            r.kind = kind;
            r.work = work;
            r.a = p->get();
            r.b = p->get();
            (void)hipEventRecord(r.a, s);
        }
    }
    ~ProfScope() {
        if (p) {
            (void)hipEventRecord(r.b, s);
            p->recs.push_back(r);
        }
    }
};

// ------------------------------------------------------------------ geometry (host) -------
// Contour z(t) = sum_m zhat_m e^{imt}; arc-length density |z'(t)| as a Fourier series
// c0 + 2 Re sum_{m>=1} c_m e^{imt}.  Nodes s_i = i L / N (uniform in arc length).
struct HostGeometry {
    int M = 0;                       // z modes -M..M
    std::vector<zd> zhat;            // 2M+1
    double c0 = 0.0;                 // mean speed
    std::vector<zd> cm;              // c_m, m = 1..Ms
    double L = 0.0, h = 0.0, radius = 0.0;
    bool convex = true;
    double min_curvature = 0.0;
};

// Fills g from the contour; returns an error text or "" on success.
std::string build_geometry(const cfie_contour &c, HostGeometry &g);
HostGeometry circle_geometry(double radius);
void gauss_legendre01(int n, std::vector<double> &x, std::vector<double> &w);

// Product-integration weights for the log part of touching element pairs.  For the
// q-point Gauss grid (xi_g, xi'_h) on [0,1]^2:
//   mom[kind][c][g*q+h] = int int l_g(xi) l_h(xi') P_c(xi, xi') log(sigma) dxi dxi'
// kind 0: sigma = |xi - xi'| (same element), 1: sigma = 1 - xi + xi' (source = next
// element), 2: sigma = 1 + xi - xi' (source = previous element); c = 2a+b for the hat
// product phi_a(xi) phi_b(xi') (phi_0 = 1 - xi, phi_1 = xi) and c = 4 for no hats.
void log_moments(int q, std::vector<double> &mom /* 3 * 5 * q * q */);

// ------------------------------------------------------------------ device tables --------
struct PointTable {                  // per element e and Gauss point g: index e*q + g
    int q = 0;
    double *x = nullptr, *y = nullptr, *tx = nullptr, *ty = nullptr, *curv = nullptr;
};

struct GeomDev {                     // device copies of the Fourier data
    int M = 0, Ms = 0;
    zd *zhat = nullptr;              // 2M+1
    zd *cm = nullptr;                // Ms
    double c0 = 0.0, L = 0.0, h = 0.0;
    int N = 0;
};

struct KernelConsts {                // wavenumbers and derived constants
    double k;                        // real wavenumber
    zd kt;                           // complex wavenumber k + i beta
};

// ------------------------------------------------------------------ launchers ------------
// Gauss points of all elements (x, y, unit tangent, curvature) from the Fourier data.
void launch_points(const GeomDev &g, const double *xi, PointTable &pt, hipStream_t s);

// Rows [r0, r1) of Dk, Nk, Dkt, Skt (out[m] + i + j*ld); far part: entries with cyclic
// |i - j| >= nb + 2 by q_far x q_far Gauss-Legendre.
struct AsmParams {
    int N;
    double h;
    KernelConsts kc;
    int nb;                          // near band
    int r0, r1;
    int64_t ld;
    zd *out[4];                      // Dk, Nk, Dkt, Skt
    zd *ws = nullptr;                // far assembly: far_band_ws_elems(*this) complex128
};
// work space of launch_assemble_far (blocks of the small-argument element pairs near the
// diagonal), in complex128 elements
size_t far_band_ws_elems(const AsmParams &p);
// half-width in elements of the band of small-argument element pairs near the diagonal
int far_band_width(int N, double k, double h, int nb);
void launch_assemble_far(const AsmParams &p, const PointTable &far, const double *xi,
                         const double *w, hipStream_t s);
// Near part: entries with cyclic |i - j| <= nb + 1; touching element pairs by product
// integration of the log singularity (moments), others by q_near Gauss-Legendre.  p.ws:
// near_ws_elems(p) complex128 (blocks of the element pairs).
size_t near_ws_elems(const AsmParams &p);
void launch_assemble_near(const AsmParams &p, const PointTable &near, const double *xi,
                          const double *w, const double *moments, hipStream_t s);

// Plane-wave right-hand-side vectors e' and h (N x m each; hvec may be NULL).
void launch_excitation(const GeomDev &g, const PointTable &pt, const double *xi,
                       const double *w, double k, const double *angles, int64_t m,
                       zd *e, zd *hvec, int64_t ld, hipStream_t s);

// ------------------------------------------------------------------ shape derivative -----
// Backward passes of the assembly (far and near element pairs), of the plane-wave vectors and
// of the point evaluation; Om = loss weights of (Dk, Nk, Dkt, Skt), column-major, ld.
// far: adj (4 x N q_far) = d loss / d(x, y, tx, ty) of the far table (written); ws:
// grad_far_ws_doubles work space; spart: grad_far_spart_pairs pairs (d/dh, d/dbeta), their
// number returned in n_pairs.
size_t grad_far_ws_doubles(int N, int q, double k, double h, int nb);
int grad_far_spart_pairs(int N, double k, double h, int nb);
void launch_grad_far(int N, double h, const KernelConsts &kc, int nb, const zd *const Om[4],
                     int64_t ld, const PointTable &pt, const double *xi, const double *w,
                     double *ws, double *spart, double *adj, int &n_pairs, hipStream_t s);
// near: adj (5 x N q_near, with curvature) written; spart: 2 per block; returns the blocks
int launch_grad_near(int N, double h, const KernelConsts &kc, int nb, const zd *const Om[4],
                     int64_t ld, const PointTable &pt, const double *xi, const double *w,
                     const double *moments, double *adj, double *spart, hipStream_t s);
// plane-wave vectors: adds to adj[0..3]; spart: d/dh per block; returns the blocks
int launch_grad_exc(int N, double h, double k, const PointTable &pt, const double *xi,
                    const double *w, const double *angles, int64_t m, const zd *WE,
                    int64_t lde, zd aE, bool cE, const zd *WH, int64_t ldh, zd aH, bool cH,
                    double *adj, double *spart, hipStream_t s);
// per point: t, 2 pi sigma - t, (d/dt)/s'(t), adjoints of z, z', z'' (10 doubles)
void launch_grad_prep(const GeomDev &g, const PointTable &pt, const double *xi,
                      const double *adj, bool has_curv, double *out, hipStream_t s);
// reductions onto the modes of z (2M+1), of the speed (Ms) and onto c0 (1)
void launch_grad_modes(int M, int Ms, int64_t n1, const double *P1, int64_t n2,
                       const double *P2, zd *out, hipStream_t s);
int launch_gdot(int N, int64_t m, double h, const zd *A, int64_t lda, const zd *B, int64_t ldb,
                zd coef, double *part, hipStream_t s);
void launch_transpose(int64_t rows, int64_t cols, const zd *src, int64_t lds, zd *dst,
                      int64_t ldd, zd alpha, bool cj, hipStream_t s);
void launch_conj_scale(int64_t rows, int64_t cols, const zd *src, int64_t lds, zd *dst,
                       int64_t ldd, zd alpha, hipStream_t s);
// adjoint of the speed coefficients (c0, c_1..c_Ms) of build_geometry onto zbar (2M+1, +=)
void speed_coeffs_adjoint(const HostGeometry &g, double c0bar, const std::vector<zd> &cmbar,
                          std::vector<zd> &zbar);

// ------------------------------------------------------------------ FFT ------------------
struct FFTPlan {
    int N = 0;                       // length of the circulant
    // transform length M = N1 * N2 (power of two, N1 <= 4096): M = N for powers of two;
    // otherwise the smallest power of two >= 2N - 1, and circulant products are computed
    // as zero-padded linear convolutions of length M
    int M = 0, N1 = 0, N2 = 0;
    double *tw1 = nullptr;           // e^{-2 pi i j / N1}, j < N1   (complex, interleaved)
    double *twM = nullptr;           // e^{-2 pi i j / M},  j < M    (complex)
    float *tw1f = nullptr, *twMf = nullptr;
    double *twN = nullptr;           // e^{-2 pi i j / N},  j < N    (aliases twM when M == N)
};
// y = IFFT(d .* FFT(x)) column by column at the transform length M (d in the transposed
// layout of length M, 1/M folded in), written to x; the input is src (ld lds) when src is
// given, else x itself.
template <typename T>
void launch_circ_apply(const FFTPlan &p, const cpx<T> *d, cpx<T> *x, int64_t ldx,
                       int64_t nb, hipStream_t s, const cpx<T> *src = nullptr,
                       int64_t lds = 0);
// the same for M > N: the input (N x nb) zero-padded into P (M x nb), transformed, and the
// first N rows copied to x (ld ldx)
template <typename T>
void launch_circ_apply_padded(const FFTPlan &p, const cpx<T> *d, cpx<T> *x, int64_t ldx,
                              int64_t nb, cpx<T> *P, hipStream_t s, const cpx<T> *src = nullptr,
                              int64_t lds = 0);
// diagonal of length M in the transposed layout from the natural-order eigenvalues d_m / N
// (m < N) of a circulant of length N: its first column by an inverse DFT, wrapped to length
// M, transformed and scaled by 1/M (direct DFTs; once per assembly)
void launch_padded_diagonal(const FFTPlan &p, const zd *eig_over_N, zd *work, zd *dT, zf *fT,
                            hipStream_t s);

// ------------------------------------------------------------------ SRFT test matrix -----
// Subsampled randomized Fourier transform (Halko, Martinsson and Tropp, SIAM Review 2011,
// Sec. 4.6): Omega = (D F)[0:N, S] with D = diag(d), |d_i| = 1 of uniform random phase, F
// the M-point DFT matrix F_ij = e^{-2 pi i i j / M} (M the smallest power of two >= N; its
// first N rows when M > N) and S a random choice of columns.  A D F is formed once by
// radix-2^b decimation-in-frequency passes along the rows of A (zero-padded to M columns),
// which leave column j of A D F at a digit-reversed position p; the sketch then takes the
// columns at the positions p = perm(t), t = 0, 1, 2, ... of a seeded bijection of [0, M).
struct SrftPlan {
    int lgN = 0, npass = 0;
    int bits[8] = {};                // log2 of each pass's radix, first pass first
};
__host__ __device__ inline SrftPlan srft_plan(int lgN) {
    SrftPlan p;
    p.lgN = lgN;
    p.npass = lgN <= 0 ? 0 : (lgN + 4) / 5;           // radices of at most 32
    // the larger radices last, where the columns of a butterfly group lie closer together
    for (int l = 0; l < p.npass; ++l)
        p.bits[l] = lgN / p.npass + (l >= p.npass - lgN % p.npass ? 1 : 0);
    return p;
}
// frequency j of the column at position p: pass l contributes its digit e_l at weight
// 2^(bits of the later passes) to the position and at 2^(bits of the earlier passes) to j
__host__ __device__ inline int srft_freq(const SrftPlan &p, int pos) {
    int j = 0, lo = 0, hi = p.lgN;
    for (int l = 0; l < p.npass; ++l) {
        hi -= p.bits[l];
        const int e = (pos >> hi) & ((1 << p.bits[l]) - 1);
        j |= e << lo;
        lo += p.bits[l];
    }
    return j;
}
// seeded bijection of [0, 2^lgN): three rounds of an odd multiply-add and an xor-shift, each
// invertible modulo 2^lgN
struct SrftPerm {
    int lgN = 0;
    uint32_t mul[3] = {}, add[3] = {};
};
SrftPerm srft_perm(uint64_t seed, int lgN);
__host__ __device__ inline uint32_t srft_perm_apply(const SrftPerm &q, uint32_t x) {
    const uint32_t mask = q.lgN >= 32 ? 0xffffffffu : ((1u << q.lgN) - 1u);
    const int sh = q.lgN / 2 > 0 ? q.lgN / 2 : 1;
    for (int r = 0; r < 3; ++r) {
        x = (x * q.mul[r] + q.add[r]) & mask;
        x ^= x >> sh;
    }
    return x;
}
// out = A D F (m x M, columns at the digit-reversed positions; M a power of two >= N, the
// columns N..M-1 of A taken as zero): the first pass reads A and d and writes out, the others
// work in place on out.  tw: e^{-2 pi i j / (M tws)}, so that w_M^j = tw[j tws].
template <typename T>
void launch_srft_rows(int64_t m, int N, int M, const cpx<T> *A, int64_t lda, const cpx<T> *d,
                      const cpx<T> *tw, int tws, cpx<T> *out, int64_t ldo, hipStream_t s);
// Om[:, t] = (D F)[0:N, j(perm(off + t))] for t < nb (N x nb, F of length M = 2^q.lgN): the
// test-matrix columns whose products are the columns of A D F gathered by launch_srft_gather
template <typename T>
void launch_srft_omega(int N, const SrftPerm &q, int64_t off, int nb, const cpx<T> *d,
                       const cpx<T> *tw, int tws, cpx<T> *Om, int64_t ldo, hipStream_t s);
// out[:, t] = AF[:, perm(off + t)] for t < nb (AF: m x N from launch_srft_rows)
template <typename T>
void launch_srft_gather(int64_t m, const SrftPerm &q, int64_t off, int nb, const cpx<T> *AF,
                        int64_t ldaf, cpx<T> *out, int64_t ldo, hipStream_t s);
// d_i = e^{2 pi i u_i}, u_i uniform from the Philox stream (seed, stream), i < n
template <typename T>
void launch_steinhaus(int64_t n, uint64_t seed, uint64_t stream, cpx<T> *d, hipStream_t s);

// complex GEMM: C = alpha * op(A) * B + beta * C, op(A) = A (GEMM_N), A^H (GEMM_C) or the
// elementwise conjugate of A (GEMM_R); GEMM_NREAL: op(A) = A and B real-valued (stored
// complex, its imaginary parts taken as zero and not read), two real products instead of
// the three of the 3M form
enum { GEMM_N = 0, GEMM_C = 1, GEMM_R = 2, GEMM_NREAL = 3 };
// release the split-K workspace of (device, stream)
void splitk_release(int device, hipStream_t s);
// process-wide switch of the GEMM tile autotuner (returns the previous mode) and the number
// of shape classes measured so far
int set_gemm_autotune(int mode);
int gemm_tuned_classes();
// process-wide switch of the wide 128 x 128 complex128 tile for large products (1 = on, the
// default); bitwise the same results either way.  Returns the previous mode.
int set_gemm_wide(int mode);
// tile autotuning for the calling thread's products (it allocates a scratch output the
// first time it meets a shape class); off: the 64 x 64 tile, bitwise the same results.
// Returns the previous setting.
bool set_gemm_tune_thread(bool on);
// split-K workspace of the calling thread's GEMMs taken from p (bytes) instead of the shared
// per-stream one while p is set (graph capture); the bytes a GEMM's split needs (0: none)
void set_splitk_override(void *p, size_t bytes);
size_t gemm_splitk_bytes(int op, int64_t m, int64_t n, int64_t k, size_t elem);
template <typename T>
void gemm(int op, int64_t m, int64_t n, int64_t k, cpx<T> alpha, const cpx<T> *A, int64_t lda,
          const cpx<T> *B, int64_t ldb, cpx<T> beta, cpx<T> *C, int64_t ldc, hipStream_t s);

}  // namespace cfie
