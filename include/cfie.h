/*
 * cfie.h - C ABI of the MI355X fast direct solver for the preconditioned 2D TE combined
 * field integral equation on a closed PEC contour.
 *
 * The operation follows the paper "On the Fast Direct Solution of a Preconditioned
 * Electromagnetic Integral Equation":
 *   - Sec. II, eqs. (1)-(4): CFIE for the tangential current j_t on the contour gamma,
 *     discretised with hat functions piecewise linear in arc length (Galerkin, bilinear
 *     pairing <f,g> = int f g ds).  Matrices N^k (hypersingular, Maue form), D^k
 *     (double layer), Gram matrix G.
 *   - Sec. III, eq. (5): the preconditioned system C j = b with
 *       C = S^kt G^-1 N^k + (G/2 + D^kt) G^-1 (G/2 - D^k),
 *       b = -(i k/eta) S^kt G^-1 e - (G/2 + D^kt) G^-1 h,
 *       kt = k + 0.4 i k^(1/3) a^(-2/3).
 *   - Sec. V, eqs. (6)-(9): C_c is C on the circle of equal perimeter (circulant,
 *     diagonalised by the FFT); the remainder C - C_c = U V^T is compressed to a skeleton;
 *     C^-1 = C_c^-1 - C_c^-1 U (I + V^T C_c^-1 U)^-1 V^T C_c^-1 (Woodbury) serves any number
 *     of right-hand sides.
 *
 * Conventions used by every entry point:
 *   - Complex numbers are interleaved (re, im) pairs: complex128 = 2 doubles.
 *   - Vectors and matrices are column-major; a "device pointer" is memory allocated on
 *     the device given to cfie_create (hipMalloc, torch CUDA tensors, ...).
 *   - Every call is enqueued on the stream given to cfie_create and returns after that
 *     stream has drained.  A context must not be used from two threads at once.
 *   - The library owns every internal buffer; the caller owns what it passes in.
 *   - Return value: CFIE_OK (0), an error (1..99; nothing was changed unless stated), or a
 *     warning (>= 100; the call completed and its result is valid).  cfie_last_error
 *     gives a text for the last non-OK status of a context.
 */
#ifndef CFIE_H
#define CFIE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct cfie_ctx cfie_ctx;

typedef enum {
    CFIE_OK = 0,
    CFIE_EINVAL = 1,      /* an argument is out of range or malformed                    */
    CFIE_ENOMEM = 2,      /* device allocation failed (or the injected failure fired)    */
    CFIE_EHIP = 3,        /* a HIP runtime call or kernel launch failed                  */
    CFIE_ESTATE = 4,      /* call out of order (e.g. solve before factor)               */
    CFIE_ESINGULAR = 5,   /* zero circulant eigenvalue or zero pivot in the capacitance */
    CFIE_ENOCONV = 6,     /* refinement did not reach refine_tol; X holds the best iterate */
    CFIE_WNONCONVEX = 100 /* warning: contour has negative curvature somewhere          */
} cfie_status;

enum { CFIE_FP64 = 0, CFIE_MIXED = 1 };

/* Matrices that cfie_export_matrix can copy out (complex128, N x N unless stated). */
enum {
    CFIE_MAT_G = 0,       /* Gram matrix (real values stored as complex)               */
    CFIE_MAT_DK = 1,      /* D^k   on gamma                                            */
    CFIE_MAT_NK = 2,      /* N^k   on gamma (Maue form)                                */
    CFIE_MAT_DKT = 3,     /* D^kt  on gamma                                            */
    CFIE_MAT_SKT = 4,     /* S^kt  on gamma                                            */
    CFIE_MAT_CC_EIG = 5,  /* N eigenvalues c_m of C_c, natural DFT order (N x 1)        */
    CFIE_MAT_CIRCLE_ROW = 6 /* first rows of D^k, N^k, D^kt, S^kt on the circle (N x 4) */
};

typedef struct {
    int32_t n_nodes;      /* 8 <= N <= 32768 nodes = elements, uniform in arc length from
                             t = 0 (the four dense matrices take 64 N^2 bytes: 69 GB at
                             N = 32768)                                                */
    int32_t n_modes;      /* M >= 1: z(t) = sum_{m=-M..M} zhat[m+M] e^{imt}, CCW       */
    const double *zhat;   /* host, 2*(2M+1) doubles (re, im); read during the call only */
} cfie_contour;

typedef struct {
    int32_t precision;    /* CFIE_FP64 or CFIE_MIXED (complex64 skeleton, GEMMs and FFTs,
                             complex128 capacitance LU, FP64 iterative refinement)      */
    double compress_tol;  /* epsilon, tau = epsilon * ||C_c||_2 (||C_c||_2 = max |c_m|):
                             sketch blocks are added until a block's projected columns all
                             have norm <= tau, or a block keeps at most block - oversample
                             directions of norm > tau (see oversample)                  */
    int32_t block;        /* columns added to the sketch per adaptive step (b)         */
    int32_t max_rank;     /* cap on the skeleton rank; 0 = N                            */
    uint64_t seed;        /* seed of the Gaussian sketch (Philox4x32-10 counter stream) */
    double refine_tol;    /* mixed precision: stop when every column has
                             ||b_j - C x_j|| <= refine_tol ||b_j||                      */
    int32_t max_refine;   /* mixed precision: maximum number of refinement sweeps       */
    int32_t quad_far;     /* Gauss-Legendre points per element, well-separated pairs    */
    int32_t quad_near;    /* Gauss-Legendre points per element, near pairs              */
    int32_t near_band;    /* element pairs at cyclic distance <= near_band are near     */
    int64_t fail_alloc_after; /* test hook: fail the (n+1)-th device allocation; -1 off */
    int32_t profile;      /* 1: time every GEMM / assembly / FFT launch with HIP events on
                             the context stream and accumulate work and time (cfie_info) */
    int32_t remainder_form; /* how cfie_factor applies C - C_c (CFIE_REMAINDER_*)         */
    int32_t solve_graphs; /* 1: FP64 cfie_solve records its kernel sequence (C_c^-1 by FFT,
                             the two Woodbury GEMMs) once per batch size nrhs <= 4096 as a HIP
                             graph on buffers it owns, and replays it on later calls with
                             that nrhs (B copied in, X copied out); bitwise identical to the
                             direct path.  For many small solves with one factorisation.   */
    int32_t oversample;   /* p >= 0: the sketch stops after a block of b >= 2p Gaussian
                             columns that keeps at most b - p directions above tau (the
                             remaining range has then been sampled with p or more columns of
                             oversampling); 0 turns the rule off, so blocks are drawn until
                             one has no column above tau                                 */
    int32_t refine_form;  /* mixed precision: how the FP64 residual b - C x of each refinement
                             sweep applies C (CFIE_REFINE_*)                                 */
    int32_t test_matrix;  /* random test matrix of the sketch blocks (CFIE_SKETCH_*)         */
} cfie_options;

/* cfie_options.test_matrix.  The first sketch block is always real Gaussian.  With
 * CFIE_SKETCH_SRFT the later blocks take columns of a subsampled randomized Fourier
 * transform Omega = (D F)[0:N, S] (Halko, Martinsson and Tropp, SIAM Review 53 (2011),
 * Sec. 4.6: D diagonal of unit-modulus entries of uniform random phase, F the DFT of length
 * M = the smallest power of two >= N, S distinct columns in a seeded random order).  With
 * C - C_c applied factor by factor, D^k D F and N^k D F are formed once by FFTs along their
 * rows (32 N M bytes more during the factorisation in FP64, 16 N M in mixed precision) and
 * each block's products with D^k and N^k become column gathers; with C - C_c formed densely,
 * (C - C_c) D F is formed once (16 N M bytes, 8 N M) and a block is a column gather.  Once
 * N Fourier columns have been drawn the blocks are Gaussian. */
enum {
    CFIE_SKETCH_GAUSSIAN = 0,    /* real Gaussian blocks (Philox4x32-10 stream of seed)        */
    CFIE_SKETCH_SRFT = 1         /* Gaussian first block, then SRFT columns                    */
};

/* cfie_options.refine_form.  Factor by factor, a residual costs four N x N complex products
 * per right-hand side (24 N^2 real flops executed in the 3M form); with C formed once in FP64
 * at cfie_factor (two N x N x N products, 12 N^3, and 16 N^2 more bytes), one (6 N^2). */
enum {
    CFIE_REFINE_FACTORED = 0,    /* D^k, N^k, D^kt, S^kt applied in turn                        */
    CFIE_REFINE_DENSE = 1        /* C formed densely in FP64 by cfie_factor                     */
};

/* cfie_options.remainder_form.  The sketch and V^T = Q^H (C - C_c) cost 64 N^2 r flops when
 * C is applied factor by factor (four N x N GEMMs per product, eq. (6)), and 16 N^3 + 16 N^2 r
 * when C - C_c is first formed as a dense N x N matrix (two N x N x N GEMMs) and then applied
 * with one GEMM; the dense form wins for ranks above N/3 and needs 16 N^2 more bytes (8 N^2
 * in mixed precision) during the factorisation. */
enum {
    CFIE_REMAINDER_AUTO = 0,     /* factor by factor; switch to the dense form once the sketch
                                    has reached rank N/2 without meeting the tolerance       */
    CFIE_REMAINDER_FACTORED = 1, /* always factor by factor                                 */
    CFIE_REMAINDER_DENSE = 2     /* form C - C_c densely before the sketch                   */
};

typedef struct {
    int32_t n_nodes;
    int32_t rank;             /* skeleton rank r after cfie_factor                     */
    double perimeter;         /* L                                                     */
    double radius;            /* a = L / (2 pi), radius of the equivalent circle       */
    double k;
    double ktilde_re, ktilde_im;
    double h;                 /* L / N                                                 */
    double cc_norm;           /* ||C_c||_2 = max_m |c_m|                               */
    double remainder_est;     /* last sketch block's largest column norm               */
    double t_assemble_ms;     /* device time of the last cfie_assemble                 */
    double t_factor_ms;       /* device time of the last cfie_factor                   */
    double t_solve_ms;        /* device time of the last cfie_solve                    */
    int32_t refine_sweeps;    /* sweeps used by the last mixed-precision cfie_solve    */
    double refine_residual;   /* max_j ||b_j - C x_j|| / ||b_j|| after the last sweep  */
    int32_t precision;
    int32_t convex;           /* 1 if curvature >= 0 everywhere sampled                */
    /* launch profile (options.profile = 1), accumulated since cfie_create or the last
     * reset; index: 0 complex128 GEMM, 1 complex64 GEMM, 2 far-pair assembly, 3 near-pair
     * assembly, 4 circulant FFT apply.  work: real flops executed (GEMM: 6 m n k for a
     * complex product in the 3M form, 4 m n k for a complex times a real matrix), Gauss point
     * pairs (assembly), bytes of one read and one write of the batch (FFT). */
    int64_t prof_launches[5];
    double prof_work[5];
    double prof_ms[5];
    /* device time of the phases of the last cfie_factor: 0 range finder (sketch blocks and
     * their orthonormalisation), 1 V^T = Q^H (C - C_c) and U~ = C_c^-1 Q, 2 the capacitance
     * matrix K = I + V^T U~ and its LU, 3 K^-1 V^T; a phase not reached is 0 */
    double t_factor_phase_ms[4];
} cfie_info;

/* Process-wide switch of the complex GEMM tile autotuner: mode 1 (the default) lets the first
 * product of each shape class whose 64 x 64 output grid cannot fill the device time the four
 * tile shapes (64 x 64, 32 x 64, 64 x 32, 32 x 32) on the caller's stream and keep the
 * fastest for the rest of the process; mode 0 always uses 64 x 64.  The tile shapes give
 * bitwise identical results (same K order per output element, split along K fixed
 * independently of the tile), so the switch changes speed only.  Returns the previous
 * mode.  cfie_gemm_tuned_classes returns how many shape classes have been measured. */
int cfie_set_gemm_autotune(int mode);
int cfie_gemm_tuned_classes(void);

/* Process-wide switch of the wide complex128 GEMM tile: mode 1 (the default) multiplies the
 * large FP64 products (K >= 8192 and enough 128 x 128 output tiles to fill the device) with
 * 128 x 128 tiles of 8 wavefronts whose operands go straight from global memory into LDS;
 * mode 0 always uses the 64 x 64 tiles.  Both run the same MFMA sequence per output element,
 * so the switch changes speed only (bitwise identical results).  Returns the previous mode. */
int cfie_set_gemm_wide(int mode);

/* Zero the accumulated launch profile of ctx. */
cfie_status cfie_profile_reset(cfie_ctx *ctx);

/* Fill *opt with defaults: FP64, compress_tol 1e-10, block 128, max_rank 0, seed 1,
 * refine_tol 1e-8, max_refine 20, quad_far 5, quad_near 10, near_band 6, no injection,
 * no profiling, remainder_form CFIE_REMAINDER_AUTO, solve_graphs 0, oversample 16,
 * refine_form CFIE_REFINE_FACTORED, test_matrix CFIE_SKETCH_SRFT. */
void cfie_default_options(cfie_options *opt);

/* Create a context on HIP device `device` using `hip_stream` (a hipStream_t, or NULL for
 * the null stream).  *out is set only on success.  EINVAL on bad options, EHIP if the
 * device cannot be selected.  Device memory comes from the device's default stream-ordered
 * pool (hipMallocAsync); while any context lives on the device the pool keeps memory that
 * contexts free (its release threshold raised) so that later factorisations reuse it, and
 * when the last one is destroyed the threshold returns to 0 and the pool is trimmed. */
cfie_status cfie_create(const cfie_options *opt, int device, void *hip_stream,
                        cfie_ctx **out);

/* Steps A1-A3 (Sec. II eq. (4), Sec. V): geometry of gamma and of its equivalent circle,
 * dense assembly of D^k, N^k, D^kt, S^kt on gamma (complex128, library-owned, 64 N^2
 * bytes), and the N eigenvalues c_m of C_c.  EINVAL: N < 8 or above the limits of
 * cfie_contour.n_nodes, k <= 0 or not finite, M < 1,
 * non-finite coefficients, clockwise or self-intersecting contour.  WNONCONVEX: the
 * contour is not convex (the algebra is unaffected).  Invalidates a previous factor. */
cfie_status cfie_assemble(cfie_ctx *ctx, const cfie_contour *contour, double k);

/* Steps A4-A5 (Sec. V eqs. (7)-(9)): randomized skeleton C - C_c ~ U V^T grown in blocks
 * until the remainder estimate drops below compress_tol * ||C_c||_2 or a block is found
 * rank-deficient at that level (see cfie_options.compress_tol; or max_rank / N),
 * then the capacitance matrix K = I + V^T C_c^-1 U and its LU factorisation with partial
 * pivoting (complex128).  ESTATE before assemble; ESINGULAR on a zero pivot. */
cfie_status cfie_factor(cfie_ctx *ctx);

/* Step A6 (+ A7 in mixed precision): X = C^-1 B for nrhs right-hand sides by eq. (9).
 * B_dev, X_dev: device, complex128, N x nrhs column-major with leading dimensions
 * ldb, ldx >= N.  B_dev == X_dev is allowed (in place); other overlaps are not.
 * nrhs == 0 is a no-op.  ESTATE before factor; ENOCONV (mixed only) if max_refine sweeps
 * do not reach refine_tol, X then holds the last iterate. */
cfie_status cfie_solve(cfie_ctx *ctx, const void *B_dev, int64_t ldb, void *X_dev,
                       int64_t ldx, int64_t nrhs);

/* cfie_solve without device allocation, for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * FP64 Woodbury solve of eq. (9) with the arithmetic of cfie_solve, its work space (the
 * rank x m block of the capacitance solve, a packed copy when ldx > N, the padded circulant
 * block when N is not a power of two, the GEMMs' split-K partial products) taken from one
 * fixed 64 MiB device array that the library holds per device until the process ends.  The
 * right-hand sides are processed in blocks of as many columns as fit (at most 4096), so the
 * results agree with cfie_solve to rounding (the products' K splits can differ), not
 * bitwise.  Every call on a device shares that device's array and leaves its contents
 * behind; nothing in it needs to start at zero.  Calls that overlap in time on one device
 * (several threads or streams) race on the array and must not be issued.  Arguments,
 * aliasing and the return after the stream drains as for cfie_solve.  Errors: ESTATE
 * before cfie_factor; EINVAL for a mixed-precision context, nrhs < 0, NULL B or X, a
 * leading dimension < N, or when one right-hand side needs more than the fixed array;
 * EHIP if the array's device address could not be resolved or a launch failed. */
cfie_status cfie_solve_noalloc(cfie_ctx *ctx, const void *B_dev, int64_t ldb, void *X_dev,
                               int64_t ldx, int64_t nrhs);

/* Adjoint solve X = C^-H B for nrhs right-hand sides with the same factorisation: with
 * C = C_c + U V^T (Sec. V eqs. (7)-(9)), C^H = C_c^H + V U^H and the Woodbury identity holds
 * with the capacitance matrix K^H and C_c^-H (conjugate eigenvalues), so no new factor is
 * needed.  Used for adjoint sensitivities (g^H C^-1 b = (C^-H g)^H b).  Arguments, aliasing
 * and errors as for cfie_solve; mixed precision refines against C^H in FP64. */
cfie_status cfie_solve_adjoint(cfie_ctx *ctx, const void *B_dev, int64_t ldb, void *X_dev,
                               int64_t ldx, int64_t nrhs);

/* Step A8 (Sec. II eq. (4), Sec. III eq. (5)): right-hand sides b of eq. (5) for unit TE
 * plane waves H_z^inc = exp(i k d.r), d = (cos alpha_j, sin alpha_j); eta cancels.
 * angles_host: host, nrhs doubles.  B_dev: device, complex128, N x nrhs, ldb >= N.
 * ESTATE before assemble. */
cfie_status cfie_plane_wave_rhs(cfie_ctx *ctx, const double *angles_host, int64_t nrhs,
                                void *B_dev, int64_t ldb);

/* Far-field pattern of the field scattered by the surface currents X (Sec. II: the unknown
 * of eq. (5) is the tangential current j_t = sum_i x_i lambda_i; with H_z^tot = -j_t on
 * gamma, Green's representation and the large-argument form of H0 give
 * H_z^s ~ exp(i k r) r^(-1/2) F(phi)), for the directions dhat = (cos phi, sin phi):
 *   F(phi) = -sqrt(k/(8 pi)) exp(-i pi/4) int j_t(s) (dhat.n) exp(-i k dhat.r(s)) ds.
 * X_dev: device, complex128, N x nrhs column-major (ldx >= N).  obs_angles_host: host,
 * n_obs doubles.  F_dev: device, complex128, n_obs x nrhs column-major (ldf >= n_obs):
 * F[o + j ldf] is the far field of column j in direction o.  ESTATE before assemble;
 * EINVAL for negative sizes, NULL pointers or non-finite angles. */
cfie_status cfie_far_field(cfie_ctx *ctx, const void *X_dev, int64_t ldx, int64_t nrhs,
                           const double *obs_angles_host, int64_t n_obs, void *F_dev,
                           int64_t ldf);

/* Reverse-mode derivative, with respect to the contour coefficients, of a real function L of
 * the far fields F = cfie_far_field(X, obs) of the solutions X = C^-1 b of eq. (5) for the
 * plane waves inc_angles_host (as from cfie_plane_wave_rhs and cfie_solve).
 *   dF_dev: dL/dRe F + i dL/dIm F, device, complex128, n_obs x nrhs (lddf >= n_obs);
 *   grad_host: host, 2 (2M+1) doubles: grad[2m] = dL/dRe zhat[m], grad[2m+1] = dL/dIm zhat[m]
 *   in the order of cfie_contour.zhat.
 * It is the derivative of the discrete problem that cfie_assemble defines (nodes uniform in
 * arc length, its quadrature rules, kt through the perimeter): the adjoint lambda = C^-H g
 * comes from cfie_solve_adjoint with the same factorisation; backward kernels of the
 * assembly, of the plane-wave vectors and of the far-field functional give the derivatives
 * with respect to the Gauss points, the element length and kt, which are chained through the
 * arc-length parametrisation to zhat.  C_c does not enter (C^-1 b does not depend on it).
 * Work space: four N x N complex128 matrices of loss weights.  ESTATE before factor; EINVAL
 * for negative sizes, NULL pointers or non-finite angles; nrhs == 0 or n_obs == 0 gives a zero
 * gradient. */
cfie_status cfie_shape_gradient(cfie_ctx *ctx, const double *inc_angles_host, int64_t nrhs,
                                const void *X_dev, int64_t ldx,
                                const double *obs_angles_host, int64_t n_obs,
                                const void *dF_dev, int64_t lddf, double *grad_host);

/* Operators that cfie_apply can apply (Sec. V eqs. (6)-(9)). */
enum {
    CFIE_OP_C = 0,        /* C of eq. (6), factor by factor from the assembled matrices  */
    CFIE_OP_CC = 1,       /* C_c, circulant, by FFT                                        */
    CFIE_OP_CC_INV = 2,   /* C_c^-1 by FFT                                                 */
    CFIE_OP_REMAINDER = 3,/* C - C_c                                                        */
    CFIE_OP_SKELETON = 4, /* U V^T, the compressed remainder (after cfie_factor)            */
    CFIE_OP_C_ADJ = 5     /* C^H, the adjoint of C, factor by factor                           */
};

/* Y = op X in complex128.  X_dev, Y_dev: device, N x nrhs column-major, ldx, ldy >= N,
 * must not overlap.  ESTATE before assemble (before factor for CFIE_OP_SKELETON); EINVAL
 * for an unknown op.  Used for residuals, diagnostics and the tests. */
cfie_status cfie_apply(cfie_ctx *ctx, int op, const void *X_dev, int64_t ldx, void *Y_dev,
                       int64_t ldy, int64_t nrhs);

/* The row transform behind CFIE_SKETCH_SRFT, for checking it: out = A_0 diag(d) F with
 * F_ij = e^{-2 pi i i j / M}, M = the smallest power of two >= N, N = the context's node
 * count, A_0 = A with M - N zero columns appended (ESTATE before cfie_assemble).  A_dev:
 * device, m x N complex128, column-major, lda >= m; d_dev: device, N complex128; out_dev:
 * device, m x M, ldo >= m, must not overlap A_dev.  Column j of A_0 diag(d) F is written to
 * column p of out with j = cfie_srft_frequency(M, p), the digit reversal of the radix
 * passes.  Runs on the context's stream. */
cfie_status cfie_srft_rows(cfie_ctx *ctx, const void *A_dev, int64_t lda, int64_t m,
                           const void *d_dev, void *out_dev, int64_t ldo);
/* The frequency j held at output position p (0 <= p < N) of cfie_srft_rows; -1 if N is not
 * a power of two or p is out of range. */
int64_t cfie_srft_frequency(int64_t n, int64_t p);

/* Copy one internal matrix (CFIE_MAT_*) to dst_dev (device, complex128, column-major,
 * leading dimension ld >= N).  ESTATE if it does not exist yet. */
cfie_status cfie_export_matrix(cfie_ctx *ctx, int which, void *dst_dev, int64_t ld);

cfie_status cfie_query(const cfie_ctx *ctx, cfie_info *out);

/* Text for the last non-OK status on ctx (or for errors of cfie_create if ctx is NULL);
 * valid until the next call on ctx. */
const char *cfie_last_error(const cfie_ctx *ctx);

const char *cfie_status_string(cfie_status s);

/* Release every device buffer of ctx.  NULL is ignored. */
void cfie_destroy(cfie_ctx *ctx);

/* One problem of a batch: a contour, its wavenumber and its plane waves (Sec. II-V). */
typedef struct {
    cfie_contour contour;     /* as for cfie_assemble; read during the call only          */
    double k;                 /* wavenumber                                                */
    const double *angles_host;/* host, nrhs plane-wave directions (cfie_plane_wave_rhs)    */
    int64_t nrhs;             /* >= 0                                                      */
    void *X_dev;              /* device, complex128, N x nrhs column-major (ld = N):
                                 receives the solutions j = C^-1 b of eq. (5)             */
    /* filled by the call */
    int32_t status;           /* cfie_status of this problem                               */
    int32_t rank;             /* skeleton rank                                             */
    double refine_residual;   /* mixed precision: final max relative residual              */
    double t_ms;              /* host wall time of this problem (assemble..solve)          */
} cfie_batch_item;

/* Solve many independent problems (uneven N, their own right-hand-side sets) on one device:
 * each item runs the whole path (cfie_assemble, cfie_factor, cfie_plane_wave_rhs,
 * cfie_solve) with the options opt, and the items are spread, largest first, over n_streams
 * HIP streams (default priority, created and destroyed by the call) driven by as many host
 * threads, so that the small problems of a batch run concurrently on the device.  Each
 * item's device buffers are released when it completes.  Returns CFIE_OK when every item
 * returned OK or a warning, else the first error; per-item results in items[i].  EINVAL for
 * n_items < 0, n_streams < 1 or > 16, or a NULL items array with n_items > 0. */
cfie_status cfie_solve_batch(const cfie_options *opt, int device, int n_streams,
                             cfie_batch_item *items, int64_t n_items);

/* Step A6 (+ A7) of eq. (9) (Sec. V) for many factored problems in one recorded launch: the
 * solves of the n contexts ctxs[i] (X_i = C_i^-1 B_i, nrhs[i] columns, device complex128
 * N_i x nrhs[i] column-major with leading dimensions ldb[i], ldx[i] >= N_i; B == X allowed)
 * are recorded as one HIP graph, one independent branch per context between a fork and a
 * join (each branch with buffers of its own, allocated before recording and released before
 * the call returns), and launched once on a stream the call creates.  An FP64 context's
 * branch is its Woodbury solve (circulant inverse by FFT, the two products), bitwise equal to
 * cfie_solve; a mixed-precision context's branch holds `sweeps` refinement sweeps (complex64
 * Woodbury solve of the residual, FP64 residual against the assembled operator) -- the same
 * arithmetic as cfie_solve, so equal to it when cfie_solve takes that many sweeps -- after
 * which contexts above refine_tol continue sweeping directly, up to max_refine in all
 * (a member records min(sweeps, max_refine) sweeps; cfie_query reports the sweeps and
 * residual of each).  The members' own streams are
 * synchronised before recording and the call returns when every solve has completed.
 * Contexts must be distinct, factored and on one device; members with nrhs[i] == 0 are
 * skipped.  Errors: EINVAL for n < 0, NULL arrays, a NULL or repeated context, contexts on
 * different devices, sweeps < 1 or > 64, nrhs[i] < 0 or > 4096, NULL B or X, leading
 * dimension < N; ESTATE before cfie_factor (message on that context); ENOCONV if some mixed member
 * did not reach refine_tol (its X holds the last iterate); EHIP/ENOMEM otherwise (message on
 * ctxs[0] unless it names another context). */
cfie_status cfie_solve_group(cfie_ctx *const *ctxs, int64_t n, const void *const *B_dev,
                             const int64_t *ldb, void *const *X_dev, const int64_t *ldx,
                             const int64_t *nrhs, int32_t sweeps);

/* cfie_solve_batch with every solve in one recorded launch: each item is assembled, factored
 * and given its plane-wave right-hand sides (in X_dev) as in cfie_solve_batch, its context
 * kept; then the solves of all items run through cfie_solve_group (in place, `sweeps`
 * recorded refinement sweeps for mixed precision) and the contexts are released.  All items'
 * contexts are alive together, so device memory holds every problem's matrices at once.
 * t_ms covers each item's path up to its right-hand sides.  Errors as for cfie_solve_batch,
 * and EINVAL for sweeps < 1 or > 64 or an item with nrhs > 4096. */
cfie_status cfie_solve_batch_grouped(const cfie_options *opt, int device, int n_streams,
                                     cfie_batch_item *items, int64_t n_items, int32_t sweeps);

/* A batch recorded as one HIP graph (the whole path of every problem in one launch). */
typedef struct cfie_batch cfie_batch;

/* Sec. II-V for many problems at once, recorded for one launch per batch.  Each item (as for
 * cfie_solve_batch; nrhs <= 4096, X_dev its N x nrhs solutions with ld = N) is first run once
 * on a HIP stream of its own with opt -- assembly, the adaptive randomized skeleton and LU,
 * the plane-wave right-hand sides, the solve (mixed precision: refinement until refine_tol)
 * -- which writes its solutions and fills status, rank, refine_residual and t_ms.  That run
 * records the sketch's block schedule (block widths, directions kept per block, Gram-Schmidt
 * passes, where it stopped) and the number of refinement sweeps, and keeps every work
 * buffer.  Then the whole batch is recorded as one HIP graph: a fork, one branch per item
 * that replays its path from the schedule with no host interaction (assembly, skeleton with
 * the recorded block widths and kept counts, capacitance LU, right-hand sides, solve with
 * the recorded sweep count), a join.  The items' contours, wavenumbers, angles and X_dev are
 * fixed by this call.  Device memory holds every item's matrices and buffers until
 * cfie_batch_destroy.  Errors: EINVAL for NULL arguments, n_items < 1, an item with nrhs
 * outside [0, 4096] or NULL X_dev / angles_host; any error of an item's path (message via
 * cfie_last_error(NULL)); EHIP if recording fails.  *out is set only on success.
 * DISABLED in this version: after the argument checks it returns EHIP (message via
 * cfie_last_error(NULL)) without any HIP call, because the recording has ended its host
 * process with a segmentation fault on the device for a cause not yet found. */
cfie_status cfie_batch_record(const cfie_options *opt, int device, cfie_batch_item *items,
                              int64_t n_items, cfie_batch **out);

/* One launch of the recorded batch: every item's whole path runs again on the device and its
 * solutions are written to the X_dev given to cfie_batch_record.  Device-side checks compare
 * each replay with its plan: a block whose kept count differs from the recorded one, or a
 * final block whose remainder is not below tau, gives ENOCONV for that item (its result is
 * then not to be used); a zero pivot ESINGULAR; mixed precision above refine_tol after the
 * recorded sweeps ENOCONV.  items (the same n_items as recorded) receive status, rank,
 * refine_residual and t_ms (the launch's wall time).  Returns the first item error, else OK. */
cfie_status cfie_batch_launch(cfie_batch *b, cfie_batch_item *items, int64_t n_items);

/* Number of nodes of the recorded graph (0 for NULL). */
int64_t cfie_batch_nodes(const cfie_batch *b);

/* Release the graph, the streams and every item's device buffers.  NULL is ignored. */
void cfie_batch_destroy(cfie_batch *b);

#ifdef __cplusplus
}
#endif
#endif /* CFIE_H */
