"""MI355X fast direct solver for the preconditioned 2D TE CFIE (Python front end).

    s = Solver(compress_tol=1e-10)
    s.assemble(zhat, n_nodes, k)       # steps A1-A3: geometry, BEM matrices, C_c spectrum
    s.factor()                          # steps A4-A5: randomized skeleton, capacitance LU
    B = s.plane_wave_rhs(angles)        # step A8: right-hand sides of the preconditioned CFIE
    X = s.solve(B)                      # step A6 (+ A7 refinement in mixed precision)

    X_list, results = solve_batch(problems)   # many contours of uneven N at once
    F = s.far_field(X, obs)             # far field of the currents (m, n_obs)
    g = s.shape_gradient(angles, X, obs, dF)  # d loss / d zhat for dF = d loss / d F
    F = far_field_of_shape(zhat_ri, N, k, angles, obs)   # the same as a torch.autograd op

Batches are (m, N) complex128 CUDA tensors (row j = right-hand side j).  The compute runs
in libcfie.so; torch is used for device memory and the current stream only.
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _lib
from ._lib import (CFIE_FP64, CFIE_MIXED, CfieError, MAT_CC_EIG, MAT_CIRCLE_ROW, MAT_DK,
                   MAT_DKT, MAT_G, MAT_NK, MAT_SKT, OP_C, OP_C_ADJ, OP_CC, OP_CC_INV,
                   OP_REMAINDER, OP_SKELETON, REFINE_DENSE, REFINE_FACTORED, REMAINDER_AUTO,
                   REMAINDER_DENSE, REMAINDER_FACTORED, SKETCH_GAUSSIAN, SKETCH_SRFT)

__all__ = ["Solver", "solve_batch", "solve_group", "RecordedBatch", "far_field_of_shape", "CfieError", "CFIE_FP64", "CFIE_MIXED", "MAT_G", "MAT_DK",
           "MAT_NK", "MAT_DKT", "MAT_SKT", "MAT_CC_EIG", "MAT_CIRCLE_ROW", "OP_C", "OP_CC",
           "OP_CC_INV", "OP_REMAINDER", "OP_SKELETON", "OP_C_ADJ", "load_library", "REMAINDER_AUTO", "REMAINDER_FACTORED", "REFINE_FACTORED", "REFINE_DENSE",
           "REMAINDER_DENSE", "SKETCH_GAUSSIAN", "SKETCH_SRFT", "srft_frequency",
           "set_gemm_autotune", "gemm_tuned_classes"]


def load_library():
    return _lib.load()


def set_gemm_autotune(enabled: bool) -> bool:
    """Process-wide GEMM tile autotuner switch (cfie_set_gemm_autotune); returns the
    previous setting.  The tile shapes give bitwise identical results."""
    return bool(_lib.load().cfie_set_gemm_autotune(1 if enabled else 0))


def set_gemm_wide(enabled: bool) -> bool:
    """Process-wide switch of the wide 128 x 128 complex128 GEMM tile (cfie_set_gemm_wide);
    returns the previous setting.  Bitwise identical results either way."""
    return bool(_lib.load().cfie_set_gemm_wide(1 if enabled else 0))


def gemm_tuned_classes() -> int:
    return int(_lib.load().cfie_gemm_tuned_classes())


def srft_frequency(n: int, p: int) -> int:
    """Frequency held at output position p of the row transform (cfie_srft_frequency)."""
    return int(_lib.load().cfie_srft_frequency(n, p))


def _torch():
    import torch
    return torch


def _ptr(t) -> int:
    return t.data_ptr()


class Solver:
    """One problem (contour, N, k) on one HIP device."""

    def __init__(self, precision: int = CFIE_FP64, compress_tol: float = 1e-10,
                 block: int = 128, max_rank: int = 0, seed: int = 1,
                 refine_tol: float = 1e-8, max_refine: int = 20, quad_far: int = 5,
                 quad_near: int = 10, near_band: int = 6, fail_alloc_after: int = -1,
                 profile: bool = False, remainder_form: int = 0, solve_graphs: bool = False,
                 oversample: int = 16, refine_form: int = 0, test_matrix: int = 1,
                 device: int = 0, stream=None):
        lib = _lib.load()
        torch = _torch()
        o = _lib.default_options()
        o.precision = precision
        o.compress_tol = compress_tol
        o.block = block
        o.max_rank = max_rank
        o.seed = seed
        o.refine_tol = refine_tol
        o.max_refine = max_refine
        o.quad_far = quad_far
        o.quad_near = quad_near
        o.near_band = near_band
        o.fail_alloc_after = fail_alloc_after
        o.profile = 1 if profile else 0
        o.remainder_form = remainder_form
        o.solve_graphs = 1 if solve_graphs else 0
        o.oversample = oversample
        o.refine_form = refine_form
        o.test_matrix = test_matrix
        self.device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self._stream = stream
        handle = ctypes.c_void_p()
        st = lib.cfie_create(ctypes.byref(o), device, ctypes.c_void_p(stream.cuda_stream),
                             ctypes.byref(handle))
        if st != 0:
            raise CfieError(st, "cfie_create", lib.cfie_last_error(None).decode())
        self._h = handle
        self._lib = lib
        self.N = 0
        self.warning = None

    # -- helpers ------------------------------------------------------------------------------
    def _check(self, st: int, where: str):
        if st == 0:
            return
        msg = self._lib.cfie_last_error(self._h).decode()
        if st >= 100:
            self.warning = (st, msg)
            return
        raise CfieError(st, where, msg)

    def close(self):
        if getattr(self, "_h", None):
            self._lib.cfie_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _batch(self, m):
        torch = _torch()
        return torch.empty((m, self.N), dtype=torch.complex128, device=self.device)

    @staticmethod
    def _check_batch(t, N, name):
        torch = _torch()
        if t.dtype != torch.complex128 or not t.is_cuda or t.dim() != 2 or t.shape[1] != N:
            raise ValueError(f"{name} must be a (m, {N}) complex128 CUDA tensor")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")

    # -- API ------------------------------------------------------------------------------------
    def assemble(self, zhat, n_nodes: int, k: float):
        z = np.ascontiguousarray(np.asarray(zhat, dtype=np.complex128))
        flat = np.ascontiguousarray(z.view(np.float64))
        c = _lib.Contour(n_nodes, (z.size - 1) // 2,
                         flat.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        self.warning = None
        self._check(self._lib.cfie_assemble(self._h, ctypes.byref(c), float(k)),
                    "cfie_assemble")
        self.N = n_nodes
        self._modes = z.size
        return self

    def factor(self):
        self._check(self._lib.cfie_factor(self._h), "cfie_factor")
        return self

    def solve(self, B, out=None):
        self._check_batch(B, self.N, "B")
        m = B.shape[0]
        X = out if out is not None else self._batch(m)
        self._check_batch(X, self.N, "X")
        self._check(self._lib.cfie_solve(self._h, _ptr(B), self.N, _ptr(X), self.N, m),
                    "cfie_solve")
        return X

    def solve_noalloc(self, B, out=None):
        """X = C^-1 B like solve, through cfie_solve_noalloc: the library allocates no device
        memory in the call (its work space is a fixed per-device array); FP64 contexts only.
        The caller's B and X (allocated here when out is None) are the only buffers."""
        self._check_batch(B, self.N, "B")
        m = B.shape[0]
        X = out if out is not None else self._batch(m)
        self._check_batch(X, self.N, "X")
        self._check(self._lib.cfie_solve_noalloc(self._h, _ptr(B), self.N, _ptr(X), self.N,
                                                 m), "cfie_solve_noalloc")
        return X

    def solve_adjoint(self, B, out=None):
        """X = C^-H B with the same factorisation (cfie_solve_adjoint)."""
        self._check_batch(B, self.N, "B")
        m = B.shape[0]
        X = out if out is not None else self._batch(m)
        self._check_batch(X, self.N, "X")
        self._check(self._lib.cfie_solve_adjoint(self._h, _ptr(B), self.N, _ptr(X), self.N,
                                                 m), "cfie_solve_adjoint")
        return X

    def plane_wave_rhs(self, angles, out=None):
        a = np.ascontiguousarray(np.asarray(angles, dtype=np.float64))
        B = out if out is not None else self._batch(a.size)
        self._check(self._lib.cfie_plane_wave_rhs(
            self._h, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), a.size, _ptr(B),
            self.N), "cfie_plane_wave_rhs")
        return B

    def far_field(self, X, obs_angles, out=None):
        """Far field F[j, o] of the currents X[j] in the directions obs_angles
        (cfie_far_field); X is (m, N) complex128, the result (m, n_obs) complex128."""
        torch = _torch()
        self._check_batch(X, self.N, "X")
        a = np.ascontiguousarray(np.asarray(obs_angles, dtype=np.float64).ravel())
        m = X.shape[0]
        F = out if out is not None else torch.empty((m, a.size), dtype=torch.complex128,
                                                    device=self.device)
        if F.shape != (m, a.size) or F.dtype != torch.complex128 or not F.is_contiguous():
            raise ValueError("F must be a contiguous (m, n_obs) complex128 tensor")
        self._check(self._lib.cfie_far_field(
            self._h, _ptr(X), self.N, m, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
            a.size, _ptr(F), a.size), "cfie_far_field")
        return F

    def shape_gradient(self, inc_angles, X, obs_angles, dF):
        """d loss / d zhat (real view: (2M+1, 2) float64 array of d/dRe, d/dIm) for a real
        loss of F = far_field(X, obs_angles), X the solutions for the plane waves inc_angles,
        given dF = d loss/d Re F + i d loss/d Im F as an (m, n_obs) complex128 tensor
        (cfie_shape_gradient)."""
        torch = _torch()
        self._check_batch(X, self.N, "X")
        inc = np.ascontiguousarray(np.asarray(inc_angles, dtype=np.float64).ravel())
        obs = np.ascontiguousarray(np.asarray(obs_angles, dtype=np.float64).ravel())
        m = X.shape[0]
        if inc.size != m:
            raise ValueError("one incident angle per row of X")
        if dF.shape != (m, obs.size) or dF.dtype != torch.complex128 or not dF.is_contiguous():
            raise ValueError("dF must be a contiguous (m, n_obs) complex128 tensor")
        grad = np.zeros((self._modes, 2))
        dp = ctypes.POINTER(ctypes.c_double)
        self._check(self._lib.cfie_shape_gradient(
            self._h, inc.ctypes.data_as(dp), m, _ptr(X), self.N, obs.ctypes.data_as(dp),
            obs.size, _ptr(dF), obs.size, grad.ctypes.data_as(dp)), "cfie_shape_gradient")
        return grad

    def apply(self, op: int, X):
        """Y = op X for op in OP_C, OP_CC, OP_CC_INV, OP_REMAINDER, OP_SKELETON, OP_C_ADJ."""
        self._check_batch(X, self.N, "X")
        Y = self._batch(X.shape[0])
        self._check(self._lib.cfie_apply(self._h, op, _ptr(X), self.N, _ptr(Y), self.N,
                                         X.shape[0]), "cfie_apply")
        return Y

    def apply_C(self, X):
        return self.apply(OP_C, X)

    def export_matrix(self, which: int):
        """Matrix as a torch tensor in natural (row, column) indexing."""
        torch = _torch()
        cols = {MAT_CC_EIG: 1, MAT_CIRCLE_ROW: 4}.get(which, self.N)
        buf = torch.empty((cols, self.N), dtype=torch.complex128, device=self.device)
        self._check(self._lib.cfie_export_matrix(self._h, which, _ptr(buf), self.N),
                    "cfie_export_matrix")
        return buf.t() if cols == self.N else buf

    def srft_rows(self, A, d):
        """A_0 diag(d) F (F_ij = e^{-2 pi i i j / M}, M the smallest power of two >= N, A_0 =
        A with M - N zero columns appended), its columns at the digit-reversed positions of
        cfie_srft_rows (column p holds frequency srft_frequency(M, p)).  A: (m, N) complex128
        CUDA tensor in natural (row, column) indexing, d: N complex128.  Returns an (m, M)
        tensor in natural indexing."""
        torch = _torch()
        self._check_batch(A, self.N, "A")
        if d.dtype != torch.complex128 or d.numel() != self.N or not d.is_contiguous():
            raise ValueError("d must be a contiguous complex128 tensor of N entries")
        m = A.shape[0]
        M = 1
        while M < self.N:
            M *= 2
        out = torch.empty((M, m), dtype=torch.complex128, device=self.device)
        # column-major m x N: A's transpose view is that matrix with leading dimension m
        At = A.t().contiguous()
        self._check(self._lib.cfie_srft_rows(self._h, _ptr(At), max(m, 1), m, _ptr(d),
                                             _ptr(out), max(m, 1)), "cfie_srft_rows")
        return out.t()

    def info(self) -> dict:
        i = _lib.Info()
        self._check(self._lib.cfie_query(self._h, ctypes.byref(i)), "cfie_query")
        out = {}
        for f, _ in i._fields_:
            v = getattr(i, f)
            out[f] = list(v) if f.startswith("prof_") or f == "t_factor_phase_ms" else v
        return out

    def profile(self) -> dict:
        """Per-kernel launch totals: {name: (launches, work, ms)}."""
        inf = self.info()
        return {n: (inf["prof_launches"][i], inf["prof_work"][i], inf["prof_ms"][i])
                for i, n in enumerate(_lib.PROF_NAMES)}

    def profile_reset(self):
        self._check(self._lib.cfie_profile_reset(self._h), "cfie_profile_reset")


class _FarFieldOfShape:
    """torch.autograd.Function built lazily (torch is imported on first use)."""
    fn = None

    @classmethod
    def get(cls):
        if cls.fn is None:
            torch = _torch()

            class FarFieldOfShape(torch.autograd.Function):
                @staticmethod
                def forward(ctx, zhat_ri, n_nodes, k, inc_angles, obs_angles, options):
                    z = zhat_ri.detach().cpu().numpy()
                    zhat = z[:, 0] + 1j * z[:, 1]
                    s = Solver(**(options or {}))
                    s.assemble(zhat, int(n_nodes), float(k))
                    s.factor()
                    X = s.solve(s.plane_wave_rhs(inc_angles))
                    F = s.far_field(X, obs_angles)
                    ctx.state = (s, X, np.asarray(inc_angles), np.asarray(obs_angles),
                                 zhat_ri.dtype, zhat_ri.device)
                    return F

                @staticmethod
                def backward(ctx, dF):
                    s, X, inc, obs, dt, dev = ctx.state
                    g = s.shape_gradient(inc, X, obs, dF.contiguous())
                    ctx.state = None
                    return torch.as_tensor(g, dtype=dt, device=dev), None, None, None, None, None

            cls.fn = FarFieldOfShape
        return cls.fn


def far_field_of_shape(zhat_ri, n_nodes: int, k: float, inc_angles, obs_angles, **options):
    """Differentiable far field of the scattered field for the contour zhat_ri.

    zhat_ri: (2M+1, 2) float64 tensor of the contour's Fourier coefficients (real and
    imaginary parts); returns F (m, n_obs) complex128 on the GPU, F[j, o] the far field of
    the plane wave inc_angles[j] in the direction obs_angles[o].  The forward pass runs the
    whole solver (assemble, factor, right-hand sides, solve, far field); the backward pass is
    cfie_shape_gradient (adjoint solve with the same factorisation and the backward kernels
    of the assembly)."""
    return _FarFieldOfShape.get().apply(zhat_ri, n_nodes, k, inc_angles, obs_angles, options)


def solve_group(solvers, rhs, sweeps: int = 2, out=None):
    """X_i = C_i^-1 B_i for many factored solvers in one recorded launch (cfie_solve_group).

    solvers: distinct factored Solver objects on one device; rhs: one (m_i, N_i) complex128
    CUDA tensor per solver (m_i <= 4096); sweeps: refinement sweeps recorded for
    mixed-precision solvers.  Returns the list of solutions (out, if given, in place)."""
    torch = _torch()
    lib = _lib.load()
    n = len(solvers)
    if len(rhs) != n or (out is not None and len(out) != n):
        raise ValueError("one right-hand-side batch (and output) per solver")
    outs = []
    for i, (s, B) in enumerate(zip(solvers, rhs)):
        Solver._check_batch(B, s.N, "B")
        X = out[i] if out is not None else s._batch(B.shape[0])
        Solver._check_batch(X, s.N, "X")
        outs.append(X)
    vp, i64 = ctypes.c_void_p, ctypes.c_int64
    hs = (vp * n)(*[s._h.value for s in solvers])
    bs = (vp * n)(*[B.data_ptr() if B.numel() else None for B in rhs])
    xs = (vp * n)(*[X.data_ptr() if X.numel() else None for X in outs])
    lds = (i64 * n)(*[s.N for s in solvers])
    ms = (i64 * n)(*[B.shape[0] for B in rhs])
    st = lib.cfie_solve_group(hs, n, bs, lds, xs, lds, ms, int(sweeps))
    if st != 0:
        msg = lib.cfie_last_error(solvers[0]._h).decode() if n else ""
        raise CfieError(st, "cfie_solve_group", msg)
    return outs


def _batch_items(problems, device, torch):
    """ctypes batch items for problems (dicts with zhat, n_nodes, k, angles), the solution
    tensors they point at and the host arrays that must outlive the call."""
    n = len(problems)
    items = (_lib.BatchItem * n)()
    keep, sols = [], []
    for i, pr in enumerate(problems):
        zh = np.ascontiguousarray(np.asarray(pr["zhat"], dtype=np.complex128))
        zbuf = np.ascontiguousarray(np.stack([zh.real, zh.imag], axis=-1).reshape(-1))
        ang = np.ascontiguousarray(np.asarray(pr["angles"], dtype=np.float64))
        N = int(pr["n_nodes"])
        X = torch.empty((ang.size, N), dtype=torch.complex128, device=f"cuda:{device}")
        keep += [zbuf, ang]
        sols.append(X)
        it = items[i]
        it.contour.n_nodes = N
        it.contour.n_modes = (zh.size - 1) // 2
        it.contour.zhat = zbuf.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        it.k = float(pr["k"])
        it.angles_host = ang.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        it.nrhs = ang.size
        it.X_dev = X.data_ptr() if ang.size else None
    return items, sols, keep


def _batch_results(items):
    return [dict(status=it.status, rank=it.rank, refine_residual=it.refine_residual,
                 t_ms=it.t_ms) for it in items]


class RecordedBatch:
    """Many problems recorded as one HIP graph (cfie_batch_record): the constructor runs every
    problem once (planning; `solutions` and `results` hold that run's output) and records the
    batch; launch() runs every problem's whole path -- assembly, skeleton, LU, right-hand sides,
    solve -- in one graph launch, writing `solutions` again, and returns the per-problem
    results (status 0 when the replay reproduced its plan).

    Disabled in this version: cfie_batch_record reports CFIE_EHIP (recording ended the host
    process with a segmentation fault on the GPU, cause not yet found), so the constructor
    raises CfieError."""

    def __init__(self, problems, precision: int = CFIE_FP64, compress_tol: float = 1e-10,
                 block: int = 128, refine_tol: float = 1e-8, device: int = 0, **options):
        torch = _torch()
        self._lib = lib = _lib.load()
        o = _lib.default_options()
        o.precision = precision
        o.compress_tol = compress_tol
        o.block = block
        o.refine_tol = refine_tol
        for key, val in options.items():
            setattr(o, key, val)
        self._items, self.solutions, self._keep = _batch_items(problems, device, torch)
        torch.cuda.synchronize(device)
        h = ctypes.c_void_p()
        st = lib.cfie_batch_record(ctypes.byref(o), device, self._items, len(problems),
                                   ctypes.byref(h))
        if st != 0:
            raise CfieError(st, "cfie_batch_record", lib.cfie_last_error(None).decode())
        self._h = h
        self.results = _batch_results(self._items)
        self.nodes = int(lib.cfie_batch_nodes(h))

    def launch(self):
        st = self._lib.cfie_batch_launch(self._h, self._items, len(self._items))
        self.results = _batch_results(self._items)
        if st != 0:
            raise CfieError(st, "cfie_batch_launch", self._lib.cfie_last_error(None).decode())
        return self.results

    def close(self):
        if getattr(self, "_h", None):
            self._lib.cfie_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def solve_batch(problems, precision: int = CFIE_FP64, compress_tol: float = 1e-10,
                block: int = 128, refine_tol: float = 1e-8, n_streams: int = 4,
                device: int = 0, grouped: bool = False, sweeps: int = 2, **options):
    """Solve independent problems concurrently (cfie_solve_batch).

    problems: sequence of dicts with keys zhat (Fourier coefficients of the contour), n_nodes,
    k and angles (plane-wave directions).  Returns (solutions, results): solutions[i] is a
    (len(angles), n_nodes) complex128 CUDA tensor, results[i] a dict with status, rank,
    refine_residual and t_ms.  The whole path of every problem runs in the library.
    grouped: the solves of all problems run in one recorded launch after every problem is
    factored (cfie_solve_batch_grouped, `sweeps` recorded refinement sweeps)."""
    torch = _torch()
    lib = _lib.load()
    o = _lib.default_options()
    o.precision = precision
    o.compress_tol = compress_tol
    o.block = block
    o.refine_tol = refine_tol
    for key, val in options.items():
        setattr(o, key, val)
    n = len(problems)
    items, sols, keep = _batch_items(problems, device, torch)
    torch.cuda.synchronize(device)
    if grouped:
        st = lib.cfie_solve_batch_grouped(ctypes.byref(o), device, n_streams, items, n,
                                          int(sweeps))
    else:
        st = lib.cfie_solve_batch(ctypes.byref(o), device, n_streams, items, n)
    results = _batch_results(items)
    if st != 0:
        bad = [i for i in range(n) if results[i]["status"] not in (0, 100)]
        raise CfieError(st, "cfie_solve_batch" + ("_grouped" if grouped else ""),
                        f"items {bad} failed")
    return sols, results
