"""ctypes binding of libcfie.so (argument marshalling only).

Every numerical step runs in the library's HIP kernels; this module only converts Python
arguments to the C ABI of include/cfie.h.  Device buffers are torch CUDA tensors, used as
plain device pointers on the current HIP stream.

Layout: a batch of m right-hand sides is a (m, N) complex128 tensor, contiguous, whose row
j is right-hand side j.  In memory that is the column-major N x m matrix the C ABI takes
(leading dimension N).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libcfie.so")

CFIE_OK, CFIE_EINVAL, CFIE_ENOMEM, CFIE_EHIP, CFIE_ESTATE = 0, 1, 2, 3, 4
CFIE_ESINGULAR, CFIE_ENOCONV, CFIE_WNONCONVEX = 5, 6, 100
CFIE_FP64, CFIE_MIXED = 0, 1
MAT_G, MAT_DK, MAT_NK, MAT_DKT, MAT_SKT, MAT_CC_EIG, MAT_CIRCLE_ROW = range(7)
OP_C, OP_CC, OP_CC_INV, OP_REMAINDER, OP_SKELETON, OP_C_ADJ = range(6)
REFINE_FACTORED, REFINE_DENSE = 0, 1
REMAINDER_AUTO, REMAINDER_FACTORED, REMAINDER_DENSE = 0, 1, 2
SKETCH_GAUSSIAN, SKETCH_SRFT = 0, 1

EXPORTED = [
    "cfie_default_options", "cfie_create", "cfie_assemble", "cfie_factor", "cfie_solve",
    "cfie_plane_wave_rhs", "cfie_apply", "cfie_export_matrix", "cfie_query",
    "cfie_last_error", "cfie_status_string", "cfie_destroy", "cfie_profile_reset",
    "cfie_solve_batch", "cfie_solve_adjoint", "cfie_far_field", "cfie_shape_gradient",
    "cfie_set_gemm_autotune", "cfie_gemm_tuned_classes", "cfie_solve_group",
    "cfie_solve_batch_grouped", "cfie_solve_noalloc", "cfie_set_gemm_wide",
    "cfie_batch_record", "cfie_batch_launch", "cfie_batch_nodes", "cfie_batch_destroy",
    "cfie_srft_rows", "cfie_srft_frequency",
]


class Contour(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int32), ("n_modes", ctypes.c_int32),
                ("zhat", ctypes.POINTER(ctypes.c_double))]


class Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("compress_tol", ctypes.c_double),
                ("block", ctypes.c_int32), ("max_rank", ctypes.c_int32),
                ("seed", ctypes.c_uint64), ("refine_tol", ctypes.c_double),
                ("max_refine", ctypes.c_int32), ("quad_far", ctypes.c_int32),
                ("quad_near", ctypes.c_int32), ("near_band", ctypes.c_int32),
                ("fail_alloc_after", ctypes.c_int64), ("profile", ctypes.c_int32),
                ("remainder_form", ctypes.c_int32), ("solve_graphs", ctypes.c_int32),
                ("oversample", ctypes.c_int32), ("refine_form", ctypes.c_int32),
                ("test_matrix", ctypes.c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("n_nodes", ctypes.c_int32), ("rank", ctypes.c_int32),
                ("perimeter", ctypes.c_double), ("radius", ctypes.c_double),
                ("k", ctypes.c_double), ("ktilde_re", ctypes.c_double),
                ("ktilde_im", ctypes.c_double), ("h", ctypes.c_double),
                ("cc_norm", ctypes.c_double), ("remainder_est", ctypes.c_double),
                ("t_assemble_ms", ctypes.c_double), ("t_factor_ms", ctypes.c_double),
                ("t_solve_ms", ctypes.c_double), ("refine_sweeps", ctypes.c_int32),
                ("refine_residual", ctypes.c_double), ("precision", ctypes.c_int32),
                ("convex", ctypes.c_int32), ("prof_launches", ctypes.c_int64 * 5),
                ("prof_work", ctypes.c_double * 5), ("prof_ms", ctypes.c_double * 5),
                ("t_factor_phase_ms", ctypes.c_double * 4)]

PROF_NAMES = ("zgemm_f64", "zgemm_f32", "assemble_far", "assemble_near", "circ_fft")


class BatchItem(ctypes.Structure):
    _fields_ = [("contour", Contour), ("k", ctypes.c_double),
                ("angles_host", ctypes.POINTER(ctypes.c_double)), ("nrhs", ctypes.c_int64),
                ("X_dev", ctypes.c_void_p), ("status", ctypes.c_int32),
                ("rank", ctypes.c_int32), ("refine_residual", ctypes.c_double),
                ("t_ms", ctypes.c_double)]


_lib = None


def load(path: str = LIB_PATH):
    """Load libcfie.so; raises if the native library is missing (no fallback path)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with __graft_entry__.build()")
    # torch ships its own HIP runtime (loaded by file name); importing it first makes the
    # library bind to that same runtime instead of loading a second one next to it, so that
    # device pointers and streams from torch are valid in the library
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    lib.cfie_default_options.argtypes = [ctypes.POINTER(Options)]
    lib.cfie_default_options.restype = None
    lib.cfie_create.argtypes = [ctypes.POINTER(Options), ctypes.c_int, vp, ctypes.POINTER(vp)]
    lib.cfie_create.restype = i32
    lib.cfie_assemble.argtypes = [vp, ctypes.POINTER(Contour), ctypes.c_double]
    lib.cfie_assemble.restype = i32
    lib.cfie_factor.argtypes = [vp]
    lib.cfie_factor.restype = i32
    lib.cfie_solve.argtypes = [vp, vp, i64, vp, i64, i64]
    lib.cfie_solve.restype = i32
    lib.cfie_solve_noalloc.argtypes = [vp, vp, i64, vp, i64, i64]
    lib.cfie_solve_noalloc.restype = i32
    lib.cfie_solve_adjoint.argtypes = [vp, vp, i64, vp, i64, i64]
    lib.cfie_solve_adjoint.restype = i32
    lib.cfie_plane_wave_rhs.argtypes = [vp, ctypes.POINTER(ctypes.c_double), i64, vp, i64]
    lib.cfie_plane_wave_rhs.restype = i32
    lib.cfie_apply.argtypes = [vp, ctypes.c_int, vp, i64, vp, i64, i64]
    lib.cfie_apply.restype = i32
    lib.cfie_export_matrix.argtypes = [vp, ctypes.c_int, vp, i64]
    lib.cfie_export_matrix.restype = i32
    lib.cfie_query.argtypes = [vp, ctypes.POINTER(Info)]
    lib.cfie_query.restype = i32
    lib.cfie_last_error.argtypes = [vp]
    lib.cfie_last_error.restype = ctypes.c_char_p
    lib.cfie_status_string.argtypes = [i32]
    lib.cfie_status_string.restype = ctypes.c_char_p
    lib.cfie_destroy.argtypes = [vp]
    lib.cfie_destroy.restype = None
    lib.cfie_profile_reset.argtypes = [vp]
    lib.cfie_profile_reset.restype = i32
    lib.cfie_solve_batch.argtypes = [ctypes.POINTER(Options), ctypes.c_int, ctypes.c_int,
                                     ctypes.POINTER(BatchItem), i64]
    lib.cfie_solve_batch.restype = i32
    lib.cfie_solve_batch_grouped.argtypes = [ctypes.POINTER(Options), ctypes.c_int,
                                             ctypes.c_int, ctypes.POINTER(BatchItem), i64, i32]
    lib.cfie_solve_batch_grouped.restype = i32
    i64p = ctypes.POINTER(i64)
    lib.cfie_solve_group.argtypes = [ctypes.POINTER(vp), i64, ctypes.POINTER(vp), i64p,
                                     ctypes.POINTER(vp), i64p, i64p, i32]
    lib.cfie_solve_group.restype = i32
    dp = ctypes.POINTER(ctypes.c_double)
    lib.cfie_far_field.argtypes = [vp, vp, i64, i64, dp, i64, vp, i64]
    lib.cfie_far_field.restype = i32
    lib.cfie_shape_gradient.argtypes = [vp, dp, i64, vp, i64, dp, i64, vp, i64, dp]
    lib.cfie_shape_gradient.restype = i32
    lib.cfie_set_gemm_autotune.argtypes = [ctypes.c_int]
    lib.cfie_set_gemm_autotune.restype = ctypes.c_int
    lib.cfie_batch_record.argtypes = [ctypes.POINTER(Options), ctypes.c_int,
                                      ctypes.POINTER(BatchItem), i64, ctypes.POINTER(vp)]
    lib.cfie_batch_record.restype = i32
    lib.cfie_batch_launch.argtypes = [vp, ctypes.POINTER(BatchItem), i64]
    lib.cfie_batch_launch.restype = i32
    lib.cfie_batch_nodes.argtypes = [vp]
    lib.cfie_batch_nodes.restype = i64
    lib.cfie_batch_destroy.argtypes = [vp]
    lib.cfie_batch_destroy.restype = None
    lib.cfie_set_gemm_wide.argtypes = [ctypes.c_int]
    lib.cfie_set_gemm_wide.restype = ctypes.c_int
    lib.cfie_gemm_tuned_classes.argtypes = []
    lib.cfie_gemm_tuned_classes.restype = ctypes.c_int
    lib.cfie_srft_rows.argtypes = [vp, vp, i64, i64, vp, vp, i64]
    lib.cfie_srft_rows.restype = i32
    lib.cfie_srft_frequency.argtypes = [i64, i64]
    lib.cfie_srft_frequency.restype = i64
    _lib = lib
    return lib


class CfieError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: status {status}: {msg}")
        self.status = status


def default_options() -> Options:
    o = Options()
    load().cfie_default_options(ctypes.byref(o))
    return o
