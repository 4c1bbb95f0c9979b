"""Spectral diagnostics of C and of C - C_c (test infrastructure only).

Sec. III (Fig. 3) and Sec. V (Fig. 4) discuss the singular values of the preconditioned
matrix C of eq. (6) and of the remainder C - C_c left after the circulant extraction, each
labelled by the spatial frequency of its singular vector.  This module computes them densely:
the SVD (LAPACK through numpy), the label of a singular value as the DFT index (in
[-N/2, N/2)) at which its right singular vector has the largest magnitude, and the exact
rank #{sigma_i > tau} of a truncation at tau.
"""
from __future__ import annotations

import numpy as np


def labelled_spectrum(A: np.ndarray):
    """Singular values (descending) of the square matrix A and the dominant spatial
    frequency of each right singular vector."""
    _, s, Vh = np.linalg.svd(A)
    N = A.shape[1]
    F = np.fft.fft(Vh.conj(), axis=1)
    m = np.argmax(np.abs(F), axis=1)
    m = np.where(m >= (N + 1) // 2, m - N, m)
    return s, m


def exact_rank(s: np.ndarray, tau: float) -> int:
    """Number of singular values strictly above tau."""
    return int(np.count_nonzero(np.asarray(s) > tau))
