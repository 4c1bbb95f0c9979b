"""The preconditioned system and its dense solution (test infrastructure only).

Follows Sec. III, eq. (5) and Sec. V, eq. (6):
  C = (G/2 + D^kt) G^{-1} (G/2 - D^k) + S^kt G^{-1} N^k
  b = -(i k / eta) S^kt G^{-1} e - (G/2 + D^kt) G^{-1} h
with kt = k + 0.4 i k^{1/3} a^{-2/3} (Sec. III).  The radius a is read as L / (2 pi), the
radius of the circle of equal perimeter, which is the arc-length harmonic mean of the radii
of curvature of a convex curve (the curvature integrates to 2 pi); the same kt then serves
the curve and its equivalent circle.

Incident field (TE, e^{-i omega t}, unit amplitude): H_z^inc = e^{i k d.r} with
d = (cos alpha, sin alpha); then E_t^inc = eta (d.n) H_z^inc with t = z x n, so eta cancels:
  e_i / eta = int lambda_i (d.n) e^{i k d.r} ds,   h_i = int lambda_i e^{i k d.r} ds.
G^{-1} is applied by a dense LU solve of G (deliberately not a closed form), and the
solution j of C j = b by a dense LU factorisation (LAPACK zgetrf/zgetrs through scipy).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla

from .assembly import assemble
from .geometry import Contour, Discretisation
from .quadrature import gauss01


def ktilde(k: float, L: float) -> complex:
    a = L / (2.0 * math.pi)
    return complex(k, 0.4 * k ** (1.0 / 3.0) * a ** (-2.0 / 3.0))


def equivalent_circle(L: float) -> np.ndarray:
    """Fourier coefficients of the circle of perimeter L (modes -1..1)."""
    return np.array([0.0, 0.0, L / (2.0 * math.pi)], dtype=np.complex128)


def form_C(M) -> np.ndarray:
    """Eq. (6) from assembled matrices M (dict with G, Dk, Nk, Dkt, Skt)."""
    G = M["G"].astype(np.complex128)
    T1 = np.linalg.solve(G, 0.5 * G - M["Dk"])
    T2 = np.linalg.solve(G, M["Nk"])
    return (0.5 * G + M["Dkt"]) @ T1 + M["Skt"] @ T2


def excitation(zhat, N: int, k: float, angles, q: int = 12):
    """e'/eta and h for plane waves from directions angles (N x m complex each)."""
    disc = Discretisation(Contour(zhat), N)
    P = disc.points(q)
    xi, w = P["xi"], P["w"]
    z, tau = P["z"], P["tau"]
    nrm = -1j * tau                                     # outward normal for a CCW curve
    d = np.exp(1j * np.asarray(angles, dtype=np.float64))
    phase = np.exp(1j * k * np.real(z[:, :, None] * np.conj(d)[None, None, :]))
    dn = np.real(nrm[:, :, None] * np.conj(d)[None, None, :])
    N_ = disc.N
    e = np.zeros((N_, d.size), dtype=np.complex128)
    hh = np.zeros((N_, d.size), dtype=np.complex128)
    for a, phi in enumerate((1.0 - xi, xi)):
        we = disc.h * (w * phi)[None, :, None]
        ce = np.sum(we * dn * phase, axis=1)
        ch = np.sum(we * phase, axis=1)
        rows = (np.arange(N_) + a) % N_
        e[rows] += ce
        hh[rows] += ch
    return e, hh


def rhs(M, e, hh, k: float) -> np.ndarray:
    """Right-hand side of eq. (5) with eta cancelled."""
    G = M["G"].astype(np.complex128)
    return -1j * k * (M["Skt"] @ np.linalg.solve(G, e)) \
        - (0.5 * G + M["Dkt"]) @ np.linalg.solve(G, hh)


def solve_dense(C, b):
    lu = sla.lu_factor(C)
    return sla.lu_solve(lu, b)


class Problem:
    """Everything the oracle knows about one (contour, N, k) problem."""

    def __init__(self, zhat, N: int, k: float, assemble_opts=None, workers: int = 1):
        self.zhat = np.asarray(zhat, dtype=np.complex128)
        self.N = N
        self.k = float(k)
        self.contour = Contour(self.zhat)
        self.L = self.contour.L
        self.kt = ktilde(self.k, self.L)
        self.workers = workers
        self.M = assemble(self.zhat, N, self.k, self.kt, assemble_opts, workers=workers)
        self.C = form_C(self.M)
        self._Mc = None
        self._Cc = None
        self._opts = assemble_opts

    def rhs(self, angles):
        e, hh = excitation(self.zhat, self.N, self.k, angles)
        return rhs(self.M, e, hh, self.k)

    def solve(self, b):
        return solve_dense(self.C, b)

    @property
    def circle(self):
        """Dense matrices on the circle of equal perimeter, same N, k, kt (Sec. V)."""
        if self._Mc is None:
            self._Mc = assemble(equivalent_circle(self.L), self.N, self.k, self.kt,
                                self._opts, workers=self.workers)
        return self._Mc

    @property
    def Cc(self):
        if self._Cc is None:
            self._Cc = form_C(self.circle)
        return self._Cc


def rel_err(x, ref) -> float:
    """max over columns of ||x_j - ref_j||_2 / ||ref_j||_2."""
    x = np.asarray(x).reshape(ref.shape)
    num = np.linalg.norm(x - ref, axis=0)
    den = np.linalg.norm(ref, axis=0)
    return float(np.max(num / den))
