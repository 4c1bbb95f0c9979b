"""Far-field functional and the reference shape gradient (test infrastructure only).

Far field.  With H_z^tot = -j_t on the contour (the reading of the TE currents used for
eq. (1)) and d(H_z^tot)/dn = 0 on a perfect conductor, Green's representation of the
scattered field outside gamma is
    H_z^s(r) = - int_gamma j_t(s') dg_k(r, r')/dn' ds',      g_k = (i/4) H0^(1)(k |r - r'|).
For |r| -> infinity in the direction dhat = (cos phi, sin phi), H0^(1)(k|r - r'|) ~
sqrt(2/(pi k |r|)) e^{i(k|r| - pi/4)} e^{-i k dhat.r'}, so H_z^s ~ e^{ik|r|} |r|^{-1/2} F(phi)
with
    F(phi) = -sqrt(k/(8 pi)) e^{-i pi/4} int_gamma j_t(s) (dhat.n(s)) e^{-i k dhat.r(s)} ds,
and j_t = sum_i x_i lambda_i for the discrete solution x of eq. (5).  On a circle this is
the Mie far field sqrt(2/(pi k)) e^{-i pi/4} sum_n (-J_n'(kR)/H_n'(kR)) e^{in(phi-alpha)}.

Loss.  L = sum over the selected (observation angle, incident wave) pairs of |F|^2.

Reference gradient.  dL/dp for real parameters p of the contour by central differences of L,
extrapolated twice (Richardson: D(h) = (L(p+h) - L(p-h)) / 2h has error c2 h^2 + c4 h^4 + ...,
and (4 D(h/2) - D(h)) / 3, then (16 D'(h/4) - D'(h/2)) / 15 remove the h^2 and h^4 terms).
Every evaluation of L is the oracle's own dense assembly and LU solve.
"""
from __future__ import annotations

import math

import numpy as np

from .geometry import Contour, Discretisation
from .system import Problem


def far_field(zhat, N: int, x, obs_angles, k: float, q: int = 12) -> np.ndarray:
    """F[o, j] for the solutions x (N x m) at the angles obs_angles (n_obs,)."""
    disc = Discretisation(Contour(np.asarray(zhat, dtype=np.complex128)), N)
    P = disc.points(q)
    xi, w = P["xi"], P["w"]
    z, tau = P["z"], P["tau"]
    nrm = -1j * tau                                     # outward normal of a CCW curve
    x = np.asarray(x, dtype=np.complex128).reshape(N, -1)
    # current at the Gauss points: element e carries hats e (1 - xi) and e + 1 (xi)
    jq = x[:, None, :] * (1.0 - xi)[None, :, None] + \
        np.roll(x, -1, axis=0)[:, None, :] * xi[None, :, None]
    d = np.exp(1j * np.asarray(obs_angles, dtype=np.float64).ravel())
    dn = np.real(nrm[:, :, None] * np.conj(d)[None, None, :])          # dhat . n
    ph = np.exp(-1j * k * np.real(z[:, :, None] * np.conj(d)[None, None, :]))
    wts = disc.h * w[None, :, None] * dn * ph                          # (N, q, n_obs)
    F = np.einsum("ego,egj->oj", wts, jq)
    return -math.sqrt(k / (8.0 * math.pi)) * np.exp(-0.25j * math.pi) * F


def backscatter_loss(zhat, N: int, k: float, inc_angles, obs, workers: int = 1):
    """L = sum_j sum_o |F(obs[j, o]; wave j)|^2 with the oracle's dense solve; returns
    (L, F) with F[j] the far field of wave j at obs[j]."""
    P = Problem(zhat, N, k, workers=workers)
    x = P.solve(P.rhs(inc_angles))
    obs = np.asarray(obs, dtype=np.float64)
    F = np.stack([far_field(zhat, N, x[:, j:j + 1], obs[j], k)[:, 0]
                  for j in range(x.shape[1])])
    return float(np.sum(np.abs(F) ** 2)), F


def richardson_gradient(fun, p, h: float, idx=None) -> np.ndarray:
    """Central differences of fun at p in each coordinate of idx (default all), with step
    h, h/2, h/4 and two Richardson extrapolations (error O(h^6))."""
    p = np.asarray(p, dtype=np.float64)
    idx = range(p.size) if idx is None else idx
    out = []
    for i in idx:
        D = []
        for hh in (h, h / 2.0, h / 4.0):
            e = np.zeros_like(p)
            e[i] = hh
            D.append((fun(p + e) - fun(p - e)) / (2.0 * hh))
        D1 = [(4.0 * D[1] - D[0]) / 3.0, (4.0 * D[2] - D[1]) / 3.0]
        out.append((16.0 * D1[1] - D1[0]) / 15.0)
    return np.asarray(out)
