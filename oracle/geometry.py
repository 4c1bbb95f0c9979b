"""Contour geometry for the oracle (test infrastructure only).

The paper discretises both the scatterer gamma and its equivalent circle with hat functions
that are piecewise linear in the curvilinear abscissa and nodes uniformly spaced in arc
length (Sec. V); gamma is a smooth convex curve (Sec. II).  Here gamma is given by a
trigonometric polynomial z(t) = sum_m zhat_m e^{imt}, counter-clockwise, and the geometry is
exact (no flat panels), so that the Gram matrix is exactly the same on gamma and on the
circle of equal perimeter.

Arc length s(t) = int_0^t |z'(u)| du uses the Fourier series of the speed |z'(t)|, taken from
an FFT on a fine grid (the speed is analytic and periodic, so its coefficients decay
geometrically).  Differences of nearby points are formed from the Fourier series with
e^{ix}-1 written as -2 sin^2(x/2) + i sin x, so that they keep full relative accuracy however
close the two points are; the singular Galerkin integrals need that.
"""
from __future__ import annotations

import math

import numpy as np


def _expm1i(x):
    """e^{ix} - 1 with full relative accuracy for small x."""
    return -2.0 * np.sin(0.5 * x) ** 2 + 1j * np.sin(x)


def _powers(t, m):
    """e^{i m_j t} for the consecutive integer modes m (ascending), by repeated products."""
    t = np.asarray(t, dtype=np.float64)[..., None]
    step = np.exp(1j * t)
    reps = np.broadcast_to(step, t.shape[:-1] + (m.size,)).copy()
    reps[..., 0] = np.exp(1j * t[..., 0] * m[0])
    return np.cumprod(reps, axis=-1)


def _expm1i_modes(delta, m):
    """e^{i m_j delta} - 1 for modes m = 1, 2, ..., by E_{j+1} = E_j + E_1 + E_j E_1,
    which keeps full relative accuracy for small delta."""
    delta = np.asarray(delta, dtype=np.float64)[..., None]
    e1 = _expm1i(delta)[..., 0]
    out = np.empty(delta.shape[:-1] + (m.size,), dtype=np.complex128)
    cur = e1
    out[..., 0] = cur
    for j in range(1, m.size):
        cur = cur + e1 + cur * e1
        out[..., j] = cur
    return out


def _expm1i_minus_ix(x):
    """e^{ix} - 1 - ix with full relative accuracy for small x."""
    x = np.asarray(x, dtype=np.float64)
    re = -2.0 * np.sin(0.5 * x) ** 2
    small = np.abs(x) < 0.5
    im = np.sin(x) - x
    xs = np.where(small, x, 0.0)
    # sin x - x = -x^3/3! + x^5/5! - ...
    x2 = xs * xs
    term = -xs * x2 / 6.0
    acc = term.copy()
    for j in range(2, 12):
        term = -term * x2 / ((2 * j) * (2 * j + 1))
        acc = acc + term
    im = np.where(small, acc, im)
    return re + 1j * im


class Contour:
    """Smooth closed counter-clockwise curve z(t) = sum_{m=-M..M} zhat[m+M] e^{imt}."""

    def __init__(self, zhat, n_fine: int = 8192, tail_tol: float = 3e-17):
        zhat = np.asarray(zhat, dtype=np.complex128)
        if zhat.ndim != 1 or zhat.size % 2 != 1:
            raise ValueError("zhat must have 2M+1 entries")
        self.zhat = zhat
        self.M = (zhat.size - 1) // 2
        self.modes = np.arange(-self.M, self.M + 1, dtype=np.float64)
        n_fine = max(n_fine, 64 * zhat.size)
        t = 2.0 * np.pi * np.arange(n_fine) / n_fine
        speed = np.abs(self.dz(t))
        c = np.fft.rfft(speed) / n_fine
        c0 = c[0].real
        mags = np.abs(c)
        # keep the speed's Fourier modes down to tail_tol relative to the mean, or to twice
        # the rounding noise of the sampled speed (the largest magnitude in the upper half
        # of the sampled spectrum, where the smooth density has none) if that is higher
        noise = mags[n_fine // 4:].max()
        last = np.nonzero(mags > max(tail_tol * c0, 2.0 * noise))[0].max()
        if last > n_fine // 4:
            raise ValueError("arc-length density not resolved; contour too irregular")
        self.speed_c0 = c0
        self.speed_c = c[1:last + 1].copy()           # c_m, m = 1..last (c_{-m} = conj)
        self.speed_m = np.arange(1, last + 1, dtype=np.float64)
        self.L = 2.0 * np.pi * c0

    # --- z and its derivatives -------------------------------------------------------------
    def _phase(self, t):
        return _powers(t, self.modes)

    def z(self, t):
        return self._phase(t) @ self.zhat

    def dz(self, t):
        return self._phase(t) @ (1j * self.modes * self.zhat)

    def d2z(self, t):
        return self._phase(t) @ (-(self.modes ** 2) * self.zhat)

    def speed(self, t):
        return np.abs(self.dz(t))

    # --- arc length --------------------------------------------------------------------------
    def s_of_t(self, t):
        """s(t) = c0 t + sum_{m>=1} 2 Re(c_m (e^{imt}-1)/(im)) for t in [0, 2 pi)."""
        t = np.asarray(t, dtype=np.float64)
        if self.speed_m.size == 0:
            return self.speed_c0 * t
        e = _powers(t, self.speed_m) - 1.0
        return self.speed_c0 * t + 2.0 * np.real(e @ (self.speed_c / (1j * self.speed_m)))

    def ds(self, t, delta):
        """s(t) - s(t - delta), accurate in relative terms for small delta."""
        t = np.asarray(t, dtype=np.float64)
        delta = np.asarray(delta, dtype=np.float64)
        if self.speed_m.size == 0:
            return self.speed_c0 * delta
        e = _powers(t - delta, self.speed_m) * _expm1i_modes(delta, self.speed_m)
        return self.speed_c0 * delta + 2.0 * np.real(e @ (self.speed_c / (1j * self.speed_m)))

    def t_of_s(self, s, iters: int = 40):
        """Invert s(t) by Newton's method (s' = |z'| > 0); two steps past 1e-13."""
        s = np.asarray(s, dtype=np.float64)
        t = 2.0 * np.pi * s / self.L
        extra = 2
        for _ in range(iters):
            step = (self.s_of_t(t) - s) / self.speed(t)
            t = t - step
            if np.all(np.abs(step) < 1e-13 * (1.0 + np.abs(t))):
                extra -= 1
                if extra == 0:
                    break
        return t

    def delta_of_ds(self, t, sigma, iters: int = 50):
        """Parameter offset delta with s(t) - s(t - delta) = sigma (signed arc length)."""
        t = np.asarray(t, dtype=np.float64)
        sigma = np.asarray(sigma, dtype=np.float64)
        d = sigma / self.speed(t)
        extra = 2
        for _ in range(iters):
            step = (self.ds(t, d) - sigma) / self.speed(t - d)
            d = d - step
            if np.all(np.abs(step) <= 1e-13 * np.abs(d)):
                extra -= 1
                if extra == 0:
                    break
        return d

    # --- accurate differences ----------------------------------------------------------------
    def dz_diff(self, t, delta):
        """z(t) - z(t - delta)."""
        ph = _powers(np.asarray(t - delta, dtype=np.float64), self.modes) * _expm1i(
            np.asarray(delta)[..., None] * self.modes)
        return ph @ self.zhat

    def dz_diff_minus_tangent(self, tp, delta):
        """z(tp + delta) - z(tp) - z'(tp) delta."""
        ph = _powers(tp, self.modes) * _expm1i_minus_ix(
            np.asarray(delta)[..., None] * self.modes)
        return ph @ self.zhat

    # --- sanity ------------------------------------------------------------------------------
    def signed_area(self, n: int = 4096):
        t = 2.0 * np.pi * np.arange(n) / n
        z = self.z(t)
        dz = self.dz(t)
        return 0.5 * np.mean(np.imag(np.conj(z) * dz)) * 2.0 * np.pi

    def curvature(self, t):
        d1 = self.dz(t)
        d2 = self.d2z(t)
        return np.imag(np.conj(d1) * d2) / np.abs(d1) ** 3


class Discretisation:
    """N nodes uniform in arc length, s_i = i L / N, starting at t = 0 (Sec. V)."""

    def __init__(self, contour: Contour, N: int):
        if N < 8:
            raise ValueError("N >= 8 required")
        self.contour = contour
        self.N = N
        self.h = contour.L / N
        self._tables = {}
        self._T = None

    def node_params(self):
        """t(s_i) for i = 0..N, with t(s_N) = 2 pi (periodic closure)."""
        if self._T is None:
            s = np.arange(self.N) * self.h
            T = self.contour.t_of_s(s)
            self._T = np.concatenate([T, [2.0 * np.pi + T[0]]])
        return self._T

    def points(self, q: int):
        """Gauss points of every element: dict of (N, q) arrays t, z, dz, speed, tau."""
        if q not in self._tables:
            from .quadrature import gauss01
            xi, w = gauss01(q)
            s = (np.arange(self.N)[:, None] + xi[None, :]) * self.h
            t = self.contour.t_of_s(s.ravel()).reshape(s.shape)
            z = self.contour.z(t)
            dz = self.contour.dz(t)
            sp = np.abs(dz)
            self._tables[q] = dict(xi=xi, w=w, t=t, z=z, tau=dz / sp)
        return self._tables[q]
