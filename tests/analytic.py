"""Closed forms that pin the oracle (no part of the solver).

* Continuous spectra of S, D, N on a circle of radius R (mode e^{in phi}):
    s_n = (i pi R / 2) J_n(x) H_n(x)
    d_n = (i pi x / 4) (J_n'(x) H_n(x) + J_n(x) H_n'(x))
    n_n = -(i pi kappa x / 2) J_n'(x) H_n'(x),        x = kappa R
  from the addition theorem for H0^(1).  For |n| >> |x| the products are formed from
  Debye's expansions (DLMF 10.19, coefficients u_k, v_k of DLMF 10.41.9-10), in which the
  exponentially large and small factors cancel exactly.
* Galerkin matrices on a circle with N hats uniform in arc length are circulant, and the
  DFT of their first column is the aliasing sum
    mu_m = h sum_{n = m mod N} a_n sinc^4(pi n / N),   sinc x = sin x / x,
  because the Fourier coefficients of a hat are (1/N) sinc^2(pi n / N).  The slowly decaying
  Laplace parts (R / 2|n| for S, |n| / 2R for N) are summed exactly with Hurwitz zeta.
* The exact PEC-cylinder (Mie) current for TE incidence H_z^inc = e^{ik d.r}:
    j_t(phi) = -H_z^tot = -sum_n i^n 2i / (pi k R H_n'(kR)) e^{in(phi - alpha)}.
* Its far field: H_z^s ~ e^{ikr} r^{-1/2} F(phi) with
    F(phi) = sqrt(2/(pi k)) e^{-i pi/4} sum_n b_n e^{in(phi - alpha)},  b_n = -J_n'(kR)/H_n'(kR)
  (large-argument form of H_n in the scattered field sum_n i^n b_n H_n(kr) e^{in(phi-alpha)}),
  and its radius derivative from Bessel's equation, f'' = -f'/x - (1 - n^2/x^2) f, and the
  Wronskian J_n H_n' - J_n' H_n = 2i/(pi x):  d b_n/dx = (1 - n^2/x^2) (2i/(pi x)) / H_n'^2.
* Gram matrix: G = h circ(2/3, 1/6, ..., 1/6); its inverse has first column
  (6/h) (rho^n + rho^{N-n}) / (2 sqrt 3 (1 - rho^N)),  rho = sqrt 3 - 2.
"""
from __future__ import annotations

from fractions import Fraction
from functools import lru_cache

import numpy as np
import scipy.special as sps


# --------------------------------------------------------------------------------------
# Debye coefficient polynomials u_k(p), v_k(p) as exact rational coefficient lists
# --------------------------------------------------------------------------------------
def _pmul(a, b):
    out = [Fraction(0)] * (len(a) + len(b) - 1)
    for i, x in enumerate(a):
        for j, y in enumerate(b):
            out[i + j] += x * y
    return out


def _padd(a, b):
    n = max(len(a), len(b))
    return [(a[i] if i < len(a) else 0) + (b[i] if i < len(b) else 0) for i in range(n)]


def _pscale(a, c):
    return [x * c for x in a]


def _pder(a):
    return [a[i] * i for i in range(1, len(a))] or [Fraction(0)]


def _pint(a):
    return [Fraction(0)] + [a[i] / (i + 1) for i in range(len(a))]


@lru_cache(maxsize=None)
def debye_coeffs(K: int = 10):
    """u_k, v_k for k = 0..K (DLMF 10.41.9, 10.41.10)."""
    one_m_p2 = [Fraction(1), Fraction(0), Fraction(-1)]
    u = [[Fraction(1)]]
    v = [[Fraction(1)]]
    for k in range(K):
        uk = u[-1]
        # u_{k+1} = 1/2 p^2 (1 - p^2) u_k' + 1/8 int_0^p (1 - 5 t^2) u_k(t) dt
        t1 = _pscale(_pmul([0, 0, Fraction(1)], _pmul(one_m_p2, _pder(uk))), Fraction(1, 2))
        t2 = _pscale(_pint(_pmul([Fraction(1), 0, Fraction(-5)], uk)), Fraction(1, 8))
        un = _padd(t1, t2)
        # v_{k+1} = u_{k+1} - 1/2 p (1 - p^2) u_k - p^2 (1 - p^2) u_k'
        vn = _padd(un, _pscale(_pmul([0, Fraction(1)], _pmul(one_m_p2, uk)), Fraction(-1, 2)))
        vn = _padd(vn, _pscale(_pmul([0, 0, Fraction(1)], _pmul(one_m_p2, _pder(uk))), -1))
        u.append(un)
        v.append(vn)
    uf = [np.array([float(c) for c in a], dtype=np.float64) for a in u]
    vf = [np.array([float(c) for c in a], dtype=np.float64) for a in v]
    return uf, vf


def _poly(c, p):
    return np.polynomial.polynomial.polyval(p, c)


def _debye_products(nu, x):
    """(J Y, J'Y', J'Y, J Y') at order nu >> |x| (x may be complex)."""
    u, v = debye_coeffs()
    w = np.sqrt(1.0 - (x / nu) ** 2 + 0j)        # tanh(alpha)
    p = 1.0 / w                                   # coth(alpha)
    Su_p = sum(_poly(u[k], p) / nu ** k for k in range(len(u)))
    Su_m = sum((-1) ** k * _poly(u[k], p) / nu ** k for k in range(len(u)))
    Sv_p = sum(_poly(v[k], p) / nu ** k for k in range(len(v)))
    Sv_m = sum((-1) ** k * _poly(v[k], p) / nu ** k for k in range(len(v)))
    cosh_a = nu / x
    JY = -Su_p * Su_m / (np.pi * nu * w)
    sinh2a = 2.0 * cosh_a * (cosh_a * w)          # 2 cosh sinh, sinh = cosh tanh
    JpYp = sinh2a / (2.0 * np.pi * nu) * Sv_p * Sv_m
    JpY = -cosh_a / (np.pi * nu) * Sv_p * Su_m
    JYp = cosh_a / (np.pi * nu) * Su_p * Sv_m
    return JY, JpYp, JpY, JYp


def circle_symbols(n, kappa, R, n_switch=None):
    """s_n, d_n, n_n for integer modes n (array) on the circle of radius R."""
    n = np.abs(np.asarray(n, dtype=np.int64))
    x = complex(kappa) * R
    if n_switch is None:
        n_switch = int(max(150, 4 * abs(x) + 60))
    s = np.empty(n.shape, dtype=np.complex128)
    d = np.empty(n.shape, dtype=np.complex128)
    nn = np.empty(n.shape, dtype=np.complex128)
    lo = n <= n_switch
    if np.any(lo):
        m = n[lo].astype(np.float64)
        J = sps.jv(m, x)
        H = sps.hankel1(m, x)
        Jp = sps.jvp(m, x)
        Hp = sps.h1vp(m, x)
        s[lo] = 0.5j * np.pi * R * J * H
        d[lo] = 0.25j * np.pi * x * (Jp * H + J * Hp)
        nn[lo] = -0.5j * np.pi * kappa * x * Jp * Hp
    hi = ~lo
    if np.any(hi):
        m = n[hi].astype(np.float64)
        JY, JpYp, JpY, JYp = _debye_products(m, x)
        # J_n^2, J_n J_n', J_n'^2 are below 1e-100 relative here and are dropped
        s[hi] = 0.5j * np.pi * R * (1j * JY)
        d[hi] = 0.25j * np.pi * x * (1j * (JpY + JYp))
        nn[hi] = -0.5j * np.pi * kappa * x * (1j * JpYp)
    return s, d, nn


def galerkin_circle_eigs(N, kappa, R, L_alias: int = 400):
    """DFT eigenvalues mu_m (m = 0..N-1) of the Galerkin S, D, N matrices on a circle."""
    h = 2.0 * np.pi * R / N
    m = np.arange(N)
    ls = np.arange(-L_alias, L_alias + 1)
    nmat = m[:, None] + ls[None, :] * N
    s, d, nn = circle_symbols(nmat.ravel(), kappa, R)
    s, d, nn = s.reshape(nmat.shape), d.reshape(nmat.shape), nn.reshape(nmat.shape)
    with np.errstate(invalid="ignore", divide="ignore"):
        arg = np.pi * nmat / N
        sinc4 = np.where(nmat == 0, 1.0, (np.sin(arg) / arg) ** 4)
    an = np.abs(nmat).astype(np.float64)
    lap_s = np.where(nmat == 0, 0.0, R / (2.0 * np.where(an == 0, 1, an)))
    lap_n = an / (2.0 * R)
    mu_s = h * np.sum((s - lap_s) * sinc4, axis=1)
    mu_d = h * np.sum(d * sinc4, axis=1)
    mu_n = h * np.sum((nn - lap_n) * sinc4, axis=1)
    # Laplace parts over all n = m mod N, n != 0, summed exactly:
    # sum |n|^{-p} = N^{-p} (zeta(p, m/N) + zeta(p, 1 - m/N)) for 0 < m < N
    frac = m / N
    with np.errstate(divide="ignore", invalid="ignore"):
        z5 = np.where(m == 0, 0.0, sps.zeta(5, np.where(m == 0, 0.5, frac))
                      + sps.zeta(5, np.where(m == 0, 0.5, 1.0 - frac)))
        z3 = np.where(m == 0, 0.0, sps.zeta(3, np.where(m == 0, 0.5, frac))
                      + sps.zeta(3, np.where(m == 0, 0.5, 1.0 - frac)))
    s4 = np.sin(np.pi * frac) ** 4 * (N / np.pi) ** 4
    mu_s = mu_s + h * (R / 2.0) * s4 * z5 / N ** 5
    mu_n = mu_n + h * (1.0 / (2.0 * R)) * s4 * z3 / N ** 3
    mu_g = h * (2.0 + np.cos(2.0 * np.pi * m / N)) / 3.0
    return dict(S=mu_s, D=mu_d, N=mu_n, G=mu_g)


def mie_current(k, R, phi, alpha, nmax=None):
    """Exact surface current j_t(phi) on a PEC circle, TE plane wave from direction alpha."""
    x = k * R
    if nmax is None:
        nmax = int(abs(x) + 40 + 4 * abs(x) ** (1 / 3))
    n = np.arange(-nmax, nmax + 1)
    Hp = sps.h1vp(np.abs(n), x) * np.where(n < 0, (-1.0) ** np.abs(n), 1.0)
    coef = (1j ** n) * 2j / (np.pi * x * Hp)
    ph = np.exp(1j * np.outer(np.asarray(phi) - alpha, n))
    return -(ph @ coef)


def mie_far_field(k, R, phi, alpha, nmax=None):
    """(F, dF/dR) of the PEC circle of radius R for the TE plane wave from direction alpha."""
    x = k * R
    if nmax is None:
        nmax = int(abs(x) + 40 + 4 * abs(x) ** (1 / 3))
    n = np.arange(-nmax, nmax + 1)
    sg = np.where(n < 0, (-1.0) ** np.abs(n), 1.0)
    Jp = sps.jvp(np.abs(n), x) * sg
    Hp = sps.h1vp(np.abs(n), x) * sg
    c = np.sqrt(2.0 / (np.pi * k)) * np.exp(-0.25j * np.pi)
    E = np.exp(1j * np.outer(np.asarray(phi, dtype=np.float64) - alpha, n))
    F = c * (E @ (-Jp / Hp))
    dF = c * (E @ (k * (1.0 - n ** 2 / x ** 2) * (2j / (np.pi * x)) / Hp ** 2))
    return F, dF


def gram_inverse_column(N, h):
    rho = np.sqrt(3.0) - 2.0
    n = np.arange(N)
    return (6.0 / h) * (rho ** n + rho ** (N - n)) / (2.0 * np.sqrt(3.0) * (1.0 - rho ** N))
