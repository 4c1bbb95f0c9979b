"""Pins of the oracle's far-field functional and reference shape gradient (CPU only).

* The far field of the dense discrete solution on a circle converges to the Mie far field
  (closed form, tests/analytic.py) at a high rate as N doubles.
* The oracle's reference derivative of the backscatter loss with respect to the radius
  (central differences with Richardson extrapolation of the dense solve) converges to the
  derivative of the Mie loss (closed form from Bessel's equation and the Wronskian).
* The loss is invariant under translation of the contour (|F| only changes phase), so the
  derivative with respect to zhat_0 vanishes.
* The differencing routine reproduces the derivative of an analytic function to O(h^6).
* The stored reference gradient (tests/golden/shapegrad128.npz, written by
  tests/golden/make_golden.py from the oracle) agrees with a directional difference of the
  oracle's loss along it, and its stored loss with a fresh evaluation.
"""
import math
import os

import numpy as np
import pytest

import analytic as An
import workloads as W
from oracle import gradient as G
from oracle import system as S

HERE = os.path.dirname(os.path.abspath(__file__))


def test_far_field_converges_to_mie():
    R, k, alpha = 1.0, 10.0, 0.3
    phi = np.linspace(0.0, 2 * np.pi, 13)
    Fm, _ = An.mie_far_field(k, R, phi, alpha)
    errs = []
    for N in (48, 96, 192):
        P = S.Problem(W.circle_coeffs(R), N, k)
        x = P.solve(P.rhs([alpha]))
        F = G.far_field(W.circle_coeffs(R), N, x, phi, k)[:, 0]
        errs.append(np.abs(F - Fm).max() / np.abs(Fm).max())
    assert errs[-1] < 5e-4, errs
    assert errs[0] / errs[1] > 6 and errs[1] / errs[2] > 6, errs


def test_radius_derivative_converges_to_mie():
    R, k, alpha = 1.0, 10.0, 0.3
    obs = W.backscatter_angles([alpha], 181)
    F, dF = An.mie_far_field(k, R, obs[0], alpha)
    dL = float(np.sum(2 * np.real(np.conj(F) * dF)))
    # the closed-form derivative itself against a difference of the closed form
    Fp, _ = An.mie_far_field(k, R + 1e-6, obs[0], alpha)
    Fn, _ = An.mie_far_field(k, R - 1e-6, obs[0], alpha)
    fd = (np.sum(np.abs(Fp) ** 2) - np.sum(np.abs(Fn) ** 2)) / 2e-6
    assert abs(fd - dL) <= 1e-7 * abs(dL)
    errs = []
    for N in (48, 96):
        def loss(p):
            return G.backscatter_loss(np.array([0, 0, p[0]], complex), N, k, [alpha], obs)[0]
        g = G.richardson_gradient(loss, np.array([R]), 1e-2)[0]
        errs.append(abs(g - dL) / abs(dL))
    assert errs[-1] < 3e-3 and errs[0] / errs[1] > 6, errs


def test_loss_is_translation_invariant():
    pr = W.shape_problem(N=64, mmax=4, n_inc=2, n_obs=9, amp=0.05)
    z0, M = pr["zhat"], (pr["zhat"].size - 1) // 2

    def loss(p):
        z = z0.copy()
        z[M] += p[0] + 1j * p[1]
        return G.backscatter_loss(z, 64, pr["k"], pr["angles"], pr["obs"])[0]

    def loss_shape(p):
        z = z0.copy()
        z[M + 3] += p[0]
        return G.backscatter_loss(z, 64, pr["k"], pr["angles"], pr["obs"])[0]

    g_tr = G.richardson_gradient(loss, np.zeros(2), 1e-2)
    g_sh = G.richardson_gradient(loss_shape, np.zeros(1), 1e-3)
    assert abs(g_sh[0]) > 1e-3
    assert np.abs(g_tr).max() <= 1e-9 * abs(g_sh[0]), (g_tr, g_sh)


def test_richardson_gradient_analytic():
    f = lambda p: math.sin(3 * p[0]) * math.exp(p[1]) + p[0] ** 5  # noqa: E731
    p = np.array([0.3, -0.2])
    g = G.richardson_gradient(f, p, 0.05)
    ref = np.array([3 * math.cos(0.9) * math.exp(-0.2) + 5 * 0.3 ** 4,
                    math.sin(0.9) * math.exp(-0.2)])
    assert np.allclose(g, ref, rtol=1e-9, atol=0)


def test_stored_reference_gradient():
    d = np.load(os.path.join(HERE, "golden", "shapegrad128.npz"))
    N, mmax, k = int(d["N"]), int(d["mmax"]), float(d["k"])
    p0 = np.concatenate([d["s"], d["t"]])
    g = d["grad"]

    def loss(p):
        return G.backscatter_loss(W.shape_to_zhat(p[:mmax], p[mmax:]), N, k, d["angles"],
                                  d["obs"], workers=os.cpu_count() or 1)[0]

    assert abs(loss(p0) - float(d["L"])) <= 1e-12 * float(d["L"])
    # the derivative along the stored gradient's direction is its norm
    u = g / np.linalg.norm(g)
    dd = G.richardson_gradient(lambda e: loss(p0 + e[0] * u), np.zeros(1), 1e-3)[0]
    assert abs(dd - np.linalg.norm(g)) <= 1e-8 * np.linalg.norm(g), (dd, np.linalg.norm(g))
