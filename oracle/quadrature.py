"""Quadrature rules on [0, 1] used by the oracle (test infrastructure only).

* Gauss-Legendre: a library primitive (numpy.polynomial.legendre.leggauss), mapped to [0, 1].
* tanh-sinh (double-exponential) rule: u = (1 + tanh(pi/2 sinh x)) / 2 sampled on a uniform
  x-grid.  It integrates functions with integrable endpoint singularities (log u, u log u)
  with exponential convergence, which is how the oracle treats the coincident and adjacent
  element pairs of the Galerkin integrals (Sec. II, eq. (4)) without splitting the kernel.
"""
from __future__ import annotations

import math
from functools import lru_cache

import numpy as np


@lru_cache(maxsize=None)
def gauss01(q: int):
    """Nodes and weights of the q-point Gauss-Legendre rule on [0, 1]."""
    x, w = np.polynomial.legendre.leggauss(q)
    return (0.5 * (x + 1.0)).copy(), (0.5 * w).copy()


@lru_cache(maxsize=None)
def tanh_sinh01(step: float = 1.0 / 8.0, umin: float = 1e-24):
    """tanh-sinh rule on [0, 1].

    Returns (u, w): nodes increasing from about umin to 1 - 1e-16 and their weights.  The
    node u is formed as 1 / (1 + exp(-2y)), y = (pi/2) sinh(x), which keeps full relative
    accuracy for the small nodes that sit next to the singular endpoint u = 0.
    """
    xs = []
    k = 0
    while True:
        x = k * step
        y = 0.5 * math.pi * math.sinh(x)
        if 1.0 / (1.0 + math.exp(2.0 * y)) < 1e-17:
            break
        xs.append(x)
        k += 1
    xs = np.array(xs)
    xs = np.concatenate([-xs[:0:-1], xs])
    y = 0.5 * np.pi * np.sinh(xs)
    u = 1.0 / (1.0 + np.exp(-2.0 * y))
    w = step * 0.25 * np.pi * np.cosh(xs) / np.cosh(y) ** 2
    keep = u >= umin
    return u[keep].copy(), w[keep].copy()
