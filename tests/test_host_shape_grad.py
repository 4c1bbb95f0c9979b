"""Host build of the point-pair derivative formulas of the shape gradient (CPU only).

The formulas in csrc/shape_grad.h (used by the backward kernels) are compiled for the host
with g++ and compared with central differences of the pair's loss term as the assembly forms
it: the smooth Gauss rule for separated points, the log-split (moment) rule for touching
elements with the forward's own expressions for A and B, and the coincident-point limits.
Differentiated variables: both points' coordinates and tangents, h, Im kt and curvature.
"""
import ctypes
import os
import subprocess
import tempfile

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
DP = ctypes.POINTER(ctypes.c_double)


@pytest.fixture(scope="module")
def sg():
    out = os.path.join(tempfile.mkdtemp(), "sg.so")
    subprocess.run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-o", out,
                    os.path.join(HERE, "host_shape_grad.cpp")], check=True)
    lib = ctypes.CDLL(out)
    for f in ("sg_smooth", "sg_coincident"):
        getattr(lib, f).restype = ctypes.c_double
        getattr(lib, f).argtypes = [ctypes.c_double, DP, DP, DP]
    lib.sg_split.restype = ctypes.c_double
    lib.sg_split.argtypes = [ctypes.c_double, ctypes.c_double, DP, DP, DP]
    return lib


def _p(a):
    return np.ascontiguousarray(a, dtype=np.float64).ctypes.data_as(DP)


def _fd(fun, p, i, step):
    """Central difference with one Richardson extrapolation."""
    def d(hh):
        e = np.zeros_like(p)
        e[i] = hh
        return (fun(p + e) - fun(p - e)) / (2 * hh)
    return (4 * d(step / 2) - d(step)) / 3


def _geometry(rng, R):
    a, b = rng.uniform(0, 2 * np.pi, 2)
    th = rng.uniform(0, 2 * np.pi)
    xo, yo = rng.normal(size=2)
    return np.array([xo, yo, np.cos(a), np.sin(a), xo - R * np.cos(th), yo - R * np.sin(th),
                     np.cos(b), np.sin(b), 0.01, 0.0, 0.0])


@pytest.mark.parametrize("R,k", [(0.003, 20.0), (0.05, 20.0), (0.4, 40.0), (2.0, 120.0)])
def test_smooth_rule_derivatives(sg, R, k):
    rng = np.random.default_rng(int(R * 1000) + int(k))
    p = _geometry(rng, R)
    p[9] = 0.4 * k ** (1 / 3) * 1.3
    w = rng.normal(size=10)
    g = np.zeros(10)
    sg.sg_smooth(k, _p(p), _p(w), g.ctypes.data_as(DP))
    fun = lambda q: sg.sg_smooth(k, _p(q), _p(w), None)  # noqa: E731
    steps = [1e-4 * R] * 2 + [1e-4] * 2 + [1e-4 * R] * 2 + [1e-4] * 2 + [1e-6, 1e-4]
    fd = np.array([_fd(fun, p, i, steps[i]) for i in range(10)])
    assert np.allclose(g, fd, rtol=1e-6, atol=1e-7 * np.abs(fd).max()), (g, fd)


@pytest.mark.parametrize("R,logl", [(0.002, np.log(0.2)), (0.01, np.log(0.9)),
                                    (0.02, np.log(1.7))])
@pytest.mark.parametrize("k", [15.0, 300.0])
def test_split_rule_derivatives(sg, R, logl, k):
    rng = np.random.default_rng(7)
    p = _geometry(rng, R)
    p[9] = 0.4 * k ** (1 / 3)
    w = rng.normal(size=20)
    g = np.zeros(10)
    sg.sg_split(k, logl, _p(p), _p(w), g.ctypes.data_as(DP))
    fun = lambda q: sg.sg_split(k, logl, _p(q), _p(w), None)  # noqa: E731
    steps = [1e-3 * R] * 2 + [1e-4] * 2 + [1e-3 * R] * 2 + [1e-4] * 2 + [1e-7, 1e-4]
    fd = np.array([_fd(fun, p, i, steps[i]) for i in range(10)])
    assert np.allclose(g, fd, rtol=1e-6, atol=1e-7 * np.abs(fd).max()), (g, fd)


@pytest.mark.parametrize("k", [15.0, 300.0])
def test_coincident_rule_derivatives(sg, k):
    rng = np.random.default_rng(3)
    p = np.zeros(11)
    p[8] = 0.01
    p[9] = 0.4 * k ** (1 / 3)
    p[10] = 1.7
    w = rng.normal(size=20)
    g = np.zeros(3)
    sg.sg_coincident(k, _p(p), _p(w), g.ctypes.data_as(DP))
    fun = lambda q: sg.sg_coincident(k, _p(q), _p(w), None)  # noqa: E731
    fd = np.array([_fd(fun, p, i, s) for i, s in ((8, 1e-6), (9, 1e-4), (10, 1e-4))])
    assert np.allclose(g, fd, rtol=1e-7, atol=1e-9), (g, fd)
