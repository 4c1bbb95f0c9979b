"""Host build of the contour geometry and of the log-singular moment tables (CPU only).

csrc/geometry.cpp is compiled for the host with g++ and checked against closed forms:

* the arc-length density: the perimeter of an ellipse (complete elliptic integral of the
  second kind) and its smallest curvature b / a^2;
* the admissibility checks of the contour (Sec. II assumes a simple closed curve; the
  method's equivalent circle needs its orientation): the hypotrochoid
  z = e^{it} + a e^{-2it} is simple for a < 1/2, has cusps (zero tangent) at a = 1/2 and
  three small loops beyond; the limacon (1 + 2 cos t) e^{it} has an inner loop; a contour
  traversed clockwise is refused;
* the moment tables of the product-integration rule for touching and coincident elements
  (Sec. V discretisation): for monomials x^a, y^b of degree below the rule's order q, the sums
  sum_{g,h} x_g^a x_h^b M[g, h] equal the integrals of log(distance) x^a y^b times the hat
  factors, which reduce to harmonic numbers and log 2 (derived in _J and _K below).
"""
import ctypes
import math
import os
import subprocess
import tempfile
from math import comb

import numpy as np
import pytest
from scipy.special import ellipe

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "..", "paper_2203_13283_amd", "csrc")
DP = ctypes.POINTER(ctypes.c_double)


@pytest.fixture(scope="module")
def geo():
    out = os.path.join(tempfile.mkdtemp(), "geo.so")
    subprocess.run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-D__HIP_PLATFORM_AMD__",
                    "-I/opt/rocm/include", "-o", out, os.path.join(HERE, "host_geometry.cpp"),
                    os.path.join(CSRC, "geometry.cpp")], check=True)
    lib = ctypes.CDLL(out)
    lib.geo_build.restype = ctypes.c_int
    lib.geo_build.argtypes = [ctypes.c_int, ctypes.c_int, DP, DP, ctypes.c_char_p, ctypes.c_int]
    lib.geo_log_moments.restype = None
    lib.geo_log_moments.argtypes = [ctypes.c_int, DP]
    return lib


def _build(lib, zhat, n_nodes):
    z = np.ascontiguousarray(np.asarray(zhat, dtype=np.complex128)).view(np.float64)
    M = (len(zhat) - 1) // 2
    out = np.zeros(5)
    err = ctypes.create_string_buffer(256)
    rc = lib.geo_build(n_nodes, M, z.ctypes.data_as(DP), out.ctypes.data_as(DP), err, 256)
    return rc, out, err.value.decode()


def _hypotrochoid(a):
    return [a, 0, 0, 1, 0]                     # zhat_{-2..2}: e^{it} + a e^{-2it}


@pytest.mark.parametrize("a,b,N", [(1.5, 0.5, 4096), (1.0, 0.2, 1000), (2.0, 1.9, 64)])
def test_ellipse_perimeter_and_curvature(geo, a, b, N):
    rc, out, err = _build(geo, [(a - b) / 2, 0, (a + b) / 2], N)
    assert rc == 0, err
    L = 4 * a * ellipe(1 - (b / a) ** 2)
    assert abs(out[1] - L) <= 1e-13 * L
    assert abs(out[0] - L / (2 * math.pi)) <= 1e-13 * L
    assert abs(out[2] - b / a ** 2) <= 1e-12 * b / a ** 2       # at t = 0, a grid point
    assert out[3] == 1.0


def test_circle_has_one_speed_mode_or_none(geo):
    rc, out, err = _build(geo, [0, 0, 1.7], 128)
    assert rc == 0, err
    assert abs(out[1] - 2 * math.pi * 1.7) <= 1e-14 * 2 * math.pi * 1.7
    assert out[4] == 0                        # constant speed: no retained modes


@pytest.mark.parametrize("N", [64, 4096, 16384])
def test_admissibility_of_hypotrochoids(geo, N):
    rc, out, err = _build(geo, _hypotrochoid(0.45), N)
    assert rc == 0, err
    assert out[3] == 0.0                      # simple but not convex
    rc, _, err = _build(geo, _hypotrochoid(0.5), N)
    assert rc == 1 and "zero tangent" in err  # cusps at t = 0, 2 pi / 3, 4 pi / 3
    rc, _, err = _build(geo, _hypotrochoid(0.55), N)
    assert rc == 1 and "intersects itself" in err


def test_limacon_loop_and_orientation(geo):
    rc, _, err = _build(geo, [0, 0, 1, 1, 1], 512)        # 1 + e^{it} + e^{2it}
    assert rc == 1 and "intersects itself" in err
    rc, _, err = _build(geo, [1.0, 0, 0.5], 256)          # clockwise ellipse
    assert rc == 1 and "counter-clockwise" in err


def test_smooth_perturbed_contour_is_admitted(geo):
    rng = np.random.default_rng(3)
    M = 12
    z = np.zeros(2 * M + 1, dtype=np.complex128)
    z[M + 1] = 1.0
    for m in range(2, M + 1):
        z[M + m] = (rng.normal() + 1j * rng.normal()) * 0.02 / m ** 2
        z[M - m] = (rng.normal() + 1j * rng.normal()) * 0.02 / m ** 2
    rc, out, err = _build(geo, z, 32768)
    assert rc == 0, err
    # perimeter by a fine trapezoidal rule (spectrally accurate for a periodic integrand)
    t = 2 * np.pi * np.arange(1 << 16) / (1 << 16)
    m = np.arange(-M, M + 1)
    dz = (1j * m * z) @ np.exp(1j * np.outer(m, t))
    L = np.abs(dz).mean() * 2 * np.pi
    assert abs(out[1] - L) <= 1e-13 * L


def _H(n):
    return sum(1.0 / i for i in range(1, n + 1))


def _J(a, b):
    """int_0^1 int_0^1 log|x - y| x^a y^b dx dy.  On y < x put y = x s:
    int x^(n) (log x + log(1 - s)) s^b, n = a + b + 1, with int_0^1 x^n log x = -1/(n+1)^2
    and int_0^1 log(1 - s) s^b ds = -H_{b+1} / (b+1); the other triangle swaps a and b."""
    n = a + b + 1

    def tri(p, q):                            # y = x s carries y^q
        return -1.0 / ((n + 1) ** 2 * (q + 1)) - _H(q + 1) / ((n + 1) * (q + 1))
    return tri(a, b) + tri(b, a)


def _A(m):
    """int_0^1 s^m / (1 + s) ds: A_0 = log 2, A_m = 1/m - A_{m-1}."""
    v = math.log(2.0)
    for i in range(1, m + 1):
        v = 1.0 / i - v
    return v


def _K(i, j):
    """int_0^1 int_0^1 log(u + v) u^i v^j du dv.  On v < u put v = u s:
    int u^n (log u + log(1 + s)) s^j, n = i + j + 1, with
    int_0^1 log(1 + s) s^j ds = (log 2 - A_{j+1}) / (j + 1) by parts."""
    n = i + j + 1

    def tri(p, q):
        return -1.0 / ((n + 1) ** 2 * (q + 1)) + (math.log(2.0) - _A(q + 1)) / ((n + 1) * (q + 1))
    return tri(i, j) + tri(j, i)


def _poly_hat(a, hat):
    """coefficients {degree: coef} of x^a times the hat factor: 1 - x (0), x (1), 1 (None)"""
    if hat is None:
        return {a: 1.0}
    return {a + 1: 1.0} if hat == 1 else {a: 1.0, a + 1: -1.0}


def _exact(kind, c, a, b):
    po = _poly_hat(a, None if c == 4 else c >> 1)
    ps = _poly_hat(b, None if c == 4 else c & 1)
    tot = 0.0
    for da, ca in po.items():
        for db, cb in ps.items():
            if kind == 0:                      # coincident: log|xi - xi'|
                v = _J(da, db)
            elif kind == 1:                    # source follows: log(1 - xi + xi'), u = 1 - xi
                v = sum(comb(da, i) * (-1) ** i * _K(i, db) for i in range(da + 1))
            else:                              # source precedes: log(xi + 1 - xi'), v = 1 - xi'
                v = sum(comb(db, j) * (-1) ** j * _K(da, j) for j in range(db + 1))
            tot += ca * cb * v
    return tot


@pytest.mark.parametrize("q", [4, 6, 10, 16])
def test_log_moments_against_closed_forms(geo, q):
    mom = np.zeros(3 * 5 * q * q)
    geo.geo_log_moments(q, mom.ctypes.data_as(DP))
    mom = mom.reshape(3, 5, q, q)
    x, _ = np.polynomial.legendre.leggauss(q)
    xs = np.sort(0.5 * (x + 1.0))
    dmax = min(q - 1, 6)
    V = np.vander(xs, dmax + 1, increasing=True)          # V[g, a] = x_g^a
    worst = 0.0
    for kind in range(3):
        for c in range(5):
            S = V.T @ mom[kind, c] @ V
            for a in range(dmax + 1):
                for b in range(dmax + 1):
                    worst = max(worst, abs(S[a, b] - _exact(kind, c, a, b)))
    assert worst <= 1e-14, worst
