"""Host build of the device Bessel/Hankel routines against scipy (AMOS) (CPU only).

The header is compiled for the host with g++, so the exact arithmetic the kernels use is
checked here without a GPU: H0, H1 for real and complex arguments across the series,
Miller-recurrence and large-argument regions, the split Y = (2/pi) log(z/2) J + Yhat, and
the Wronskian J1 Y0 - J0 Y1 = 2 / (pi z).
"""
import ctypes
import os
import subprocess
import tempfile

import numpy as np
import pytest
import scipy.special as sps

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def hb():
    out = os.path.join(tempfile.mkdtemp(), "hb.so")
    subprocess.run(["g++", "-O2", "-std=c++17", "-shared", "-fPIC", "-o", out,
                    os.path.join(HERE, "host_bessel.cpp")], check=True)
    return ctypes.CDLL(out)


def _call(lib, fn, z, w=4):
    z = np.ascontiguousarray(np.asarray(z, complex))
    out = np.zeros(len(z) * w)
    getattr(lib, fn)(len(z), z.ctypes.data_as(ctypes.c_void_p),
                     out.ctypes.data_as(ctypes.c_void_p))
    o = out.reshape(-1, w)
    return o[:, 0::2] + 1j * o[:, 1::2]


@pytest.mark.parametrize("lo,hi,tol", [(1e-4, 1, 3e-15), (1, 5, 3e-14), (5, 22, 2e-14),
                                       (22, 60, 5e-15), (60, 5000, 5e-15)])
@pytest.mark.parametrize("cplx", [False, True])
def test_hankel_against_amos(hb, lo, hi, tol, cplx):
    rng = np.random.default_rng(1)
    r = np.exp(rng.uniform(np.log(lo), np.log(hi), 4000))
    z = r + (1j * rng.uniform(0, 1.2, r.size) if cplx else 0.0)
    H = _call(hb, "hb_hankel01", z)
    for nu in (0, 1):
        ref = sps.hankel1(nu, z)
        assert np.max(np.abs(H[:, nu] - ref) / np.abs(ref)) <= tol


def test_split_form_and_wronskian(hb):
    z = np.array([1e-3, 0.3 + 0.01j, 3.0, 4.9 + 0.5j, 5.1 + 0.2j, 9.0 + 0.3j, 15.0, 21.0])
    S = _call(hb, "hb_split", z, 8)
    J0, J1 = sps.jv(0, z), sps.jv(1, z)
    assert np.max(np.abs(S[:, 0] - J0) / np.abs(J0)) <= 1e-13
    assert np.max(np.abs(S[:, 1] - J1) / np.abs(J1)) <= 1e-13
    Y0 = 2 / np.pi * np.log(z / 2) * S[:, 0] + S[:, 2]
    Y1 = 2 / np.pi * np.log(z / 2) * S[:, 1] - 2 / (np.pi * z) + S[:, 3]
    assert np.max(np.abs(Y0 - sps.yv(0, z)) / np.abs(sps.hankel1(0, z))) <= 1e-13
    assert np.max(np.abs(Y1 - sps.yv(1, z)) / np.abs(sps.hankel1(1, z))) <= 1e-13
    W = S[:, 1] * Y0 - S[:, 0] * Y1
    assert np.max(np.abs(W * np.pi * z / 2 - 1.0)) <= 1e-12
