"""The largest problem the library accepts, N = 32768 (GPU, through the C ABI).

* A circle at 10 nodes per wavelength, N = 32768 (FFT of a power of two, four-step with
  N1 = 4096, N2 = 8) and N = 32767 (zero-padded circulant product of length 65536): C equals
  C_c to rounding, so the skeleton is empty once epsilon is above the rounding floor of the
  assembled C (entrywise about 1e-11 of C_c x at this N, measured 9e-12 and 1.4e-11; a
  Gaussian sketch column sums N such errors, about 2e-9 of ||C_c||, so epsilon = 1e-8 here);
  the FFT solve must satisfy the system applied factor by factor with the full-size GEMMs
  (residual <= 1e-10) and agree with the Mie series to the discretisation error of P1
  elements at kh = 0.63 and k R = 3277 (measured 2.0e-2: the phase error of the discrete
  waves accumulates over the circumference, so at fixed nodes per wavelength it grows with k).
* An ellipse (semi-axes 1 and 0.5) at N = 32768 with epsilon = 1e-4: the whole factorisation
  at full size; the residual of the solve against the assembled operator is at the
  compression level.
"""
import math
import time

import numpy as np
import pytest

import analytic as An
import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2203_13283_amd")


def _residual(s, X, B):
    R = s.apply(P.OP_C, X) - B
    return float((R.abs().pow(2).sum(1).sqrt() / B.abs().pow(2).sum(1).sqrt()).max())


@pytest.mark.parametrize("N", [32768, 32767])
def test_circle_at_maximum_size(N):
    R, k = 1.0, N / 10.0
    s = P.Solver(compress_tol=1e-8)
    t0 = time.time()
    s.assemble(W.circle_coeffs(R), N, k).factor()
    t1 = time.time()
    assert s.info()["rank"] == 0
    ang = np.array([0.0, 0.7, 2.0, 4.5])
    B = s.plane_wave_rhs(ang)
    X = s.solve(B)
    res = _residual(s, X, B)
    phi = 2 * np.pi * np.arange(N) / N
    x = X.cpu().numpy()
    err = max(np.linalg.norm(x[j] - An.mie_current(k, R, phi, a)) /
              np.linalg.norm(An.mie_current(k, R, phi, a)) for j, a in enumerate(ang))
    print(f"N={N}: assemble+factor {t1 - t0:.2f} s, residual {res:.2e}, vs Mie {err:.2e}")
    assert res <= 1e-10
    assert err <= 5e-2


def test_ellipse_factorisation_at_maximum_size():
    N = 32768
    zh = W.ellipse_coeffs(1.0, 0.5)
    k = 2 * math.pi * N / (10 * 4.844224110273)
    s = P.Solver(compress_tol=1e-4, block=256)
    t0 = time.time()
    s.assemble(zh, N, k)
    t1 = time.time()
    s.factor()
    t2 = time.time()
    B = s.plane_wave_rhs(W.plane_wave_angles(8))
    X = s.solve(B)
    res = _residual(s, X, B)
    info = s.info()
    print(f"N={N}: assemble {t1 - t0:.2f} s, factor {t2 - t1:.2f} s, rank {info['rank']}, "
          f"residual {res:.2e}")
    assert 0 < info["rank"] < N
    assert res <= 1e-3
