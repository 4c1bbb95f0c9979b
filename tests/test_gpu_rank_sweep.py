"""Rank and accuracy of the skeleton as functions of k at a fixed compression parameter
(Sec. VI, Fig. 5): the 2:1 ellipse (semi-axes 2 and 1) at 10 nodes per wavelength, k doubling
with N, epsilon = 0.015 (GPU, through the C ABI), against the oracle
(tests/golden/fig5_ellipse.npz: dense-LU solutions for 16 plane waves and the singular values
of C - C_c at N = 256 ... 2048).

The paper reports that at fixed epsilon the accuracy of the solution improves as k grows,
and that the inner rank grows no faster than k^(1/3).  Asserted here:
* accuracy: the rel.err of the epsilon = 0.015 Woodbury solution against the oracle's dense
  LU is below epsilon and falls monotonically with k;
* rank: the randomized range finder keeps a direction while a test column of the
  remaining remainder has norm above tau = epsilon ||C_c||_2 -- a Gaussian column, or (the
  default) a column of the SRFT D F, whose entries are independent of unit modulus, scaled
  for the columns already drawn -- and such a column's squared norm has the squared
  Frobenius norm of the remaining singular values as its mean.  So its rank lies between the exact rank r*(epsilon) =
  #{sigma_i > tau} and the Frobenius rank r_F(epsilon) = min{r : (sum_{i>r} sigma_i^2)^(1/2)
  <= tau}, plus what a randomized range finder needs beyond r_F to capture those
  directions: r* <= r <= 1.15 r_F + 16 (measured r / r_F = 1.16, 1.12, 1.11, 1.10 with the
  SRFT blocks; 1.14, 1.14, 1.12, 1.10 with Gaussian ones);
* the rank fraction r*/N of the oracle does not grow with k.
The k^(1/3) bound on the rank is not reproduced with the readings of the paper used here
(nodes uniform in arc length, tau = epsilon max |c_m|): r*/N only decreases slowly (0.24,
0.22, 0.20, 0.18); the measured values are printed.
"""
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import system as S

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2203_13283_amd")

HERE = os.path.dirname(os.path.abspath(__file__))
EPS = 0.015


def _golden():
    path = os.path.join(HERE, "golden", "fig5_ellipse.npz")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated (tests/golden/make_golden.py fig5)")
    return np.load(path)


def _ranks(s, tau):
    r_star = int(np.count_nonzero(s > tau))
    tail = np.sqrt(np.cumsum((s ** 2)[::-1])[::-1])       # tail[r] = |sigma_{r..}|_2
    below = np.nonzero(tail <= tau)[0]
    r_f = int(below[0]) if below.size else s.size
    return r_star, r_f


def test_rank_and_accuracy_vs_k_against_oracle():
    g = _golden()
    zh = W.ellipse_coeffs(2.0, 1.0)
    L = S.Contour(zh).L
    ang = W.plane_wave_angles(int(g["n_rhs"]))
    rows = []
    for N in [int(n) for n in g["Ns"]]:
        k = 2 * math.pi * N / (10 * L)
        assert abs(k - float(g[f"k_{N}"])) <= 1e-12 * k
        s = P.Solver(compress_tol=EPS, block=64)
        s.assemble(zh, N, k).factor()
        X = s.solve(s.plane_wave_rhs(ang)).cpu().numpy().T
        info = s.info()
        del s
        torch.cuda.empty_cache()
        x_ref = g[f"x_{N}"]
        err = float(np.max(np.linalg.norm(X - x_ref, axis=0) / np.linalg.norm(x_ref, axis=0)))
        cc = float(g[f"cc_max_{N}"])
        assert abs(info["cc_norm"] - cc) <= 1e-10 * cc
        r_star, r_f = _ranks(g[f"sR_{N}"], EPS * cc)
        r = info["rank"]
        rows.append((N, k, r, r_star, r_f, err))
        print(f"N={N:5d} k={k:8.3f} rank {r:5d} r*={r_star:5d} r_F={r_f:5d} r*/N "
              f"{r_star / N:.3f} r*/k^(1/3) {r_star / k ** (1 / 3):7.2f} rel.err {err:.2e}")
        assert r_star <= r <= 1.15 * r_f + 16, (N, r, r_star, r_f)
    errs = [e for (*_, e) in rows]
    assert all(e <= EPS for e in errs), errs
    assert all(b < a for a, b in zip(errs, errs[1:])), errs
    fracs = [rs / N for (N, _, _, rs, _, _) in rows]
    assert all(b <= a for a, b in zip(fracs, fracs[1:])), fracs


def test_full_rank_solution_matches_oracle():
    """At epsilon = 1e-12 the same solver reproduces the oracle's dense LU at every size of the
    sweep (the reference the accuracy above would otherwise need)."""
    g = _golden()
    zh = W.ellipse_coeffs(2.0, 1.0)
    ang = W.plane_wave_angles(int(g["n_rhs"]))
    for N in [int(n) for n in g["Ns"]]:
        s = P.Solver(compress_tol=1e-12, block=256)
        s.assemble(zh, N, float(g[f"k_{N}"])).factor()
        X = s.solve(s.plane_wave_rhs(ang)).cpu().numpy().T
        del s
        torch.cuda.empty_cache()
        x_ref = g[f"x_{N}"]
        err = float(np.max(np.linalg.norm(X - x_ref, axis=0) / np.linalg.norm(x_ref, axis=0)))
        print(f"N={N}: epsilon 1e-12 rel.err {err:.2e}")
        assert err <= 1e-10
