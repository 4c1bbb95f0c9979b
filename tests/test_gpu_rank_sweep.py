"""Rank and accuracy of the skeleton as functions of k at a fixed compression parameter
(Sec. VI, Fig. 5): the 2:1 ellipse (semi-axes 2 and 1) at 10 nodes per wavelength, k doubling
with N, epsilon = 0.015 (GPU, through the C ABI).

The paper reports that at fixed epsilon the accuracy of the solution improves as k grows,
and that the inner rank grows no faster than k^(1/3).  Accuracy here is the rel.err of the
epsilon = 0.015 Woodbury solution against the same solver at epsilon = 1e-12 (full rank,
which matches the oracle's dense LU to 1e-12 at these sizes).  Asserted: the accuracy is
within epsilon and improves monotonically with k; the rank fraction r/N does not grow.
The k^(1/3) bound on the rank is not reproduced with the readings of the paper used here
(nodes uniform in arc length, tau = epsilon max |c_m|): r/N only decreases slowly (the
measured values are printed; see the design notes).
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import system as S

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2203_13283_amd")


def _sweep(Ns, eps=0.015):
    zh = W.ellipse_coeffs(2.0, 1.0)
    L = S.Contour(zh).L
    ang = W.plane_wave_angles(16)
    rows = []
    for N in Ns:
        k = 2 * math.pi * N / (10 * L)
        ref = P.Solver(compress_tol=1e-12, block=256)
        ref.assemble(zh, N, k).factor()
        B = ref.plane_wave_rhs(ang)
        Xr = ref.solve(B)
        del ref
        s = P.Solver(compress_tol=eps, block=64)
        s.assemble(zh, N, k).factor()
        X = s.solve(B)
        err = float(((X - Xr).abs().pow(2).sum(1).sqrt() / Xr.abs().pow(2).sum(1).sqrt()).max())
        r = s.info()["rank"]
        del s, B, X, Xr
        torch.cuda.empty_cache()
        rows.append((N, k, r, err))
        print(f"N={N:5d} k={k:8.3f} rank {r:5d} r/N {r / N:.3f} r/k^(1/3) {r / k ** (1/3):7.2f} "
              f"rel.err {err:.2e}")
    return rows


def test_rank_and_accuracy_vs_k():
    rows = _sweep([256, 512, 1024, 2048, 4096])
    errs = [e for (_, _, _, e) in rows]
    fracs = [r / N for (N, _, r, _) in rows]
    assert all(e <= 0.015 for e in errs)
    assert all(b < a for a, b in zip(errs, errs[1:])), errs
    assert all(b <= a * 1.02 for a, b in zip(fracs, fracs[1:])), fracs
