"""GEMM tile autotuner (GPU, through the C ABI): the four tile shapes give bitwise identical
results, so solutions with the autotuner off, while it measures, and after it has decided are
equal bit for bit; small shapes get measured."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2203_13283_amd")


def _solve(zhat, N, k, m, **opt):
    s = P.Solver(**opt)
    s.assemble(zhat, N, k)
    s.factor()
    X = s.solve(s.plane_wave_rhs(W.plane_wave_angles(m)))
    return X.cpu().numpy(), s.info()["rank"]


@pytest.mark.parametrize("prec", [P.CFIE_FP64, P.CFIE_MIXED])
def test_autotuned_tiles_are_bitwise_neutral(prec):
    zh = W.ellipse_coeffs(1.0, 0.55)
    N, k, m = 600, 60.0, 40
    old = P.set_gemm_autotune(False)
    try:
        X0, r0 = _solve(zh, N, k, m, precision=prec, compress_tol=1e-8, block=64)
        P.set_gemm_autotune(True)
        before = P.gemm_tuned_classes()
        X1, r1 = _solve(zh, N, k, m, precision=prec, compress_tol=1e-8, block=64)
        X2, r2 = _solve(zh, N, k, m, precision=prec, compress_tol=1e-8, block=64)
        after = P.gemm_tuned_classes()
    finally:
        P.set_gemm_autotune(old)
    print(f"rank {r0}, shape classes measured {after - before} (total {after})")
    assert r0 == r1 == r2
    assert after >= before
    assert np.array_equal(X0, X1) and np.array_equal(X1, X2)
