"""The wide 128 x 128 complex128 GEMM tile against the 64 x 64 tile (GPU, through the C ABI).

The wide tile takes the large FP64 products of the metric workload (N = 16384: the sketch's
N x N x 256 products and their adjoints, V^T U~, the solve's W Y).  It runs the same MFMA
sequence per output element as the 64 x 64 tile (k ascending in steps of 4, the same K split,
3M form), so the whole path -- rank, skeleton and solutions -- must come out bitwise equal
with the wide tile on and off.  The second case has N = 4000 (not a multiple of the 128-row
tile: the last tile is shifted inside the matrix and writes only its own rows) at
epsilon = 1e-10 (rank close to N), so that the solve's products W Y (ragged rows) and
X - U~ Z (ragged rows, beta = 1) take the wide tile with K of about 4000 and 256 or more
tiles.
"""
import math

import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2203_13283_amd")


def _run(w, eps):
    s = P.Solver(compress_tol=eps, block=256)
    s.assemble(w.zhat, w.n_nodes, w.k).factor()
    B = s.plane_wave_rhs(w.angles[:300])
    X = s.solve(B)
    torch.cuda.synchronize()
    out = (s.info()["rank"], X.clone())
    del s, B, X
    torch.cuda.empty_cache()
    return out


def test_wide_tile_is_bitwise_neutral_on_the_metric_workload():
    w = W.get("perturbed16384")
    prev = P.set_gemm_wide(False)
    try:
        r0, X0 = _run(w, 1e-5)
    finally:
        P.set_gemm_wide(prev)
    P.set_gemm_wide(True)
    r1, X1 = _run(w, 1e-5)
    print(f"rank {r0} (64 x 64 tiles) vs {r1} (wide tiles); max |dX| "
          f"{float((X0 - X1).abs().max()):.3e}")
    assert r0 == r1
    assert torch.equal(X0, X1)


def test_wide_tile_ragged_edges_and_beta_one():
    zh = W.ellipse_coeffs(1.0, 0.6)
    N = 4000
    k = 2 * math.pi * N / (10 * 5.1054)          # 10 nodes per wavelength (perimeter 5.1054)
    ang = W.plane_wave_angles(1024)

    def run():
        s = P.Solver(compress_tol=1e-10, block=256)
        s.assemble(zh, N, k).factor()
        X = s.solve(s.plane_wave_rhs(ang))
        torch.cuda.synchronize()
        out = (s.info()["rank"], X.clone())
        del s, X
        torch.cuda.empty_cache()
        return out

    prev = P.set_gemm_wide(False)
    try:
        r0, X0 = run()
    finally:
        P.set_gemm_wide(prev)
    P.set_gemm_wide(True)
    r1, X1 = run()
    print(f"N={N}: rank {r0} / {r1}; max |dX| {float((X0 - X1).abs().max()):.3e}")
    assert r0 == r1 and r0 >= 2048
    assert torch.equal(X0, X1)
