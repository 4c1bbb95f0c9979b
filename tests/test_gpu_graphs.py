"""Recorded FP64 solves (options.solve_graphs, GPU through the C ABI): every replay of the
recorded kernel sequence equals the direct solve of the same right-hand sides bit for bit,
with direct work and synchronisations between the replays, for a power-of-two N (FFT in
place) and another N (padded circulant product), batch sizes that change, in-place solves,
and after a new factorisation (the recorded graphs are dropped with the old factors)."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2203_13283_amd")


@pytest.mark.parametrize("N", [512, 600, 2048])
def test_graph_replays_equal_direct_solves(N):
    zh = W.ellipse_coeffs(1.0, 0.6)
    k = 2 * np.pi * N / (10 * 5.1054)
    opt = dict(compress_tol=1e-9, block=64)
    sd = P.Solver(**opt)
    sg = P.Solver(solve_graphs=True, **opt)
    for s in (sd, sg):
        s.assemble(zh, N, k).factor()
    assert sd.info()["rank"] == sg.info()["rank"]
    rng = np.random.default_rng(0)
    for it, m in enumerate((3, 8, 3, 8, 1, 3)):
        ang = rng.uniform(0, 2 * np.pi, m)
        B = sd.plane_wave_rhs(ang)
        Xd = sd.solve(B)
        torch.cuda.synchronize()
        Xg = sg.solve(B)
        assert torch.equal(Xd, Xg), (N, it, m)
        if it == 3:                                  # in place
            Bi = B.clone()
            sg.solve(Bi, out=Bi)
            assert torch.equal(Bi, Xd)
    sg.close()
    # a new factorisation drops the recorded graphs with the old factors
    sd2 = P.Solver(compress_tol=1e-5, block=64)
    sg2 = P.Solver(solve_graphs=True, compress_tol=1e-5, block=64)
    for s in (sd2, sg2):
        s.assemble(zh, N, k).factor()
    B = sd2.plane_wave_rhs(rng.uniform(0, 2 * np.pi, 4))
    X1 = sg2.solve(B)
    sg2.factor()
    X2 = sg2.solve(B)
    assert torch.equal(X1, sd2.solve(B)) and torch.equal(X1, X2)
