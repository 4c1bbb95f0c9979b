"""Batched solves of many contours of uneven N (cfie_solve_batch, GPU tests through the C
ABI): seeded perturbed ellipses, sizes that are and are not powers of two, their own
plane-wave sets.  Each item must equal the same problem solved alone (same kernels, its
own stream), and the smallest ones the oracle's dense LU."""
import numpy as np
import pytest

import workloads as W
from oracle import system as S

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2203_13283_amd")


@pytest.fixture(scope="module")
def problems():
    return W.batch_problems(count=7, seed=3, n_range=(96, 700), rhs_range=(3, 20))


def _alone(pr, **opt):
    s = P.Solver(**opt)
    s.assemble(pr["zhat"], pr["n_nodes"], pr["k"]).factor()
    return s.solve(s.plane_wave_rhs(pr["angles"])), s.info()["rank"]


def _rel(a, b):
    return float(((a - b).abs().pow(2).sum(1).sqrt() / b.abs().pow(2).sum(1).sqrt()).max())


def test_batch_equals_single_problem_solves(problems):
    opt = dict(compress_tol=1e-10, block=64)
    sols, res = P.solve_batch(problems, n_streams=3, **opt)
    for pr, X, r in zip(problems, sols, res):
        Xa, ra = _alone(pr, **opt)
        d = _rel(X, Xa)
        print(f"N={pr['n_nodes']:4d} m={pr['angles'].size:3d} rank {r['rank']} "
              f"vs alone {d:.1e} ({r['t_ms']:.1f} ms)")
        assert r["status"] == 0 and r["rank"] == ra
        assert d <= 1e-13


def test_batch_against_oracle(problems):
    small = sorted(problems, key=lambda p: p["n_nodes"])[:2]
    sols, _ = P.solve_batch(small, compress_tol=1e-10, block=64, n_streams=2)
    for pr, X in zip(small, sols):
        prob = S.Problem(pr["zhat"], pr["n_nodes"], pr["k"])
        err = S.rel_err(X.cpu().numpy().T, prob.solve(prob.rhs(pr["angles"])))
        print(f"N={pr['n_nodes']}: rel.err vs oracle {err:.2e}")
        assert err <= 1e-10


def test_batch_mixed_precision(problems):
    sols, res = P.solve_batch(problems, precision=P.CFIE_MIXED, compress_tol=1e-3,
                              refine_tol=1e-8, block=64, n_streams=4)
    for pr, X, r in zip(problems, sols, res):
        Xa, _ = _alone(pr, compress_tol=1e-10, block=64)
        assert r["status"] == 0 and r["refine_residual"] <= 1e-8
        assert _rel(X, Xa) <= 1e-6


def test_batch_argument_errors():
    with pytest.raises(P.CfieError):
        P.solve_batch([dict(zhat=W.ellipse_coeffs(1.0, 0.5), n_nodes=4, k=1.0,
                            angles=np.zeros(2))])
    sols, res = P.solve_batch([])
    assert sols == [] and res == []
