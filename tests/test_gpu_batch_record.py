"""Recorded batches (cfie_batch_record / cfie_batch_launch) through the C ABI (GPU).

A recorded batch runs every problem once adaptively (planning), then records all problems'
whole paths -- assembly, randomized skeleton, capacitance LU, plane-wave right-hand sides
(Sec. II-V eqs. (5)-(9)), solve -- as one HIP graph that replays the planned block schedule.
Checked: each launch reproduces the planning run's solutions bitwise (the same kernels on the
same data in the same order), a second launch too, the members against the oracle's dense LU
(FP64 to 1e-10, mixed precision to 1e-6), and the schedule's special paths (a rank-0
circle, a full-rank member that switches to the dense remainder at rank N/2).
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import system as S

pytestmark = [
    pytest.mark.gpu,
    pytest.mark.skip(reason="cfie_batch_record is disabled: recording ended the host process "
                            "with a segmentation fault on the GPU, cause not yet found"),
]

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2203_13283_amd")


def _problems():
    probs = W.batch_problems(count=5, seed=3, n_range=(200, 1100), rhs_range=(3, 12))
    # a circle (the remainder vanishes: rank 0) and a member with no right-hand sides
    probs.append(dict(zhat=W.circle_coeffs(1.0), n_nodes=256, k=2 * math.pi * 256 / (10 * 2 * math.pi),
                      angles=W.plane_wave_angles(4)))
    probs.append(dict(zhat=W.ellipse_coeffs(1.0, 0.6), n_nodes=300, k=20.0, angles=np.zeros(0)))
    return probs


def _oracle_check(probs, sols, tol, nmax=560):
    worst = 0.0
    for pr, X in zip(probs, sols):
        if pr["n_nodes"] > nmax or len(pr["angles"]) == 0:
            continue
        prob = S.Problem(pr["zhat"], pr["n_nodes"], pr["k"])
        x_ref = prob.solve(prob.rhs(pr["angles"]))
        e = S.rel_err(X.cpu().numpy().T, x_ref)
        worst = max(worst, e)
        print(f"N={pr['n_nodes']}: rel.err vs oracle {e:.2e}")
        assert e <= tol
    return worst


@pytest.mark.parametrize("prec,eps,tol", [(0, 1e-10, 1e-10), (1, 1e-3, 1e-6)])
def test_recorded_batch_replays_bitwise_and_matches_oracle(prec, eps, tol):
    probs = _problems()
    rb = P.RecordedBatch(probs, precision=prec, compress_tol=eps, refine_tol=1e-8)
    planned = [X.clone() for X in rb.solutions]
    ranks = [r["rank"] for r in rb.results]
    print(f"precision {prec}: {rb.nodes} graph nodes, ranks {ranks}, N "
          f"{[p['n_nodes'] for p in probs]}")
    assert ranks[5] == 0                                   # the circle
    for _ in range(2):
        for X in rb.solutions:
            X.fill_(complex(float("nan"), 0.0))
        res = rb.launch()
        torch.cuda.synchronize()
        assert all(r["status"] == 0 for r in res), res
        assert [r["rank"] for r in res] == ranks
        for X, Xp in zip(rb.solutions, planned):
            assert torch.equal(X, Xp)
    _oracle_check(probs, rb.solutions, tol)
    rb.close()


def test_recorded_batch_dense_switch_and_full_rank():
    """A member whose remainder has no numerical low rank at epsilon = 1e-13 keeps every
    direction; the automatic mode forms C - C_c densely once the rank reaches N/2, in the
    planning run and in the replay alike."""
    probs = [dict(zhat=W.ellipse_coeffs(1.0, 0.4), n_nodes=384, k=15.0,
                  angles=W.plane_wave_angles(5)),
             dict(zhat=W.ellipse_coeffs(1.0, 0.7), n_nodes=200, k=9.0,
                  angles=W.plane_wave_angles(3))]
    rb = P.RecordedBatch(probs, compress_tol=1e-13, block=64)
    planned = [X.clone() for X in rb.solutions]
    print("ranks", [r["rank"] for r in rb.results])
    assert rb.results[0]["rank"] == 384
    rb.launch()
    torch.cuda.synchronize()
    for X, Xp in zip(rb.solutions, planned):
        assert torch.equal(X, Xp)
    _oracle_check(probs, rb.solutions, 1e-10)
    rb.close()


def test_recorded_batch_arguments():
    lib = P._lib.load()
    probs = _problems()[:1]
    with pytest.raises(P.CfieError):
        P.RecordedBatch([dict(probs[0], angles=np.zeros(4097))])
    rb = P.RecordedBatch(probs, compress_tol=1e-8)
    assert lib.cfie_batch_launch(rb._h, rb._items, 2) == 1
    assert lib.cfie_batch_launch(None, rb._items, 1) == 1
    assert rb.launch()[0]["status"] == 0
    rb.close()
    lib.cfie_batch_destroy(None)
