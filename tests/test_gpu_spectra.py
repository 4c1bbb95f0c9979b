"""Spectra of C and of the remainder C - C_c (Sec. III Fig. 3, Sec. V Fig. 4) from the HIP
path, against the oracle's dense SVD (GPU tests, through the C ABI).

C, C - C_c and the skeleton U V^T are formed on the GPU by applying the operators of
cfie_apply to the identity; their singular values (LAPACK on the host) are compared with
the stored oracle spectra of tests/golden/spectra_ellipse512.npz (2:1 ellipse with semi-axes
2 and 1, N = 512, 10 nodes per wavelength).  Singular values are unique, so they are compared
entry by entry (Weyl: |d sigma| <= ||d A||_2).  The statements of the paper checked on the GPU
spectra, each singular value labelled by the dominant spatial frequency m of its singular
vector (ka = k L / (2 pi)):
  * the spectrum of C is maximal near the surface resonance |m| ~ ka (Sec. III);
  * for |m| >> ka it is flat (the deviation from a multiple of the identity is small);
  * the spectrum of C - C_c decreases at high spatial frequencies (Sec. V): below 1e-3 of
    its maximum for |m| >= 2 ka and below 1e-4 for |m| >= 4 ka.
"""
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import diagnostics as Dg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2203_13283_amd")

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def spectra():
    path = os.path.join(HERE, "golden", "spectra_ellipse512.npz")
    if not os.path.exists(path):
        pytest.skip(f"{path} not generated (tests/golden/make_golden.py spectra512)")
    g = np.load(path)
    N, k = int(g["N"]), float(g["k"])
    s = P.Solver(compress_tol=0.015, block=64)
    s.assemble(W.ellipse_coeffs(2.0, 1.0), N, k)
    I = torch.eye(N, dtype=torch.complex128, device="cuda")
    C = s.apply(P.OP_C, I).T.cpu().numpy()
    R = s.apply(P.OP_REMAINDER, I).T.cpu().numpy()
    s.factor()
    UV = s.apply(P.OP_SKELETON, I).T.cpu().numpy()
    return g, s, C, R, UV


def test_singular_values_match_oracle(spectra):
    g, _, C, R, _ = spectra
    sC, mC = Dg.labelled_spectrum(C)
    sR, _ = Dg.labelled_spectrum(R)
    errC = np.abs(sC - g["sC"]).max() / g["sC"][0]
    errR = np.abs(sR - g["sR"]).max() / g["sC"][0]
    print(f"sigma(C) {errC:.2e}, sigma(C - C_c) {errR:.2e} (relative to sigma_max(C))")
    assert errC <= 1e-10 and errR <= 1e-10


def test_paper_statements_on_gpu_spectra(spectra):
    g, _, C, R, _ = spectra
    ka = float(g["k"]) * float(g["L"]) / (2 * math.pi)
    sC, mC = Dg.labelled_spectrum(C)
    sR, mR = Dg.labelled_spectrum(R)
    am = np.abs(mC) / ka
    assert 0.4 <= am[0] <= 1.2, am[0]
    high = np.abs(mC) >= 4 * ka
    assert high.sum() > 50 and sC[high].max() / sC[high].min() <= 1.3
    aR = np.abs(mR) / ka
    assert sR[aR >= 2].max() <= 1e-3 * sR[0]
    assert sR[aR >= 4].max() <= 1e-4 * sR[0]


def test_skeleton_spectrum(spectra):
    g, s, _, R, UV = spectra
    tau = 0.015 * float(g["cc_max"])
    r = s.info()["rank"]
    rstar = Dg.exact_rank(g["sR"], tau)
    sUV = np.linalg.svd(UV, compute_uv=False)
    sR = np.linalg.svd(R, compute_uv=False)
    print(f"rank {r} (exact at tau: {rstar}); max |sigma_i(UV^T) - sigma_i(R)| / tau = "
          f"{np.abs(sUV[:r] - sR[:r]).max() / tau:.3f}")
    assert rstar <= r <= 1.3 * rstar
    assert np.abs(sUV[:r] - sR[:r]).max() <= tau
    assert sUV[r:].max() <= 1e-12 * sUV[0]
