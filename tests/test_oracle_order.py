"""Pins of the order of the non-commuting factors in C (Sec. V, eq. (6)) and in the
right-hand side of the preconditioned equation (Sec. III, eq. (5)), CPU only.

On a circle every Galerkin matrix is circulant and all of them commute, so the circle pins
cannot tell (G/2 + D^kt) G^-1 (G/2 - D^k) from (G/2 - D^k) G^-1 (G/2 + D^kt), nor
S^kt G^-1 N^k from N^k G^-1 S^kt.  These tests run on the 2:1 ellipse, where they differ,
and pin the order against two facts that do not involve the oracle's formula:

* Calderon's identity for the single layer V, the double layer K and the hypersingular
  operator W of one wavenumber: V W = I/4 - K^2 (W with the sign of eq. (2)).  In Galerkin
  form S G^-1 N + D G^-1 D - G/4 -> 0 as the mesh is refined, at the rate of the
  discretisation; the other order N G^-1 S belongs to the identity with the adjoint double
  layer and stays O(1) away.
* The preconditioned equation (5) combines the discrete EFIE and MFIE parts of the
  unpreconditioned CFIE (4) (Sec. II) each with its own left factor, so both discrete
  solutions approximate the same current and their difference falls at the rate of the
  discretisation.  A factor in the wrong order makes eq. (5) inconsistent with eq. (4): the
  difference then stalls (operator) or falls at a lower rate (right-hand side).
"""

import numpy as np
import pytest

import workloads as W
from oracle import assembly as A
from oracle import system as S
from oracle.geometry import Contour

ZH = W.ellipse_coeffs(1.0, 0.5)
K = 5.0
NS = (32, 64, 128)
ANGLES = [0.3, 1.7]


@pytest.fixture(scope="module")
def ladder():
    """Oracle matrices on the 2:1 ellipse at k = 5 for N = 32, 64, 128: at the paper's kt and
    at kt = k (one wavenumber, where Calderon's identity applies)."""
    L = Contour(ZH).L
    out = []
    for N in NS:
        out.append(dict(N=N, L=L,
                        M=A.assemble(ZH, N, K, S.ktilde(K, L)),
                        M1=A.assemble(ZH, N, K, complex(K, 0.0))))
    return out


def _smooth(N, L):
    """Hat coefficients of a smooth function of arc length (nodes uniform in s)."""
    s = np.arange(N) * L / N
    return np.cos(2 * np.pi * s / L) + 0.5 * np.sin(4 * np.pi * s / L + 0.3)


def _rates(errs):
    return [errs[i] / errs[i + 1] for i in range(len(errs) - 1)]


def test_calderon_identity_of_assembled_operators(ladder):
    """S G^-1 N + D G^-1 D - G/4 -> 0 on the ellipse at one wavenumber (second order in h);
    the transposed product N G^-1 S does not satisfy it."""
    good, swapped = [], []
    for P in ladder:
        M = P["M1"]
        G = M["G"].astype(np.complex128)
        x = _smooth(P["N"], P["L"])
        Gi = lambda y: np.linalg.solve(G, y)  # noqa: E731
        DD = M["Dk"] @ Gi(M["Dk"] @ x)
        nGx = np.linalg.norm(G @ x)
        good.append(np.linalg.norm(M["Skt"] @ Gi(M["Nk"] @ x) + DD - 0.25 * G @ x) / nGx)
        swapped.append(np.linalg.norm(M["Nk"] @ Gi(M["Skt"] @ x) + DD - 0.25 * G @ x) / nGx)
    assert all(r >= 6.0 for r in _rates(good)), good
    assert good[-1] < 1e-5, good
    assert min(swapped) > 1e-2, swapped


def test_form_C_order_at_one_wavenumber(ladder):
    """At kt = k eq. (6) reads C = G/4 - D G^-1 D + S G^-1 N; with Calderon's identity this
    is G/2 - 2 D G^-1 D up to the discretisation error.  Pins the order of S G^-1 N in
    form_C (the first term's order is invisible at kt = k; the next test covers it)."""
    errs = []
    for P in ladder:
        M = P["M1"]
        G = M["G"].astype(np.complex128)
        x = _smooth(P["N"], P["L"])
        C = S.form_C(M)
        ref = 0.5 * G @ x - 2.0 * M["Dk"] @ np.linalg.solve(G, M["Dk"] @ x)
        errs.append(np.linalg.norm(C @ x - ref) / np.linalg.norm(G @ x))
    assert all(r >= 6.0 for r in _rates(errs)), errs
    assert errs[-1] < 1e-5, errs


def test_preconditioned_solution_converges_to_cfie_solution(ladder):
    """The solution of eq. (5) (form_C and rhs of the oracle) and the solution of the
    unpreconditioned discrete CFIE (4), (1/ik) N^k j + (G/2 - D^k) j = -e/eta - h, approach
    each other at the discretisation rate (about 8 per doubling of N measured: 4.6e-3,
    5.5e-4, 6.8e-5).  Swapping the first term of C stalls the difference at 0.16, swapping
    N^k G^-1 S^kt at 0.16, and G^-1 S^kt in the right-hand side lowers the rate to 4."""
    errs = []
    for P in ladder:
        M, N = P["M"], P["N"]
        G = M["G"].astype(np.complex128)
        e, hh = S.excitation(ZH, N, K, ANGLES)
        j5 = S.solve_dense(S.form_C(M), S.rhs(M, e, hh, K))
        A4 = M["Nk"] / (1j * K) + 0.5 * G - M["Dk"]
        j4 = np.linalg.solve(A4, -e - hh)
        errs.append(S.rel_err(j5, j4))
    assert all(r >= 6.0 for r in _rates(errs)), errs
    assert errs[-1] < 2e-4, errs


def test_ktilde_radius_is_harmonic_mean_of_curvature_radii():
    """Sec. III takes a as an average of the radii of curvature; the reading used is their
    arc-length harmonic mean L / int kappa ds.  The curvature integral is taken here by
    quadrature of the contour's own curvature, independently of the perimeter formula."""
    for zh in (W.ellipse_coeffs(1.0, 0.5), W.perturbed_circle_coeffs(0)):
        c = Contour(zh)
        t = 2 * np.pi * np.arange(20000) / 20000
        turning = np.sum(c.curvature(t) * c.speed(t)) * (2 * np.pi / t.size)
        a = c.L / turning
        k = 300.0
        kt = S.ktilde(k, c.L)
        assert abs(kt.real - k) == 0.0
        assert abs(kt.imag - 0.4 * k ** (1 / 3) * a ** (-2 / 3)) <= 1e-12 * kt.imag
