"""Pins of the CPU oracle against what the paper and the mathematics fix (CPU only).

Each test checks the oracle against something that is not the oracle: closed forms,
exact identities, an independent brute-force integration, or the analytic PEC-cylinder
solution.
"""

import numpy as np
import pytest
import scipy.integrate as sint
import scipy.special as sps

import analytic as An
import workloads as W
from oracle import assembly as A
from oracle import system as S
from oracle.geometry import Contour, Discretisation


# ---------------------------------------------------------------- geometry (Sec. V) ---------
@pytest.mark.parametrize("a,b", [(1.0, 0.6), (1.0, 0.5), (2.0, 1.0), (0.7, 0.7)])
def test_perimeter_matches_elliptic_integral(a, b):
    c = Contour(W.ellipse_coeffs(a, b))
    exact = 4.0 * a * sps.ellipe(1.0 - (b / a) ** 2)
    assert abs(c.L - exact) <= 1e-13 * exact


def test_nodes_uniform_in_arc_length():
    c = Contour(W.ellipse_coeffs(1.0, 0.6))
    d = Discretisation(c, 64)
    T = d.node_params()[:-1]
    # independent arc length of the ellipse x = cos t, y = 0.6 sin t: a E(phi | e^2)
    m = 1.0 - 0.36
    s = sps.ellipeinc(np.pi / 2, m) - sps.ellipeinc(np.pi / 2 - T, m)
    assert np.max(np.abs(s - np.arange(64) * d.h)) <= 1e-13


def test_convexity_and_orientation_of_workloads():
    for name in ("ellipse256", "ellipse4096", "perturbed16384"):
        c = Contour(W.get(name).zhat)
        assert c.signed_area() > 0
        assert c.curvature(np.linspace(0, 2 * np.pi, 4000)).min() > 0


# ---------------------------------------------------------------- Gram matrix ---------------
def test_gram_closed_form_and_inverse():
    N = 40
    d = Discretisation(Contour(W.ellipse_coeffs(1.0, 0.6)), N)
    Gq = A.gram_by_quadrature(d)
    Gc = A.gram_closed_form(N, d.h)
    assert np.max(np.abs(Gq - Gc)) <= 1e-16 * 10
    inv = np.linalg.inv(Gc)
    assert np.max(np.abs(inv[:, 0] - An.gram_inverse_column(N, d.h))) <= 1e-12 * np.max(
        np.abs(inv))


# ---------------------------------------------------------------- circle spectra (T4) -------
@pytest.fixture(scope="module")
def circle64():
    R, k = 0.8125, 20.0
    kt = S.ktilde(k, 2 * np.pi * R)
    M = A.assemble(W.circle_coeffs(R), 64, k, kt)
    return R, k, kt, M


def test_circle_matrices_match_aliasing_sums(circle64):
    R, k, kt, M = circle64
    ek = An.galerkin_circle_eigs(64, k, R)
    et = An.galerkin_circle_eigs(64, kt, R)
    for name, ref in (("Dk", ek["D"]), ("Nk", ek["N"]), ("Dkt", et["D"]), ("Skt", et["S"]),
                      ("G", ek["G"])):
        got = np.fft.fft(M[name][:, 0])
        err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
        assert err <= 1e-11, (name, err)


def test_circle_matrices_are_circulant(circle64):
    _, _, _, M = circle64
    for name in ("Dk", "Nk", "Dkt", "Skt"):
        X = M[name]
        sh = np.roll(np.roll(X, 1, axis=0), 1, axis=1)
        assert np.max(np.abs(sh - X)) <= 1e-13 * np.max(np.abs(X)), name


def test_labelled_spectrum_of_circulant(circle64):
    """On the circle C is circulant and normal: its singular values are |c_m| and each
    singular vector is a Fourier mode, so the labels are the mode numbers (up to the sign,
    c_m = c_-m)."""
    from oracle import diagnostics as Dg
    _, _, _, M = circle64
    C = S.form_C(M)
    s, m = Dg.labelled_spectrum(C)
    c = np.fft.fft(C[:, 0])
    N = C.shape[0]
    freq = np.fft.fftfreq(N, 1.0 / N).astype(int)
    assert np.max(np.abs(s - np.sort(np.abs(c))[::-1])) <= 1e-12 * s[0]
    by_mode = {int(abs(f)): abs(v) for f, v in zip(freq, c)}
    for sv, lab in zip(s, m):
        assert abs(by_mode[int(abs(lab))] - sv) <= 1e-10 * s[0], (sv, lab)
    assert Dg.exact_rank(s, s[3]) == 3


# ---------------------------------------------------------------- invariants (T5, T6) -------
@pytest.fixture(scope="module")
def ellipse64():
    zh = W.ellipse_coeffs(1.0, 0.6)
    k = 6.0
    L = Contour(zh).L
    return zh, k, S.ktilde(k, L), A.assemble(zh, 64, k, S.ktilde(k, L))


def test_reciprocity_symmetry(ellipse64):
    _, _, _, M = ellipse64
    for name in ("Skt", "Nk"):
        X = M[name]
        assert np.max(np.abs(X - X.T)) <= 1e-14 * np.max(np.abs(X)), name
    assert np.max(np.abs(M["G"] - M["G"].T)) == 0.0


@pytest.mark.parametrize("zhat", [W.ellipse_coeffs(1.0, 0.6), W.perturbed_circle_coeffs(0)],
                         ids=["ellipse", "perturbed"])
def test_gauss_identity_double_layer(zhat):
    """Laplace limit: D 1 = -1/2 on a smooth closed curve, so row sums of D = -h/2."""
    N = 64
    M = A.assemble(zhat, N, 1e-9, complex(1e-9, 0.0))
    rs = M["Dk"].sum(axis=1)
    assert np.max(np.abs(rs + M["h"] / 2)) <= 1e-12 * M["h"]


def test_quadrature_converged(ellipse64):
    zh, k, kt, M = ellipse64
    Mr = A.assemble(zh, 64, k, kt, A.QuadOptions().refined())
    for name in ("Dk", "Nk", "Dkt", "Skt"):
        err = np.linalg.norm(M[name] - Mr[name]) / np.linalg.norm(Mr[name])
        assert err <= 1e-13, (name, err)


# ---------------------------------------------------------------- brute force (T7) ----------
def _brute_entry(a_ax, b_ax, N, kappa, i, j, kind):
    """Galerkin entry by nested adaptive QUADPACK integration in the ellipse angle t,
    with the closed-form elliptic arc length; independent of the oracle's rules."""
    m = 1.0 - (b_ax / a_ax) ** 2
    L = 4 * a_ax * sps.ellipe(m)
    h = L / N

    def s_of(t):
        return a_ax * (sps.ellipeinc(np.pi / 2, m) - sps.ellipeinc(np.pi / 2 - t, m))

    def t_of(s):
        from scipy.optimize import brentq
        return brentq(lambda t: s_of(t) - s, -1.0, 2 * np.pi + 1.0, xtol=1e-15)

    def hat(idx, t):
        s = s_of(t)
        x = (s - idx * h) / h
        x = (x + N / 2) % N - N / 2
        return max(0.0, 1.0 - abs(x))

    def pos(t):
        return np.array([a_ax * np.cos(t), b_ax * np.sin(t)])

    def tang(t):
        v = np.array([-a_ax * np.sin(t), b_ax * np.cos(t)])
        return v, np.linalg.norm(v)

    ti = [t_of((i + q) * h) for q in (-1, 0, 1)]
    tj = [t_of((j + q) * h) for q in (-1, 0, 1)]

    def inner(t):
        r = pos(t)
        li = hat(i, t)
        _, sp = tang(t)

        def f(tp, part):
            rp = pos(tp)
            v, spp = tang(tp)
            n_p = np.array([v[1], -v[0]]) / spp
            d = r - rp
            R = np.hypot(*d)
            if kind == "S":
                K = 0.25j * sps.hankel1(0, kappa * R)
            else:
                K = 0.25j * kappa * sps.hankel1(1, kappa * R) * (d @ n_p) / R
            val = K * hat(j, tp) * spp
            return val.real if part == 0 else val.imag

        pts = sorted(set([tj[0], tj[1], tj[2]] + ([t] if tj[0] < t < tj[2] else [])))
        out = 0j
        for lo, hi in zip(pts[:-1], pts[1:]):
            for part in (0, 1):
                v = sint.quad(f, lo, hi, args=(part,), epsabs=1e-15, epsrel=1e-13,
                              limit=200)[0]
                out += v if part == 0 else 1j * v
        return out * li * sp

    total = 0j
    for lo, hi in ((ti[0], ti[1]), (ti[1], ti[2])):
        for part in (0, 1):
            v = sint.quad(lambda t: (inner(t).real if part == 0 else inner(t).imag), lo, hi,
                          epsabs=1e-15, epsrel=1e-12, limit=100)[0]
            total += v if part == 0 else 1j * v
    return total


@pytest.mark.parametrize("i,j,kind", [(0, 0, "S"), (0, 1, "S"), (3, 1, "D"), (2, 2, "D")])
def test_brute_force_entries(i, j, kind):
    a_ax, b_ax, N, k = 1.0, 0.6, 8, 2.0
    zh = W.ellipse_coeffs(a_ax, b_ax)
    kt = complex(k, 0.0)
    M = A.assemble(zh, N, k, kt)
    ref = _brute_entry(a_ax, b_ax, N, k, i, j, kind)
    got = M["Skt" if kind == "S" else "Dk"][i, j]
    scale = np.max(np.abs(M["Skt" if kind == "S" else "Dk"]))
    assert abs(got - ref) <= 1e-11 * scale, (got, ref)


# ---------------------------------------------------------------- Woodbury identity (T10) ---
def test_woodbury_equals_dense_lu():
    """Eqs. (8)-(9): C^{-1} b through C_c (diagonalised by the FFT) and an exact skeleton
    U V^T = C - C_c equals the dense LU solution."""
    zh = W.ellipse_coeffs(1.0, 0.6)
    P = S.Problem(zh, 32, 5.0)
    b = P.rhs(W.plane_wave_angles(3))
    x_ref = P.solve(b)
    Cc = P.Cc
    c = np.fft.fft(Cc[:, 0])                        # eigenvalues of the circulant C_c
    assert np.max(np.abs(np.fft.ifft(c[:, None] * np.fft.fft(np.eye(32), axis=0), axis=0)
                         - Cc)) <= 1e-13 * np.max(np.abs(Cc))

    def Ccinv(y):
        return np.fft.ifft(np.fft.fft(y, axis=0) / c[:, None], axis=0)

    Uf, s, Vh = np.linalg.svd(P.C - Cc)
    U = Uf * s
    Vt = Vh
    K = np.eye(U.shape[1]) + Vt @ Ccinv(U)
    y = Ccinv(b)
    x = y - Ccinv(U) @ np.linalg.solve(K, Vt @ y)
    assert S.rel_err(x, x_ref) <= 1e-12


# ---------------------------------------------------------------- Mie series (T12) ----------
def test_circle_solution_converges_to_mie_series():
    R, k, alpha = 1.0, 10.0, 0.3
    errs = []
    for N in (48, 96, 192):
        P = S.Problem(W.circle_coeffs(R), N, k)
        j = P.solve(P.rhs([alpha]))[:, 0]
        phi = 2 * np.pi * np.arange(N) / N
        jm = An.mie_current(k, R, phi, alpha)
        errs.append(np.linalg.norm(j - jm) / np.linalg.norm(jm))
    assert errs[-1] < 1e-2
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 3.0 < r1 < 5.0 and 3.0 < r2 < 5.0, errs
