"""Parity of the HIP path with the CPU oracle (GPU tests, through the C ABI).

Tolerances: the FP64 path must reproduce the oracle's solution to rel.err <= 1e-10 (max
over columns of ||x - x_ref|| / ||x_ref||); assembled matrices agree to 1e-11 of their
largest entry (both sides converge to the exact Galerkin integrals with different
quadrature); the mixed-precision path reaches rel.err <= 1e-6 after FP64 refinement.
"""
import numpy as np
import pytest

import analytic as An
import workloads as W
from oracle import system as S

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
P = pytest.importorskip("paper_2203_13283_amd")


def _np(t):
    return t.detach().cpu().numpy()


@pytest.fixture(scope="module")
def cfg1():
    w = W.get("ellipse256")
    prob = S.Problem(w.zhat, w.n_nodes, w.k)
    return w, prob


@pytest.fixture(scope="module")
def cfg1_solver(cfg1):
    w, _ = cfg1
    s = P.Solver(compress_tol=w.compress_tol)
    s.assemble(w.zhat, w.n_nodes, w.k)
    return s


def test_geometry_and_constants(cfg1, cfg1_solver):
    w, prob = cfg1
    info = cfg1_solver.info()
    assert abs(info["perimeter"] - prob.L) <= 1e-13 * prob.L
    assert abs(info["ktilde_re"] - prob.kt.real) == 0.0
    assert abs(info["ktilde_im"] - prob.kt.imag) <= 1e-14 * prob.kt.imag


def test_assembled_matrices_match_oracle(cfg1, cfg1_solver):
    _, prob = cfg1
    s = cfg1_solver
    for which, name in ((P.MAT_DK, "Dk"), (P.MAT_NK, "Nk"), (P.MAT_DKT, "Dkt"),
                        (P.MAT_SKT, "Skt")):
        got = _np(s.export_matrix(which))
        ref = prob.M[name]
        emax = np.abs(got - ref).max() / np.abs(ref).max()
        efro = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        print(f"{name}: max-entry {emax:.2e}  frobenius {efro:.2e}")
        assert emax <= 1e-11 and efro <= 1e-12, name
    G = _np(s.export_matrix(P.MAT_G)).real
    assert np.abs(G - prob.M["G"]).max() <= 1e-16 * 8


def test_circulant_eigenvalues_match_oracle(cfg1, cfg1_solver):
    _, prob = cfg1
    c_gpu = _np(cfg1_solver.export_matrix(P.MAT_CC_EIG))[0]
    c_ref = np.fft.fft(prob.Cc[:, 0])
    err = np.abs(c_gpu - c_ref).max() / np.abs(c_ref).max()
    print(f"C_c eigenvalues: {err:.2e}")
    assert err <= 1e-11


def test_plane_wave_rhs_matches_oracle(cfg1, cfg1_solver):
    w, prob = cfg1
    B = _np(cfg1_solver.plane_wave_rhs(w.angles)).T
    ref = prob.rhs(w.angles)
    err = S.rel_err(B, ref)
    print(f"rhs: {err:.2e}")
    assert err <= 1e-11


def test_apply_C_matches_oracle(cfg1, cfg1_solver):
    _, prob = cfg1
    rng = np.random.default_rng(5)
    x = rng.standard_normal((256, 3)) + 1j * rng.standard_normal((256, 3))
    X = torch.from_numpy(np.ascontiguousarray(x.T)).cuda()
    Y = _np(cfg1_solver.apply_C(X)).T
    err = S.rel_err(Y, prob.C @ x)
    print(f"apply_C: {err:.2e}")
    assert err <= 1e-11


def test_solve_fp64_matches_dense_lu(cfg1, cfg1_solver):
    w, prob = cfg1
    s = cfg1_solver
    s.factor()
    B = s.plane_wave_rhs(w.angles)
    X = s.solve(B)
    x_ref = prob.solve(prob.rhs(w.angles))
    err = S.rel_err(_np(X).T, x_ref)
    print(f"solve fp64: rank {s.info()['rank']} rel.err {err:.2e}")
    assert err <= 1e-10


def test_solve_in_place_and_ragged_batch(cfg1, cfg1_solver):
    w, prob = cfg1
    s = cfg1_solver
    ang = np.array([0.1, 1.7, 2.9])
    B = s.plane_wave_rhs(ang)
    X = s.solve(B.clone())
    s.solve(B, out=B)                                   # B_dev == X_dev
    assert torch.equal(B, X)
    x_ref = prob.solve(prob.rhs(ang))
    assert S.rel_err(_np(X).T, x_ref) <= 1e-10


@pytest.mark.parametrize("prec,adjoint,m", [(P.CFIE_FP64, False, 4100),
                                             (P.CFIE_MIXED, False, 2050),
                                             (P.CFIE_FP64, True, 1030)])
def test_solve_leading_dimensions_and_chunks(cfg1, prec, adjoint, m):
    """The C ABI with leading dimensions larger than N (B and X padded rows of different
    widths) and more right-hand sides than one internal chunk (4096 FP64, 2048 mixed, 1024
    adjoint): bitwise equal to the packed solve, the padding left untouched, and sampled
    columns on both sides of the chunk boundary against the oracle's dense LU."""
    w, prob = cfg1
    N = w.n_nodes
    eps = 1e-10 if prec == P.CFIE_FP64 else 1e-3
    s = P.Solver(precision=prec, compress_tol=eps, refine_tol=1e-9)
    s.assemble(w.zhat, N, w.k).factor()
    ang = 2 * np.pi * np.arange(m) / m
    B = s.plane_wave_rhs(ang)
    Xp = s.solve_adjoint(B) if adjoint else s.solve(B)
    ldb, ldx = N + 7, N + 3
    Bw = torch.zeros((m, ldb), dtype=torch.complex128, device="cuda")
    Bw[:, :N] = B
    Xw = torch.full((m, ldx), 7 + 7j, dtype=torch.complex128, device="cuda")
    fn = s._lib.cfie_solve_adjoint if adjoint else s._lib.cfie_solve
    s._check(fn(s._h, P._ptr(Bw), ldb, P._ptr(Xw), ldx, m), "strided solve")
    assert torch.equal(Xw[:, :N], Xp)
    assert bool((Xw[:, N:] == 7 + 7j).all())
    chunk = {P.CFIE_FP64: 1024 if adjoint else 4096, P.CFIE_MIXED: 2048}[prec]
    cols = [0, chunk - 1, chunk, m - 1]
    Bn = prob.rhs(ang[cols])
    ref = np.linalg.solve(prob.C.conj().T, _np(B[cols]).T) if adjoint else prob.solve(Bn)
    err = S.rel_err(_np(Xp[cols]).T, ref)
    print(f"precision {prec} adjoint {adjoint} m={m}: rel.err {err:.2e}")
    assert err <= (1e-10 if prec == P.CFIE_FP64 else 1e-6)


def test_adjoint_solve_matches_dense_lu(cfg1, cfg1_solver):
    """C^H x = g with the same factorisation (adjoint Woodbury, conjugate circulant
    eigenvalues, K^H from the LU of K) against a dense LU of the oracle's C^H; the adjoint
    operator against the oracle's C^H; the adjoint identity g^H C^-1 b = (C^-H g)^H b."""
    w, prob = cfg1
    s = cfg1_solver
    s.factor()
    g = torch.randn((3, w.n_nodes), dtype=torch.complex128, device="cuda",
                    generator=torch.Generator(device="cuda").manual_seed(5))
    lam = _np(s.solve_adjoint(g)).T
    ref = np.linalg.solve(prob.C.conj().T, _np(g).T)
    err = S.rel_err(lam, ref)
    print(f"adjoint fp64: rel.err {err:.2e}")
    assert err <= 1e-10
    y = _np(s.apply(P.OP_C_ADJ, g)).T
    assert np.abs(y - prob.C.conj().T @ _np(g).T).max() <= 1e-12 * np.abs(y).max()
    B = s.plane_wave_rhs(w.angles[:3])
    X = _np(s.solve(B)).T
    lhs = np.einsum("ij,ij->j", _np(g).T.conj(), X)
    rhs = np.einsum("ij,ij->j", lam.conj(), _np(B).T)
    assert np.abs(lhs - rhs).max() <= 1e-11 * np.abs(lhs).max()
    sm = P.Solver(precision=P.CFIE_MIXED, compress_tol=1e-3, refine_tol=1e-9)
    sm.assemble(w.zhat, w.n_nodes, w.k).factor()
    errm = S.rel_err(_np(sm.solve_adjoint(g)).T, ref)
    print(f"adjoint mixed: sweeps {sm.info()['refine_sweeps']} rel.err {errm:.2e}")
    assert errm <= 1e-6


def test_circle_remainder_vanishes():
    """Circle: C = C_c up to rounding (the same rules on the same mesh), so at the FP64
    tolerance the skeleton has rank 0 and the FFT solve alone is the answer."""
    R, k = 0.9, 12.0
    zh = W.circle_coeffs(R)
    s = P.Solver(compress_tol=1e-10)
    s.assemble(zh, 128, k)
    x = torch.randn((2, 128), dtype=torch.complex128, device="cuda")
    yc, ycc = s.apply(P.OP_C, x), s.apply(P.OP_CC, x)
    assert float((yc - ycc).abs().max() / ycc.abs().max()) <= 1e-11
    s.factor()
    assert s.info()["rank"] == 0
    ang = W.plane_wave_angles(2)
    X = _np(s.solve(s.plane_wave_rhs(ang))).T
    prob = S.Problem(zh, 128, k)
    assert S.rel_err(X, prob.solve(prob.rhs(ang))) <= 1e-10
    # and the current converges to the Mie series like h^2 (conventions pinned)
    phi = 2 * np.pi * np.arange(128) / 128
    jm = An.mie_current(k, R, phi, ang[1])
    assert np.linalg.norm(X[:, 1] - jm) / np.linalg.norm(jm) < 2e-2


@pytest.mark.parametrize("N", [8, 32, 512, 2048, 4096, 8192, 16384, 32768, 9, 100, 1000, 3000, 6000,
                               20000, 32767])
def test_circulant_fft_lengths(N):
    """C_c x and C_c^-1 x by the library's FFT path against numpy's FFT with the exported
    eigenvalues: odd and even powers of two, one pass (N <= 4096, the radix-16 kernel at
    4096) and the four-step split (N1 = 4096, N2 = 2, 4, 8); other lengths through the
    zero-padded convolution (transform lengths 32 ... 65536)."""
    zh = W.ellipse_coeffs(1.0, 0.6)
    L = S.Contour(zh).L
    s = P.Solver(compress_tol=1e-10)
    s.assemble(zh, N, 2 * np.pi * N / (10 * L))
    c = _np(s.export_matrix(P.MAT_CC_EIG))[0]
    g = torch.Generator(device="cuda").manual_seed(N)
    x = torch.randn((3, N), dtype=torch.complex128, device="cuda", generator=g)
    xn = _np(x)
    for op, ref in ((P.OP_CC, np.fft.ifft(c * np.fft.fft(xn, axis=1), axis=1)),
                    (P.OP_CC_INV, np.fft.ifft(np.fft.fft(xn, axis=1) / c, axis=1))):
        y = _np(s.apply(op, x))
        err = np.abs(y - ref).max() / np.abs(ref).max()
        assert err <= 1e-13, (op, err)


@pytest.mark.parametrize("N", [61, 64, 100, 1000, 2047, 2048, 2049, 4157])
def test_apply_C_matches_dense_product(N):
    """C X by the library (eq. (6) applied factor by factor, G^-1 as the 61-tap band) against
    the same product formed with numpy from the exported matrices and the exact inverse of
    the exported G: isolates the banded G^-1 kernel, including columns shorter than the
    band's 2048-row workgroup segments and segments that wrap around the column."""
    zh = W.ellipse_coeffs(1.0, 0.6)
    L = S.Contour(zh).L
    s = P.Solver(compress_tol=1e-10)
    s.assemble(zh, N, 2 * np.pi * N / (10 * L))
    G, Dk, Nk, Dkt, Skt = (_np(s.export_matrix(w)) for w in
                           (P.MAT_G, P.MAT_DK, P.MAT_NK, P.MAT_DKT, P.MAT_SKT))
    C = G / 4 + (Dkt - Dk) / 2 - Dkt @ np.linalg.solve(G, Dk) + Skt @ np.linalg.solve(G, Nk)
    g = torch.Generator(device="cuda").manual_seed(N)
    x = torch.randn((3, N), dtype=torch.complex128, device="cuda", generator=g)
    ref = (C @ _np(x).T).T
    y = _np(s.apply(P.OP_C, x))
    err = np.abs(y - ref).max() / np.abs(ref).max()
    print(f"N={N}: C X vs dense numpy product {err:.2e}")
    assert err <= 1e-12


@pytest.mark.parametrize("N", [200, 333])
def test_solve_non_power_of_two(N):
    """Lengths that are not powers of two (circulant products by zero-padded convolution):
    the full path against the oracle's dense LU, FP64 at epsilon = 1e-10 and mixed."""
    zh = W.ellipse_coeffs(1.0, 0.6)
    k = 2 * np.pi * N / (10 * S.Contour(zh).L)
    prob = S.Problem(zh, N, k)
    ang = W.plane_wave_angles(4)
    x_ref = prob.solve(prob.rhs(ang))
    for prec, eps, tol in ((P.CFIE_FP64, 1e-10, 1e-10), (P.CFIE_MIXED, 1e-3, 1e-6)):
        s = P.Solver(precision=prec, compress_tol=eps, block=64)
        s.assemble(zh, N, k).factor()
        X = _np(s.solve(s.plane_wave_rhs(ang))).T
        err = S.rel_err(X, x_ref)
        print(f"N={N} precision {prec}: rank {s.info()['rank']} rel.err {err:.2e}")
        assert err <= tol


@pytest.mark.parametrize("form", [0, 1])
def test_mixed_precision_refinement(cfg1, form):
    """Mixed precision with FP64 refinement, the residual applied factor by factor (form 0)
    or with C formed densely in FP64 (form 1): both against the oracle, and the adjoint solve
    against the oracle's C^H."""
    w, prob = cfg1
    s = P.Solver(precision=P.CFIE_MIXED, compress_tol=1e-3, refine_tol=1e-8, refine_form=form)
    s.assemble(w.zhat, w.n_nodes, w.k).factor()
    B = s.plane_wave_rhs(w.angles)
    X = s.solve(B)
    info = s.info()
    x_ref = prob.solve(prob.rhs(w.angles))
    err = S.rel_err(_np(X).T, x_ref)
    print(f"mixed (refine form {form}): rank {info['rank']} sweeps {info['refine_sweeps']} "
          f"residual {info['refine_residual']:.2e} rel.err {err:.2e}")
    assert info["refine_residual"] <= 1e-8
    assert err <= 1e-6
    Xa = s.solve_adjoint(B)
    xa_ref = np.linalg.solve(prob.C.conj().T, _np(B).T)
    erra = S.rel_err(_np(Xa).T, xa_ref)
    print(f"mixed adjoint (refine form {form}): rel.err {erra:.2e}")
    assert erra <= 1e-6


def test_smallest_mesh():
    zh = W.ellipse_coeffs(1.0, 0.7)
    s = P.Solver(compress_tol=0.0)
    s.assemble(zh, 8, 1.5).factor()
    ang = [0.3]
    X = _np(s.solve(s.plane_wave_rhs(ang))).T
    prob = S.Problem(zh, 8, 1.5)
    err = S.rel_err(X, prob.solve(prob.rhs(ang)))
    print(f"N=8: rel.err {err:.2e}")
    assert err <= 1e-9


def test_state_machine_and_errors(cfg1):
    w, _ = cfg1
    s = P.Solver()
    with pytest.raises(P.CfieError) as e:
        s.factor()
    assert e.value.status == 4
    with pytest.raises(P.CfieError) as e:
        s.assemble(w.zhat, 6, w.k)
    assert e.value.status == 1
    with pytest.raises(P.CfieError) as e:
        s.assemble(w.zhat, 64, -1.0)
    assert e.value.status == 1
    with pytest.raises(P.CfieError) as e:
        s.assemble(w.zhat, 32769, 3.0)                    # above the size limit
    assert e.value.status == 1
    with pytest.raises(P.CfieError) as e:
        s.assemble(w.zhat[::-1].copy(), 64, 3.0)          # clockwise
    assert e.value.status == 1
    s.assemble(w.zhat, 64, 3.0)
    with pytest.raises(P.CfieError) as e:
        s.solve(torch.zeros((1, 64), dtype=torch.complex128, device="cuda"))
    assert e.value.status == 4
    s2 = P.Solver(fail_alloc_after=3)
    with pytest.raises(P.CfieError) as e:
        s2.assemble(w.zhat, 64, 3.0)
    assert e.value.status == 2


def test_empty_batches(cfg1, cfg1_solver):
    """Zero right-hand sides, zero observation directions: every entry point returns at once
    with an empty result and leaves the context usable."""
    w, prob = cfg1
    s = cfg1_solver
    s.factor()
    N = w.n_nodes
    E = torch.zeros((0, N), dtype=torch.complex128, device="cuda")
    assert s.plane_wave_rhs([]).shape == (0, N)
    assert s.solve(E).shape == (0, N)
    assert s.solve_adjoint(E).shape == (0, N)
    assert s.apply(P.OP_C, E).shape == (0, N)
    assert s.far_field(E, [0.1, 0.2]).shape == (0, 2)
    B = s.plane_wave_rhs(w.angles[:2])
    X = s.solve(B)
    assert s.far_field(X, []).shape == (2, 0)
    assert S.rel_err(_np(X).T, prob.solve(prob.rhs(w.angles[:2]))) <= 1e-10


def test_skeleton_approximates_remainder(cfg1):
    """U V^T approximates C - C_c to the compression tolerance (Sec. V eq. (7))."""
    w, _ = cfg1
    eps = 1e-6
    s = P.Solver(compress_tol=eps)
    s.assemble(w.zhat, w.n_nodes, w.k).factor()
    info = s.info()
    assert 0 < info["rank"] < w.n_nodes
    x = torch.randn((6, w.n_nodes), dtype=torch.complex128, device="cuda")
    d = s.apply(P.OP_REMAINDER, x) - s.apply(P.OP_SKELETON, x)
    ratio = float((d.abs().pow(2).sum(1).sqrt() / x.abs().pow(2).sum(1).sqrt()).max())
    tau = eps * info["cc_norm"]
    print(f"skeleton: rank {info['rank']} ||(R - UV^T) x|| / ||x|| = {ratio:.2e}, tau {tau:.2e}")
    assert ratio <= 10 * tau


@pytest.mark.parametrize("form,prec,tol,bar", [
    (P.REMAINDER_DENSE, P.CFIE_FP64, 1e-10, 1e-10),
    (P.REMAINDER_AUTO, P.CFIE_FP64, 1e-13, 1e-10),
    (P.REMAINDER_DENSE, P.CFIE_MIXED, 1e-4, 1e-6),
])
def test_dense_remainder_form(cfg1, form, prec, tol, bar):
    """C - C_c formed densely (two N x N x N GEMMs) before the sketch, or once the rank passes
    N/2 (automatic mode at a tolerance that needs almost full rank): same solution as the
    oracle's dense LU to the FP64 (or mixed-precision) bar."""
    w, prob = cfg1
    s = P.Solver(precision=prec, compress_tol=tol, remainder_form=form, block=64,
                 refine_tol=1e-9)
    s.assemble(w.zhat, w.n_nodes, w.k).factor()
    B = s.plane_wave_rhs(w.angles)
    X = _np(s.solve(B)).T
    ref = prob.solve(_np(B).T)
    err = S.rel_err(X, ref)
    print(f"form {form} prec {prec}: rank {s.info()['rank']} rel.err {err:.2e}")
    assert err <= bar
    if form == P.REMAINDER_AUTO:
        assert 2 * s.info()["rank"] >= w.n_nodes
