"""Write the oracle reference values used by the full-size GPU parity tests.

Calls only the CPU oracle (oracle/) and the input generators (workloads/).  For each
workload it stores, in tests/golden/<name>.npz:
  rows, cols, entries[m]   sampled entries of Dk, Nk, Dkt, Skt (by the oracle's own rules)
  cc_eig                   eigenvalues of C_c (DFT of the first column of the dense C_c)
                           -- only where N <= 4096 (the dense circle matrices are needed)
  cols_rhs                 indices of the stored right-hand sides (angles 2 pi j / m)
  b, x                     right-hand sides of eq. (5) and dense-LU solutions for them
  L, k, kt_re, kt_im, N    constants

Also spectra<N>: singular values of C and C - C_c with their spatial-frequency labels, and
shapegrad<N>: the backscatter loss of the shape-differentiation workload at N nodes (shape
modes 1..8, four incident waves, 181 observation angles each), its far fields and the
reference gradient with respect to the 16 shape coefficients (central differences with two
Richardson extrapolations of the oracle's dense solve).

fig5_ellipse: the sweep of Sec. VI (Fig. 5) on the 2:1 ellipse at N = 256 ... 2048 (dense-LU
solutions for 16 plane waves, singular values of C - C_c, ||C_c||_2), and shapegrad_dir<N>:
the full shape workload's loss and its derivative along one seeded direction of the 128
shape coefficients.

Run:  python tests/golden/make_golden.py ellipse4096 perturbed16384 spectra512 shapegrad128
      fig5 shapegrad_dir2048 [--workers 8]
(about 2 minutes for ellipse4096 and 40 minutes for perturbed16384 on 8 cores; the
larger one needs about 40 GB of host memory).
"""
import argparse
import os
import sys
import time

import numpy as np
import scipy.linalg as sla

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import workloads as W  # noqa: E402
from oracle import assembly as A  # noqa: E402
from oracle import system as S  # noqa: E402

STORED_COLUMNS = {"ellipse4096": [0, 37, 64, 128, 201, 255],
                  "perturbed16384": [0, 301, 512, 777]}


def make(name: str, workers: int, n_samples: int = 2048):
    w = W.get(name)
    N = w.n_nodes
    contour = S.Contour(w.zhat)
    L = contour.L
    kt = S.ktilde(w.k, L)
    t0 = time.time()
    M = A.assemble(w.zhat, N, w.k, kt, workers=workers)
    t_asm = time.time() - t0
    print(f"{name}: assembly {t_asm:.1f} s", flush=True)
    rng = np.random.default_rng(1234)
    rows = rng.integers(0, N, n_samples)
    cols = np.concatenate([rng.integers(0, N, n_samples // 2),
                           (rows[n_samples // 2:] + rng.integers(-8, 9, n_samples - n_samples // 2)) % N])
    entries = {m: M[m][rows, cols].copy() for m in A.MATS}
    cols_rhs = np.array(STORED_COLUMNS[name])
    angles = w.angles[cols_rhs]
    e, hh = S.excitation(w.zhat, N, w.k, angles)
    b = S.rhs(M, e, hh, w.k)
    t1 = time.time()
    C = S.form_C(M)
    del M
    lu = sla.lu_factor(C, overwrite_a=True, check_finite=False)
    x = sla.lu_solve(lu, b)
    t_lu = time.time() - t1
    print(f"{name}: form C + LU + solve {t_lu:.1f} s", flush=True)
    out = dict(rows=rows, cols=cols, cols_rhs=cols_rhs, b=b, x=x, L=L, k=w.k, kt_re=kt.real,
               kt_im=kt.imag, N=N, t_assemble_s=t_asm, t_lu_s=t_lu)
    for m in A.MATS:
        out["entries_" + m] = entries[m]
    del lu, C
    if N <= 4096:
        Mc = A.assemble(S.equivalent_circle(L), N, w.k, kt, workers=workers)
        out["cc_eig"] = np.fft.fft(S.form_C(Mc)[:, 0])
    np.savez_compressed(os.path.join(HERE, name + ".npz"), **out)
    print(f"{name}: written", flush=True)


def make_spectra(N: int, workers: int):
    """Singular values of C and C - C_c on the 2:1 ellipse (semi-axes 2 and 1) at 10 nodes
    per wavelength, labelled by spatial frequency (Sec. III Fig. 3, Sec. V Fig. 4)."""
    import math
    from oracle import diagnostics as Dg
    zh = W.ellipse_coeffs(2.0, 1.0)
    L = S.Contour(zh).L
    k = 2 * math.pi * N / (10 * L)
    pr = S.Problem(zh, N, k, workers=workers)
    sC, mC = Dg.labelled_spectrum(pr.C)
    sR, mR = Dg.labelled_spectrum(pr.C - pr.Cc)
    cc = np.fft.fft(pr.Cc[:, 0])
    np.savez_compressed(os.path.join(HERE, f"spectra_ellipse{N}.npz"), N=N, k=k, L=L, sC=sC,
                        mC=mC, sR=sR, mR=mR, cc_max=np.abs(cc).max())
    print(f"spectra_ellipse{N}: written", flush=True)


def make_shapegrad(N: int, workers: int, mmax: int = 8, n_inc: int = 4, fd_step: float = 1e-3):
    from oracle import gradient as G
    pr = W.shape_problem(N=N, mmax=mmax, n_inc=n_inc)
    s, t = pr["s"], pr["t"]
    p0 = np.concatenate([s, t])

    def loss(p):
        return G.backscatter_loss(W.shape_to_zhat(p[:mmax], p[mmax:]), N, pr["k"],
                                  pr["angles"], pr["obs"], workers=workers)[0]

    t0 = time.time()
    L0, F = G.backscatter_loss(pr["zhat"], N, pr["k"], pr["angles"], pr["obs"], workers=workers)
    grad = G.richardson_gradient(loss, p0, fd_step)
    print(f"shapegrad{N}: loss {L0:.6e}, gradient in {time.time() - t0:.0f} s", flush=True)
    np.savez_compressed(os.path.join(HERE, f"shapegrad{N}.npz"), N=N, mmax=mmax, k=pr["k"],
                        s=s, t=t, zhat=pr["zhat"], angles=pr["angles"], obs=pr["obs"], L=L0,
                        F=F, grad=grad, fd_step=fd_step)
    print(f"shapegrad{N}: written", flush=True)


def make_fig5(Ns, workers: int, n_rhs: int = 16):
    """The sweep of Sec. VI (Fig. 5): the 2:1 ellipse with semi-axes 2 and 1 at 10 nodes per
    wavelength for each N of Ns.  Stores, per N, k, the dense-LU solutions of eq. (5) for
    n_rhs plane waves at 2 pi j / n_rhs, the singular values of C - C_c (dense SVD) and
    ||C_c||_2 = max |c_m| (the DFT of the dense circle C_c's first column)."""
    import math
    zh = W.ellipse_coeffs(2.0, 1.0)
    L = S.Contour(zh).L
    out = dict(Ns=np.asarray(Ns), L=L, n_rhs=n_rhs)
    for N in Ns:
        t0 = time.time()
        k = 2 * math.pi * N / (10 * L)
        pr = S.Problem(zh, N, k, workers=workers)
        ang = W.plane_wave_angles(n_rhs)
        b = pr.rhs(ang)
        x = pr.solve(b)
        sR = np.linalg.svd(pr.C - pr.Cc, compute_uv=False)
        out[f"k_{N}"] = k
        out[f"x_{N}"] = x
        out[f"sR_{N}"] = sR
        out[f"cc_max_{N}"] = float(np.abs(np.fft.fft(pr.Cc[:, 0])).max())
        print(f"fig5: N={N} in {time.time() - t0:.0f} s", flush=True)
        del pr
    np.savez_compressed(os.path.join(HERE, "fig5_ellipse.npz"), **out)
    print("fig5_ellipse: written", flush=True)


def make_shapegrad_direction(N: int, workers: int, mmax: int = 64, n_inc: int = 16,
                             fd_step: float = 2e-5, seed: int = 7):
    """The shape-differentiation workload's loss (16 waves, 181 backscatter angles each) at N
    nodes with all 128 shape coefficients, and its derivative along one seeded unit direction
    of the coefficients by central differences with two Richardson extrapolations of the
    oracle's dense solve (six solves).

    Step: a unit step along the direction moves the contour by up to about ten units of
    length (the sum of the direction's 128 components), so the loss's phases (k about 200 at
    N = 2048) vary on steps of about 1/(10 k) = 5e-4; h = 2e-5 keeps the extrapolation's
    O(h^6) remainder below 1e-9 relative, and the loss's rounding (about 1e-14 relative)
    gives about 1e-8 after the differences.  (h = 1e-3 left a 7e-6 remainder.)"""
    from oracle import gradient as G
    pr = W.shape_problem(N=N, mmax=mmax, n_inc=n_inc)
    p0 = np.concatenate([pr["s"], pr["t"]])
    d = np.random.default_rng(seed).normal(size=p0.size)
    d /= np.linalg.norm(d)

    def loss_along(u):
        p = p0 + u[0] * d
        return G.backscatter_loss(W.shape_to_zhat(p[:mmax], p[mmax:]), N, pr["k"],
                                  pr["angles"], pr["obs"], workers=workers)[0]

    t0 = time.time()
    L0, F = G.backscatter_loss(pr["zhat"], N, pr["k"], pr["angles"], pr["obs"],
                               workers=workers)
    dL = float(G.richardson_gradient(loss_along, np.zeros(1), fd_step)[0])
    print(f"shapegrad_dir{N}: loss {L0:.6e}, dL/du {dL:.9e} in {time.time() - t0:.0f} s",
          flush=True)
    np.savez_compressed(os.path.join(HERE, f"shapegrad_dir{N}.npz"), N=N, mmax=mmax,
                        k=pr["k"], direction=d, L=L0, F=F, dL=dL, fd_step=fd_step)
    print(f"shapegrad_dir{N}: written", flush=True)


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("names", nargs="+")
    ap.add_argument("--workers", type=int, default=os.cpu_count() or 1)
    a = ap.parse_args()
    for n in a.names:
        if n.startswith("spectra"):
            make_spectra(int(n[len("spectra"):]), a.workers)
        elif n == "fig5":
            make_fig5([256, 512, 1024, 2048], a.workers)
        elif n.startswith("shapegrad_dir"):
            make_shapegrad_direction(int(n[len("shapegrad_dir"):]), a.workers)
        elif n.startswith("shapegrad"):
            make_shapegrad(int(n[len("shapegrad"):]), a.workers)
        else:
            make(n, a.workers)
