"""Dense Galerkin boundary-element matrices for the oracle (test infrastructure only).

Definitions followed (Sec. II, eqs. (2)-(4); Sec. III, eq. (5)):
  [A]_ij = <lambda_i, A lambda_j>, with the bilinear pairing <f, g> = int_gamma f g ds
  (no complex conjugation), lambda_i the hat functions piecewise linear in arc length.
  g_kappa(R) = (i/4) H0^(1)(kappa R)                       Green's function
  S^kappa : int g_kappa(|r - r'|) j(r') ds'                single layer (used in eq. (5),
                                                          not written out in the paper)
  D^kappa : int d/dn' g_kappa j ds'  ->  kernel (i kappa/4) H1^(1)(kappa R) (r - r').n' / R
  N^k     : -d/dn int d/dn' g_k j ds'  in the integrated-by-parts (Maue) form
            <lambda_i, N lambda_j> = int int g_k(R) [lambda_i'(s) lambda_j'(s')
                                     - k^2 n(s).n(s') lambda_i(s) lambda_j(s')] ds ds'
  G       : <lambda_i, lambda_j>
Here n is the outward unit normal, (r - r').n' uses the normal at the source point r', and
d/ds is the derivative in arc length.

Quadrature (this oracle's own; deliberately heavier than anything the GPU path uses):
  element pairs at cyclic distance d >= 8: tensor Gauss-Legendre, QF points per direction
  4 <= d <= 7: Gauss-Legendre QM points; d = 2, 3: Gauss-Legendre QN points
  d = 0 (coincident) and d = 1 (adjacent): Duffy-type substitutions that put the log
  singularity at an endpoint of one variable, tanh-sinh in that variable and Gauss-Legendre
  in the other; the kernel is evaluated with accurate point differences so that it keeps
  its relative accuracy next to the singularity.
Hankel functions come from scipy.special.hankel1 (AMOS), a library primitive.
"""
from __future__ import annotations

import numpy as np
import scipy.special as sps

from .geometry import Contour, Discretisation
from .quadrature import gauss01, tanh_sinh01

MATS = ("Dk", "Nk", "Dkt", "Skt")


class QuadOptions:
    def __init__(self, qf=6, qm=8, qn=12, qs=16, ts_step=1.0 / 8.0):
        self.qf, self.qm, self.qn, self.qs, self.ts_step = qf, qm, qn, qs, ts_step

    @staticmethod
    def for_mesh(kh: float):
        """Default rules; the far-pair order grows when elements are long compared with the
        wavelength (|kappa| h > 1) so that the oscillation stays resolved."""
        extra = 2 * int(np.ceil(max(0.0, kh - 1.0)))
        return QuadOptions(qf=min(16, 6 + extra), qm=min(16, 8 + extra),
                           qn=min(20, 12 + extra))

    def refined(self):
        """Every rule made clearly finer (used to check convergence)."""
        return QuadOptions(self.qf + 4, self.qm + 4, self.qn + 6, self.qs + 8,
                           self.ts_step * 0.5)


def _kernels(R, nu, nn, k, kt):
    """Point-pair kernel values.

    R = |r - r'|, nu = (r - r').n' / R, nn = n.n'.  Returns g_k, nn, D^k, D^kt and S^kt
    kernels (complex arrays with the shape of R)."""
    H0k = sps.hankel1(0, k * R)
    H1k = sps.hankel1(1, k * R)
    H0t = sps.hankel1(0, kt * R)
    H1t = sps.hankel1(1, kt * R)
    gk = 0.25j * H0k
    Dk = 0.25j * k * H1k * nu
    Dt = 0.25j * kt * H1t * nu
    St = 0.25j * H0t
    return gk, Dk, Dt, St


def _accumulate(wts, phio, phis, gk, nn, Dk, Dt, St, k, h):
    """Sum point-pair kernels into 2x2 local blocks.

    wts: quadrature weights (already including h^2 and Jacobians), phio/phis: (2, ...) hat
    values at the observation / source point; returns dict of (..., 2, 2) local blocks
    summed over the trailing point axes."""
    dphi = np.array([-1.0 / h, 1.0 / h])
    res = {}
    for name, K in (("Dk", Dk), ("Dkt", Dt), ("Skt", St)):
        blk = np.empty(K.shape[:1] + (2, 2), dtype=np.complex128)
        for a in range(2):
            for b in range(2):
                blk[:, a, b] = np.sum((wts * phio[a] * phis[b] * K).reshape(K.shape[0], -1),
                                      axis=1)
        res[name] = blk
    blk = np.empty(gk.shape[:1] + (2, 2), dtype=np.complex128)
    for a in range(2):
        for b in range(2):
            c = dphi[a] * dphi[b] - k * k * nn * phio[a] * phis[b]
            blk[:, a, b] = np.sum((wts * c * gk).reshape(gk.shape[0], -1), axis=1)
    res["Nk"] = blk
    return res


def _blocks_regular(disc: Discretisation, E, F, q, k, kt):
    """Local blocks of element pairs (E[i], F[i]) by q x q Gauss-Legendre (non-touching)."""
    P = disc.points(q)
    h = disc.h
    xi, w = P["xi"], P["w"]
    zo = P["z"][E][:, :, None]
    zs = P["z"][F][:, None, :]
    to = P["tau"][E][:, :, None]
    ts = P["tau"][F][:, None, :]
    dz = zo - zs
    R = np.abs(dz)
    nu = -np.imag(dz * np.conj(ts)) / R
    nn = np.real(to * np.conj(ts))
    gk, Dk, Dt, St = _kernels(R, nu, nn, k, kt)
    wts = (h * h) * (w[:, None] * w[None, :])[None, :, :]
    phio = np.stack([1.0 - xi, xi])[:, None, :, None]
    phis = np.stack([1.0 - xi, xi])[:, None, None, :]
    wts = np.broadcast_to(wts, R.shape)
    return _accumulate(wts, phio, phis, gk, nn, Dk, Dt, St, k, h)


def _touching_rule(kind: str, opts: QuadOptions):
    """Quadrature on [0,1]^2 for an element pair that shares a point.

    Local coordinates are the element's own parameter fraction.  Returned arrays
    (to, ts, w, c_o, c_s): observation and source local coordinates, weights, and the
    coefficients of the parameter difference t - t' = c_o l_obs + c_s l_src in terms of the
    two elements' parameter lengths (so that t - t' is formed without cancellation).

    'coincident': Duffy split along the diagonal; u = |to - ts| is the tanh-sinh variable,
    the other variable Gauss-Legendre.  'right': source element e+1, shared node e+1;
    'left': source element e-1, shared node e.  For the latter two a = distance of the
    observation point to the shared node, b = that of the source point (in element
    fractions); each triangle a >= b / a < b is mapped to (rho, v) with rho tanh-sinh."""
    u, wu = tanh_sinh01(opts.ts_step)
    x, wx = gauss01(opts.qs)
    U = u[:, None]
    WU = wu[:, None]
    X = x[None, :]
    WX = wx[None, :]
    if kind == "coincident":
        xi1 = U + (1.0 - U) * X          # to in [u, 1], ts = to - u
        xi2 = (1.0 - U) * X              # to in [0, 1 - u], ts = to + u
        wt = (WU * (1.0 - U) * WX).ravel()
        Uf = np.broadcast_to(U, xi1.shape).ravel()
        to = np.concatenate([xi1.ravel(), xi2.ravel()])
        ts = np.concatenate([(xi1 - U).ravel(), (xi2 + U).ravel()])
        w = np.concatenate([wt, wt])
        c_o = np.concatenate([Uf, -Uf])
        return to, ts, w, c_o, np.zeros_like(c_o)
    rho, v = U, X
    wt = ((WU * WX) * rho).ravel()
    a = np.concatenate([(rho * np.ones_like(v)).ravel(), (rho * v).ravel()])
    b = np.concatenate([(rho * v).ravel(), (rho * np.ones_like(v)).ravel()])
    w = np.concatenate([wt, wt])
    if kind == "right":
        return 1.0 - a, b, w, -a, -b
    if kind == "left":
        return b, 1.0 - a, w, b, a
    raise ValueError(kind)


def _blocks_touching(disc: Discretisation, E, kind, k, kt, opts: QuadOptions,
                     chunk_points: int = 400_000):
    """Local blocks of the pairs (e, e) / (e, e+1) / (e, e-1) for e in E.

    The integrals are taken in the curve parameter t: ds = |z'(t)| dt, hats evaluated at
    s(t).  Point differences come from the Fourier series in difference form, so R and
    (r - r').n' keep full relative accuracy next to the singular point."""
    c: Contour = disc.contour
    h, N = disc.h, disc.N
    T = disc.node_params()
    to, ts, w, c_o, c_s = _touching_rule(kind, opts)
    src_off = {"coincident": 0, "right": 1, "left": -1}[kind]
    res = {m: np.empty((len(E), 2, 2), dtype=np.complex128) for m in MATS}
    per = max(1, chunk_points // to.size)
    for i0 in range(0, len(E), per):
        Eo = np.asarray(E[i0:i0 + per])
        Es = (Eo + src_off) % N
        lo = (T[Eo + 1] - T[Eo])[:, None]
        ls = (T[Es + 1] - T[Es])[:, None]
        t = T[Eo][:, None] + lo * to[None, :]
        delta = c_o[None, :] * lo + c_s[None, :] * ls
        tp = t - delta
        dz_o = c.dz(t)
        dz_s = c.dz(tp)
        sp_o = np.abs(dz_o)
        sp_s = np.abs(dz_s)
        R = np.abs(c.dz_diff(t, delta))
        rem = c.dz_diff_minus_tangent(tp, delta)
        nu = -np.imag(rem * np.conj(dz_s)) / (sp_s * R)
        nn = np.real((dz_o / sp_o) * np.conj(dz_s / sp_s))
        gk, Dk, Dt, St = _kernels(R, nu, nn, k, kt)
        xi_o = c.ds(t, lo * to[None, :]) / h
        xi_s = c.ds(T[Es][:, None] + ls * ts[None, :], ls * ts[None, :]) / h
        wts = w[None, :] * lo * ls * sp_o * sp_s
        phio = np.stack([1.0 - xi_o, xi_o])
        phis = np.stack([1.0 - xi_s, xi_s])
        blk = _accumulate(wts, phio, phis, gk, nn, Dk, Dt, St, k, h)
        for m in MATS:
            res[m][i0:i0 + len(Eo)] = blk[m]
    return res


def _scatter(Ms, E, F, blocks, N):
    for m in MATS:
        B = blocks[m]
        for a in range(2):
            for b in range(2):
                np.add.at(Ms[m], ((E + a) % N, (F + b) % N), B[:, a, b])


def gram_closed_form(N: int, h: float) -> np.ndarray:
    """G for hats uniform in arc length: circulant h [1/6, 2/3, 1/6] (exact)."""
    G = np.zeros((N, N))
    i = np.arange(N)
    G[i, i] = 2.0 * h / 3.0
    G[i, (i + 1) % N] = h / 6.0
    G[i, (i - 1) % N] = h / 6.0
    return G


def gram_by_quadrature(disc: Discretisation) -> np.ndarray:
    """G_ij = int lambda_i lambda_j ds by Gauss-Legendre on each element (the definition)."""
    N, h = disc.N, disc.h
    xi, w = gauss01(4)
    phi = np.stack([1.0 - xi, xi])
    loc = h * np.einsum("g,ag,bg->ab", w, phi, phi)
    G = np.zeros((N, N))
    e = np.arange(N)
    for a in range(2):
        for b in range(2):
            np.add.at(G, ((e + a) % N, (e + b) % N), loc[a, b])
    return G


def near_offsets(N: int):
    """Cyclic offsets f - e (mod N) treated as near pairs, grouped by distance class."""
    out = {}
    for d in range(0, 8):
        for sgn in (1, -1):
            off = (sgn * d) % N
            dist = min(off, N - off)
            out[off] = dist
    return out


_WORK = {}     # problem shared with forked worker processes


def _single_thread_blas():
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except ImportError:
        pass


def _far_rows(args):
    """Far-pair contributions of element rows [e0, e1) to matrix rows e0 .. e1 (mod N)."""
    e0, e1 = args
    disc, k, kt, opts = _WORK["disc"], _WORK["k"], _WORK["kt"], _WORK["opts"]
    N = disc.N
    E = np.repeat(np.arange(e0, e1), N)
    F = np.tile(np.arange(N), e1 - e0)
    off = (F - E) % N
    sel = np.minimum(off, N - off) >= 8
    blk = _blocks_regular(disc, E[sel], F[sel], opts.qf, k, kt)
    nb = e1 - e0
    out = {}
    for m in MATS:
        full = np.zeros((nb * N, 2, 2), dtype=np.complex128)
        full[sel] = blk[m]
        full = full.reshape(nb, N, 2, 2)
        rows = np.zeros((nb + 1, N), dtype=np.complex128)
        for a in range(2):
            for b in range(2):
                rows[a:a + nb] += np.roll(full[:, :, a, b], b, axis=1)
        out[m] = rows
    return e0, out


def _near_chunk(args):
    """Near-pair local blocks of offset `off` for the elements E."""
    off, dist, E = args
    disc, k, kt, opts = _WORK["disc"], _WORK["k"], _WORK["kt"], _WORK["opts"]
    N = disc.N
    F = (E + off) % N
    if dist == 0:
        blk = _blocks_touching(disc, E, "coincident", k, kt, opts)
    elif dist == 1 and off == 1:
        blk = _blocks_touching(disc, E, "right", k, kt, opts)
    elif dist == 1:
        blk = _blocks_touching(disc, E, "left", k, kt, opts)
    else:
        q = opts.qn if dist <= 3 else opts.qm
        blk = _blocks_regular(disc, E, F, q, k, kt)
    return off, E, blk


def assemble(zhat, N: int, k: float, kt: complex, opts: QuadOptions | None = None,
             row_block: int | None = None, workers: int = 1):
    """Dense Dk, Nk, Dkt, Skt (complex128 N x N) and G (float64) on the contour zhat.

    workers > 1 spreads the element pairs over forked processes (same arithmetic)."""
    contour = Contour(zhat)
    disc = Discretisation(contour, N)
    h = disc.h
    opts = opts or QuadOptions.for_mesh(max(abs(k), abs(kt)) * h)
    for q in {opts.qf, opts.qm, opts.qn}:
        disc.points(q)
    disc.node_params()
    Ms = {m: np.zeros((N, N), dtype=np.complex128) for m in MATS}
    near = near_offsets(N)
    _WORK.update(disc=disc, k=k, kt=kt, opts=opts)
    far_jobs = []
    if N > 15:
        if row_block is None:
            row_block = max(1, 2_000_000 // (N * opts.qf * opts.qf))
        far_jobs = [(e0, min(N, e0 + row_block)) for e0 in range(0, N, row_block)]
    near_jobs = []
    E = np.arange(N)
    per = max(1, -(-N // max(1, 4 * workers)))
    for off, dist in near.items():
        for i0 in range(0, N, per):
            near_jobs.append((off, dist, E[i0:i0 + per]))

    def add_far(res):
        e0, out = res
        for m in MATS:
            nb = out[m].shape[0] - 1
            Ms[m][e0:e0 + nb, :] += out[m][:nb]          # rows e0 .. e1-1
            Ms[m][(e0 + nb) % N, :] += out[m][nb]         # row e1 (wraps to 0 at the end)

    def add_near(res):
        off, Eb, blk = res
        _scatter(Ms, Eb, (Eb + off) % N, blk, N)

    if workers > 1:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(workers, initializer=_single_thread_blas) as pool:
            for r in pool.imap_unordered(_far_rows, far_jobs):
                add_far(r)
            for r in pool.imap_unordered(_near_chunk, near_jobs):
                add_near(r)
    else:
        for j in far_jobs:
            add_far(_far_rows(j))
        for j in near_jobs:
            add_near(_near_chunk(j))
    _WORK.clear()
    Ms["G"] = gram_by_quadrature(disc)
    Ms["h"] = h
    Ms["L"] = contour.L
    return Ms
