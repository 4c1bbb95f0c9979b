"""Seeded synthetic workloads shared by the tests, the benchmark and the oracle scripts.

This module only describes inputs: contours as Fourier coefficients of z(t), wavenumbers,
plane-wave incidence angles and seeds.  It holds none of the solver's arithmetic, so both
the HIP path and the CPU oracle can take their inputs from here without sharing any code.

Contour convention: z(t) = sum_{m=-M..M} zhat[m+M] exp(i m t), t in [0, 2*pi),
counter-clockwise, complex plane identified with R^2.

The paper (Sec. VI) works on an ellipse with semi-axes 2 m and 1 m at increasing k with the
mesh a fixed fraction of the wavelength.  The named workloads below are synthetic stand-ins
shaped like that: ellipses and a smooth, convex, seeded perturbation of the unit circle,
all discretised at about 10 nodes per wavelength (the first one is coarser, 15.7 nodes per
wavelength, and small enough for a dense CPU solve).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Workload",
    "ellipse_coeffs",
    "perturbed_circle_coeffs",
    "circle_coeffs",
    "plane_wave_angles",
    "batch_problems",
    "shape_coeffs",
    "shape_to_zhat",
    "shape_jacobian",
    "backscatter_angles",
    "shape_problem",
    "WORKLOADS",
    "get",
]


def ellipse_coeffs(a: float, b: float) -> np.ndarray:
    """x = a cos t, y = b sin t  ->  z = (a+b)/2 e^{it} + (a-b)/2 e^{-it}; modes -1..1."""
    return np.array([(a - b) / 2.0, 0.0, (a + b) / 2.0], dtype=np.complex128)


def circle_coeffs(radius: float) -> np.ndarray:
    return ellipse_coeffs(radius, radius)


def perturbed_circle_coeffs(seed: int = 0, mmin: int = 2, mmax: int = 8,
                            amp: float = 0.02) -> np.ndarray:
    """r(theta) = 1 + sum_{m=mmin..mmax} c_m cos(m theta + phi_m),
    c_m ~ U(0, amp/m^2) drawn as one vector, then phi_m ~ U(0, 2 pi) as one vector,
    from numpy.random.default_rng(seed).  z(theta) = r(theta) e^{i theta} expanded in
    Fourier modes -(mmax-1) .. mmax+1."""
    rng = np.random.default_rng(seed)
    ms = np.arange(mmin, mmax + 1)
    c = rng.uniform(0.0, amp / ms.astype(np.float64) ** 2)
    phi = rng.uniform(0.0, 2.0 * math.pi, size=ms.size)
    M = mmax + 1
    zhat = np.zeros(2 * M + 1, dtype=np.complex128)
    zhat[M + 1] += 1.0
    for mi, cm, ph in zip(ms, c, phi):
        zhat[M + mi + 1] += 0.5 * cm * np.exp(1j * ph)
        zhat[M + 1 - mi] += 0.5 * cm * np.exp(-1j * ph)
    return zhat


def plane_wave_angles(m: int) -> np.ndarray:
    """Propagation directions alpha_j = 2 pi j / m, j = 0..m-1."""
    return 2.0 * math.pi * np.arange(m, dtype=np.float64) / m


@dataclass(frozen=True)
class Workload:
    name: str
    zhat: np.ndarray = field(repr=False)
    n_nodes: int
    k: float
    nrhs: int
    compress_tol: float
    description: str
    sketch_seed: int = 1

    @property
    def angles(self) -> np.ndarray:
        return plane_wave_angles(self.nrhs)

    @property
    def n_modes(self) -> int:
        return (len(self.zhat) - 1) // 2


# Wavenumbers of the 10-nodes-per-wavelength workloads: k = 2 pi N / (10 L), with the
# perimeter L of the contour (ellipse 1 x 0.5: L = 4.844224110273; perturbed circle,
# seed 0: L = 6.283280042604).  They are fixed here as plain input numbers.
_K_ELLIPSE_4096 = 531.2703630624
_K_PERTURBED_16384 = 1638.375300000

WORKLOADS = {
    "ellipse256": Workload(
        name="ellipse256", zhat=ellipse_coeffs(1.0, 0.6), n_nodes=256, k=20.0, nrhs=8,
        compress_tol=1e-10,
        description="ellipse a=1, b=0.6, k=20, N=256, 8 plane waves"),
    "ellipse4096": Workload(
        name="ellipse4096", zhat=ellipse_coeffs(1.0, 0.5), n_nodes=4096, k=_K_ELLIPSE_4096,
        nrhs=256, compress_tol=1e-10,
        description="ellipse a=1, b=0.5, 10 nodes/wavelength, N=4096, 256 plane waves"),
    "perturbed16384": Workload(
        name="perturbed16384", zhat=perturbed_circle_coeffs(0), n_nodes=16384,
        k=_K_PERTURBED_16384, nrhs=1024, compress_tol=1e-4,
        description="seed-0 convex Fourier-perturbed circle, 10 nodes/wavelength, "
                    "N=16384, 1024 plane waves"),
}


def get(name: str) -> Workload:
    return WORKLOADS[name]


def _perimeter(zhat: np.ndarray, n: int = 4096) -> float:
    """Length of z(t) by the periodic trapezoid rule on |z'(t)| (spectrally accurate)."""
    M = (zhat.size - 1) // 2
    t = 2.0 * math.pi * np.arange(n) / n
    m = np.arange(-M, M + 1)
    dz = (1j * m * zhat)[None, :] * np.exp(1j * np.outer(t, m))
    return float(np.abs(dz.sum(axis=1)).mean() * 2.0 * math.pi)


def _convex(zhat: np.ndarray, n: int = 4096) -> bool:
    """Im(conj(z') z'') > 0 on n samples (counter-clockwise and convex)."""
    M = (zhat.size - 1) // 2
    t = 2.0 * math.pi * np.arange(n) / n
    m = np.arange(-M, M + 1)
    E = np.exp(1j * np.outer(t, m))
    d1 = (E * (1j * m * zhat)[None, :]).sum(axis=1)
    d2 = (E * (-(m ** 2) * zhat)[None, :]).sum(axis=1)
    return bool(np.all(np.imag(np.conj(d1) * d2) > 0.0))


def batch_problems(count: int = 64, seed: int = 0, n_range=(512, 8192), rhs_range=(32, 512),
                   nodes_per_wavelength: float = 10.0):
    """Seeded batch of perturbed ellipses of uneven size.

    Per problem, from numpy.random.default_rng(seed) in this order: semi-axes a ~ U(0.8, 1.2)
    and b ~ U(0.4, 0.8); radial perturbation 1 + sum_{m=2..8} c_m cos(m t + phi_m) of the
    ellipse z = a cos t + i b sin t with c_m ~ U(0, 0.02/m^2) (one vector) and
    phi_m ~ U(0, 2 pi) (one vector), redrawn until the contour is convex; N log-uniform in
    n_range (rounded); the number of plane waves uniform in rhs_range; k from the perimeter L
    at nodes_per_wavelength: k = 2 pi N / (nodes_per_wavelength L).  The contour's Fourier
    coefficients (modes -9..9) come from 64 samples of the band-limited z(t).
    Returns a list of dicts with zhat, n_nodes, k, angles."""
    rng = np.random.default_rng(seed)
    ms = np.arange(2, 9)
    out = []
    for _ in range(count):
        a = rng.uniform(0.8, 1.2)
        b = rng.uniform(0.4, 0.8)
        while True:
            c = rng.uniform(0.0, 0.02 / ms.astype(np.float64) ** 2)
            phi = rng.uniform(0.0, 2.0 * math.pi, size=ms.size)
            t = 2.0 * math.pi * np.arange(64) / 64
            r = 1.0 + (c[:, None] * np.cos(np.outer(ms, t) + phi[:, None])).sum(axis=0)
            z = (a * np.cos(t) + 1j * b * np.sin(t)) * r
            f = np.fft.fft(z) / 64
            M = 9
            zhat = np.concatenate([f[-M:], f[:M + 1]]).astype(np.complex128)
            if _convex(zhat):
                break
        N = int(round(math.exp(rng.uniform(math.log(n_range[0]), math.log(n_range[1])))))
        m = int(rng.integers(rhs_range[0], rhs_range[1] + 1))
        k = 2.0 * math.pi * N / (nodes_per_wavelength * _perimeter(zhat))
        out.append(dict(zhat=zhat, n_nodes=N, k=k, angles=plane_wave_angles(m)))
    return out

def shape_coeffs(seed: int = 0, mmax: int = 64, amp: float = 0.01):
    """Shape coefficients of r(theta) = 1 + sum_{m=1..mmax} s_m cos(m theta) + t_m sin(m theta)
    with s_m, t_m ~ N(0, (amp/m)^2): s drawn as one vector, then t, from
    numpy.random.default_rng(seed).  Returns (s, t)."""
    rng = np.random.default_rng(seed)
    ms = np.arange(1, mmax + 1, dtype=np.float64)
    s = rng.normal(0.0, 1.0, mmax) * (amp / ms)
    t = rng.normal(0.0, 1.0, mmax) * (amp / ms)
    return s, t


def shape_to_zhat(s, t) -> np.ndarray:
    """z(theta) = r(theta) e^{i theta} for the radial series of shape_coeffs, as Fourier
    modes -(mmax-1) .. mmax+1 (M = mmax + 1): cos(m th) e^{i th} = (e^{i(m+1)th} +
    e^{-i(m-1)th})/2 and sin(m th) e^{i th} = (e^{i(m+1)th} - e^{-i(m-1)th})/(2i)."""
    s = np.asarray(s, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    mmax = s.size
    M = mmax + 1
    zhat = np.zeros(2 * M + 1, dtype=np.complex128)
    zhat[M + 1] += 1.0
    for m in range(1, mmax + 1):
        zhat[M + 1 + m] += 0.5 * (s[m - 1] - 1j * t[m - 1])
        zhat[M + 1 - m] += 0.5 * (s[m - 1] + 1j * t[m - 1])
    return zhat


def shape_jacobian(mmax: int) -> np.ndarray:
    """d(Re zhat, Im zhat interleaved) / d(s_1..s_mmax, t_1..t_mmax): the real
    (2 (2M+1)) x (2 mmax) matrix of the linear map shape_to_zhat (M = mmax + 1)."""
    M = mmax + 1
    J = np.zeros((2 * (2 * M + 1), 2 * mmax))
    for m in range(1, mmax + 1):
        up, dn = M + 1 + m, M + 1 - m
        J[2 * up, m - 1] += 0.5
        J[2 * dn, m - 1] += 0.5
        J[2 * up + 1, mmax + m - 1] += -0.5
        J[2 * dn + 1, mmax + m - 1] += 0.5
    return J


def backscatter_angles(inc_angles, n_obs: int = 181) -> np.ndarray:
    """Observation angles around the backscatter direction of each incident wave: for the
    wave propagating along alpha_j, n_obs angles alpha_j + pi + (o - (n_obs-1)/2) pi/(n_obs-1),
    o = 0..n_obs-1 (the half circle facing the source, 1 degree apart for 181 angles, the
    exact backscatter direction in the middle).  Returns a (m, n_obs) array."""
    a = np.asarray(inc_angles, dtype=np.float64)
    o = np.arange(n_obs, dtype=np.float64)
    step = math.pi / max(n_obs - 1, 1)
    return a[:, None] + math.pi + (o[None, :] - (n_obs - 1) / 2.0) * step


def shape_problem(N: int = 8192, mmax: int = 64, seed: int = 0, n_inc: int = 16,
                  n_obs: int = 181, amp: float = 0.01, nodes_per_wavelength: float = 10.0):
    """The shape-differentiation workload: the seeded contour of shape_coeffs, N nodes, k at
    nodes_per_wavelength for the seed's perimeter, n_inc plane waves at 2 pi j / n_inc and
    n_obs backscatter observation angles per wave.  Returns a dict with s, t, zhat, n_nodes,
    k, angles (incident), obs (n_inc x n_obs)."""
    s, t = shape_coeffs(seed, mmax, amp)
    zhat = shape_to_zhat(s, t)
    k = 2.0 * math.pi * N / (nodes_per_wavelength * _perimeter(zhat, 8192))
    ang = plane_wave_angles(n_inc)
    return dict(s=s, t=t, zhat=zhat, n_nodes=N, k=k, angles=ang,
                obs=backscatter_angles(ang, n_obs))
