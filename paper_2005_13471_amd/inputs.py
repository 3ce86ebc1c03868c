"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle's
callers.

This module holds none of the method's arithmetic: no footprint, Gram filter,
interpolation or back projection.  It only draws the problem data that the
paper's experiments use (Sec. 6): uniformly spaced view angles, "Spots"
phantoms made of randomly placed ellipses rasterised to pixel coefficients,
uniform random coefficient images, Gaussian sinogram noise, and the analytic
line integrals of the continuous ellipse phantom (the data model g_s = S P f_c
of Sec. 2, applied to the continuous object rather than to its pixel
discretisation).

Everything is generated on the host in float64 with numpy's PCG64.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np


def angles(n: int) -> np.ndarray:
    """theta_i = i * pi / n, i = 0..n-1 (uniform in [0, pi))."""
    return np.arange(n, dtype=np.float64) * (np.pi / n)


@dataclass
class Ellipse:
    cx: float   # centre, pixel units, image centred at the origin
    cy: float
    a: float    # semi-axes, pixel units
    b: float
    phi: float  # rotation of the a-axis from the x1 axis
    rho: float  # density (added where ellipses overlap)


def random_ellipses(N: int, count: int, seed: int) -> list[Ellipse]:
    """Draw `count` ellipses, per ellipse in this order: centre x1, centre x2
    ~ U[-0.8, 0.8] * N/2; semi-axes ~ U[2, 20] * N/64; rotation ~ U[0, pi);
    density ~ U[-0.5, 1]."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for _ in range(count):
        cx, cy = rng.uniform(-0.8, 0.8, size=2) * (N / 2)
        a, b = rng.uniform(2.0, 20.0, size=2) * (N / 64)
        phi = rng.uniform(0.0, np.pi)
        rho = rng.uniform(-0.5, 1.0)
        out.append(Ellipse(float(cx), float(cy), float(a), float(b), float(phi), float(rho)))
    return out


def rasterize(N: int, ells: list[Ellipse], sub: int = 8) -> np.ndarray:
    """c[k2, k1] = sum_e rho_e * (fraction of the sub x sub sub-pixel centres
    of pixel k inside ellipse e).  Pixel k is centred at k - (N-1)/2."""
    img = np.zeros((N, N))
    offs = (np.arange(sub) + 0.5) / sub - 0.5
    for e in ells:
        r = max(e.a, e.b) + 1.0
        k1lo = max(int(np.floor(e.cx + (N - 1) / 2 - r)), 0)
        k1hi = min(int(np.ceil(e.cx + (N - 1) / 2 + r)), N - 1)
        k2lo = max(int(np.floor(e.cy + (N - 1) / 2 - r)), 0)
        k2hi = min(int(np.ceil(e.cy + (N - 1) / 2 + r)), N - 1)
        if k1lo > k1hi or k2lo > k2hi:
            continue
        x1 = (np.arange(k1lo, k1hi + 1) - (N - 1) / 2)[None, :, None, None] + offs[None, None, None, :]
        x2 = (np.arange(k2lo, k2hi + 1) - (N - 1) / 2)[:, None, None, None] + offs[None, None, :, None]
        dx, dy = x1 - e.cx, x2 - e.cy
        cp, sp = np.cos(e.phi), np.sin(e.phi)
        u = dx * cp + dy * sp
        v = -dx * sp + dy * cp
        inside = (u / e.a) ** 2 + (v / e.b) ** 2 <= 1.0
        img[k2lo:k2hi + 1, k1lo:k1hi + 1] += e.rho * inside.mean(axis=(2, 3))
    return img


def phantom(N: int, count: int, seed: int) -> tuple[np.ndarray, list[Ellipse]]:
    ells = random_ellipses(N, count, seed)
    return rasterize(N, ells), ells


def uniform_coeffs(N: int, seed: int) -> np.ndarray:
    """c ~ U[0, 1], i.i.d. per pixel."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(0.0, 1.0, size=(N, N))


def add_noise(sino: np.ndarray, eta: float, seed: int) -> np.ndarray:
    """g + N(0, sigma^2) with sigma = eta * RMS(g) over the whole sinogram."""
    if eta == 0.0:
        return sino.copy()
    rng = np.random.Generator(np.random.PCG64(seed))
    sigma = eta * float(np.sqrt(np.mean(np.square(sino))))
    return sino + rng.normal(0.0, sigma, size=sino.shape)


def analytic_sinogram(ells: list[Ellipse], theta: np.ndarray, M: int, ly: float = 1.0,
                      zeta: float = 0.0) -> np.ndarray:
    """Line integrals of the continuous ellipse phantom at y_m = ly (m - (M-1)/2),
    averaged over the detector cell [y_m - zeta/2, y_m + zeta/2] when zeta > 0.
    An ellipse with support function h in direction u has chord length
    (2ab/h^2) sqrt(h^2 - t^2) at offset t from its centre."""
    y = ly * (np.arange(M) - 0.5 * (M - 1))
    out = np.zeros((theta.size, M))
    c, s = np.cos(theta)[:, None], np.sin(theta)[:, None]
    for e in ells:
        cp, sp = np.cos(e.phi), np.sin(e.phi)
        ua = c * cp + s * sp           # u . a-axis
        ub = -c * sp + s * cp          # u . b-axis
        h = np.sqrt((e.a * ua) ** 2 + (e.b * ub) ** 2)
        t = y[None, :] - (e.cx * c + e.cy * s)
        k = 2.0 * e.a * e.b / h ** 2
        if zeta <= 0.0:
            out += e.rho * k * np.sqrt(np.clip(h * h - t * t, 0.0, None))
        else:
            def prim(v):
                v = np.clip(v, -h, h)
                return 0.5 * (v * np.sqrt(np.clip(h * h - v * v, 0.0, None)) + h * h * np.arcsin(v / h))
            out += e.rho * k * (prim(t + 0.5 * zeta) - prim(t - 0.5 * zeta)) / zeta
    return out


def detector_bins(N: int, zeta: float) -> int:
    """Smallest even M >= N sqrt(2) + zeta + 2: covers the projected support of
    an N x N image at every angle."""
    m = int(np.ceil(N * np.sqrt(2.0) + zeta + 2.0))
    return m + (m % 2)


# Workloads of the benchmark and the parity tests (sizes of the paper's
# experiments, Sec. 6: 64^2 ... 1024^2 images, up to 2048^2 for precision).
WORKLOADS = {
    "n64_a90_m92_z0": dict(N=64, n=90, M=92, ly=1.0, zeta=0.0, ellipses=10, eta=0.0,
                           seed=1000, coeff_seed=2000),
    "n512_a720_m730_z1": dict(N=512, n=720, M=730, ly=1.0, zeta=1.0, ellipses=40, eta=0.01,
                              seed=1000, coeff_seed=2000),
    "n2048_a1800_m2900_z1": dict(N=2048, n=1800, M=2900, ly=1.0, zeta=1.0, ellipses=100,
                                 eta=0.005, seed=1000, coeff_seed=2000),
    "n256_a180_m366_z1": dict(N=256, n=180, M=366, ly=1.0, zeta=1.0, ellipses=40, eta=0.01,
                              seed=1000, coeff_seed=2000),
}

NOISE_SEED_BASE = 1_000_000
