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


def random_ellipses_inside(N: float, count: int, seed: int, radius: float | None = None) -> list[Ellipse]:
    """As random_ellipses (same distributions, same generator), keeping only
    ellipses that lie inside the disc of `radius` (default N/2, the disc
    inscribed in the image) until `count` are kept: a phantom wholly inside
    the field of view, so that exact data contain nothing the image cannot
    represent."""
    rng = np.random.Generator(np.random.PCG64(seed))
    R = 0.5 * N if radius is None else float(radius)
    out = []
    while len(out) < count:
        cx, cy = rng.uniform(-0.8, 0.8, size=2) * (N / 2)
        a, b = rng.uniform(2.0, 20.0, size=2) * (N / 64)
        phi = rng.uniform(0.0, np.pi)
        rho = rng.uniform(-0.5, 1.0)
        if np.hypot(cx, cy) + max(a, b) <= R:
            out.append(Ellipse(float(cx), float(cy), float(a), float(b), float(phi), float(rho)))
    return out


def rasterize(N: int, ells: list[Ellipse], sub: int = 8, lx=(1.0, 1.0)) -> np.ndarray:
    """c[k2, k1] = sum_e rho_e * (fraction of the sub x sub sub-pixel centres
    of pixel k inside ellipse e).  Pixel k is the lx[0] x lx[1] rectangle
    centred at (lx[0] (k1 - (N-1)/2), lx[1] (k2 - (N-1)/2)).  Counted
    exactly per sub-row: the ellipse cuts each sub-row in one interval of x,
    and the sub-sample centres of a pixel inside an interval are counted
    arithmetically."""
    img = np.zeros((N, N))
    offs = (np.arange(sub) + 0.5) / sub - 0.5
    h = 0.5 * (N - 1)
    l1, l2 = float(lx[0]), float(lx[1])
    for e in ells:
        r = max(e.a, e.b) + max(l1, l2)
        k1lo = max(int(np.floor((e.cx - r) / l1 + h)), 0)
        k1hi = min(int(np.ceil((e.cx + r) / l1 + h)), N - 1)
        k2lo = max(int(np.floor((e.cy - r) / l2 + h)), 0)
        k2hi = min(int(np.ceil((e.cy + r) / l2 + h)), N - 1)
        if k1lo > k1hi or k2lo > k2hi:
            continue
        cp, sp = np.cos(e.phi), np.sin(e.phi)
        ia2, ib2 = 1.0 / e.a ** 2, 1.0 / e.b ** 2
        # sub-row y values, shape (rows * sub,)
        y = (l2 * ((np.arange(k2lo, k2hi + 1) - h)[:, None] + offs[None, :])).reshape(-1)
        dy = y - e.cy
        A = cp * cp * ia2 + sp * sp * ib2
        B = 2.0 * dy * cp * sp * (ia2 - ib2)
        C = dy * dy * (sp * sp * ia2 + cp * cp * ib2) - 1.0
        disc = B * B - 4.0 * A * C
        ok = disc >= 0.0
        sq = np.sqrt(np.where(ok, disc, 0.0))
        xlo = np.where(ok, e.cx + (-B - sq) / (2.0 * A), np.inf)[:, None] / l1
        xhi = np.where(ok, e.cx + (-B + sq) / (2.0 * A), -np.inf)[:, None] / l1
        x1 = (np.arange(k1lo, k1hi + 1) - h)[None, :]
        qlo = np.ceil((xlo - x1 + 0.5) * sub - 0.5)
        qhi = np.floor((xhi - x1 + 0.5) * sub - 0.5)
        cnt = np.clip(np.minimum(qhi, sub - 1) - np.maximum(qlo, 0) + 1, 0, None)
        cnt = cnt.reshape(k2hi - k2lo + 1, sub, k1hi - k1lo + 1).sum(axis=1)
        img[k2lo:k2hi + 1, k1lo:k1hi + 1] += e.rho * cnt / (sub * sub)
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


def noise_normals(n: int, M: int, seed: int) -> np.ndarray:
    """The standard normals that add_noise(., eta, seed) scales by sigma for
    an n x M sinogram (same generator and draw order)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.standard_normal(size=(n, M))


def draw_slice(args) -> tuple[np.ndarray, np.ndarray]:
    """Phantom coefficients and sinogram noise normals of one training or
    test slice: args = (N, ellipses, n, M, seed); the noise uses seed
    NOISE_SEED_BASE + seed.  Returned as float32 (a process-pool worker)."""
    N, count, n, M, seed = args
    c, _ = phantom(N, count, seed)
    z = noise_normals(n, M, NOISE_SEED_BASE + seed)
    return c.astype(np.float32), z.astype(np.float32)


def analytic_sinogram(ells: list[Ellipse], theta: np.ndarray, M: int, ly: float = 1.0,
                      zeta: float = 0.0) -> np.ndarray:
    """Line integrals of the continuous ellipse phantom at y_m = ly (m - (M-1)/2),
    averaged over the detector cell [y_m - zeta/2, y_m + zeta/2] when zeta > 0.
    An ellipse with support function h in direction u has chord length
    (2ab/h^2) sqrt(h^2 - t^2) at offset t from its centre.  Only the bins
    inside each ellipse's shadow are evaluated."""
    n = theta.size
    out = np.zeros(n * M)
    c, s = np.cos(theta), np.sin(theta)
    half = 0.5 * zeta
    for e in ells:
        cp, sp = np.cos(e.phi), np.sin(e.phi)
        h = np.sqrt((e.a * (c * cp + s * sp)) ** 2 + (e.b * (-c * sp + s * cp)) ** 2)
        ctr = e.cx * c + e.cy * s
        k = 2.0 * e.a * e.b / h ** 2
        # bins whose (cell-averaged) sample can touch the shadow [ctr - h, ctr + h]
        mlo = np.maximum(np.ceil((ctr - h - half) / ly + 0.5 * (M - 1)).astype(np.int64), 0)
        mhi = np.minimum(np.floor((ctr + h + half) / ly + 0.5 * (M - 1)).astype(np.int64), M - 1)
        cnt = np.maximum(mhi - mlo + 1, 0)
        if cnt.sum() == 0:
            continue
        a_idx = np.repeat(np.arange(n), cnt)
        start = np.repeat(np.cumsum(cnt) - cnt, cnt)
        m = np.repeat(mlo, cnt) + (np.arange(cnt.sum()) - start)
        hh, kk = h[a_idx], k[a_idx]
        t = ly * (m - 0.5 * (M - 1)) - ctr[a_idx]
        if zeta <= 0.0:
            val = kk * np.sqrt(np.clip(hh * hh - t * t, 0.0, None))
        else:
            def prim(v):
                v = np.clip(v, -hh, hh)
                return 0.5 * (v * np.sqrt(np.clip(hh * hh - v * v, 0.0, None)) + hh * hh * np.arcsin(v / hh))
            val = kk * (prim(t + half) - prim(t - half)) / zeta
        np.add.at(out, a_idx * M + m, e.rho * val)
    return out.reshape(n, M)


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
