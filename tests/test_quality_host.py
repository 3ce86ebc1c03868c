"""CPU checks of the reconstruction-quality metrics: SNR against its
closed form, SSIM against a direct windowed sum written out here and
against the properties that define it."""
import math

import numpy as np
import pytest

from paper_2005_13471_amd import quality


def test_snr_closed_form():
    rng = np.random.default_rng(0)
    ref = rng.uniform(0.5, 1.5, size=(32, 32))
    e = rng.normal(size=ref.shape)
    e *= 0.1 * np.linalg.norm(ref) / np.linalg.norm(e)   # ||e|| = 0.1 ||ref||
    assert quality.snr_db(ref + e, ref) == pytest.approx(20.0, abs=1e-9)
    assert quality.snr_db(2.0 * ref, ref) == pytest.approx(0.0, abs=1e-12)


def _ssim_direct(x, y, L, sigma=1.5, k1=0.01, k2=0.03):
    """Gaussian-weighted local statistics by explicit sums over an 11 x 11
    window with reflected borders (x[-1] = x[0], numpy 'symmetric'),
    averaged over the pixels whose window fits."""
    r = int(3.5 * sigma + 0.5)
    t = np.arange(-r, r + 1)
    w1 = np.exp(-0.5 * (t / sigma) ** 2)
    w1 /= w1.sum()
    w = np.outer(w1, w1)
    c1, c2 = (k1 * L) ** 2, (k2 * L) ** 2
    xp, yp = np.pad(x, r, mode="symmetric"), np.pad(y, r, mode="symmetric")
    n1, n2 = x.shape
    vals = []
    for i in range(r, n1 - r):
        for j in range(r, n2 - r):
            px = xp[i:i + 2 * r + 1, j:j + 2 * r + 1]
            py = yp[i:i + 2 * r + 1, j:j + 2 * r + 1]
            mx, my = (w * px).sum(), (w * py).sum()
            sxx = (w * px * px).sum() - mx * mx
            syy = (w * py * py).sum() - my * my
            sxy = (w * px * py).sum() - mx * my
            vals.append(((2 * mx * my + c1) * (2 * sxy + c2)) / ((mx * mx + my * my + c1) * (sxx + syy + c2)))
    return float(np.mean(vals))


def test_ssim_against_direct_sum():
    rng = np.random.default_rng(1)
    y = rng.uniform(0.0, 1.0, size=(20, 23))
    x = y + 0.2 * rng.normal(size=y.shape)
    got = quality.ssim(x, y)
    ref = _ssim_direct(x, y, float(y.max() - y.min()))
    assert got == pytest.approx(ref, rel=1e-10)


def test_ssim_properties():
    rng = np.random.default_rng(2)
    y = rng.uniform(0.0, 1.0, size=(24, 24))
    assert quality.ssim(y, y) == pytest.approx(1.0, abs=1e-12)
    x = y + 0.1 * rng.normal(size=y.shape)
    assert quality.ssim(x, y) == pytest.approx(quality.ssim(y, x, data_range=float(y.max() - y.min())), abs=1e-12)
    assert quality.ssim(x, y) < quality.ssim(0.5 * (x + y), y) < 1.0


def test_detector_bins_cover_the_image():
    for N in (64, 128):
        for ly in (0.25, 0.5, 1.0, 2.0):
            M = quality.detector_bins(N, 1.0, ly)
            assert M % 2 == 0 and M * ly >= N * math.sqrt(2.0) + 1.0 + 2 * ly
