"""The seeded generators shared by tests, benchmark and training data: the
warm-start slice draw reproduces add_noise's normals, rasterisation
conserves ellipse area, and draws are deterministic per seed."""
import numpy as np
import pytest

from paper_2005_13471_amd import inputs


def test_noise_normals_match_add_noise():
    g = np.random.default_rng(0).normal(size=(7, 11))
    sigma = 0.01 * np.sqrt(np.mean(g * g))
    a = inputs.add_noise(g, 0.01, 123)
    assert np.array_equal(a, g + sigma * inputs.noise_normals(7, 11, 123))


def test_draw_slice_is_deterministic_and_consistent():
    c1, z1 = inputs.draw_slice((32, 5, 6, 50, 77))
    c2, z2 = inputs.draw_slice((32, 5, 6, 50, 77))
    assert np.array_equal(c1, c2) and np.array_equal(z1, z2)
    c, _ = inputs.phantom(32, 5, 77)
    assert np.array_equal(c1, c.astype(np.float32))
    assert np.array_equal(z1, inputs.noise_normals(6, 50, inputs.NOISE_SEED_BASE + 77).astype(np.float32))
    assert c1.dtype == np.float32 and z1.shape == (6, 50)


def test_rasterised_area_matches_ellipse():
    """A lone ellipse well inside the image covers pi a b pixels (sub-pixel
    counting error O(perimeter / sub))."""
    e = inputs.Ellipse(1.3, -2.1, 9.5, 5.25, 0.7, 1.0)
    img = inputs.rasterize(64, [e], sub=16)
    assert abs(img.sum() - np.pi * e.a * e.b) < 2.0 * np.pi * (e.a + e.b) / 16


@pytest.mark.parametrize("lx", [(1.0, 1.0), (0.8, 1.25), (1.3, 0.6)])
def test_rasterize_pixel_sides_keep_the_ellipse_area(lx):
    """Coefficients times the pixel area sum to the ellipse's area (to the
    sub-sampling error), whatever the pixel sides."""
    e = [inputs.Ellipse(1.5, -2.0, 11.0, 6.5, 0.3, 1.0)]
    c = inputs.rasterize(64, e, sub=24, lx=lx)
    assert abs(c.sum() * lx[0] * lx[1] - np.pi * 11.0 * 6.5) < 2e-3 * np.pi * 11.0 * 6.5


def test_ellipses_inside_the_disc():
    """The in-field phantoms keep the distributions' draw order and lie in
    the inscribed disc."""
    e = inputs.random_ellipses_inside(64, 20, 4243)
    assert len(e) == 20
    assert all(np.hypot(x.cx, x.cy) + max(x.a, x.b) <= 32.0 for x in e)
    assert e == inputs.random_ellipses_inside(64, 20, 4243)
