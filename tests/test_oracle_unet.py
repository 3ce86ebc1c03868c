"""Pins of the FP64 reference U-Net in oracle/unet.py: its building blocks
against explicit loops on tiny inputs, the documented tap orientation by
exact shifts, its gradients against central finite differences, and the
first Adam step against its closed form."""
import numpy as np
import pytest
import torch

from oracle import unet as ou


def _rng(seed):
    return np.random.Generator(np.random.PCG64(seed))


def test_conv3x3_matches_loops():
    r = _rng(1)
    x = r.normal(size=(2, 3, 5, 4))
    w = r.normal(size=(9, 2, 3))
    b = r.normal(size=2)
    got = ou.conv3x3(torch.tensor(x), torch.tensor(w), torch.tensor(b)).numpy()
    ref = np.zeros((2, 2, 5, 4))
    for n in range(2):
        for co in range(2):
            for i in range(5):
                for j in range(4):
                    s = b[co]
                    for dy in range(3):
                        for dx in range(3):
                            ii, jj = i + dy - 1, j + dx - 1
                            if 0 <= ii < 5 and 0 <= jj < 4:
                                s += sum(w[3 * dy + dx, co, ci] * x[n, ci, ii, jj] for ci in range(3))
                    ref[n, co, i, j] = s
    assert np.max(np.abs(got - ref)) < 1e-12


def test_upconv_matches_loops():
    r = _rng(2)
    x = r.normal(size=(1, 3, 3, 2))
    w = r.normal(size=(4, 2, 3))
    b = r.normal(size=2)
    got = ou.upconv(torch.tensor(x), torch.tensor(w), torch.tensor(b)).numpy()
    ref = np.zeros((1, 2, 6, 4))
    for co in range(2):
        ref[0, co] += b[co]
        for i in range(3):
            for j in range(2):
                for a in range(2):
                    for bb in range(2):
                        ref[0, co, 2 * i + a, 2 * j + bb] += sum(
                            w[2 * a + bb, co, ci] * x[0, ci, i, j] for ci in range(3))
    assert np.max(np.abs(got - ref)) < 1e-12


def test_conv1x1_matches_loops():
    r = _rng(3)
    x = r.normal(size=(2, 4, 3, 3))
    w = r.normal(size=(1, 1, 4))
    b = r.normal(size=1)
    got = ou.conv1x1(torch.tensor(x), torch.tensor(w), torch.tensor(b)).numpy()[:, 0]
    ref = np.einsum("c,ncij->nij", w[0, 0], x) + b[0]
    assert np.max(np.abs(got - ref)) < 1e-12


def _identity_net(tap):
    """One level, C0 = 16: conv1 moves input channel 0 by `tap`, conv2 and the
    final 1x1 pass channel 0 through."""
    lys, n = ou.layout(1, 16)
    p = np.zeros(n)
    c1, c2, fin = lys
    p[c1["w_off"] + (tap * 16 + 0) * 16 + 0] = 1.0
    p[c2["w_off"] + (4 * 16 + 0) * 16 + 0] = 1.0
    p[fin["w_off"]] = 1.0
    return p


@pytest.mark.parametrize("tap", range(9))
def test_forward_tap_orientation(tap):
    """With only tap t = 3 dy + dx of the first convolution set, the network
    output is the input moved by (dy - 1, dx - 1), zero outside."""
    x = _rng(4).uniform(0.0, 1.0, size=(1, 6, 5))
    y = ou.forward(_identity_net(tap), x, 1, 16, in_scale=2.0, out_scale=0.5).numpy()
    dy, dx = divmod(tap, 3)
    ref = np.zeros_like(x)
    for i in range(6):
        for j in range(5):
            ii, jj = i + dy - 1, j + dx - 1
            if 0 <= ii < 6 and 0 <= jj < 5:
                ref[0, i, j] = x[0, ii, jj]
    assert np.max(np.abs(y - ref)) < 1e-14


def test_upconv_path_places_pixels():
    """Two levels with the decoder's skip half zeroed: the output at (2i+a,
    2j+b) is the pooled value times the transposed-convolution tap 2a+b."""
    lys, n = ou.layout(2, 16)
    p = np.zeros(n)
    e1, e2, b1, b2, up, d1, d2, fin = lys
    p[e1["w_off"] + (4 * 16 + 0) * 16 + 0] = 1.0        # level 0: pass channel 0
    p[e2["w_off"] + (4 * 16 + 0) * 16 + 0] = 1.0
    p[b1["w_off"] + (4 * 32 + 0) * 16 + 0] = 1.0        # bottleneck: pass channel 0
    p[b2["w_off"] + (4 * 32 + 0) * 32 + 0] = 1.0
    taps = [1.0, 2.0, 3.0, 4.0]
    for t in range(4):
        p[up["w_off"] + (t * 16 + 0) * 32 + 0] = taps[t]  # up: channel 0 -> 0 scaled by tap
    p[d1["w_off"] + (4 * 16 + 0) * 32 + 0] = 1.0         # decoder conv1 reads the up half only
    p[d2["w_off"] + (4 * 16 + 0) * 16 + 0] = 1.0
    p[fin["w_off"]] = 1.0
    x = _rng(5).uniform(0.0, 1.0, size=(1, 4, 6))
    y = ou.forward(p, x, 2, 16).numpy()[0]
    pooled = x[0].reshape(2, 2, 3, 2).max(axis=(1, 3))
    ref = np.zeros((4, 6))
    for i in range(2):
        for j in range(3):
            for a in range(2):
                for b in range(2):
                    ref[2 * i + a, 2 * j + b] = taps[2 * a + b] * pooled[i, j]
    assert np.max(np.abs(y - ref)) < 1e-14


def _random_params(levels, base, seed, scale=1.0):
    lys, n = ou.layout(levels, base)
    r = _rng(seed)
    p = np.zeros(n)
    for ly in lys:
        fan = ly["taps"] * (1 if ly["w_off"] == 0 else ly["cin"])
        nw = ly["taps"] * ly["cout"] * ly["cin"]
        p[ly["w_off"]:ly["w_off"] + nw] = r.normal(0.0, scale * np.sqrt(2.0 / fan), size=nw)
        p[ly["b_off"]:ly["b_off"] + ly["cout"]] = r.normal(0.0, 0.1, size=ly["cout"])
    return p


def test_gradient_matches_finite_differences():
    levels, base = 2, 16
    r = _rng(6)
    x = r.uniform(-1.0, 1.0, size=(2, 8, 8))
    t = r.uniform(-1.0, 1.0, size=(2, 8, 8))
    p = _random_params(levels, base, 7)
    loss, _, g = ou.loss_and_grad(p, x, t, levels, base, in_scale=1.5, out_scale=0.7)
    lys, _ = ou.layout(levels, base)
    h = 1e-6
    checked = 0
    for ly in lys:
        cin = 1 if ly["w_off"] == 0 else ly["cin"]   # first layer: only channel 0 is fed
        idx = [ly["w_off"] + (tap * ly["cout"] + co) * ly["cin"] + ci
               for tap, co, ci in [(0, 0, 0), (ly["taps"] - 1, ly["cout"] - 1, cin - 1),
                                   (ly["taps"] // 2, ly["cout"] // 2, cin // 2)]]
        idx.append(ly["b_off"] + ly["cout"] - 1)
        for i in idx:
            pp, pm = p.copy(), p.copy()
            pp[i] += h
            pm[i] -= h
            fd = (ou.loss_only(pp, x, t, levels, base, 1.5, 0.7) -
                  ou.loss_only(pm, x, t, levels, base, 1.5, 0.7)) / (2 * h)
            assert abs(fd - g[i]) <= 1e-6 * max(1.0, abs(g[i])) + 1e-8, (ly, i, fd, g[i])
            checked += 1
    assert checked == 4 * len(lys)
    # dead input channels of the first layer see zeros: exactly zero gradient
    first = lys[0]
    w = g[first["w_off"]:first["w_off"] + 9 * base * 16].reshape(9, base, 16)
    assert np.all(w[:, :, 1:] == 0.0) and np.any(w[:, :, 0] != 0.0)


def test_loss_gradient_of_output_scale():
    """d loss / d(final bias) = out_scale * mean(2 (y - t)): the chain rule
    through the output scale, checked without differentiation."""
    levels, base = 1, 16
    r = _rng(8)
    x = r.uniform(-1.0, 1.0, size=(3, 4, 4))
    t = r.uniform(-1.0, 1.0, size=(3, 4, 4))
    p = _random_params(levels, base, 9)
    _, y, g = ou.loss_and_grad(p, x, t, levels, base, out_scale=2.5)
    fin = ou.layout(levels, base)[0][-1]
    assert abs(g[fin["b_off"]] - 2.5 * np.mean(2 * (y - t))) < 1e-12


def test_adam_first_step_is_signed_lr():
    """After one step from zero moments the bias-corrected update is
    lr g / (|g| + eps): lr times the sign of g up to eps."""
    r = _rng(10)
    w = r.normal(size=50)
    g = r.normal(size=50)
    w1, m, v = ou.adam(w, g, np.zeros(50), np.zeros(50), 1, 1e-3, 0.9, 0.999, 1e-12)
    assert np.allclose(w - w1, 1e-3 * np.sign(g), atol=1e-12)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
