"""Warm-start U-Net through the C ABI against the FP64 CPU reference
(oracle/unet.py): parameter layout, forward output, loss, every layer's
weight and bias gradient, and the Adam step.

Inputs and weights are drawn BF16-representable, so both sides start from
the same values; the differences left are the GPU's BF16 rounding of every
activation and activation gradient (unit roundoff u = 2^-9) and its FP32
accumulation.  Tolerances: a rounding error of relative size u enters at
each of the D layers on the path and the errors add up about like a random
walk, so the normwise error of the output is about sqrt(D) u ~ 1e-2 for the
18 layers of the 4-level net; bounds are 2.5e-2 for outputs and loss and
6e-2 for gradients (which cross the path twice)."""
import numpy as np
import pytest
import torch

from oracle import unet as ou
from gpu_helpers import say

pytestmark = pytest.mark.gpu

TOL_Y, TOL_G = 2.5e-2, 6e-2


def bf16(a):
    """Round to the nearest BF16 value (ties to even), returned as float64."""
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def rel(a, b):
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / max(np.linalg.norm(np.ravel(b)), 1e-300))


def he_params(levels, base, seed):
    lys, n = ou.layout(levels, base)
    r = np.random.Generator(np.random.PCG64(seed))
    p = np.zeros(n)
    for i, ly in enumerate(lys):
        fan = ly["taps"] * (1 if i == 0 else ly["cin"])
        nw = ly["taps"] * ly["cout"] * ly["cin"]
        w = r.normal(0.0, np.sqrt(2.0 / fan), size=nw)
        if i == 0:
            w = w.reshape(ly["taps"], ly["cout"], ly["cin"])
            w[:, :, 1:] = 0.0
            w = w.reshape(-1)
        p[ly["w_off"]:ly["w_off"] + nw] = w
        p[ly["b_off"]:ly["b_off"] + ly["cout"]] = r.normal(0.0, 0.05, size=ly["cout"])
    return bf16(p)


def _gpu(a):
    return torch.as_tensor(np.asarray(a, dtype=np.float32), device="cuda").contiguous()


@pytest.fixture(scope="module")
def gct():
    from paper_2005_13471_amd import gramct
    return gramct


@pytest.mark.parametrize("levels,base", [(1, 16), (3, 16), (4, 32)])
def test_layout_matches_reference(gct, levels, base):
    net = gct.UNet(levels, base, 16 << (levels - 1), 16 << (levels - 1), 1)
    lys, n = ou.layout(levels, base)
    assert net.n_params == n
    assert len(net.layers) == len(lys)
    for a, b in zip(net.layers, lys):
        assert (a["kind"], a["taps"], a["cin"], a["cout"], a["w_off"], a["b_off"]) == \
            (b["kind"], b["taps"], b["cin"], b["cout"], b["w_off"], b["b_off"])


def _case(gct, levels, base, H, W, B, seed):
    say("unet case", levels, base, H, W, B, seed)
    p = he_params(levels, base, seed)
    r = np.random.Generator(np.random.PCG64(seed + 1))
    x = bf16(r.uniform(-1.0, 1.0, size=(B, H, W)))
    t = r.uniform(-1.0, 1.0, size=(B, H, W))
    net = gct.UNet(levels, base, H, W, B)
    gct.unet_set_params(net, _gpu(p))
    xg, tg = _gpu(x), _gpu(t)
    y = torch.empty_like(xg)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    gct.unet_forward(net, xg, y, in_scale=0.5, out_scale=2.0)
    gct.unet_backward(net, y, tg, loss)
    g = torch.empty(net.n_params, dtype=torch.float32, device="cuda")
    gct.unet_get_grads(net, g)
    torch.cuda.synchronize()
    l_ref, y_ref, g_ref = ou.loss_and_grad(p, x, t.astype(np.float32).astype(np.float64), levels, base,
                                           in_scale=0.5, out_scale=2.0)
    return net, p, y.double().cpu().numpy(), float(loss.item()), g.double().cpu().numpy(), y_ref, l_ref, g_ref


@pytest.mark.parametrize("levels,base,H,W,B", [(1, 16, 16, 24, 2), (3, 16, 32, 32, 2), (4, 32, 256, 256, 1)])
def test_forward_backward_match_reference(gct, levels, base, H, W, B):
    net, p, y, loss, g, y_ref, l_ref, g_ref = _case(gct, levels, base, H, W, B, 11 + levels)
    ey = rel(y, y_ref)
    say("  y", ey, "loss", loss, l_ref)
    assert ey <= TOL_Y
    assert abs(loss - l_ref) <= TOL_Y * l_ref
    lys, _ = ou.layout(levels, base)
    worst = 0.0
    for i, ly in enumerate(lys):
        nw = ly["taps"] * ly["cout"] * ly["cin"]
        ws = slice(ly["w_off"], ly["w_off"] + nw)
        bs = slice(ly["b_off"], ly["b_off"] + ly["cout"])
        ew, eb = rel(g[ws], g_ref[ws]), rel(g[bs], g_ref[bs])
        say("  layer", i, "kind", ly["kind"], "cin", ly["cin"], "cout", ly["cout"], "dW", ew, "db", eb)
        worst = max(worst, ew, eb)
        assert ew <= TOL_G and eb <= TOL_G, (i, ew, eb)
    # the gaps between blocks and the unfed input channels stay exactly zero
    used = np.zeros(g.size, bool)
    for ly in lys:
        used[ly["w_off"]:ly["w_off"] + ly["taps"] * ly["cout"] * ly["cin"]] = True
        used[ly["b_off"]:ly["b_off"] + ly["cout"]] = True
    assert np.all(g[~used] == 0.0)
    first = g[:9 * base * 16].reshape(9, base, 16)
    assert np.all(first[:, :, 1:] == 0.0)
    say("  worst gradient error", worst)


def test_adam_step_matches_reference(gct):
    levels, base, H, W, B = 2, 16, 16, 16, 2
    net, p, y, loss, g, *_ = _case(gct, levels, base, H, W, B, 31)
    w = p.copy()
    m = np.zeros_like(w)
    v = np.zeros_like(w)
    # the hyper-parameters are FP32 arguments: the reference takes the same
    # rounded values (1 - float32(0.999) differs from 0.001 by 1.3e-5)
    lr, b1, b2, eps = (float(np.float32(a)) for a in (1e-3, 0.9, 0.999, 1e-8))
    for step in (1, 2, 3):
        gct.unet_adam_step(net, lr, step, b1, b2, eps)
        w, m, v = ou.adam(w, g, m, v, step, lr, b1, b2, eps)
    wg = torch.empty(net.n_params, dtype=torch.float32, device="cuda")
    mg, vg = torch.empty_like(wg), torch.empty_like(wg)
    gct.unet_get_params(net, wg)
    gct.unet_get_moments(net, mg, vg)
    torch.cuda.synchronize()
    assert np.max(np.abs(wg.double().cpu().numpy() - w)) <= 1e-6 * max(1.0, np.max(np.abs(w)))
    assert rel(mg.double().cpu().numpy(), m) <= 1e-6
    assert rel(vg.double().cpu().numpy(), v) <= 1e-6


def test_training_steps_reduce_loss(gct):
    """Adam on one fixed batch: the loss after 30 steps is well below the
    first (the kernels' gradients point downhill)."""
    levels, base, H, W, B = 3, 16, 32, 32, 4
    p = he_params(levels, base, 41)
    r = np.random.Generator(np.random.PCG64(42))
    x = r.uniform(0.0, 1.0, size=(B, H, W))
    t = 0.5 * x + 0.25 * np.roll(x, 1, axis=2)
    net = gct.UNet(levels, base, H, W, B)
    gct.unet_set_params(net, _gpu(p))
    xg, tg = _gpu(x), _gpu(t)
    y = torch.empty_like(xg)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    hist = []
    for step in range(1, 31):
        gct.unet_forward(net, xg, y)
        gct.unet_backward(net, y, tg, loss)
        gct.unet_adam_step(net, 2e-3, step)
        hist.append(float(loss.item()))
    say("  loss", hist[0], "->", hist[-1])
    assert np.all(np.isfinite(hist))
    assert hist[-1] < 0.2 * hist[0]


def test_forward_replays_follow_buffers_and_weights(gct):
    """The forward is replayed from captured graphs keyed by its arguments:
    a replay reads the current contents of x and the current weights, and
    more argument sets than the cache holds still give the same outputs."""
    levels, base, H, W = 2, 16, 16, 16
    p1, p2 = he_params(levels, base, 51), he_params(levels, base, 52)
    r = np.random.Generator(np.random.PCG64(53))
    x1, x2 = _gpu(r.uniform(-1, 1, size=(H, W))), _gpu(r.uniform(-1, 1, size=(H, W)))
    net = gct.UNet(levels, base, H, W, 1)
    gct.unet_set_params(net, _gpu(p1))
    ya, yb = torch.empty_like(x1), torch.empty_like(x1)
    gct.unet_forward(net, x1, ya)
    gct.unet_forward(net, x2, yb)
    ref1, ref2 = ya.clone(), yb.clone()
    assert not torch.equal(ref1, ref2)
    # same addresses, new contents: the replay follows x
    xs = x1.clone()
    gct.unet_forward(net, xs, ya)
    xs.copy_(x2)
    gct.unet_forward(net, xs, ya)
    assert torch.equal(ya, ref2)
    # more argument sets than cached graphs, then the first again
    outs = [torch.empty_like(x1) for _ in range(10)]
    for y in outs:
        gct.unet_forward(net, x1, y)
    for y in outs:
        assert torch.equal(y, ref1)
    gct.unet_forward(net, x2, ya)
    assert torch.equal(ya, ref2)
    # new weights: the replay reads them; a fresh net agrees
    gct.unet_set_params(net, _gpu(p2))
    gct.unet_forward(net, x1, ya)
    fresh = gct.UNet(levels, base, H, W, 1)
    gct.unet_set_params(fresh, _gpu(p2))
    gct.unet_forward(fresh, x1, yb)
    torch.cuda.synchronize()
    assert torch.equal(ya, yb) and not torch.equal(ya, ref1)
    # scales are part of the key
    gct.unet_forward(net, x1, ya, in_scale=1.0, out_scale=3.0)
    gct.unet_forward(net, x1, yb, in_scale=1.0, out_scale=1.0)
    torch.cuda.synchronize()
    assert torch.allclose(ya, 3.0 * yb, rtol=1e-6, atol=0)


def test_unet_rejects_bad_calls(gct):
    net = gct.UNet(2, 16, 16, 16, 2)
    x = torch.zeros(3 * 256, dtype=torch.float32, device="cuda")
    y = torch.zeros_like(x)
    with pytest.raises(gct.GramctError) as e:
        gct.unet_forward(net, x, y, batch=3)
    assert e.value.code == gct.GCT_EINVAL
    gct.unet_forward(net, x, y, batch=2)
    with pytest.raises(gct.GramctError) as e:
        gct.unet_backward(net, y, x, batch=1)
    assert e.value.code == gct.GCT_EINVAL
    with pytest.raises(gct.GramctError) as e:
        gct.unet_adam_step(net, 1e-3, 0)
    assert e.value.code == gct.GCT_EINVAL
