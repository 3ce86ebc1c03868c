"""FP64 CPU reference of the warm-start U-Net (forward, loss, gradients).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: only ``tests/`` may
import it.  It shares no code with the product library; it follows the
network, parameter layout and loss that the library's U-Net interface
documents, written with plain PyTorch CPU operations in float64:

* 3x3 convolution with zero padding 1 and bias (cross-correlation:
  output(i, j) takes input (i + dy - 1, j + dx - 1) with weight tap
  t = 3 dy + dx, stored w[t][co][ci]);
* 2x2 max pooling;
* 2x2 stride-2 transposed convolution, w[2a + b][co][ci]: input pixel (i, j)
  feeds output pixel (2i + a, 2j + b);
* concatenation [up | skip], ReLU after every 3x3 convolution, a final 1x1
  convolution to one channel; input times in_scale, output times out_scale;
* loss = mean squared error; gradients by reverse-mode differentiation.

The paper reconstructs from zero (Sec. 6) and has no network; this is the
reference for the library's own addition.  Pins (tests): the building
blocks against explicit loops on tiny inputs, the gradients against central
finite differences.
"""
from __future__ import annotations

import numpy as np
import torch
import torch.nn.functional as F

CONV3, UPCONV, FINAL = 0, 1, 2


def _al64(n: int) -> int:
    return (n + 63) // 64 * 64


def layout(levels: int, base: int):
    """Layers in parameter order: list of dicts (kind, taps, cin, cout,
    nw, w_off, b_off) and the flat length.  Encoder (conv1, conv2) per level
    0..L-1, then per decoder level L-2..0 (upconv, conv1, conv2), then the
    final 1x1; weight then bias, each at a multiple of 64 elements."""
    C = [base << l for l in range(levels)]
    spec = []
    for l in range(levels):
        spec.append((CONV3, 16 if l == 0 else C[l - 1], C[l]))
        spec.append((CONV3, C[l], C[l]))
    for l in range(levels - 2, -1, -1):
        spec.append((UPCONV, C[l + 1], C[l]))
        spec.append((CONV3, 2 * C[l], C[l]))
        spec.append((CONV3, C[l], C[l]))
    spec.append((FINAL, base, 1))
    out, off = [], 0
    for kind, cin, cout in spec:
        taps = {CONV3: 9, UPCONV: 4, FINAL: 1}[kind]
        w_off = off
        off = _al64(off + taps * cout * cin)
        b_off = off
        off = _al64(off + cout)
        out.append(dict(kind=kind, taps=taps, cin=cin, cout=cout, w_off=w_off, b_off=b_off))
    return out, off


def _weights(p: torch.Tensor, ly: dict):
    n = ly["taps"] * ly["cout"] * ly["cin"]
    w = p[ly["w_off"]:ly["w_off"] + n].reshape(ly["taps"], ly["cout"], ly["cin"])
    b = p[ly["b_off"]:ly["b_off"] + ly["cout"]]
    return w, b


def conv3x3(x: torch.Tensor, w: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    """x [B][ci][H][W], w [9][co][ci] -> [B][co][H][W]."""
    wk = w.reshape(3, 3, w.shape[1], w.shape[2]).permute(2, 3, 0, 1)
    return F.conv2d(x, wk, b, padding=1)


def upconv(x: torch.Tensor, w: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    """x [B][ci][H][W], w [4][co][ci] -> [B][co][2H][2W]."""
    wk = w.reshape(2, 2, w.shape[1], w.shape[2]).permute(3, 2, 0, 1)
    return F.conv_transpose2d(x, wk, b, stride=2)


def conv1x1(x: torch.Tensor, w: torch.Tensor, b: torch.Tensor) -> torch.Tensor:
    return F.conv2d(x, w.reshape(w.shape[1], w.shape[2], 1, 1), b)


def forward(params, x, levels: int, base: int, in_scale: float = 1.0, out_scale: float = 1.0):
    """y = out_scale * net(in_scale * x); params flat (length from layout),
    x [B][H][W].  Accepts numpy or torch; computes in float64."""
    p = torch.as_tensor(params, dtype=torch.float64)
    xin = torch.as_tensor(x, dtype=torch.float64)
    return _forward(p, xin, levels, base, in_scale, out_scale)


def _forward(p, x, levels, base, in_scale, out_scale):
    lys, n = layout(levels, base)
    assert p.numel() == n
    Bn = x.shape[0]
    h = torch.zeros(Bn, 16, x.shape[1], x.shape[2], dtype=torch.float64)
    h[:, 0] = x * in_scale
    it = iter(lys)
    skips = []
    for l in range(levels):
        h = torch.relu(conv3x3(h, *_weights(p, next(it))))
        h = torch.relu(conv3x3(h, *_weights(p, next(it))))
        if l < levels - 1:
            skips.append(h)
            h = F.max_pool2d(h, 2)
    for l in range(levels - 2, -1, -1):
        up = upconv(h, *_weights(p, next(it)))
        h = torch.cat([up, skips[l]], dim=1)
        h = torch.relu(conv3x3(h, *_weights(p, next(it))))
        h = torch.relu(conv3x3(h, *_weights(p, next(it))))
    y = conv1x1(h, *_weights(p, next(it)))
    return out_scale * y[:, 0]


def loss_and_grad(params, x, target, levels: int, base: int, in_scale: float = 1.0,
                  out_scale: float = 1.0):
    """(loss, y, grad): loss = mean((y - target)^2) over all pixels, grad the
    gradient of the loss with respect to the flat parameters (numpy fp64)."""
    p = torch.tensor(np.asarray(params, dtype=np.float64), requires_grad=True)
    xin = torch.as_tensor(x, dtype=torch.float64)
    t = torch.as_tensor(target, dtype=torch.float64)
    y = _forward(p, xin, levels, base, in_scale, out_scale)
    loss = torch.mean((y - t) ** 2)
    loss.backward()
    return float(loss.detach()), y.detach().numpy(), p.grad.numpy().copy()


def loss_only(params, x, target, levels: int, base: int, in_scale: float = 1.0,
              out_scale: float = 1.0) -> float:
    with torch.no_grad():
        y = forward(params, x, levels, base, in_scale, out_scale)
        return float(torch.mean((y - torch.as_tensor(target, dtype=torch.float64)) ** 2))


def adam(w, g, m, v, step: int, lr: float, b1: float, b2: float, eps: float):
    """One Adam step (Kingma & Ba, Algorithm 1) in float64; returns (w, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return w - lr * mh / (np.sqrt(vh) + eps), m, v
