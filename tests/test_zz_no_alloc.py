"""gct_gram_apply_static (the entry point for callers that cannot allocate)
against gct_gram_apply through the C ABI: the same kernels on the same data,
so the outputs must agree bit for bit; two calls in a row, the second on a
smaller plan (the static scratch keeps the first call's contents), in FP32
and FP64; and a plan too large for the static scratch is refused."""
import numpy as np
import pytest
import torch

from paper_2005_13471_amd import inputs
from gpu_helpers import say

pytestmark = pytest.mark.gpu


def _setup(gct, N, n, zeta, dt):
    P = gct.Plan(N, inputs.angles(n), inputs.detector_bins(N, zeta), zeta=zeta)
    G = torch.empty(P.info.gram_elems, dtype=dt, device="cuda")
    gct.gram_build(P, G)
    Ghat = torch.empty(P.info.spectrum_elems, dtype=dt, device="cuda")
    gct.gram_spectrum(P, G, Ghat, P.workspace(gct.OP_GRAM_SPECTRUM, dt))
    return P, Ghat


@pytest.mark.parametrize("dt", [torch.float32, torch.float64])
def test_static_apply_equals_workspace_apply(dt):
    from paper_2005_13471_amd import gramct as gct
    for N, n, zeta, seed in ((300, 90, 1.0, 11), (64, 45, 0.0, 12)):
        say("gram_apply_static", N, n, zeta, dt)
        P, Ghat = _setup(gct, N, n, zeta, dt)
        c = torch.as_tensor(inputs.uniform_coeffs(N, seed).reshape(-1), dtype=dt, device="cuda")
        y_ws = torch.empty(N * N, dtype=dt, device="cuda")
        gct.gram_apply(P, Ghat, c, y_ws, P.workspace(gct.OP_GRAM_APPLY, dt))
        y_st = torch.full((N * N,), float("nan"), dtype=dt, device="cuda")
        gct.gram_apply_static(P, Ghat, c, y_st)
        torch.cuda.synchronize()
        assert torch.equal(y_st, y_ws), float((y_st - y_ws).abs().max())


def test_static_apply_refuses_too_large_plan():
    from paper_2005_13471_amd import gramct as gct
    dt = torch.float64
    N = 800  # needs 2 x 1025 x 800 x 16 bytes > 24 MiB in FP64
    P = gct.Plan(N, inputs.angles(8), inputs.detector_bins(N, 0.0))
    t = torch.zeros(N * N, dtype=dt, device="cuda")
    gh = torch.zeros(P.info.spectrum_elems, dtype=dt, device="cuda")
    with pytest.raises(gct.GramctError) as e:
        gct.gram_apply_static(P, gh, t, torch.empty_like(t))
    assert e.value.code == gct.GCT_EINVAL and "static" in str(e.value)
