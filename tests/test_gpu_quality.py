"""Reconstruction quality on the GPU (the paper's 2D reconstruction
experiments, Sec. 6.2, 6.3) at a small size: exact sinograms of an ellipse
phantom, steepest descent and CG to the stopping rule, SNR and SSIM against
the 10x pixel-basis ground truth."""
import numpy as np
import pytest

from gpu_helpers import say
from paper_2005_13471_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def Q():
    from paper_2005_13471_amd import quality
    return quality


def test_noise_lowers_quality_and_both_solvers_converge(Q):
    N, n = 64, 180
    ells = inputs.random_ellipses(N, 12, 77)
    ref = Q.ground_truth(N, ells)
    out = {}
    for eta in (0.0, 0.05):
        for solver in ("sd", "cg"):
            x, res = Q.reconstruct(N, n, 1.0, 1.0, ells, eta, 78, solver=solver)
            out[eta, solver] = (Q.snr_db(x, ref), Q.ssim(x, ref), res)
            say("eta", eta, solver, "iters", res.iters, "snr", out[eta, solver][0], "ssim", out[eta, solver][1])
            assert res.status == 0 and res.rel_res_true <= 1.1e-4
    for solver in ("sd", "cg"):
        assert out[0.0, solver][0] > out[0.05, solver][0]
        assert out[0.0, solver][1] > out[0.05, solver][1]
        assert 0.0 < out[0.05, solver][1] < out[0.0, solver][1] <= 1.0
    # the same system to the same stopping rule: the two solvers agree in quality
    assert abs(out[0.0, "sd"][0] - out[0.0, "cg"][0]) < 1.0
    # exact data of a phantom outside the pixel basis: the structure is kept
    # (SSIM), the edges carry the model mismatch (SNR about 10 dB here)
    assert out[0.0, "cg"][1] > 0.9 and out[0.0, "cg"][0] > 5.0
    # data from the plan's own forward model of the ground truth (the inverse
    # crime): the pipeline is consistent, the ground truth comes back far
    # more closely than from exact data (28.6 dB measured at 1e-4)
    x, res = Q.reconstruct(N, n, 1.0, 1.0, ells, 0.0, 78, solver="cg", model_data=True)
    snr_ic = Q.snr_db(x, ref)
    say("inverse crime: iters", res.iters, "snr", snr_ic)
    assert res.status == 0 and snr_ic > 20.0 and snr_ic > out[0.0, "cg"][0] + 10.0


@pytest.mark.parametrize("rate", [0.5, 2.0])
def test_downsampling_rates_reconstruct(Q, rate):
    N, n = 48, 180
    ells = inputs.random_ellipses(N, 8, 91)
    ref = Q.ground_truth(N, ells)
    x, res = Q.reconstruct(N, n, rate, 1.0, ells, 0.0, 92, solver="cg")
    snr = Q.snr_db(x, ref)
    say("rate", rate, "iters", res.iters, "snr", snr, "ssim", Q.ssim(x, ref))
    assert res.status == 0 and res.rel_res_true <= 1.1e-4
    assert snr > 5.0
