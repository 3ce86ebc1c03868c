"""The learned warm start through the C ABI: the trained U-Net's initial
iterate cuts the CG iterations to ||r|| <= 1e-4 ||b|| on held-out slices of
the warm-start workload (N = 256, 180 angles, blur 1, 1% noise), every
warm solve still meets the stopping rule, and a net whose output is useless
is dropped by the solver's fallback to x0 = 0."""
import numpy as np
import pytest
import torch

from gpu_helpers import say

pytestmark = pytest.mark.gpu

SLICES = 32


@pytest.fixture(scope="module")
def setup():
    from paper_2005_13471_amd import gramct as gct
    from paper_2005_13471_amd import warmstart as W
    assert W.have_trained(), "trained warm-start weights are missing from the package"
    cfg = W.WarmConfig()
    prob = W.Problem(cfg, batch_slices=SLICES)
    # the default transform tilings rather than the autotuner's choice, which
    # depends on timings: the iteration counts compared below move with the
    # rounding of the passes, so the comparison should not depend on the box
    gct.plan_set_pass_elems(prob.plan, 0, 0)
    seeds = range(W.TEST_SEEDS[0], W.TEST_SEEDS[0] + SLICES)
    b, xs, iters = W.generate(prob, seeds, None, log=lambda *a: None, normalize=False)
    return gct, W, prob, b, xs, iters


def test_trained_net_cuts_cg_iterations(setup):
    gct, W, prob, b, xs, iters = setup
    ws = W.WarmStart(prob, W.trained_path())
    cmp = W.compare(prob, ws, b)
    rep = W.summarize(cmp)
    say("plain iters", rep["plain"]["iters"], "warm iters", rep["warm"]["iters"])
    say("plain ms", rep["plain"]["ms"], "warm ms", rep["warm"]["ms"], "rel_res0", rep["warm"]["rel_res0"])
    # the single-slice solve (Chronopoulos-Gear arrangement) and the batched
    # solver that made the targets (textbook arrangement) take about as many
    # iterations: equal in exact arithmetic, a few apart in FP32 (rounding
    # moves the iteration at which the residual crosses the threshold; the
    # FFT blocking chosen by the plan's tuning moves it too)
    d = np.abs(cmp["plain_iters"] - iters)
    say("single-slice vs batched iterations: mean |d|", np.mean(d), "max", np.max(d))
    assert np.mean(d) <= 1.5 and np.max(d) <= max(5, int(0.15 * np.max(iters)))
    # both forms meet the same stopping rule (true residual, FP32 slack)
    assert np.all(cmp["plain_res"] <= 1.05e-4) and np.all(cmp["warm_res"] <= 1.05e-4)
    assert int(np.sum(cmp["fell_back"])) == 0
    # the net's x0 starts well inside the unit ball and saves iterations
    assert np.median(cmp["warm_res0"]) < 0.1
    assert rep["warm"]["iters"]["mean"] <= 0.9 * rep["plain"]["iters"]["mean"]
    assert np.mean(cmp["warm_iters"] < cmp["plain_iters"]) >= 0.75


def test_pipelined_warm_start_matches_sequential(setup):
    """Inference of the next slice on a second stream during each solve:
    the same start vectors, hence the same iterations as the sequential
    warm solves, every solve meeting the stopping rule."""
    gct, W, prob, b, xs, iters = setup
    ws = W.WarmStart(prob, W.trained_path())
    cmp = W.compare(prob, ws, b)
    ms, res = W.pipelined(prob, ws, b)
    say("pipelined warm ms per slice", ms, "sequential warm", np.mean(cmp["warm_ms"]),
        "plain", np.mean(cmp["plain_ms"]))
    assert [r.iters for r in res] == list(cmp["warm_iters"])
    assert all(r.status == gct.GCT_OK and r.rel_res_true <= 1.05e-4 for r in res)


def test_batched_inference_warm_start(setup):
    """Inference for a group of slices in one forward of a batch-16 net
    with the trained weights: start vectors equal to the batch-1 net's to
    rounding (the layers may take other tilings at another batch), the mean
    iteration count that of the sequential warm solves to within half an
    iteration (a start vector perturbed at 1e-3 can move one solve's count by
    a few where its residual curve is flat at the threshold) and below the
    plain one, every solve meeting the stopping rule."""
    gct, W, prob, b, xs, iters = setup
    ws = W.WarmStart(prob, W.trained_path())
    cmp = W.compare(prob, ws, b)
    ms, res, dev = W.batched(prob, ws, b, batch=16)
    say("batched warm ms per slice", ms, "sequential warm", np.mean(cmp["warm_ms"]),
        "plain", np.mean(cmp["plain_ms"]), "start deviation", dev)
    assert dev <= 1e-2
    assert len(res) == b.shape[0]
    it_b = np.array([r.iters for r in res])
    say("iteration differences batched - sequential", (it_b - cmp["warm_iters"]).tolist())
    assert abs(it_b.mean() - np.mean(cmp["warm_iters"])) <= 0.5
    assert it_b.mean() < np.mean(cmp["plain_iters"])
    assert all(r.status == gct.GCT_OK and r.rel_res_true <= 1.05e-4 for r in res)


def test_stacked_warm_start_through_the_batched_solver(setup):
    """The slices as one stack through the batched solver: from zero and
    from the U-Net's start vectors (gct_batch_cg_solve_x0).  Every slice of
    both meets the stopping rule, no start falls back, and the warm stack
    takes fewer iterations on average."""
    gct, W, prob, b, xs, iters = setup
    ws = W.WarmStart(prob, W.trained_path())
    st = W.stacked(prob, ws, b)
    (ms_p, rp), (ms_w, rw) = st["plain"], st["warm"]
    ip, iw = np.mean([r.iters for r in rp]), np.mean([r.iters for r in rw])
    say("stack ms per slice plain", ms_p, "warm", ms_w, "iters", ip, iw)
    assert len(rp) == len(rw) == b.shape[0]
    assert all(r.status == gct.GCT_OK and r.rel_res_true <= 1.05e-4 for r in rp + rw)
    assert not any(r.fell_back for r in rw)
    assert iw < ip - 3


def test_warm_iterate_is_close_to_the_cg_target(setup):
    """x0 from the net is a rough reconstruction: relative error against the
    plain-CG solution well below 1 on every slice."""
    gct, W, prob, b, xs, iters = setup
    ws = W.WarmStart(prob, W.trained_path())
    x0 = torch.empty(prob.cfg.N, prob.cfg.N, dtype=torch.float32, device="cuda")
    errs = []
    for s in range(SLICES):
        ws.initial(b[s].contiguous(), x0)
        errs.append(float(torch.linalg.norm(x0 - xs[s]) / torch.linalg.norm(xs[s])))
    say("x0 relative error: median", np.median(errs), "max", np.max(errs))
    assert np.max(errs) < 0.5


def test_useless_net_falls_back_to_zero(setup):
    """All-zero parameters give x0 = 0, whose residual equals ||b||: the
    solver reports the fallback and runs exactly the plain iterations."""
    gct, W, prob, b, xs, iters = setup
    cfg = prob.cfg
    net = gct.UNet(cfg.levels, cfg.base_channels, cfg.N, cfg.N, 1)
    gct.unet_set_params(net, torch.zeros(net.n_params, dtype=torch.float32, device="cuda"))
    ws = W.WarmStart(prob, net=net, meta=dict(s_in=1.0, s_out=1.0))
    x = torch.empty(cfg.N, cfg.N, dtype=torch.float32, device="cuda")
    for s in range(3):
        bs = b[s].contiguous()
        rw = ws.solve(bs, x)
        rp = gct.cg_solve(prob.plan, prob.Ghat, bs, x, prob.ws_cg, rtol=cfg.rtol)
        assert rw.fell_back == 1 and rw.status == gct.GCT_OK
        assert rw.iters == rp.iters
