"""Learned warm start for the CG solve of the normal equations.

A U-Net (include/gramct_unet.h) maps the back projection b = H^T g of a
slice, normalised by the central Gram tap (b~ = b / G[0]), to an initial
iterate x0; CG then runs to the same stopping rule as from zero, and falls
back to x0 = 0 when ||b - A x0|| >= ||b||.  The training pairs are made by
the method itself: seeded ellipse phantoms, the exact box-spline forward
model (Sec. 4), Gaussian noise, box-spline back projection (Sec. 5) and plain
CG to the stopping tolerance for the target.

Everything that touches the data runs in libgramct's kernels; torch only
holds device memory and does the bookkeeping between calls (stacking
slices, noise scaling, index gathers for mini-batches).  The phantoms are
drawn on the host by a process pool, ahead of the GPU work.
"""
from __future__ import annotations

import json
import multiprocessing as mp
import os
import time
from dataclasses import dataclass, asdict

import numpy as np
import torch

from . import gramct as gct
from . import inputs

WEIGHTS_DIR = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights")
WEIGHTS_NAME = "unet_n256_a180_m366_z1"

TRAIN_SEEDS = (0, 20000)
TEST_SEEDS = (20000, 21024)


@dataclass
class WarmConfig:
    """Slice geometry and data recipe of the warm-start workload, and the
    network shape."""
    N: int = 256
    n_angles: int = 180
    M: int = 366
    ly: float = 1.0
    zeta: float = 1.0
    eta: float = 0.01
    ellipses: int = 40
    rtol: float = 1e-4
    levels: int = 4
    base_channels: int = 32


class Problem:
    """Plan, Gram spectrum and work buffers of one slice geometry."""

    def __init__(self, cfg: WarmConfig, batch_slices: int = 256):
        self.cfg = cfg
        self.theta = inputs.angles(cfg.n_angles)
        self.plan = gct.Plan(cfg.N, self.theta, cfg.M, ly=cfg.ly, zeta=cfg.zeta)
        P = self.plan
        G = torch.empty(P.info.gram_elems, dtype=torch.float32, device="cuda")
        gct.gram_build(P, G)
        self.Ghat = torch.empty(P.info.spectrum_elems, dtype=torch.float32, device="cuda")
        gct.gram_spectrum(P, G, self.Ghat, P.workspace(gct.OP_GRAM_SPECTRUM))
        W = 2 * cfg.N - 1
        self.G0 = float(G[(cfg.N - 1) * W + (cfg.N - 1)].item())
        self.ws_bp = P.workspace(gct.OP_BACKPROJECT)
        self.ws_cg = P.workspace(gct.OP_CG)
        # transform tilings of the apply and the fused CG passes for this size
        gct.plan_autotune(P, self.Ghat, self.ws_cg, reps=10)
        self.S = int(batch_slices)
        self.batch = gct.Batch([P] * self.S)
        self.bGhat = torch.empty(self.batch.spectrum_elems, dtype=torch.float32, device="cuda")
        bG = torch.empty(self.batch.gram_elems, dtype=torch.float32, device="cuda")
        gct.batch_gram_build(self.batch, bG)
        gct.batch_gram_spectrum(self.batch, bG, self.bGhat, self.batch.workspace(gct.OP_GRAM_SPECTRUM))
        del bG
        self.ws_bcg = self.batch.workspace(gct.OP_CG)

    def rhs(self, c: torch.Tensor, z: torch.Tensor) -> torch.Tensor:
        """b = H^T (H c + sigma z) per slice, sigma = eta RMS(H c).
        c: [S][N][N], z: [S][n][M] on the GPU.  Returns [S][N][N]."""
        cfg, P = self.cfg, self.plan
        S = c.shape[0]
        g = torch.empty(S, cfg.n_angles, cfg.M, dtype=torch.float32, device="cuda")
        for s in range(S):
            gct.forward_project(P, c[s], g[s])
        sigma = cfg.eta * torch.sqrt(torch.mean(g.double() ** 2, dim=(1, 2))).float()
        g += sigma[:, None, None] * z
        b = torch.empty(S, cfg.N, cfg.N, dtype=torch.float32, device="cuda")
        for s in range(S):
            gct.backproject_boxspline(P, g[s], b[s], self.ws_bp)
        return b

    def solve_batch(self, b: torch.Tensor, max_iter: int = 1000):
        """Plain CG from zero for S slices at once (the batched solver)."""
        S = b.shape[0]
        assert S <= self.S
        bb = torch.zeros(self.batch.image_elems, dtype=torch.float32, device="cuda")
        bb[: b.numel()] = b.reshape(-1)
        x = torch.zeros_like(bb)
        res = gct.batch_cg_solve(self.batch, self.bGhat, bb, x, self.ws_bcg, rtol=self.cfg.rtol,
                                 max_iter=max_iter, check_every=8)
        return x[: b.numel()].view_as(b), res[:S]


def _pool(workers: int):
    return mp.get_context("spawn").Pool(workers)


def generate(prob: Problem, seeds, pool=None, out_b=None, out_x=None, log=print, chunk=None,
             normalize: bool = True):
    """(b~, x*) for each seed: b~ = b / G[0] (b itself if not normalize) and
    x* the plain-CG solution.  Returns GPU tensors [len(seeds)][N][N] and
    the CG iteration counts.  `pool` (a process pool) draws the phantoms
    ahead of the GPU work; None draws them in this process."""
    cfg = prob.cfg
    seeds = list(seeds)
    S = prob.S if chunk is None else chunk
    n = len(seeds)
    if out_b is None:
        out_b = torch.empty(n, cfg.N, cfg.N, dtype=torch.float32, device="cuda")
    if out_x is None:
        out_x = torch.empty(n, cfg.N, cfg.N, dtype=torch.float32, device="cuda")
    iters = np.zeros(n, np.int32)
    args = [(cfg.N, cfg.ellipses, cfg.n_angles, cfg.M, s) for s in seeds]
    it = pool.imap(inputs.draw_slice, args, chunksize=4) if pool is not None else map(inputs.draw_slice, args)
    t0 = time.time()
    last = t0
    for lo in range(0, n, S):
        hi = min(n, lo + S)
        cs, zs = zip(*[next(it) for _ in range(hi - lo)])
        c = torch.from_numpy(np.stack(cs)).cuda()
        z = torch.from_numpy(np.stack(zs)).cuda()
        b = prob.rhs(c, z)
        x, res = prob.solve_batch(b)
        bad = [r.status for r in res if r.status != gct.GCT_OK]
        if bad:
            raise RuntimeError(f"target CG failed for {len(bad)} slices (status {bad[:4]})")
        out_b[lo:hi] = b / prob.G0 if normalize else b
        out_x[lo:hi] = x
        iters[lo:hi] = [r.iters for r in res]
        if time.time() - last > 20 or hi == n:
            last = time.time()
            log(f"  data {hi}/{n} slices, {last - t0:.1f} s, CG iters mean {iters[:hi].mean():.1f}")
    return out_b, out_x, iters


def he_init(levels: int, base: int, seed: int, net: gct.UNet) -> np.ndarray:
    """He-normal weights (std sqrt(2 / fan_in)), zero biases; the unfed
    input channels of the first layer stay zero."""
    r = np.random.Generator(np.random.PCG64(seed))
    p = np.zeros(net.n_params, np.float32)
    for i, ly in enumerate(net.layers):
        cin_fed = 1 if i == 0 else ly["cin"]
        fan = ly["taps"] * cin_fed
        if ly["kind"] == gct.UNET_UPCONV:
            fan = ly["cin"]
        w = r.normal(0.0, np.sqrt(2.0 / fan), size=(ly["taps"], ly["cout"], ly["cin"]))
        if i == 0:
            w[:, :, 1:] = 0.0
        if ly["kind"] == gct.UNET_FINAL:
            w *= 0.5
        n = w.size
        p[ly["w_off"]:ly["w_off"] + n] = w.reshape(-1)
    return p


@dataclass
class TrainConfig:
    batch: int = 16
    epochs: float = 4.0
    lr: float = 1e-3
    lr_final: float = 2e-5
    warmup: int = 200
    seed: int = 7
    log_every_s: float = 20.0


def lr_at(tc: TrainConfig, step: int, total: int) -> float:
    """Linear warm-up, then cosine decay to lr_final."""
    if step <= tc.warmup:
        return tc.lr * step / tc.warmup
    f = (step - tc.warmup) / max(1, total - tc.warmup)
    return tc.lr_final + 0.5 * (tc.lr - tc.lr_final) * (1.0 + np.cos(np.pi * min(1.0, f)))


def train(net: gct.UNet, bt: torch.Tensor, xs: torch.Tensor, s_in: float, s_out: float, tc: TrainConfig,
          step0: int = 0, total_steps: int | None = None, time_limit: float | None = None, log=print):
    """Adam on mini-batches of (b~ * s_in -> x* / s_out) pairs.  Returns the
    last step done and the loss history (per logged window)."""
    n = bt.shape[0]
    B = tc.batch
    per_epoch = n // B
    total = int(tc.epochs * per_epoch) if total_steps is None else int(total_steps)
    gen = torch.Generator(device="cpu")
    gen.manual_seed(tc.seed)
    H, W = bt.shape[1], bt.shape[2]
    xb = torch.empty(B, H, W, dtype=torch.float32, device="cuda")
    tb = torch.empty_like(xb)
    yb = torch.empty_like(xb)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    acc = torch.zeros(1, dtype=torch.float64, device="cuda")
    hist = []
    t0 = time.time()
    last = t0
    cnt = 0
    perm = None
    step = step0
    # the permutation sequence is a function of the seed and the epoch only
    for epoch in range(step0 // per_epoch, 10 ** 9):
        gen.manual_seed(tc.seed * 1000003 + epoch)
        perm = torch.randperm(n, generator=gen).cuda()
        start = step - epoch * per_epoch
        for k in range(start, per_epoch):
            if step >= total:
                break
            idx = perm[k * B:(k + 1) * B]
            torch.index_select(bt, 0, idx, out=xb)
            torch.index_select(xs, 0, idx, out=tb)
            gct.unet_forward(net, xb, yb, in_scale=s_in, out_scale=s_out)
            gct.unet_backward(net, yb, tb, loss)
            step += 1
            gct.unet_adam_step(net, lr_at(tc, step, total), step)
            acc += loss
            cnt += 1
            now = time.time()
            if now - last > tc.log_every_s or step == total:
                torch.cuda.synchronize()
                m = float(acc.item()) / cnt
                hist.append((step, m))
                log(f"  train step {step}/{total} epoch {epoch} loss {m:.4e} "
                    f"lr {lr_at(tc, step, total):.2e} {now - t0:.0f} s")
                acc.zero_()
                cnt = 0
                last = time.time()
            if time_limit is not None and now - t0 > time_limit:
                torch.cuda.synchronize()
                return step, hist
        if step >= total:
            break
    torch.cuda.synchronize()
    return step, hist


def save_checkpoint(path: str, net: gct.UNet, meta: dict, moments: bool = True):
    """FP32 master weights (and Adam moments) as .npy, metadata as JSON."""
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    w = torch.empty(net.n_params, dtype=torch.float32, device="cuda")
    gct.unet_get_params(net, w)
    np.save(path + ".weights.npy", w.cpu().numpy())
    if moments:
        m, v = torch.empty_like(w), torch.empty_like(w)
        gct.unet_get_moments(net, m, v)
        np.save(path + ".adam_m.npy", m.cpu().numpy())
        np.save(path + ".adam_v.npy", v.cpu().numpy())
    with open(path + ".json", "w") as f:
        json.dump(meta, f, indent=1, sort_keys=True)


def load_checkpoint(path: str, net: gct.UNet, moments: bool = False) -> dict:
    with open(path + ".json") as f:
        meta = json.load(f)
    w = np.load(path + ".weights.npy", allow_pickle=False)
    if w.size != net.n_params:
        raise ValueError(f"checkpoint has {w.size} parameters, the net {net.n_params}")
    gct.unet_set_params(net, torch.from_numpy(w).cuda())
    if moments and os.path.exists(path + ".adam_m.npy"):
        m = torch.from_numpy(np.load(path + ".adam_m.npy", allow_pickle=False)).cuda()
        v = torch.from_numpy(np.load(path + ".adam_v.npy", allow_pickle=False)).cuda()
        gct.unet_set_moments(net, m, v)
    return meta


def trained_path() -> str:
    return os.path.join(WEIGHTS_DIR, WEIGHTS_NAME)


def have_trained() -> bool:
    return os.path.exists(trained_path() + ".weights.npy") and os.path.exists(trained_path() + ".json")


class WarmStart:
    """Inference: x0 = U-Net(b) with the scales of a trained checkpoint,
    then CG from x0 (falls back to zero inside cg_solve)."""

    def __init__(self, prob: Problem, path: str | None = None, net: gct.UNet | None = None,
                 meta: dict | None = None):
        cfg = prob.cfg
        self.prob = prob
        if net is None:
            net = gct.UNet(cfg.levels, cfg.base_channels, cfg.N, cfg.N, 1)
            meta = load_checkpoint(path, net)
        self.net = net
        self.meta = meta
        # b~ = b / G[0] folded into the input scale
        self.in_scale = float(meta["s_in"]) / prob.G0
        self.out_scale = float(meta["s_out"])
        self.x0 = torch.empty(cfg.N, cfg.N, dtype=torch.float32, device="cuda")
        # the net replays a captured forward per (input, output) address
        # pair: b is staged into one buffer so every slice reuses it
        self.b_in = torch.empty(cfg.N, cfg.N, dtype=torch.float32, device="cuda")

    def initial(self, b: torch.Tensor, x0: torch.Tensor):
        self.b_in.copy_(b.view(self.b_in.shape))
        gct.unet_forward(self.net, self.b_in, x0, in_scale=self.in_scale, out_scale=self.out_scale, batch=1)
        return x0

    def solve(self, b: torch.Tensor, x: torch.Tensor, max_iter: int = 1000, check_every: int = 8):
        self.initial(b, x)
        return gct.cg_solve(self.prob.plan, self.prob.Ghat, b, x, self.prob.ws_cg, use_x0=True,
                            rtol=self.prob.cfg.rtol, max_iter=max_iter, check_every=check_every)


def compare(prob: Problem, ws: WarmStart, b_all: torch.Tensor, log=print, check_every: int = 8):
    """Plain (x0 = 0) vs warm CG on each slice of b_all [S][N][N]: iterations,
    wall time (host clock around each solve, U-Net inference included in
    warm) and final true relative residuals."""
    P = prob.plan
    x = torch.empty(prob.cfg.N, prob.cfg.N, dtype=torch.float32, device="cuda")
    out = dict(plain_iters=[], warm_iters=[], plain_ms=[], warm_ms=[], plain_res=[], warm_res=[],
               warm_res0=[], fell_back=[])
    # one untimed solve of each kind (graph capture, first launches)
    b0 = b_all[0].contiguous()
    gct.cg_solve(P, prob.Ghat, b0, x, prob.ws_cg, rtol=prob.cfg.rtol, check_every=check_every)
    ws.solve(b0, x, check_every=check_every)
    for s in range(b_all.shape[0]):
        b = b_all[s].contiguous()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = gct.cg_solve(P, prob.Ghat, b, x, prob.ws_cg, rtol=prob.cfg.rtol, check_every=check_every)
        t1 = time.perf_counter()
        out["plain_iters"].append(r.iters)
        out["plain_ms"].append(1e3 * (t1 - t0))
        out["plain_res"].append(r.rel_res_true)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = ws.solve(b, x, check_every=check_every)
        t1 = time.perf_counter()
        out["warm_iters"].append(r.iters)
        out["warm_ms"].append(1e3 * (t1 - t0))
        out["warm_res"].append(r.rel_res_true)
        out["warm_res0"].append(r.rel_res0)
        out["fell_back"].append(r.fell_back)
    return {k: np.asarray(v) for k, v in out.items()}


def pipelined(prob: Problem, ws: WarmStart, b_all: torch.Tensor, check_every: int = 8):
    """Warm-started CG over a run of slices with the U-Net inference of
    slice s + 1 on a second stream while slice s is solved (the inference
    does not depend on the solve, and a 256^2 solve leaves most CUs idle).
    Returns (milliseconds per slice over the whole run, host clock; the
    solver results).  Plain CG has nothing to overlap: its per-slice time is
    the sequential one."""
    cfg = prob.cfg
    S = b_all.shape[0]
    N = cfg.N
    main_s = torch.cuda.current_stream()
    side = torch.cuda.Stream()  # default priority
    x0 = [torch.empty(N, N, dtype=torch.float32, device="cuda") for _ in range(2)]
    b_in = [torch.empty(N, N, dtype=torch.float32, device="cuda") for _ in range(2)]
    ready = [torch.cuda.Event() for _ in range(2)]
    bs = [b_all[s].contiguous() for s in range(S)]

    def infer(s):
        k = s % 2
        with torch.cuda.stream(side):
            side.wait_stream(main_s)  # b_all and the slot's previous solve are done
            b_in[k].copy_(bs[s])
            gct.unet_forward(ws.net, b_in[k], x0[k], in_scale=ws.in_scale, out_scale=ws.out_scale, batch=1)
            ready[k].record(side)

    def run():
        res = []
        infer(0)
        for s in range(S):
            if s + 1 < S:
                infer(s + 1)
            main_s.wait_event(ready[s % 2])
            res.append(gct.cg_solve(prob.plan, prob.Ghat, bs[s], x0[s % 2], prob.ws_cg, use_x0=True,
                                    rtol=cfg.rtol, check_every=check_every))
        torch.cuda.synchronize()
        return res

    run()  # captures (graphs of both buffer slots)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = run()
    ms = (time.perf_counter() - t0) * 1e3 / S
    return ms, res


def batched(prob: Problem, ws: WarmStart, b_all: torch.Tensor, batch: int = 16, check_every: int = 8):
    """Warm-started CG over a run of slices with the U-Net inference done
    for `batch` slices at a time (one forward of a batch-`batch` net sharing
    the trained weights; a batch costs little more than one slice, since the
    layers of a 256^2 inference leave most of the GPU idle), then each slice
    solved from its start vector.  Returns (milliseconds per slice over the
    whole run, host clock, inference included; the solver results; the start
    vectors' largest relative deviation from the batch-1 net's)."""
    cfg = prob.cfg
    S = b_all.shape[0]
    N = cfg.N
    net = gct.UNet(cfg.levels, cfg.base_channels, N, N, batch)
    w = torch.empty(ws.net.n_params, dtype=torch.float32, device="cuda")
    gct.unet_get_params(ws.net, w)
    gct.unet_set_params(net, w)
    b_in = torch.zeros(batch, N, N, dtype=torch.float32, device="cuda")
    x0 = torch.empty(batch, N, N, dtype=torch.float32, device="cuda")
    x = torch.empty(N, N, dtype=torch.float32, device="cuda")  # one solve buffer: one cached CG graph
    bs = [b_all[s].contiguous() for s in range(S)]

    def run(check=None):
        res = []
        for s0 in range(0, S, batch):
            k = min(batch, S - s0)
            b_in[:k].copy_(b_all[s0:s0 + k])
            # the full batch every time (one captured forward); rows past k are stale
            gct.unet_forward(net, b_in, x0, in_scale=ws.in_scale, out_scale=ws.out_scale, batch=batch)
            for i in range(k):
                if check is not None:
                    check.append(x0[i].clone())
                x.copy_(x0[i])
                res.append(gct.cg_solve(prob.plan, prob.Ghat, bs[s0 + i], x, prob.ws_cg, use_x0=True,
                                        rtol=cfg.rtol, check_every=check_every))
        torch.cuda.synchronize()
        return res

    starts = []
    run(starts)  # captures, and keeps the start vectors for the check below
    ref = torch.empty(N, N, dtype=torch.float32, device="cuda")
    dev = 0.0
    for s in range(S):
        ws.initial(bs[s], ref)
        dev = max(dev, float(torch.linalg.norm(starts[s] - ref) / torch.linalg.norm(ref)))
    del starts
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = run()
    ms = (time.perf_counter() - t0) * 1e3 / S
    return ms, res, dev


def stacked(prob: Problem, ws: WarmStart, b_all: torch.Tensor, net_batch: int = 32, check_every: int = 8):
    """A stack of slices (one geometry, as the slices of a parallel-beam
    volume) through the batched solver, prob.S slices per solve, plain (from
    zero) and warm (start vectors from the U-Net, net_batch slices per
    forward, then gct_batch_cg_solve_x0).  Returns {"plain": (ms per slice,
    results), "warm": (...)}; host clock over the whole stack, inference
    included in warm."""
    cfg = prob.cfg
    S_all, N, G = b_all.shape[0], cfg.N, prob.S
    net = gct.UNet(cfg.levels, cfg.base_channels, N, N, net_batch)
    w = torch.empty(ws.net.n_params, dtype=torch.float32, device="cuda")
    gct.unet_get_params(ws.net, w)
    gct.unet_set_params(net, w)
    b_in = torch.zeros(net_batch, N, N, dtype=torch.float32, device="cuda")
    x0 = torch.empty(net_batch, N, N, dtype=torch.float32, device="cuda")
    bb = torch.zeros(prob.batch.image_elems, dtype=torch.float32, device="cuda")
    x = torch.zeros_like(bb)
    bv, xv = bb.view(G, N, N), x.view(G, N, N)

    def run(warm):
        res = []
        for g0 in range(0, S_all, G):
            k = min(G, S_all - g0)
            bv[:k].copy_(b_all[g0:g0 + k])
            if k < G:
                bv[k:].zero_()
            if warm:
                for s0 in range(0, k, net_batch):
                    m = min(net_batch, k - s0)
                    b_in[:m].copy_(b_all[g0 + s0:g0 + s0 + m])
                    gct.unet_forward(net, b_in, x0, in_scale=ws.in_scale, out_scale=ws.out_scale, batch=net_batch)
                    xv[s0:s0 + m].copy_(x0[:m])
                if k < G:
                    xv[k:].zero_()
            r = gct.batch_cg_solve(prob.batch, prob.bGhat, bb, x, prob.ws_bcg, rtol=cfg.rtol, max_iter=1000,
                                   check_every=check_every, use_x0=warm)
            res += r[:k]
        torch.cuda.synchronize()
        return res

    out = {}
    for warm in (False, True):
        run(warm)  # captures
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = run(warm)
        out["warm" if warm else "plain"] = ((time.perf_counter() - t0) * 1e3 / S_all, res)
    return out


def summarize(cmp: dict) -> dict:
    def st(a):
        a = np.asarray(a, dtype=np.float64)
        return dict(mean=float(a.mean()), p50=float(np.percentile(a, 50)), p95=float(np.percentile(a, 95)))
    return dict(slices=int(len(cmp["plain_iters"])),
                plain=dict(iters=st(cmp["plain_iters"]), ms=st(cmp["plain_ms"]),
                           max_rel_res_true=float(np.max(cmp["plain_res"]))),
                warm=dict(iters=st(cmp["warm_iters"]), ms=st(cmp["warm_ms"]),
                          max_rel_res_true=float(np.max(cmp["warm_res"])),
                          rel_res0=st(cmp["warm_res0"]), fell_back=int(np.sum(cmp["fell_back"]))))


def main(argv=None):
    """Generate data, train, evaluate; writes a checkpoint and a JSON report."""
    import argparse
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--train", type=int, default=TRAIN_SEEDS[1] - TRAIN_SEEDS[0])
    ap.add_argument("--test", type=int, default=TEST_SEEDS[1] - TEST_SEEDS[0])
    ap.add_argument("--epochs", type=float, default=4.0)
    ap.add_argument("--batch", type=int, default=16)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--workers", type=int, default=min(16, os.cpu_count() or 1))
    ap.add_argument("--time-limit", type=float, default=None, help="seconds of training")
    ap.add_argument("--out", default=os.path.join(WEIGHTS_DIR, WEIGHTS_NAME))
    ap.add_argument("--report", default=None)
    ap.add_argument("--resume", default=None)
    ap.add_argument("--eval", default=None, metavar="CHECKPOINT",
                    help="evaluate a trained checkpoint on the held-out slices only (no training)")
    a = ap.parse_args(argv)

    def log(*x):
        print(*x, flush=True)

    pool = _pool(a.workers)        # before the GPU is touched
    cfg = WarmConfig()
    t0 = time.time()
    prob = Problem(cfg)
    log(f"problem ready: G[0] = {prob.G0:.6f}, {time.time() - t0:.1f} s")
    if a.eval:
        ws = WarmStart(prob, a.eval)
        b_test, _, it_test = generate(prob, range(TEST_SEEDS[0], TEST_SEEDS[0] + a.test), pool, log=log,
                                      normalize=False)
        cmp = compare(prob, ws, b_test, log=log)
        rep = summarize(cmp)
        ms_pipe, res_pipe = pipelined(prob, ws, b_test)
        rep["warm_pipelined"] = dict(ms_per_slice=ms_pipe, iters_mean=float(np.mean([r.iters for r in res_pipe])),
                                     max_rel_res_true=float(max(r.rel_res_true for r in res_pipe)))
        ms_b, res_b, dev_b = batched(prob, ws, b_test)
        rep["warm_batched16"] = dict(ms_per_slice=ms_b, iters_mean=float(np.mean([r.iters for r in res_b])),
                                     max_rel_res_true=float(max(r.rel_res_true for r in res_b)),
                                     start_dev_vs_batch1=dev_b)
        st = stacked(prob, ws, b_test)
        rep["stack_batched_solver"] = {k: dict(ms_per_slice=v[0], iters_mean=float(np.mean([r.iters for r in v[1]])),
                                               max_rel_res_true=float(max(r.rel_res_true for r in v[1])),
                                               converged=int(sum(r.status == gct.GCT_OK for r in v[1])))
                                       for k, v in st.items()}
        rep["stack_batched_solver"]["slices_per_solve"] = prob.S
        rep.update(checkpoint=os.path.basename(a.eval), step=int(ws.meta.get("step", 0)),
                   batched_target_iters_mean=float(it_test.mean()), seconds=time.time() - t0)
        log(json.dumps(rep))
        if a.report:
            with open(a.report, "w") as f:
                json.dump(rep, f, indent=1)
        pool.close()
        return
    bt, xs, it_train = generate(prob, range(TRAIN_SEEDS[0], TRAIN_SEEDS[0] + a.train), pool, log=log)
    s_in = float(1.0 / torch.sqrt(torch.mean(bt[:1000].double() ** 2)).item())
    s_out = float(torch.sqrt(torch.mean(xs[:1000].double() ** 2)).item())
    log(f"training data: {a.train} slices, s_in {s_in:.4e} s_out {s_out:.4e}, "
        f"target CG iters mean {it_train.mean():.1f}, {time.time() - t0:.1f} s")
    net = gct.UNet(cfg.levels, cfg.base_channels, cfg.N, cfg.N, a.batch)
    tc = TrainConfig(batch=a.batch, epochs=a.epochs, lr=a.lr)
    step0 = 0
    meta = dict(config=asdict(cfg), train=asdict(tc), s_in=s_in, s_out=s_out, train_seeds=[0, a.train],
                G0=prob.G0)
    if a.resume:
        old = load_checkpoint(a.resume, net, moments=True)
        step0 = int(old.get("step", 0))
        meta["s_in"], meta["s_out"] = old["s_in"], old["s_out"]
        s_in, s_out = old["s_in"], old["s_out"]
        log(f"resumed at step {step0}")
    else:
        p = he_init(cfg.levels, cfg.base_channels, tc.seed, net)
        gct.unet_set_params(net, torch.from_numpy(p).cuda())
    step, hist = train(net, bt, xs, s_in, s_out, tc, step0=step0, time_limit=a.time_limit, log=log)
    meta.update(step=step, loss_history=hist)
    save_checkpoint(a.out, net, meta)
    log(f"checkpoint at step {step}: {a.out}")
    del bt, xs
    # held-out evaluation with a batch-1 net sharing the weights
    inf = gct.UNet(cfg.levels, cfg.base_channels, cfg.N, cfg.N, 1)
    w = torch.empty(net.n_params, dtype=torch.float32, device="cuda")
    gct.unet_get_params(net, w)
    gct.unet_set_params(inf, w)
    ws = WarmStart(prob, net=inf, meta=meta)
    b_test, _, _ = generate(prob, range(TEST_SEEDS[0], TEST_SEEDS[0] + a.test), pool, log=log,
                            normalize=False)
    cmp = compare(prob, ws, b_test, log=log)
    rep = summarize(cmp)
    rep.update(step=step, train_slices=a.train, epochs=a.epochs, seconds=time.time() - t0)
    log(json.dumps(rep))
    if a.report:
        with open(a.report, "w") as f:
            json.dump(rep, f, indent=1)
    pool.close()


if __name__ == "__main__":
    main()
