"""Benchmark of the pixel-basis (box-spline) CT hot path on one MI355X.

Workload n512_a720_m730_z1: N = 512 pixels per side (unit pixels), 720
angles uniform in [0, pi), 730 detector bins of unit width, detector blur
zeta = 1, a 40-ellipse random phantom whose sinogram comes from the exact
box-spline forward model plus 1% Gaussian noise.  Everything is synthetic
and seeded; all inputs are resident in GPU memory before timing starts.

One step = the whole path on that slice: Gram filter build, its spectrum,
prefilter + box-spline back projection, CG to ||r|| <= 1e-4 ||b|| from zero,
then a burst of back-to-back Gram-filter applies (H^T H c) that measures the
apply rate.  The burst is a captured HIP graph of APPLY_GRAPH applies
replayed APPLY_BURST / APPLY_GRAPH times (CG issues its applies the same
way); `value` is H^T H applies per second over the bursts.  The rate of
applies issued one C-ABI call at a time, the CG time and iteration count are
reported alongside.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# FP32 vector rate without packed instructions (which this build does not
# emit): 256 CUs x 64 lanes x 2 flop (FMA) x 2.4 GHz
FP32_VALU_PEAK_TFLOPS = 78.6
WORKLOAD = "n512_a720_m730_z1"
APPLY_BURST = 200
APPLY_GRAPH = 50


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default=WORKLOAD)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--batch-slices", type=int, default=256,
                    help="slices of the uneven batch reported beside the main line (0: skip)")
    ap.add_argument("--warm-slices", type=int, default=1024,
                    help="held-out slices for the plain vs warm-start CG comparison (0: skip)")
    ap.add_argument("--fft-elems", default="",
                    help="elements per thread of the Gram-filtering transforms: E for every pass, or "
                         "ROWS,COLS for the row passes and the column pass (empty: autotune)")
    ap.add_argument("--pmc-probe", action="store_true",
                    help="for counter runs: set up the workload, then 20 applies and one "
                         "256 MiB elementwise copy (the counters' calibration), and exit")
    ap.add_argument("--phase-probe", action="store_true",
                    help="for counter runs: set up the workload, run gram_build 4 times and the back "
                         "projection 3 times, and exit")
    ap.add_argument("--pmc-summarize", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="turn the FETCH_SIZE and WRITE_SIZE runs of --pmc-probe (rocprofv3 csv output "
                         "directories) into the per-apply HBM traffic kept under profiles/, and exit")
    ap.add_argument("--cpu-sample", type=int, default=0,
                    help="output pixels of the oracle's direct-sum apply timed for cpu_baseline "
                         "(0: all N^2, one whole apply)")
    return ap.parse_args()


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(cfg, theta, sample):
    """The FP64 oracle's normal operator (direct spatial sum with the exactly
    integrated Gram filter), timed on the host cores on a bounded sample of
    output pixels and scaled to whole applies per second: once on all the
    threads OpenMP uses, once on one thread (a 1/32 sample)."""
    import oracle
    from paper_2005_13471_amd import inputs
    oracle.build(force=False)
    N = cfg["N"]
    og = oracle.Geometry(N, theta, cfg["M"], ly=cfg["ly"], zeta=cfg["zeta"])
    G = oracle.gram(og)
    c = inputs.uniform_coeffs(N, cfg["coeff_seed"])
    if sample <= 0 or sample > N * N:
        sample = N * N
    idx = np.arange(0, N * N, max(1, (N * N) // sample), dtype=np.int32)[:sample]
    threads = oracle.max_threads()
    t0 = time.perf_counter()
    oracle.apply_at(G, c, idx)
    dt = time.perf_counter() - t0
    idx1 = idx[::32]
    oracle.set_threads(1)
    try:
        t0 = time.perf_counter()
        oracle.apply_at(G, c, idx1)
        dt1 = time.perf_counter() - t0
    finally:
        oracle.set_threads(threads)
    return {"value": (idx.size / (N * N)) / dt, "unit": "applies/s", "cores": threads,
            "kind": "oracle", "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "value_1core": (idx1.size / (N * N)) / dt1,
            "sample": f"direct-sum H^T H c (FP64, exact Gram filter) at {idx.size} of {N*N} "
                      f"output pixels on {threads} threads, {dt:.2f} s wall, scaled by "
                      f"{N*N/idx.size:.0f}; one thread: {idx1.size} pixels, {dt1:.2f} s, scaled by "
                      f"{N*N/idx1.size:.0f}"}


def batch_main(args):
    out = batch_run(args.batch_slices, args.steps, args.warmup, args.pmc_probe)
    if out is not None:
        print(json.dumps(out), flush=True)


def fft_flops(N: int, P: int) -> float:
    """Flops of one Gram-filtering apply of an N x N slice by the three
    passes, counted as 5 P log2 P per complex transform of size P: N/2 row
    transforms (two real rows each) forward and inverse, and P/2 + 1 column
    transforms forward and inverse."""
    return 5.0 * P * np.log2(P) * (2 * ((N + 1) // 2) + 2 * (P // 2 + 1))


def batch_run(S, steps, warmup, pmc_probe=False):
    """256 independent slices of uneven size through one batch: N from
    {128, 256, 384, 512, 768, 1024}, angle counts from {180, 360, 720, 1440},
    blur from {0, 0.5, 1}, each drawn from a seeded generator; 40-ellipse
    phantoms (2 x 2 sub-pixel rasterisation, to keep the setup short), exact
    box-spline forward model on the GPU plus 1% noise, back projection per
    slice.  One step = batched Gram-filter build, spectra and CG to 1e-4 on
    every slice; then graph-replayed bursts of the batched apply measure the
    aggregate Gram-filtering rate against the HBM roofline."""
    import torch
    from paper_2005_13471_amd import gramct as gct
    from paper_2005_13471_amd import inputs

    torch.cuda.set_device(0)
    dt = torch.float32
    rng = np.random.Generator(np.random.PCG64(3000))
    Ns = rng.choice([128, 256, 384, 512, 768, 1024], size=S)
    ns = rng.choice([180, 360, 720, 1440], size=S)
    zs = rng.choice([0.0, 0.5, 1.0], size=S)
    plans, bs = [], []
    for i in range(S):
        N, n, z = int(Ns[i]), int(ns[i]), float(zs[i])
        th = inputs.angles(n)
        M = inputs.detector_bins(N, z)
        P = gct.Plan(N, th, M, zeta=z)
        plans.append(P)
        ells = inputs.random_ellipses(N, 40, 1000 + i)
        c = inputs.rasterize(N, ells, sub=2)
        g = torch.empty(n * M, dtype=dt, device="cuda")
        gct.forward_project(P, torch.as_tensor(c.reshape(-1), dtype=dt, device="cuda"), g)
        gn = inputs.add_noise(g.double().cpu().numpy(), 0.01, inputs.NOISE_SEED_BASE + 1000 + i)
        b = torch.empty(N * N, dtype=dt, device="cuda")
        gct.backproject_boxspline(P, torch.as_tensor(gn, dtype=dt, device="cuda"), b,
                                  P.workspace(gct.OP_BACKPROJECT, dt))
        bs.append(b)
    B = gct.Batch(plans)
    bpk = torch.empty(B.image_elems, dtype=dt, device="cuda")
    for i in range(S):
        B.image(bpk, i).copy_(bs[i].view(plans[i].N, plans[i].N))
    del bs
    G = torch.empty(B.gram_elems, dtype=dt, device="cuda")
    Ghat = torch.empty(B.spectrum_elems, dtype=dt, device="cuda")
    x = torch.empty(B.image_elems, dtype=dt, device="cuda")
    y = torch.empty(B.image_elems, dtype=dt, device="cuda")
    ws_spec = B.workspace(gct.OP_GRAM_SPECTRUM, dt)
    ws_cg = B.workspace(gct.OP_CG, dt)
    ws_apply = B.workspace(gct.OP_GRAM_APPLY, dt)
    gct.batch_gram_build(B, G)
    gct.batch_gram_spectrum(B, G, Ghat, ws_spec)
    if not pmc_probe:
        # (counter runs keep the default tilings, so that every run of a
        # counter set times the same kernels)
        gct.batch_autotune(B, Ghat, ws_cg, reps=3)
    torch.cuda.synchronize()
    if pmc_probe:
        # counter runs: BATCH_PMC_APPLIES batched applies, then the calibration copy
        for _ in range(BATCH_PMC_APPLIES):
            gct.batch_gram_apply(B, Ghat, bpk, y, ws_apply)
        torch.cuda.synchronize()
        src = torch.ones(PMC_COPY_BYTES // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        print(json.dumps({"pmc_probe": True, "workload": "batch_uneven_256", "applies": BATCH_PMC_APPLIES,
                          "passes_per_apply": 3 * B.groups, "copy_bytes": PMC_COPY_BYTES,
                          "batch_source_sha": batch_source_sha()}))
        return None
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        for _ in range(4):
            gct.batch_gram_apply(B, Ghat, bpk, y, ws_apply)
    torch.cuda.synchronize()
    ev = lambda: torch.cuda.Event(enable_timing=True)

    def step(rec):
        e = [ev() for _ in range(5)]
        e[0].record()
        gct.batch_gram_build(B, G)
        e[1].record()
        gct.batch_gram_spectrum(B, G, Ghat, ws_spec)
        e[2].record()
        res = gct.batch_cg_solve(B, Ghat, bpk, x, ws_cg, rtol=1e-4, max_iter=3000, check_every=16)
        e[3].record()
        for _ in range(5):
            graph.replay()
        e[4].record()
        rec.append((e, res))

    warm = []
    for _ in range(warmup):
        step(warm)
    torch.cuda.synchronize()
    rec = []
    t0 = time.perf_counter()
    for _ in range(steps):
        step(rec)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ph = np.array([[e[i].elapsed_time(e[i + 1]) for i in range(4)] for e, _ in rec])
    apply_ms = ph[:, 3].sum() / (steps * 20)
    res = rec[-1][1]
    alg = sum(8 * p.N * p.N + 4 * (p.info.fft_size // 2 + 1) * p.info.fft_size for p in plans)
    flops = sum(fft_flops(p.N, p.info.fft_size) for p in plans)
    achieved = alg / (apply_ms * 1e-3) / 1e9
    tflops = flops / (apply_ms * 1e-3) / 1e12
    iters = np.array([r.iters for r in res])
    out = {
        "metric": "batched uneven slices: slices/s (build + spectrum + CG to 1e-4) and aggregate Gram-filtering GB/s",
        "value": round(S / (np.median(ph[:, 0] + ph[:, 1] + ph[:, 2]) * 1e-3), 2),
        "unit": "slices/s",
        "n_gpus": 1, "steps": steps, "warmup": warmup,
        "ms_per_step": round(wall * 1e3 / steps, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": "batch_uneven_256", "slices": S, "seed": 3000,
                   "N_values": sorted(set(int(v) for v in Ns)), "image_elems": B.image_elems,
                   "fft_groups": B.groups,
                   "autotuned_elems_per_thread": [list(e) for e in gct.batch_get_pass_elems(B, dt)]},
        "phase_ms": {"gram_build": round(float(np.median(ph[:, 0])), 3),
                     "gram_spectrum": round(float(np.median(ph[:, 1])), 3),
                     "cg_solve": round(float(np.median(ph[:, 2])), 3),
                     "batched_apply": round(apply_ms, 4)},
        "cg": {"iters_max": int(iters.max()), "iters_mean": float(iters.mean()),
               "all_converged": all(r.status == 0 for r in res),
               "rel_res_true_max": max(r.rel_res_true for r in res)},
        "roofline": {"kernel": "batched gram_apply (all slices, rows / columns / rows passes)",
                     "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": batch_measured_traffic(),
                     "alg_bytes_per_launch": alg},
        "roofline_alu": {"kernel": "batched gram_apply FFT arithmetic (5 P log2 P per complex transform)",
                         "bound": "alu", "achieved": round(tflops, 2), "peak": FP32_VALU_PEAK_TFLOPS,
                         "unit": "TFLOP/s", "frac": round(tflops / FP32_VALU_PEAK_TFLOPS, 4),
                         "alg_flops_per_launch": flops},
    }
    return out


PMC_APPLIES = 20
PMC_COPY_BYTES = 256 << 20
PMC_FILE = os.path.join(ROOT, "profiles", "gram_apply_n512_a720_pmc.json")
BATCH_PMC_APPLIES = 5
BATCH_PMC_FILE = os.path.join(ROOT, "profiles", "batch_apply_uneven256_pmc.json")
BATCH_SOURCES = ["batch.hip", "fft_passes.h", "fft_common.h"]


def batch_source_sha() -> str:
    """Hash of the batched Gram-filtering kernel sources."""
    import hashlib
    h = hashlib.sha256()
    for f in BATCH_SOURCES:
        with open(os.path.join(ROOT, "paper_2005_13471_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def pmc_summarize_batch(fetch_dir: str, write_dir: str):
    """HBM bytes per batched apply from the two counter runs of
    `--workload batch_uneven_256 --pmc-probe`: the counters of the last
    BATCH_PMC_APPLIES applies' pass dispatches (after the autotuner's), summed
    and divided by the applies, scaled by the calibration copy as for the
    single-slice apply.  Written to BATCH_PMC_FILE."""
    import csv
    import glob

    def load(d, counter):
        rows = []
        for f in glob.glob(os.path.join(d, "*counter_collection.csv")):
            with open(f) as fh:
                rows += [r for r in csv.DictReader(fh) if r["Counter_Name"] == counter]
        per = {}
        for r in rows:
            k = (int(r["Dispatch_Id"]), r["Kernel_Name"].split("(")[0].replace("void ", ""))
            per[k] = per.get(k, 0.0) + float(r["Counter_Value"])
        disp = sorted(per.items())
        passes = [(k, v) for k, v in disp if any(t in k[1] for t in ("kb_rows_fwd", "kb_cols<", "kb_rows_inv"))]
        # the calibration copy is the run's last dispatch outside the library
        # (the set-up's own large fills come earlier)
        copy = next((v for k, v in reversed(disp) if "gct::" not in k[1]), 0.0)
        return passes, copy

    fetch, copy_f = load(fetch_dir, "FETCH_SIZE")
    write, copy_w = load(write_dir, "WRITE_SIZE")
    # passes of one apply: 3 per FFT size (log2 P, the second template
    # argument); the probe's applies are the last dispatches
    groups = {k[1].split("<")[1].split(",")[1].strip() for k, _ in fetch[-30:]}
    n_last = 3 * len(groups) * BATCH_PMC_APPLIES
    sf, sw = PMC_COPY_BYTES / (copy_f * 1024), PMC_COPY_BYTES / (copy_w * 1024)
    fb = sum(v for _, v in fetch[-n_last:]) * 1024 * sf / BATCH_PMC_APPLIES
    wb = sum(v for _, v in write[-n_last:]) * 1024 * sw / BATCH_PMC_APPLIES
    entry = {"workload": "batch_uneven_256", "batch_source_sha": batch_source_sha(), "fft_sizes": len(groups),
             "scale_fetch": sf, "scale_write": sw, "hbm_fetch_bytes_per_apply": int(round(fb)),
             "hbm_write_bytes_per_apply": int(round(wb)), "hbm_bytes_per_apply": int(round(fb + wb))}
    with open(BATCH_PMC_FILE, "w") as fh:
        json.dump(entry, fh, indent=1)
    print(json.dumps(entry))


def batch_measured_traffic():
    try:
        with open(BATCH_PMC_FILE) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    return d.get("hbm_bytes_per_apply") if d.get("batch_source_sha") == batch_source_sha() else None
APPLY_SOURCES = ["gram_apply.hip", "fft_passes.h", "fft_common.h"]


def apply_source_sha() -> str:
    """Hash of the Gram-filtering kernel sources: counters taken on other
    sources do not describe the kernels that run."""
    import hashlib
    h = hashlib.sha256()
    for f in APPLY_SOURCES:
        with open(os.path.join(ROOT, "paper_2005_13471_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def pmc_probe(gct, plan, Ghat, c, y, ws, fft_elems):
    """PMC_APPLIES applies, then one elementwise copy of PMC_COPY_BYTES whose
    FETCH_SIZE / WRITE_SIZE calibrate the counters to bytes."""
    import torch
    for _ in range(PMC_APPLIES):
        gct.gram_apply(plan, Ghat, c, y, ws)
    torch.cuda.synchronize()
    src = torch.ones(PMC_COPY_BYTES // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    print(json.dumps({"pmc_probe": True, "applies": PMC_APPLIES, "copy_bytes": PMC_COPY_BYTES,
                      "fft_elems_per_thread": fft_elems, "apply_source_sha": apply_source_sha()}))


def pmc_summarize(fetch_dir: str, write_dir: str):
    """Per-apply HBM bytes from the two counter runs of --pmc-probe: the
    median over dispatches of each transform pass's counter, scaled by what
    the same counter read for the calibration copy (the largest non-library
    dispatch of the run).  Merged into PMC_FILE under the run's elements per
    thread; prints the markdown table of the profile summary."""
    import csv
    import glob

    def load(d, counter):
        rows = []
        for f in glob.glob(os.path.join(d, "*counter_collection.csv")):
            with open(f) as fh:
                rows += [r for r in csv.DictReader(fh) if r["Counter_Name"] == counter]
        if not rows:
            raise SystemExit(f"no {counter} rows under {d}")
        per = {}
        for r in rows:
            per.setdefault(r["Kernel_Name"].split("(")[0], []).append(float(r["Counter_Value"]))
        passes = {k: float(np.median(v)) for k, v in per.items()
                  if any(t in k for t in ("k_rows_fwd<", "k_cols<", "k_rows_inv<"))}
        copy = max((max(v) for k, v in per.items() if "gct::" not in k), default=0.0)
        return passes, copy

    fetch, copy_f = load(fetch_dir, "FETCH_SIZE")
    write, copy_w = load(write_dir, "WRITE_SIZE")
    def elems_of(tag):
        e = {int(k.split(",")[-1].strip(" >")) for k in fetch if tag in k}
        if len(e) != 1:
            raise SystemExit(f"expected one tiling of {tag} in the run, found {sorted(e)}")
        return e.pop()

    E = elems_key(elems_of("k_rows_fwd<"), elems_of("k_cols<"))
    if elems_of("k_rows_inv<") != elems_of("k_rows_fwd<"):
        raise SystemExit("row passes with different tilings")
    sf, sw = PMC_COPY_BYTES / (copy_f * 1024), PMC_COPY_BYTES / (copy_w * 1024)
    fb = sum(fetch.values()) * 1024 * sf
    wb = sum(write.values()) * 1024 * sw
    N, P = 512, 1024
    entry = {"copy_bytes": PMC_COPY_BYTES, "copy_fetch_kib": copy_f, "copy_write_kib": copy_w,
             "scale_fetch": sf, "scale_write": sw, "per_kernel_fetch_kib": fetch, "per_kernel_write_kib": write,
             "hbm_fetch_bytes_per_apply": int(round(fb)), "hbm_write_bytes_per_apply": int(round(wb)),
             "hbm_bytes_per_apply": int(round(fb + wb)),
             "alg_bytes_per_apply": 4 * N * N * 2 + 4 * (P // 2 + 1) * P}
    try:
        with open(PMC_FILE) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        d = {}
    if d.get("apply_source_sha") != apply_source_sha():
        d = {}
    d.update({"workload": WORKLOAD, "apply_source_sha": apply_source_sha()})
    d.setdefault("by_fft_elems", {})[E] = entry
    with open(PMC_FILE, "w") as fh:
        json.dump(d, fh, indent=1)
    print(f"elements per thread {E}: scale fetch {sf:.4f}, write {sw:.4f}")
    print("| kernel | FETCH_SIZE KiB / dispatch | fetched MB (scaled) | WRITE_SIZE KiB / dispatch | written MB (scaled) |")
    print("|---|---:|---:|---:|---:|")
    for k in fetch:
        print(f"| `{k.replace('void ', '')}` | {fetch[k]:.1f} | {fetch[k] * 1024 * sf / 1e6:.3f} | "
              f"{write.get(k, 0.0):.1f} | {write.get(k, 0.0) * 1024 * sw / 1e6:.3f} |")
    print(f"per apply: {fb / 1e6:.2f} MB fetched + {wb / 1e6:.2f} MB written = {(fb + wb) / 1e6:.2f} MB")


def elems_key(rows: int, cols: int) -> str:
    """Name of a transform tiling: "E" when every pass uses E elements per
    thread, else "ROWS,COLS"."""
    return str(rows) if rows == cols else f"{rows},{cols}"


def measured_traffic(fft_elems: str):
    """HBM bytes per apply from the committed counter runs, if they were taken
    on these kernel sources with this tiling; else None."""
    try:
        with open(PMC_FILE) as fh:
            d = json.load(fh)
    except (OSError, ValueError):
        return None
    if d.get("apply_source_sha") != apply_source_sha():
        return None
    e = d.get("by_fft_elems", {}).get(fft_elems)
    return e.get("hbm_bytes_per_apply") if e else None


def sd_plain(gct, plan, Ghat, b, ws):
    """Steepest descent (the paper's solver) from zero to the same 1e-4 on
    the same right-hand side, outside the timed steps: iterations and wall
    time next to CG's."""
    import torch
    x = torch.zeros_like(b)
    gct.sd_solve(plan, Ghat, b, x, ws, rtol=1e-4, max_iter=20000, check_every=64)  # graph capture
    x.zero_()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = gct.sd_solve(plan, Ghat, b, x, ws, rtol=1e-4, max_iter=20000, check_every=64)
    ms = (time.perf_counter() - t0) * 1e3
    return {"iters": r.iters, "ms": round(ms, 3), "rel_res_true": r.rel_res_true, "status": r.status}


def warm_compare(slices: int):
    """Plain vs learned-warm-start CG on held-out slices of the warm-start
    workload (N = 256, 180 angles, 366 bins, blur 1, 40 ellipses, 1% noise;
    seeds 20000, 20001, ...): iterations and wall time to ||r|| <= 1e-4 ||b||,
    U-Net inference included in the warm time."""
    from paper_2005_13471_amd import warmstart as W
    if not W.have_trained():
        return {"error": "no trained weights at " + os.path.relpath(W.trained_path(), ROOT)}
    cfg = W.WarmConfig()
    prob = W.Problem(cfg, batch_slices=min(256, slices))
    ws = W.WarmStart(prob, W.trained_path())
    seeds = range(W.TEST_SEEDS[0], W.TEST_SEEDS[0] + slices)
    b, _, _ = W.generate(prob, seeds, None, log=lambda *a: None, normalize=False)
    rep = W.summarize(W.compare(prob, ws, b))
    ms_pipe, res_pipe = W.pipelined(prob, ws, b)
    rep["warm_pipelined"] = {"ms_per_slice": ms_pipe,
                             "iters_mean": float(np.mean([r.iters for r in res_pipe])),
                             "max_rel_res_true": float(max(r.rel_res_true for r in res_pipe)),
                             "note": "U-Net of the next slice on a second stream during each solve"}
    ms_b, res_b, dev_b = W.batched(prob, ws, b)
    rep["warm_batched16"] = {"ms_per_slice": ms_b,
                             "iters_mean": float(np.mean([r.iters for r in res_b])),
                             "max_rel_res_true": float(max(r.rel_res_true for r in res_b)),
                             "start_dev_vs_batch1": dev_b,
                             "note": "U-Net inference for 16 slices at a time, then each CG from its start"}
    st = W.stacked(prob, ws, b)
    rep["stack_batched_solver"] = {k: {"ms_per_slice": v[0], "iters_mean": float(np.mean([r.iters for r in v[1]])),
                                       "max_rel_res_true": float(max(r.rel_res_true for r in v[1]))}
                                   for k, v in st.items()}
    rep["stack_batched_solver"]["note"] = (f"the slices as one stack through the batched solver ({prob.S} per solve), "
                                           "plain from zero vs warm from the U-Net (32 slices per forward)")
    rep.update(workload="n256_a180_m366_z1", seeds=[W.TEST_SEEDS[0], W.TEST_SEEDS[0] + slices],
               net=f"U-Net {cfg.levels} levels, {cfg.base_channels} base channels, bf16",
               trained_steps=ws.meta.get("step"))
    return rep


def bp_sizes_main(args):
    """The step the paper times (Sec. 6.1): back projection (prefilter,
    tiled kernel, group reduction) at 64^2 ... 1024^2 with 180 views and
    lambda_y = lambda_x, without and with detector blur (zeta = 1).
    Median of 20 timed calls after 3 warm-ups per case; random sinogram
    values (the kernels' work does not depend on them)."""
    import torch
    from paper_2005_13471_amd import gramct as gct
    from paper_2005_13471_amd import inputs

    torch.cuda.set_device(0)
    dt = torch.float32
    n = 180
    rows = []
    for N in (64, 128, 256, 512, 1024):
        row = {"N": N}
        for zeta in (0.0, 1.0):
            M = inputs.detector_bins(N, zeta)
            P = gct.Plan(N, inputs.angles(n), M, zeta=zeta)
            g = torch.rand(n * M, dtype=dt, device="cuda")
            b = torch.empty(N * N, dtype=dt, device="cuda")
            ws = P.workspace(gct.OP_BACKPROJECT, dt)
            for _ in range(3):
                gct.backproject_boxspline(P, g, b, ws)
            ts = []
            for _ in range(20):
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                gct.backproject_boxspline(P, g, b, ws)
                e1.record()
                torch.cuda.synchronize()
                ts.append(e0.elapsed_time(e1))
            row["ms_blur" if zeta else "ms_noblur"] = round(float(np.median(ts)), 4)
        row["blur_over_noblur"] = round(row["ms_blur"] / row["ms_noblur"], 3)
        rows.append(row)
    print(json.dumps({"metric": "back projection time by image size, 180 views (unblurred and zeta = 1)",
                      "unit": "ms", "higher_is_better": False, "n_gpus": 1, "dtype": "f32",
                      "data": "synthetic", "config": {"workload": "bp_sizes_a180"}, "rows": rows}))


def main():
    args = parse()
    if args.pmc_summarize:
        if args.workload == "batch_uneven_256":
            return pmc_summarize_batch(*args.pmc_summarize)
        return pmc_summarize(*args.pmc_summarize)
    if args.workload == "bp_sizes_a180":
        if args.gpus != 1:
            print(json.dumps({"error": "this benchmark runs on one GPU", "n_gpus": args.gpus}))
            sys.exit(2)
        return bp_sizes_main(args)
    if args.workload == "batch_uneven_256":
        if args.gpus != 1:
            print(json.dumps({"error": "this benchmark runs on one GPU", "n_gpus": args.gpus}))
            sys.exit(2)
        return batch_main(args)
    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU; multi-GPU runs are not implemented",
                          "n_gpus": args.gpus}))
        sys.exit(2)
    import torch
    from paper_2005_13471_amd import gramct as gct
    from paper_2005_13471_amd import inputs

    cfg = inputs.WORKLOADS[args.workload]
    N, n, M, ly, zeta = cfg["N"], cfg["n"], cfg["M"], cfg["ly"], cfg["zeta"]
    theta = inputs.angles(n)
    torch.cuda.set_device(0)
    dt = torch.float32
    plan = gct.Plan(N, theta, M, ly=ly, zeta=zeta)
    P = plan.info.fft_size

    # ---- synthetic input, resident before timing --------------------------------
    c_true, _ = inputs.phantom(N, cfg["ellipses"], cfg["seed"])
    g_clean = torch.empty(n * M, dtype=dt, device="cuda")
    gct.forward_project(plan, torch.as_tensor(c_true.reshape(-1), dtype=dt, device="cuda"), g_clean)
    torch.cuda.synchronize()
    g_np = inputs.add_noise(g_clean.double().cpu().numpy().reshape(n, M), cfg["eta"],
                            inputs.NOISE_SEED_BASE + cfg["seed"])
    g_s = torch.as_tensor(g_np.reshape(-1), dtype=dt, device="cuda")
    c_apply = torch.as_tensor(inputs.uniform_coeffs(N, cfg["coeff_seed"]).reshape(-1), dtype=dt,
                              device="cuda")

    G = torch.empty(plan.info.gram_elems, dtype=dt, device="cuda")
    Ghat = torch.empty(plan.info.spectrum_elems, dtype=dt, device="cuda")
    b = torch.empty(N * N, dtype=dt, device="cuda")
    x = torch.empty(N * N, dtype=dt, device="cuda")
    y = torch.empty(N * N, dtype=dt, device="cuda")
    ws_spec = plan.workspace(gct.OP_GRAM_SPECTRUM, dt)
    ws_bp = plan.workspace(gct.OP_BACKPROJECT, dt)
    ws_apply = plan.workspace(gct.OP_GRAM_APPLY, dt)
    ws_cg = plan.workspace(gct.OP_CG, dt)

    ev = lambda: torch.cuda.Event(enable_timing=True)

    # setup: Gram spectrum, then the plan's transform tiling chosen by the
    # autotuner; capture a burst of applies once (inputs are fixed buffers)
    gct.gram_build(plan, G)
    gct.gram_spectrum(plan, G, Ghat, ws_spec)
    if args.phase_probe:
        # for counter runs of the two VALU-bound phases
        for _ in range(3):
            gct.gram_build(plan, G)
            gct.backproject_boxspline(plan, g_s, b, ws_bp)
        torch.cuda.synchronize()
        print(json.dumps({"phase_probe": True, "gram_build": 4, "backproject": 3}))
        return
    if args.fft_elems:
        er, ec = (list(map(int, args.fft_elems.split(","))) * 2)[:2]
        gct.plan_set_pass_elems(plan, er, ec)
        fft_elems = elems_key(er, ec)
    else:
        fft_elems = elems_key(*gct.plan_autotune(plan, Ghat, ws_cg, reps=20))
    torch.cuda.synchronize()
    if args.pmc_probe:
        return pmc_probe(gct, plan, Ghat, c_apply, y, ws_apply, fft_elems)
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        for _ in range(APPLY_GRAPH):
            gct.gram_apply(plan, Ghat, c_apply, y, ws_apply)
    torch.cuda.synchronize()

    def step(rec):
        e = [ev() for _ in range(6)]
        e[0].record()
        gct.gram_build(plan, G)
        e[1].record()
        gct.gram_spectrum(plan, G, Ghat, ws_spec)
        e[2].record()
        gct.backproject_boxspline(plan, g_s, b, ws_bp)
        e[3].record()
        res = gct.cg_solve(plan, Ghat, b, x, ws_cg, rtol=1e-4, max_iter=5000, check_every=16)
        e[4].record()
        for _ in range(APPLY_BURST // APPLY_GRAPH):
            graph.replay()
        e[5].record()
        rec.append((e, res))

    warm = []
    for _ in range(args.warmup):
        step(warm)
    torch.cuda.synchronize()
    rec = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(rec)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    # applies issued one C-ABI call at a time (host launch included)
    e0, e1 = ev(), ev()
    e0.record()
    for _ in range(APPLY_BURST):
        gct.gram_apply(plan, Ghat, c_apply, y, ws_apply)
    e1.record()
    torch.cuda.synchronize()
    eager_ms = e0.elapsed_time(e1) / APPLY_BURST

    ph = np.array([[e[i].elapsed_time(e[i + 1]) for i in range(5)] for e, _ in rec])  # ms
    apply_ms = ph[:, 4].sum() / (args.steps * APPLY_BURST)
    applies_per_s = 1e3 / apply_ms
    res = rec[-1][1]
    alg_bytes = 4 * N * N * 2 + 4 * (P // 2 + 1) * P  # c + y + real spectrum
    achieved = alg_bytes / (apply_ms * 1e-3) / 1e9

    out = {
        "metric": "H^T H applies/sec at 512^2, 720 angles + CG time to 1e-4 residual (plain vs warm)",
        "value": round(applies_per_s, 1),
        "unit": "applies/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "N": N, "n_angles": n, "M": M, "lambda_y": ly,
                   "zeta_blur": zeta, "fft_size": P, "ellipses": cfg["ellipses"],
                   "noise": cfg["eta"], "cg_rtol": 1e-4, "apply_burst": APPLY_BURST,
                   "apply_graph": APPLY_GRAPH, "fft_elems_per_thread": fft_elems,
                   "cg_elems_per_thread": elems_key(*gct.plan_get_pass_elems(plan)[2:])},
        "phase_ms": {"gram_build": round(float(np.median(ph[:, 0])), 4),
                     "gram_spectrum": round(float(np.median(ph[:, 1])), 4),
                     "backproject": round(float(np.median(ph[:, 2])), 4),
                     "cg_solve": round(float(np.median(ph[:, 3])), 4),
                     "gram_apply": round(apply_ms, 5),
                     "gram_apply_eager_call": round(eager_ms, 5)},
        "eager_applies_per_s": round(1e3 / eager_ms, 1),
        "cg_plain": {"iters": res.iters, "ms": round(float(np.median(ph[:, 3])), 3),
                     "rel_res": res.rel_res, "rel_res_true": res.rel_res_true,
                     "status": res.status, "dot_dtype": "f64"},
        "cg_warm": warm_compare(args.warm_slices) if args.warm_slices > 0 else None,
        "sd_plain": sd_plain(gct, plan, Ghat, b, ws_cg),
        "roofline": {"kernel": "gram_apply (rows / columns / rows FFT passes)", "bound": "hbm",
                     "achieved": round(achieved, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 5), "traffic": measured_traffic(fft_elems),
                     "alg_bytes_per_launch": alg_bytes},
    }
    if args.batch_slices > 0:
        del graph
        torch.cuda.synchronize()
        bt = batch_run(args.batch_slices, 3, 1)
        out["batch_uneven_256"] = {k: bt[k] for k in ("value", "unit", "metric", "phase_ms", "cg", "roofline",
                                                       "roofline_alu")}
        out["batch_uneven_256"]["config"] = {k: bt["config"][k] for k in ("slices", "seed", "N_values",
                                                                          "fft_groups")}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, theta, args.cpu_sample)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
