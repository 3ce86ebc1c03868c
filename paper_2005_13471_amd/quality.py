"""Reconstruction quality, after the paper's experiments (Sec. 6.2, 6.3).

Quality is measured as SNR (dB) and SSIM of a reconstruction against the
ground truth. The ground truth is the phantom in the pixel basis at ten times
the reconstruction's resolution, averaged over each reconstruction pixel.
The sinograms are exact line integrals of the continuous ellipse phantom,
so the forward model that reconstructs is not the one that measured (no
inverse crime).

The sweeps follow the paper's: image size (64^2 ... 1024^2), downsampling
rate lambda_y = n lambda_x, Gaussian noise level, and pixel sides
Lambda_x, each over several random phantoms. 180 views. Unregularised
steepest descent, the paper's solver, and CG next to it, both to the
stopping rule ||r|| <= rtol ||b||.

    python -m paper_2005_13471_amd.quality [--seeds 3] [--out results.json]
"""
from __future__ import annotations

import argparse
import json
import math

import numpy as np
import torch

from . import gramct as gct
from . import inputs


def snr_db(x: np.ndarray, ref: np.ndarray) -> float:
    """10 log10(||ref||^2 / ||x - ref||^2)."""
    ref = np.asarray(ref, dtype=np.float64)
    err = np.asarray(x, dtype=np.float64) - ref
    return 10.0 * math.log10(float(np.sum(ref * ref)) / float(np.sum(err * err)))


def ssim(x: np.ndarray, ref: np.ndarray, data_range: float | None = None, sigma: float = 1.5,
         k1: float = 0.01, k2: float = 0.03) -> float:
    """Mean structural similarity (Wang, Bovik, Sheikh and Simoncelli, 2004).

    Local statistics use a Gaussian window: standard deviation sigma,
    truncated at 3.5 sigma (11 x 11 at sigma = 1.5), reflecting boundaries.
    C1 = (k1 L)^2 and C2 = (k2 L)^2, with L the data range of ref.  The
    result is the mean over the pixels whose window lies inside the image."""
    from scipy.ndimage import gaussian_filter

    x = np.asarray(x, dtype=np.float64)
    y = np.asarray(ref, dtype=np.float64)
    L = float(y.max() - y.min()) if data_range is None else float(data_range)
    c1, c2 = (k1 * L) ** 2, (k2 * L) ** 2
    f = lambda a: gaussian_filter(a, sigma, mode="reflect", truncate=3.5)
    mx, my = f(x), f(y)
    sxx = f(x * x) - mx * mx
    syy = f(y * y) - my * my
    sxy = f(x * y) - mx * my
    s = ((2 * mx * my + c1) * (2 * sxy + c2)) / ((mx * mx + my * my + c1) * (sxx + syy + c2))
    pad = int(3.5 * sigma + 0.5)
    return float(s[pad:-pad, pad:-pad].mean())


def ground_truth(N: int, ells: list, lx=(1.0, 1.0)) -> np.ndarray:
    """Pixel-basis phantom at 10x resolution, averaged per reconstruction
    pixel (10 x 10 sub-pixel samples of each lx[0] x lx[1] pixel)."""
    return inputs.rasterize(N, ells, sub=10, lx=lx)


def detector_bins(N: int, zeta: float, ly: float, lx=(1.0, 1.0)) -> int:
    """Smallest even M with M ly >= (image diagonal) + zeta + 2 ly."""
    m = int(math.ceil((N * math.hypot(lx[0], lx[1]) + zeta) / ly + 2.0))
    return m + (m % 2)


def phantom_ellipses(N: int, count: int, seed: int, lx=(1.0, 1.0)) -> list:
    """Random ellipses (the usual distributions, scaled to the image's
    shorter side N min(lx)) that lie wholly inside the disc inscribed in the
    field of view: exact data of an object partly outside the image would
    measure what no coefficient can represent, and the unregularised solvers
    would fit it with border artefacts."""
    return inputs.random_ellipses_inside(N * min(lx[0], lx[1]), count, seed)


def reconstruct(N: int, n_angles: int, ly: float, zeta: float, ells: list, eta: float, seed: int,
                solver: str = "sd", rtol: float = 1e-4, max_iter: int = 20000, model_data: bool = False,
                lx=(1.0, 1.0)):
    """Exact sinogram of `ells` (+ Gaussian noise eta * RMS), back
    projection, then `solver` ("sd" or "cg") from zero.  Returns the
    reconstruction (N x N, float64 on the host) and the solver result.
    model_data: the sinogram is instead the plan's own forward model of the
    ground truth (the inverse crime: a consistency check of the pipeline,
    not a quality measurement).  lx: pixel sides (Lambda_x)."""
    theta = inputs.angles(n_angles)
    M = detector_bins(N, zeta, ly, lx)
    plan = gct.Plan(N, theta, M, ly=ly, zeta=zeta, lx=lx)
    dt = torch.float32
    G = torch.empty(plan.info.gram_elems, dtype=dt, device="cuda")
    gct.gram_build(plan, G)
    Ghat = torch.empty(plan.info.spectrum_elems, dtype=dt, device="cuda")
    gct.gram_spectrum(plan, G, Ghat, plan.workspace(gct.OP_GRAM_SPECTRUM, dt))
    if model_data:
        gt = torch.as_tensor(ground_truth(N, ells, lx).reshape(-1), dtype=dt, device="cuda")
        gm = torch.empty(n_angles * M, dtype=dt, device="cuda")
        gct.forward_project(plan, gt, gm)
        g = inputs.add_noise(gm.double().cpu().numpy().reshape(n_angles, M), eta, seed)
    else:
        g = inputs.add_noise(inputs.analytic_sinogram(ells, theta, M, ly=ly, zeta=zeta), eta, seed)
    b = torch.empty(N * N, dtype=dt, device="cuda")
    gct.backproject_boxspline(plan, torch.as_tensor(g.reshape(-1), dtype=dt, device="cuda"), b,
                              plan.workspace(gct.OP_BACKPROJECT, dt))
    x = torch.zeros_like(b)
    solve = gct.sd_solve if solver == "sd" else gct.cg_solve
    res = solve(plan, Ghat, b, x, plan.workspace(gct.OP_CG, dt), rtol=rtol, max_iter=max_iter,
                check_every=64 if solver == "sd" else 8)
    return x.double().cpu().numpy().reshape(N, N), res


def study(sizes=(64, 128, 256, 512, 1024), rates=(0.25, 0.5, 1.0, 2.0), etas=(0.0, 0.01, 0.02, 0.05),
          pixels=((1.0, 1.0), (0.5, 0.5), (2.0, 2.0), (0.8, 1.25), (1.25, 0.8), (0.6, 1.0)),
          seeds=(4242, 4243, 4244), n_angles: int = 180, zeta: float = 1.0, ellipses: int = 20,
          log=print):
    """The paper's sweeps, each over several phantoms (seeds): size (rate 1,
    no noise), downsampling rate lambda_y = n lambda_x (N = 64, no noise),
    noise level (N = 128, rate 1), and pixel sides Lambda_x (N = 64,
    lambda_y = 1, no noise; isotropic sizes change the rate relative to the
    pixel, the others are anisotropic), each with steepest descent and CG.
    Returns a list of result rows, one per (case, phantom, solver)."""
    cases = [("size", N, 1.0, 0.0, (1.0, 1.0)) for N in sizes]
    cases += [("rate", 64, r, 0.0, (1.0, 1.0)) for r in rates]
    cases += [("noise", 128, 1.0, e, (1.0, 1.0)) for e in etas]
    cases += [("pixel", 64, 1.0, 0.0, tuple(lx)) for lx in pixels]
    rows = []
    for sweep, N, ly, eta, lx in cases:
        for seed in seeds:
            ells = phantom_ellipses(N, ellipses, seed, lx)
            ref = ground_truth(N, ells, lx)
            for solver in ("sd", "cg"):
                x, res = reconstruct(N, n_angles, ly, zeta, ells, eta, seed + 1, solver=solver, lx=lx)
                row = dict(sweep=sweep, N=N, rate=ly, eta=eta, lx=list(lx), seed=seed, solver=solver,
                           iters=int(res.iters), status=int(res.status),
                           rel_res_true=float(res.rel_res_true), snr_db=snr_db(x, ref), ssim=ssim(x, ref))
                log(json.dumps(row))
                rows.append(row)
    return rows


def summarize(rows):
    """Mean and standard deviation over the phantoms of each (case, solver)."""
    groups = {}
    for r in rows:
        k = (r["sweep"], r["N"], r["rate"], r["eta"], tuple(r["lx"]), r["solver"])
        groups.setdefault(k, []).append(r)
    out = []
    for k, g in groups.items():
        snr = np.array([r["snr_db"] for r in g])
        ss = np.array([r["ssim"] for r in g])
        it = np.array([r["iters"] for r in g])
        out.append(dict(sweep=k[0], N=k[1], rate=k[2], eta=k[3], lx=list(k[4]), solver=k[5], phantoms=len(g),
                        iters=float(it.mean()), snr_db=float(snr.mean()), snr_std=float(snr.std()),
                        ssim=float(ss.mean()), ssim_std=float(ss.std()),
                        all_converged=all(r["status"] == 0 for r in g)))
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--out", default=None)
    ap.add_argument("--seeds", type=int, default=3, help="phantoms per case")
    a = ap.parse_args(argv)
    rows = study(seeds=tuple(4242 + i for i in range(a.seeds)), log=lambda s: print(s, flush=True))
    summ = summarize(rows)
    print("| sweep | N | rate | Lambda_x | noise | solver | iterations | SNR dB | SSIM |")
    print("|---|---:|---:|---|---:|---|---:|---:|---:|")
    for r in summ:
        print(f"| {r['sweep']} | {r['N']} | {r['rate']} | {r['lx'][0]} x {r['lx'][1]} | {r['eta']} | {r['solver']} | "
              f"{r['iters']:.0f} | {r['snr_db']:.2f} ± {r['snr_std']:.2f} | {r['ssim']:.4f} ± {r['ssim_std']:.4f} |")
    if a.out:
        with open(a.out, "w") as f:
            json.dump({"rows": rows, "summary": summ}, f, indent=1)


if __name__ == "__main__":
    main()
