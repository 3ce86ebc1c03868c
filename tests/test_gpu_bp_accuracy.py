"""Back-projection accuracy against sampling (Sec. 6.1): 64 x 64 pixels,
180 views, downsampling rate lambda_y = n lambda_x with n from 0.5 to 2, a
random-ellipse phantom (the paper's "Spots" image is random ellipses; its
640 x 640 image is the object at ten times the resolution, here the
continuous ellipses themselves).

Reading of the ground truth: the exact adjoint of the model applied to the
continuous data, b_gt[k] = sum_theta integral F_k(y) q_theta(y) dy, with
q_theta the line integrals of the ellipses (cell-averaged over the detector
blur for the blurred model) known at every y.  The oracle computes it from
q sampled 40x finer than the finest rate (its own interpolation error there
is checked against a 20x-finer sampling).  The GPU back projection works
from the samples at rate n (the box-spline interpolation of Sec. 5), so
the error isolates what the sampling and interpolation lose.  SNR =
10 log10(||b_gt||^2 / ||b - b_gt||^2).  Two detector models: point samples
(zeta = 0) and cells as wide as the sampling step (zeta = lambda_y).  If
GCT_REPORT_DIR is set the table is written there as bp_accuracy_n64.json."""
import json
import os

import numpy as np
import pytest
import torch

import oracle
from gpu_helpers import say
from paper_2005_13471_amd import inputs

pytestmark = pytest.mark.gpu

N, NA = 64, 180
RATES = (0.5, 0.75, 1.0, 1.5, 2.0)


def _bins(zeta, ly):
    m = int(np.ceil((N * np.sqrt(2.0) + zeta) / ly + 2.0))
    return m + (m & 1)


def _snr(x, ref):
    return 10.0 * np.log10(np.sum(ref * ref) / np.sum((x - ref) ** 2))


def _truth(ells, theta, zeta, ly_fine):
    M = _bins(zeta, ly_fine)
    q = inputs.analytic_sinogram(ells, theta, M, ly=ly_fine, zeta=zeta)
    return oracle.backproject(oracle.Geometry(N, theta, M, ly=ly_fine, zeta=zeta), q)


@pytest.mark.parametrize("blur", [False, True], ids=["point", "cell"])
def test_backprojection_accuracy_against_sampling_rate(blur):
    from paper_2005_13471_amd import gramct as gct
    theta = inputs.angles(NA)
    ells = inputs.random_ellipses(N, 20, 4242)
    rows = []
    for n in RATES:
        zeta = n if blur else 0.0
        b_gt = _truth(ells, theta, zeta, n / 40.0)
        b_gt2 = _truth(ells, theta, zeta, n / 20.0)
        M = _bins(zeta, n)
        P = gct.Plan(N, theta, M, ly=n, zeta=zeta)
        g = inputs.analytic_sinogram(ells, theta, M, ly=n, zeta=zeta)
        b = torch.empty(N * N, dtype=torch.float32, device="cuda")
        gct.backproject_boxspline(P, torch.as_tensor(g.reshape(-1), dtype=torch.float32, device="cuda"), b,
                                  P.workspace(gct.OP_BACKPROJECT, torch.float32))
        torch.cuda.synchronize()
        bh = b.double().cpu().numpy().reshape(N, N)
        row = {"rate": n, "zeta": zeta, "snr_db": _snr(bh, b_gt), "truth_snr_db": _snr(b_gt2, b_gt)}
        say("bp accuracy", row)
        rows.append(row)
        # the ground truth is converged far beyond the error being measured
        assert row["truth_snr_db"] > row["snr_db"] + 15.0
    snr = [r["snr_db"] for r in rows]
    # finer sampling, better back projection
    assert all(a > b for a, b in zip(snr[:-1], snr[1:])), snr
    assert snr[RATES.index(1.0)] > 20.0
    out = os.environ.get("GCT_REPORT_DIR")
    if out:
        os.makedirs(out, exist_ok=True)
        path = os.path.join(out, "bp_accuracy_n64.json")
        old = json.load(open(path)) if os.path.exists(path) else {}
        old["cell" if blur else "point"] = rows
        json.dump(old, open(path, "w"), indent=1)
