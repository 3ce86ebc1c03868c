"""Detector kernels of several boxes (Sec. 2: boxes of different heights and
lengths) through the C ABI: Gram filter, forward model and back projection
against the FP64 oracle on whole arrays, in FP32 and FP64; CG on the normal
equations with the oracle's re-check; a batch holding a multi-box slice.
Tolerances as in test_gpu_parity (normwise)."""
import numpy as np
import pytest
import torch

import oracle
from paper_2005_13471_amd import inputs
from gpu_helpers import normwise, say

pytestmark = pytest.mark.gpu

TOL = {"gram": (1e-5, 1e-11), "fp": (1e-4, 1e-11), "bp": (1e-4, 1e-11)}
DTYPES = [torch.float32, torch.float64]


def _bins(N, wmax, ly):
    m = int(np.ceil((N * np.sqrt(2.0) + wmax) / ly)) + 2
    return m + (m & 1)


class DCase:
    # regs: breakpoints the tiled back projection holds in registers per
    # angle in (FP32, FP64), 0 for a search in memory (13 sub-intervals with
    # boxes of widths 1 and 1/2, 17 and 25 for the others)
    def __init__(self, N, n, boxes, ly=1.0, lx=(1.0, 1.0), shift=0.0, regs=(0, 0)):
        self.N, self.boxes, self.ly, self.lx, self.regs = N, boxes, ly, lx, regs
        self.theta = inputs.angles(n) + shift
        self.n = n
        self.M = _bins(N, max(w for w, _ in boxes), ly)

    def plan(self, gct):
        return gct.Plan(self.N, self.theta, self.M, ly=self.ly, lx=self.lx, boxes=self.boxes)

    def og(self):
        return oracle.Geometry(self.N, self.theta, self.M, ly=self.ly, lx=self.lx, boxes=self.boxes)

    def __repr__(self):
        return f"N={self.N} n={self.n} boxes={self.boxes} ly={self.ly} lx={self.lx}"


CASES = [DCase(32, 24, [(1.0, 0.6), (0.5, 0.8)], regs=(16, 0)),
         DCase(27, 17, [(1.2, 0.3), (0.7, 0.5), (0.3, 0.8)], ly=0.8, lx=(0.9, 1.1), shift=0.013),
         DCase(20, 12, [(0.8, 1.0), (0.4, -0.5)])]


@pytest.fixture(scope="module")
def gct():
    from paper_2005_13471_amd import gramct
    assert torch.cuda.is_available()
    return gramct


def _host(t):
    torch.cuda.synchronize()
    return t.detach().double().cpu().numpy()


def tol(kind, dt):
    return TOL[kind][0 if dt == torch.float32 else 1]


@pytest.mark.parametrize("dt", DTYPES)
@pytest.mark.parametrize("case", CASES, ids=repr)
def test_multibox_gram_forward_backproject(gct, case, dt):
    say("multibox", case, dt)
    P = case.plan(gct)
    og = case.og()
    W = 2 * case.N - 1
    G = torch.empty(P.info.gram_elems, dtype=dt, device="cuda")
    gct.gram_build(P, G)
    eg = normwise(_host(G).reshape(W, W), oracle.gram(og))
    say("  gram", eg)
    assert eg <= tol("gram", dt)
    c = inputs.uniform_coeffs(case.N, 21)
    gs = torch.empty(case.n * case.M, dtype=dt, device="cuda")
    gct.forward_project(P, torch.as_tensor(c.reshape(-1), dtype=dt, device="cuda"), gs)
    ef = normwise(_host(gs).reshape(case.n, case.M), oracle.forward(og, c))
    say("  forward", ef)
    assert ef <= tol("fp", dt)
    ells = inputs.random_ellipses(case.N, 8, 22)
    sino = inputs.add_noise(inputs.analytic_sinogram(ells, case.theta, case.M, ly=case.ly, zeta=0.0),
                            0.01, inputs.NOISE_SEED_BASE + 22)
    b = torch.empty(case.N * case.N, dtype=dt, device="cuda")
    gct.backproject_boxspline(P, torch.as_tensor(sino.reshape(-1), dtype=dt, device="cuda"), b,
                              P.workspace(gct.OP_BACKPROJECT, dt))
    eb = normwise(_host(b).reshape(case.N, case.N), oracle.backproject(og, sino))
    shape = gct.plan_get_bp_shape(P, dt)
    say("  backproject", eb, "shape", shape)
    assert eb <= tol("bp", dt)
    if shape[0] > 0:
        assert shape[3] == case.regs[0 if dt == torch.float32 else 1], shape


def test_multibox_cg_converges_with_oracle_recheck(gct):
    case = CASES[0]
    dt = torch.float32
    P = case.plan(gct)
    og = case.og()
    G = torch.empty(P.info.gram_elems, dtype=dt, device="cuda")
    gct.gram_build(P, G)
    Ghat = torch.empty(P.info.spectrum_elems, dtype=dt, device="cuda")
    gct.gram_spectrum(P, G, Ghat, P.workspace(gct.OP_GRAM_SPECTRUM, dt))
    c_true, _ = inputs.phantom(case.N, 6, 23)
    b_or = oracle.backproject(og, oracle.forward(og, c_true))
    b = torch.as_tensor(b_or.reshape(-1), dtype=dt, device="cuda")
    x = torch.zeros_like(b)
    res = gct.cg_solve(P, Ghat, b, x, P.workspace(gct.OP_CG, dt), rtol=1e-4, max_iter=2000)
    say("multibox cg", res.status, res.iters, res.rel_res_true)
    assert res.status == gct.GCT_OK
    xh = _host(x).reshape(case.N, case.N)
    rel = np.linalg.norm(b_or - oracle.apply(oracle.gram(og), xh)) / np.linalg.norm(b_or)
    assert rel <= 1.01e-4


def test_multibox_slice_in_a_batch(gct):
    """A batch mixing a multi-box slice with blurred and unblurred ones:
    the batched Gram filters against the oracle per slice."""
    dt = torch.float32
    specs = [(CASES[0], None), (None, (24, 20, 1.0)), (None, (18, 15, 0.0))]
    plans, ogs = [], []
    for case, simple in specs:
        if case is not None:
            plans.append(case.plan(gct))
            ogs.append(case.og())
        else:
            N, n, z = simple
            th = inputs.angles(n) + 0.02
            M = inputs.detector_bins(N, z)
            plans.append(gct.Plan(N, th, M, zeta=z))
            ogs.append(oracle.Geometry(N, th, M, zeta=z))
    B = gct.Batch(plans)
    G = torch.empty(B.gram_elems, dtype=dt, device="cuda")
    gct.batch_gram_build(B, G)
    for i, p in enumerate(plans):
        W = 2 * p.N - 1
        o = int(B.gram_offsets[i])
        e = normwise(_host(G[o:o + W * W]).reshape(W, W), oracle.gram(ogs[i]))
        say("  batch slice", i, e)
        assert e <= 1e-5, i
