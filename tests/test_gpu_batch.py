"""Batched uneven slices through the C ABI: Gram filters, spectra, Gram
filtering and CG for several slices of different N, angle sets and blur in
one launch per phase, against the FP64 oracle per slice, against the
single-slice path, and after autotuning."""
import numpy as np
import pytest
import torch

import oracle
from paper_2005_13471_amd import inputs
from gpu_helpers import normwise, sample_pixels, sample_taps, say

pytestmark = pytest.mark.gpu

# (N, n_angles, zeta): FFT sizes 32, 64, 128, 128, 256 -> four groups
SLICES = [(16, 12, 0.0), (23, 17, 1.0), (37, 45, 1.0), (64, 90, 0.0), (100, 150, 0.5)]


@pytest.fixture(scope="module")
def batch_setup():
    from paper_2005_13471_amd import gramct as gct
    plans, ogs = [], []
    for i, (N, n, z) in enumerate(SLICES):
        th = inputs.angles(n) + 0.01 * i
        M = inputs.detector_bins(N, z)
        plans.append(gct.Plan(N, th, M, zeta=z))
        ogs.append(oracle.Geometry(N, th, M, zeta=z))
    return gct, gct.Batch(plans), plans, ogs


def _packed(batch, arrays, dt):
    out = torch.zeros(batch.image_elems, dtype=dt, device="cuda")
    for i, a in enumerate(arrays):
        batch.image(out, i).copy_(torch.as_tensor(a, dtype=dt, device="cuda"))
    return out


@pytest.mark.parametrize("dt", [torch.float32, torch.float64])
def test_batch_gram_build_and_apply_match_oracle(batch_setup, dt):
    gct, B, plans, ogs = batch_setup
    say("batch gram_build / apply", dt)
    # the first slice's uniform even angle set: one octant of taps evaluated
    assert [p.info.gram_symmetry for p in plans] == [8, 2, 2, 2, 2]
    G = torch.empty(B.gram_elems, dtype=dt, device="cuda")
    gct.batch_gram_build(B, G)
    Ghat = torch.empty(B.spectrum_elems, dtype=dt, device="cuda")
    gct.batch_gram_spectrum(B, G, Ghat, B.workspace(gct.OP_GRAM_SPECTRUM, dt))
    cs = [inputs.uniform_coeffs(N, 2000 + i) for i, (N, _, _) in enumerate(SLICES)]
    y = torch.empty(B.image_elems, dtype=dt, device="cuda")
    gct.batch_gram_apply(B, Ghat, _packed(B, cs, dt), y, B.workspace(gct.OP_GRAM_APPLY, dt))
    torch.cuda.synchronize()
    tg = 1e-5 if dt == torch.float32 else 1e-11
    ta = 1e-4 if dt == torch.float32 else 1e-11
    for i, (N, _, _) in enumerate(SLICES):
        W = 2 * N - 1
        o = int(B.gram_offsets[i])
        g_gpu = G[o:o + W * W].double().cpu().numpy().reshape(W, W)
        g_or = oracle.gram(ogs[i])
        assert normwise(g_gpu, g_or) <= tg, i
        y_or = oracle.apply(g_or, cs[i])
        assert normwise(B.image(y, i).double().cpu().numpy(), y_or) <= ta, i


def test_batch_apply_bitwise_equals_single_slice(batch_setup):
    """Same device bodies and tile shapes: from the same Gram filter the
    batched spectrum and apply reproduce the single-slice ones bit for bit
    (before autotuning) at the power-of-two transform sizes; at three times
    a power of two the apply agrees to a few units in the last place (the
    same arithmetic in separately compiled kernels, where the compiler
    contracts the radix-3 butterflies' products and sums differently).  The
    Gram builds themselves use different tile shapes (the single-slice build
    splits each tile's angles over the block's waves), so their sums are
    ordered differently and agree to FP32 rounding."""
    gct, B, plans, ogs = batch_setup
    dt = torch.float32
    G = torch.empty(B.gram_elems, dtype=dt, device="cuda")
    gct.batch_gram_build(B, G)
    Ghat = torch.empty(B.spectrum_elems, dtype=dt, device="cuda")
    gct.batch_gram_spectrum(B, G, Ghat, B.workspace(gct.OP_GRAM_SPECTRUM, dt))
    cs = [inputs.uniform_coeffs(N, 3000 + i) for i, (N, _, _) in enumerate(SLICES)]
    y = torch.empty(B.image_elems, dtype=dt, device="cuda")
    gct.batch_gram_apply(B, Ghat, _packed(B, cs, dt), y, B.workspace(gct.OP_GRAM_APPLY, dt))
    for i, P in enumerate(plans):
        Gi = torch.empty(P.info.gram_elems, dtype=dt, device="cuda")
        gct.gram_build(P, Gi)
        o = int(B.gram_offsets[i])
        Gb = G[o:o + P.info.gram_elems]
        assert normwise(Gi.double().cpu().numpy(), Gb.double().cpu().numpy()) <= 1e-6
        Gh = torch.empty(P.info.spectrum_elems, dtype=dt, device="cuda")
        gct.gram_spectrum(P, Gb.contiguous(), Gh, P.workspace(gct.OP_GRAM_SPECTRUM, dt))
        so = int(B.spectrum_offsets[i])
        assert torch.equal(Gh, Ghat[so:so + P.info.spectrum_elems])
        yi = torch.empty(P.N * P.N, dtype=dt, device="cuda")
        gct.gram_apply(P, Gh, torch.as_tensor(cs[i].reshape(-1), dtype=dt, device="cuda"), yi,
                       P.workspace(gct.OP_GRAM_APPLY, dt))
        size = P.info.fft_size
        if size & (size - 1) == 0:
            assert torch.equal(yi.view(P.N, P.N), B.image(y, i)), size
        else:
            d = float((yi.view(P.N, P.N) - B.image(y, i)).abs().max())
            assert d <= 1e-6 * float(yi.abs().max()), (size, d)


@pytest.mark.parametrize("dt", [torch.float32, torch.float64])
def test_batch_cg_matches_single_slice_and_oracle(batch_setup, dt):
    gct, B, plans, ogs = batch_setup
    say("batch cg", dt)
    G = torch.empty(B.gram_elems, dtype=dt, device="cuda")
    gct.batch_gram_build(B, G)
    Ghat = torch.empty(B.spectrum_elems, dtype=dt, device="cuda")
    gct.batch_gram_spectrum(B, G, Ghat, B.workspace(gct.OP_GRAM_SPECTRUM, dt))
    bs = []
    for i, (N, n, z) in enumerate(SLICES):
        ells = inputs.random_ellipses(N, 8, 1000 + i)
        sino = inputs.add_noise(inputs.analytic_sinogram(ells, plans[i].theta, plans[i].M, zeta=z),
                                0.01, inputs.NOISE_SEED_BASE + 1000 + i)
        bi = torch.empty(N * N, dtype=dt, device="cuda")
        gct.backproject_boxspline(plans[i], torch.as_tensor(sino.reshape(-1), dtype=dt, device="cuda"),
                                  bi, plans[i].workspace(gct.OP_BACKPROJECT, dt))
        bs.append(bi.view(N, N))
    b = torch.zeros(B.image_elems, dtype=dt, device="cuda")
    for i in range(len(SLICES)):
        B.image(b, i).copy_(bs[i])
    x = torch.empty_like(b)
    res = gct.batch_cg_solve(B, Ghat, b, x, B.workspace(gct.OP_CG, dt), rtol=1e-4, max_iter=500,
                             check_every=4)
    for i, P in enumerate(plans):
        gi = torch.empty(P.info.gram_elems, dtype=dt, device="cuda")
        gct.gram_build(P, gi)
        gh = torch.empty(P.info.spectrum_elems, dtype=dt, device="cuda")
        gct.gram_spectrum(P, gi, gh, P.workspace(gct.OP_GRAM_SPECTRUM, dt))
        xi = torch.zeros(P.N * P.N, dtype=dt, device="cuda")
        ri = gct.cg_solve(P, gh, bs[i].reshape(-1).contiguous(), xi, P.workspace(gct.OP_CG, dt),
                          rtol=1e-4, max_iter=500)
        say("  slice", i, "batch iters", res[i].iters, "single", ri.iters, "true", res[i].rel_res_true)
        assert res[i].status == gct.GCT_OK
        # the batched solver (textbook arrangement) and the single-slice one
        # (Chronopoulos-Gear arrangement) agree in exact arithmetic only
        assert abs(res[i].iters - ri.iters) <= max(5, (3 * ri.iters) // 20)
        # the oracle re-checks the batched iterate
        G_or = oracle.gram(ogs[i])
        bh = bs[i].double().cpu().numpy()
        xh = B.image(x, i).double().cpu().numpy()
        rel = np.linalg.norm(bh - oracle.apply(G_or, xh)) / np.linalg.norm(bh)
        assert rel <= (1.1e-4 if dt == torch.float32 else 1.0001e-4)
    # from start vectors: the converged iterates restart converged; a start
    # worse than zero (10 b, far from the solution) falls back to zero and
    # repeats the plain solve's iterations
    ws = B.workspace(gct.OP_CG, dt)
    x2 = x.clone()
    res2 = gct.batch_cg_solve(B, Ghat, b, x2, ws, rtol=1e-4, max_iter=500, check_every=4, use_x0=True)
    assert all(r.status == gct.GCT_OK and r.iters <= 3 and not r.fell_back and r.rel_res0 <= 1.1e-4 for r in res2)
    x3 = (10.0 * b).contiguous()
    res3 = gct.batch_cg_solve(B, Ghat, b, x3, ws, rtol=1e-4, max_iter=500, check_every=4, use_x0=True)
    say("  fallback iters", [r.iters for r in res3], "plain", [r.iters for r in res])
    assert all(r.fell_back and r.status == gct.GCT_OK for r in res3)
    assert [r.iters for r in res3] == [r.iters for r in res]


def test_batch_autotune_keeps_results(batch_setup):
    gct, B, plans, ogs = batch_setup
    dt = torch.float32
    G = torch.empty(B.gram_elems, dtype=dt, device="cuda")
    gct.batch_gram_build(B, G)
    Ghat = torch.empty(B.spectrum_elems, dtype=dt, device="cuda")
    gct.batch_gram_spectrum(B, G, Ghat, B.workspace(gct.OP_GRAM_SPECTRUM, dt))
    chosen = gct.batch_autotune(B, Ghat, B.workspace(gct.OP_CG, dt), reps=2)
    both = gct.batch_get_pass_elems(B, dt)
    say("autotune choice per FFT size (rows, cols)", both)
    assert B.groups == 4
    assert len(chosen) == B.groups and all(e in (4, 8, 16, 12, 24) for e in chosen)
    assert [r for r, _ in both] == chosen and all(c in (4, 8, 16, 12, 24) for _, c in both)
    cs = [inputs.uniform_coeffs(N, 4000 + i) for i, (N, _, _) in enumerate(SLICES)]
    y = torch.empty(B.image_elems, dtype=dt, device="cuda")
    gct.batch_gram_apply(B, Ghat, _packed(B, cs, dt), y, B.workspace(gct.OP_GRAM_APPLY, dt))
    for i in range(len(SLICES)):
        y_or = oracle.apply(oracle.gram(ogs[i]), cs[i])
        assert normwise(B.image(y, i).double().cpu().numpy(), y_or) <= 1e-4


def test_batch_rejects_bad_arguments(batch_setup):
    gct, B, plans, ogs = batch_setup
    t = torch.zeros(B.image_elems, dtype=torch.float32, device="cuda")
    gh = torch.zeros(B.spectrum_elems, dtype=torch.float32, device="cuda")
    with pytest.raises(gct.GramctError) as e:
        gct.batch_gram_apply(B, gh, t, t, B.workspace(gct.OP_GRAM_APPLY))
    assert e.value.code == gct.GCT_EINVAL


# long transforms: 1024- and 2048-point groups, where FP32 row passes take
# two row pairs per block when every slice of the group has even N (the
# second batch has an odd N in the 1024-point group, which keeps the
# one-pair kernels there), and 1536-point groups (three times a power of two)
LONG = [[(400, 60, 1.0), (390, 40, 0.0), (800, 30, 1.0), (402, 20, 0.5), (600, 20, 1.0)],
        [(400, 60, 1.0), (401, 24, 0.5), (800, 30, 1.0), (700, 16, 0.5)]]
# slices whose group takes the two-pair row kernels
LONG_PAIRED = [{400, 390, 800, 402}, {800}]


@pytest.mark.parametrize("which", [0, 1])
def test_batch_long_transforms_match_single_slice_and_oracle(which):
    """Batched spectrum and apply of long-transform slices against the
    single-slice ones from the same Gram filter: the spectrum bit for bit;
    the apply to a few units in the last place (the same arithmetic in
    separately compiled kernels, where the compiler may contract products and
    sums differently; LONG_PAIRED marks the slices that also take the
    two-pair row kernels).  Sampled outputs against the oracle's direct sum;
    batched CG meets the stopping rule with the oracle's re-check of sampled
    residual entries."""
    from paper_2005_13471_amd import gramct as gct
    dt = torch.float32
    spec = LONG[which]
    plans, ogs = [], []
    for i, (N, n, z) in enumerate(spec):
        th = inputs.angles(n) + 0.013 * i
        M = inputs.detector_bins(N, z)
        plans.append(gct.Plan(N, th, M, zeta=z))
        ogs.append(oracle.Geometry(N, th, M, zeta=z))
    say("batch long", which, [p.N for p in plans])
    B = gct.Batch(plans)
    G = torch.empty(B.gram_elems, dtype=dt, device="cuda")
    gct.batch_gram_build(B, G)
    Ghat = torch.empty(B.spectrum_elems, dtype=dt, device="cuda")
    gct.batch_gram_spectrum(B, G, Ghat, B.workspace(gct.OP_GRAM_SPECTRUM, dt))
    cs = [inputs.uniform_coeffs(N, 4000 + i) for i, (N, _, _) in enumerate(spec)]
    y = torch.empty(B.image_elems, dtype=dt, device="cuda")
    gct.batch_gram_apply(B, Ghat, _packed(B, cs, dt), y, B.workspace(gct.OP_GRAM_APPLY, dt))
    for i, P in enumerate(plans):
        o = int(B.gram_offsets[i])
        Gb = G[o:o + P.info.gram_elems].contiguous()
        Gh = torch.empty(P.info.spectrum_elems, dtype=dt, device="cuda")
        gct.gram_spectrum(P, Gb, Gh, P.workspace(gct.OP_GRAM_SPECTRUM, dt))
        so = int(B.spectrum_offsets[i])
        say("  slice", i, "N", P.N, "spectrum max diff",
            float((Gh - Ghat[so:so + P.info.spectrum_elems]).abs().max()))
        assert torch.equal(Gh, Ghat[so:so + P.info.spectrum_elems]), i
        yi = torch.empty(P.N * P.N, dtype=dt, device="cuda")
        gct.gram_apply(P, Gh, torch.as_tensor(cs[i].reshape(-1), dtype=dt, device="cuda"), yi,
                       P.workspace(gct.OP_GRAM_APPLY, dt))
        d = float((yi.view(P.N, P.N) - B.image(y, i)).abs().max())
        say("  slice", i, "apply max diff", d)
        assert d <= 1e-6 * float(yi.abs().max()), (i, P.N in LONG_PAIRED[which])
        # sampled outputs against the oracle's exact filter
        g_or = oracle.gram(ogs[i])
        idx = sample_pixels(P.N, 60, 10 + i)
        ref = oracle.apply_at(g_or, cs[i], idx)
        got = B.image(y, i).double().cpu().numpy().reshape(-1)[idx]
        assert np.max(np.abs(got - ref)) <= 1e-4 * np.max(np.abs(ref)), i
    # batched CG (dot partials of the two-pair kernels) to 1e-4
    bs = [torch.as_tensor(inputs.uniform_coeffs(N, 5000 + i), dtype=dt, device="cuda")
          for i, (N, _, _) in enumerate(spec)]
    bpk = torch.zeros(B.image_elems, dtype=dt, device="cuda")
    for i, bi in enumerate(bs):
        gct.gram_apply(plans[i], Ghat[int(B.spectrum_offsets[i]):int(B.spectrum_offsets[i]) + plans[i].info.spectrum_elems],
                       bi.reshape(-1), B.image(bpk, i).reshape(-1), plans[i].workspace(gct.OP_GRAM_APPLY, dt))
    x = torch.zeros_like(bpk)
    res = gct.batch_cg_solve(B, Ghat, bpk, x, B.workspace(gct.OP_CG, dt), rtol=1e-4, max_iter=500,
                             check_every=4)
    for i, P in enumerate(plans):
        say("  slice", i, "N", P.N, "iters", res[i].iters, "true", res[i].rel_res_true)
        assert res[i].status == gct.GCT_OK and res[i].rel_res_true <= 1.2e-4
        g_or = oracle.gram(ogs[i])
        idx = sample_pixels(P.N, 60, 20 + i)
        bh = B.image(bpk, i).double().cpu().numpy()
        xh = B.image(x, i).double().cpu().numpy()
        r = bh.reshape(-1)[idx] - oracle.apply_at(g_or, xh, idx)
        assert np.sqrt(np.mean(r ** 2)) <= 3e-4 * np.linalg.norm(bh) / P.N


# slices at the sizes of the 256-slice benchmark batch: the largest N and
# angle count (the batched Gram build takes its angular windows in several
# runs of 256 angles), a 2048-point transform of N = 768, and a small slice
LARGE_SLICES = [(1024, 1440, 0.5), (768, 720, 1.0), (128, 180, 0.0)]


def test_batch_large_slices_match_oracle():
    """Batch of benchmark-sized slices against the oracle: sampled Gram taps
    (oracle.gram_at), sampled outputs of the batched apply (the oracle's
    direct sum with its exact filter), and batched CG to 1e-4 on back
    projections of noisy phantom sinograms with the oracle's recomputation of
    sampled residual entries of each returned iterate."""
    from paper_2005_13471_amd import gramct as gct
    dt = torch.float32
    plans, ogs = [], []
    for i, (N, n, z) in enumerate(LARGE_SLICES):
        th = inputs.angles(n)
        M = inputs.detector_bins(N, z)
        plans.append(gct.Plan(N, th, M, zeta=z))
        ogs.append(oracle.Geometry(N, th, M, zeta=z))
    say("batch large slices", [(p.N, p.info.n_angles) for p in plans])
    B = gct.Batch(plans)
    G = torch.empty(B.gram_elems, dtype=dt, device="cuda")
    gct.batch_gram_build(B, G)
    Ghat = torch.empty(B.spectrum_elems, dtype=dt, device="cuda")
    gct.batch_gram_spectrum(B, G, Ghat, B.workspace(gct.OP_GRAM_SPECTRUM, dt))
    cs = [inputs.uniform_coeffs(N, 6000 + i) for i, (N, _, _) in enumerate(LARGE_SLICES)]
    y = torch.empty(B.image_elems, dtype=dt, device="cuda")
    gct.batch_gram_apply(B, Ghat, _packed(B, cs, dt), y, B.workspace(gct.OP_GRAM_APPLY, dt))
    # right-hand sides as in the benchmark: back projections of noisy
    # sinograms of 40-ellipse phantoms (line integrals of the ellipses)
    rhs = []
    for i, (N, n, z) in enumerate(LARGE_SLICES):
        ells = inputs.random_ellipses(N, 40, 7000 + i)
        sino = inputs.add_noise(inputs.analytic_sinogram(ells, plans[i].theta, plans[i].M, zeta=z),
                                0.01, inputs.NOISE_SEED_BASE + 7000 + i)
        bi = torch.empty(N * N, dtype=dt, device="cuda")
        gct.backproject_boxspline(plans[i], torch.as_tensor(sino.reshape(-1), dtype=dt, device="cuda"),
                                  bi, plans[i].workspace(gct.OP_BACKPROJECT, dt))
        rhs.append(bi.double().cpu().numpy().reshape(N, N))
    bpk = _packed(B, rhs, dt)
    x = torch.zeros_like(bpk)
    res = gct.batch_cg_solve(B, Ghat, bpk, x, B.workspace(gct.OP_CG, dt), rtol=1e-4, max_iter=3000,
                             check_every=16)
    torch.cuda.synchronize()
    for i, P in enumerate(plans):
        N = P.N
        W = 2 * N - 1
        o = int(B.gram_offsets[i])
        Gb = G[o:o + W * W].double().cpu().numpy().reshape(W, W)
        taps = sample_taps(N, 300, 30 + i)
        g_at = oracle.gram_at(ogs[i], taps)
        got = Gb[taps[:, 1] + N - 1, taps[:, 0] + N - 1]
        eg = normwise(got, g_at)
        say("  slice", i, "N", N, "sampled taps normwise", eg)
        assert eg <= 1e-5, i
        say("  slice", i, "oracle Gram filter")
        g_or = oracle.gram(ogs[i])
        idx = sample_pixels(N, 200, 40 + i)
        ref = oracle.apply_at(g_or, cs[i], idx)
        ya = B.image(y, i).double().cpu().numpy().reshape(-1)[idx]
        ea = normwise(ya, ref)
        say("  slice", i, "sampled apply normwise", ea)
        assert ea <= 1e-4, i
        say("  slice", i, "cg iters", res[i].iters, "status", res[i].status, "true", res[i].rel_res_true)
        assert res[i].status == gct.GCT_OK and res[i].rel_res_true <= 1.2e-4
        idx = sample_pixels(N, 300, 50 + i)
        xh = B.image(x, i).double().cpu().numpy()
        r = rhs[i].reshape(-1)[idx] - oracle.apply_at(g_or, xh, idx)
        # sampled residual entries consistent with ||r|| <= 1e-4 ||b||
        assert np.sqrt(np.mean(r ** 2)) <= 3e-4 * np.linalg.norm(rhs[i]) / N, i


@pytest.mark.parametrize("dt,rtol", [(torch.float32, 1e-7), (torch.float64, 1e-10)])
def test_batch_cg_success_means_true_residual(batch_setup, dt, rtol):
    """As for the single-slice solver: a slice reports success only when its
    recomputed residual meets rtol (far below FP32's attainable accuracy the
    recursive residual alone would); FP64 reaches the same tolerance, and the
    oracle's recomputed residual of each FP64 iterate agrees."""
    gct, B, plans, ogs = batch_setup
    G = torch.empty(B.gram_elems, dtype=dt, device="cuda")
    gct.batch_gram_build(B, G)
    Ghat = torch.empty(B.spectrum_elems, dtype=dt, device="cuda")
    gct.batch_gram_spectrum(B, G, Ghat, B.workspace(gct.OP_GRAM_SPECTRUM, dt))
    rhs = []
    for i, (N, n, z) in enumerate(SLICES):
        ells = inputs.random_ellipses(N, 8, 8000 + i)
        sino = inputs.add_noise(inputs.analytic_sinogram(ells, plans[i].theta, plans[i].M, zeta=z),
                                0.01, inputs.NOISE_SEED_BASE + 8000 + i)
        bi = torch.empty(N * N, dtype=dt, device="cuda")
        gct.backproject_boxspline(plans[i], torch.as_tensor(sino.reshape(-1), dtype=dt, device="cuda"),
                                  bi, plans[i].workspace(gct.OP_BACKPROJECT, dt))
        rhs.append(bi.double().cpu().numpy().reshape(N, N))
    b = _packed(B, rhs, dt)
    x = torch.zeros_like(b)
    res = gct.batch_cg_solve(B, Ghat, b, x, B.workspace(gct.OP_CG, dt), rtol=rtol, max_iter=1500,
                             check_every=8)
    say("batch cg rtol", rtol, dt, [(r.status, r.iters, r.rel_res, r.rel_res_true) for r in res])
    for i, r in enumerate(res):
        assert r.status in (gct.GCT_OK, gct.GCT_ENOTCONV), i
        assert r.iters <= 1500
        if r.status == gct.GCT_OK:
            assert r.rel_res_true <= rtol, i
        if dt == torch.float64:
            assert r.status == gct.GCT_OK, i
            xh = B.image(x, i).double().cpu().numpy()
            true_rel = np.linalg.norm(rhs[i] - oracle.apply(oracle.gram(ogs[i]), xh)) / np.linalg.norm(rhs[i])
            assert true_rel <= 1.001 * rtol, i
