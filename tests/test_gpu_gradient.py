"""Adjoint (path-replay) gradients on the GPU: against the FP64 oracle's
gradient on the same Philox streams, against central finite differences
with common random numbers on the differentiable workload, and through the
torch.autograd.Function."""
import math

import numpy as np
import pytest
import torch

from paper_2402_03106_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def D():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2402_03106_amd import darts
    darts.lib()
    return darts


@pytest.mark.parametrize("wname,mode", [("box_point", "darts"), ("box_point", "uniform"),
                                        ("box_hg_small", "darts"), ("box_hg_small", "da_only"),
                                        ("infinite_point", "darts"), ("box_hg_grad", "darts")])
def test_gradient_matches_oracle(D, oracle, wname, mode):
    """Replay gradient of sum_c G_c I_c (G uniform random per cell) against
    the FP64 oracle's on the same paths, to 2e-3 of the largest component;
    box_hg_grad is the differentiable workload at its own size (128x128
    pixels x 512 bins, 2^22 paths)."""
    w = getattr(W, wname)()
    sc, pr, dm = w["scene"], w["params"], w["dims"]
    gimg = np.random.default_rng(1).random(oracle.image_shape(sc))
    table = D.build_da_tables(sc["medium"], dm)
    g = D.render_transient_backward(sc, pr, mode, table, torch.from_numpy(gimg).float().cuda())
    torch.cuda.synchronize()
    g = g.cpu().numpy()
    _, cdf = oracle.build_table(sc["medium"], dm)
    go = oracle.render_gradient(sc, pr, mode, gimg.astype(np.float32).astype(np.float64), cdf, dm)
    print(wname, mode, g, go)
    assert np.max(np.abs(g - go)) <= 2e-3 * np.max(np.abs(go)), (g, go)


def _render(D, w, med, seed, n_paths):
    sc, dm = dict(w["scene"], medium=med), w["dims"]
    pr = dict(w["params"], seed=seed, n_paths=n_paths)
    table = D.build_da_tables(med, dm)
    hi, lo, _, _ = D.render_transient(sc, pr, "darts", table)
    n = D.paths_per_cell(sc, pr, "darts").cuda().clamp(min=1)   # cells without paths read 0
    return (hi.double() + lo.double()) / n, n, sc, pr, table


@pytest.mark.parametrize("loss,h_abs", [("l2_residual", None), ("time_weighted", None), ("time_weighted", 1e-3)])
def test_gradient_matches_finite_differences_c4(D, loss, h_abs):
    """The differentiable workload (128x128 sensor, 512 bins, 2^22 paths).
    l2_residual: gradient of the L2 loss against the target medium's image,
    with the residual 2 (I - I_target) taken from an independent render (so
    that the gradient is a linear functional of the replayed render, without
    the variance term a shared sample would add); at this sampling density
    the residual is mostly noise, so this checks agreement within noise.
    time_weighted: sum_c exp(-bin/64) I_c, a functional whose gradient is well
    resolved.  Replay gradients vs central differences (h = 3% of each
    parameter, or h = 1e-3 absolute, where the differences are noisier: a
    perturbation flips a fraction ~h of the paths' discrete choices; common
    random numbers, tables rebuilt at each perturbed medium) over 8 seeds,
    tested on the per-seed differences (replay and differences share each
    seed's paths, so their errors are correlated and only the paired
    difference has the right spread)."""
    w = W.box_hg_grad()
    n_paths = w["params"]["n_paths"]
    tmed, med = w["target_medium"], w["scene"]["medium"]
    if loss == "l2_residual":
        target, _, _, _, _ = _render(D, w, tmed, 0xEF, n_paths * 4)
        img_a, _, _, _, _ = _render(D, w, med, 0xA0, n_paths * 4)
        weight = 2 * (img_a - target)                      # dL/dI at the current medium
    else:
        nb = w["scene"]["bins"]["n_bins"]
        weight = torch.exp(-torch.arange(nb, dtype=torch.float64, device="cuda") / 64.0)[:, None, None] \
            .expand(nb, w["scene"]["sensor"]["height"], w["scene"]["sensor"]["width"]).contiguous()
    G, F = [], []
    for seed in range(8):
        img, n, sc, pr, table = _render(D, w, med, seed + 1, n_paths)
        g = D.render_transient_backward(sc, pr, "darts", table, (weight / n).float())
        torch.cuda.synchronize()
        G.append(g.cpu().numpy())
        fd = []
        for key in ["sigma_s", "sigma_a", "g"]:
            h = h_abs if h_abs else 0.03 * max(abs(med[key]), 0.1)
            ip, _, _, _, _ = _render(D, w, dict(med, **{key: med[key] + h}), seed + 1, n_paths)
            im, _, _, _, _ = _render(D, w, dict(med, **{key: med[key] - h}), seed + 1, n_paths)
            fd.append(((weight * (ip - im)).sum() / (2 * h)).item())
        F.append(fd)
    G, F = np.array(G), np.array(F)
    n = len(G)
    diff = G - F
    se = diff.std(0, ddof=1) / math.sqrt(n)
    z = diff.mean(0) / se
    print(loss, "replay", G.mean(0), "+-", G.std(0, ddof=1) / math.sqrt(n), "fd", F.mean(0), "+-",
          F.std(0, ddof=1) / math.sqrt(n), "paired difference", diff.mean(0), "+-", se, "z", z)
    assert np.max(np.abs(z)) < 4.0, (G.mean(0), F.mean(0), z)
    if loss == "time_weighted":   # resolved: each component at least 5 standard errors from zero
        assert np.all(np.abs(G.mean(0)) > 5 * G.std(0, ddof=1) / math.sqrt(n))


def test_autograd_function(D):
    w = W.box_hg_small()
    sc, pr, dm = w["scene"], w["params"], w["dims"]
    theta = torch.tensor([4.75, 0.25, 0.7], dtype=torch.float64, requires_grad=True)
    img = D.transient_image(theta, sc, pr, "darts", dm)
    target = torch.zeros_like(img)
    loss = ((img - target) ** 2).sum()
    loss.backward()
    n = D.paths_per_cell(sc, pr, "darts").cuda()
    table = D.build_da_tables(sc["medium"], dm)
    g = D.render_transient_backward(sc, pr, "darts", table, (2 * img.detach() / n).float())
    torch.cuda.synchronize()
    assert torch.allclose(theta.grad, g.cpu(), rtol=1e-6, atol=0)


@pytest.mark.parametrize("wname,mode,n", [("box_hg_small", "darts", 1 << 16), ("box_hg_small", "da_only", 1 << 12),
                                          ("box_hg_grad", "darts", 1 << 22), ("fog_slab_small", "darts", 1 << 16)])
def test_tangent_images_sum_to_the_adjoint_gradient(D, wname, mode, n):
    """Forward-mode derivative images (darts_render_transient_tangent) of the
    same paths, weighted by a grad_image and summed over the cells, equal the
    path-replay gradient of darts_render_transient_backward (itself checked
    against the FP64 oracle): to 1e-5 of the largest component, under the
    tile decomposition (many paths per cell) and id ranges (few)."""
    w = getattr(W, wname)()
    sc, pr, dm = w["scene"], dict(w["params"], n_paths=n), w["dims"]
    table = D.build_da_tables(sc["medium"], dm) if D.MODES[mode] & D.EDA_DIR else None
    t = D.render_transient_tangent(sc, pr, mode, table)
    G = torch.rand(t.shape[1:], device="cuda", dtype=torch.float32, generator=torch.Generator("cuda").manual_seed(7))
    g = D.render_transient_backward(sc, pr, mode, table, G)
    torch.cuda.synchronize()
    got = (t.double() * G.double()).sum((1, 2, 3)).cpu().numpy()
    want = g.cpu().numpy()
    print(wname, mode, got, want)
    assert np.max(np.abs(got - want)) <= 1e-5 * np.max(np.abs(want))
