"""Batched persistent render (darts_batch_*): many media in one launch.

Each scene of a batch runs the same estimator on the same path ids as a
separate darts_render_transient call, so the batch image must equal the
separate renders up to the order of the floating-point additions (both sides
use compensated sums: agreement to 1e-6 of the largest cell), and the
separate renders are held to the oracle by test_gpu_render.  One small batch
is also compared with the FP64 oracle directly, with the image bar."""
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


def small(ws, width=8, n_bins=32, l_hi=10.0, dims=(32, 32, 32)):
    for w in ws:
        w["scene"]["sensor"]["width"] = w["scene"]["sensor"]["height"] = width
        w["scene"]["bins"] = {"l_lo": 0.0, "l_hi": l_hi, "n_bins": n_bins}
        w["dims"] = {"n_cs": dims[0], "n_s": dims[1], "n_cos": dims[2], "s_max": l_hi}
    return ws


def items_of(D, ws, mode="darts"):
    out = []
    for w in ws:
        t = D.build_da_tables(w["scene"]["medium"], w["dims"]) if D.MODES[mode] & D.EDA_DIR else None
        out.append((w["scene"], w["params"], mode, t))
    return out


def separate(D, items):
    imgs = []
    for sc, p, mode, t in items:
        hi, lo, _, _ = D.render_transient(sc, p, mode, t)
        imgs.append(hi.double() + lo.double())
    torch.cuda.synchronize()
    return [x.cpu().numpy() for x in imgs]


def batch_images(D, b, hi, lo):
    torch.cuda.synchronize()
    return [(h.double() + l.double()).cpu().numpy() for h, l in zip(b.images(hi), b.images(lo))]


def assert_same(got, want):
    for i, (g, e) in enumerate(zip(got, want)):
        scale = max(np.abs(e).max(), 1e-30)
        err = np.abs(g - e).max() / scale
        assert err <= 1e-6, (i, err)


PLANS = [
    {"order": "tiles", "block_threads": 256, "waves_per_cu": 16, "unit_paths": 8192},
    {"order": "tiles", "block_threads": 64, "waves_per_cu": 8, "unit_paths": 64},
    {"order": "ids", "block_threads": 256, "waves_per_cu": 16, "unit_paths": 2048},
    {"order": "ids", "block_threads": 64, "waves_per_cu": 32, "unit_paths": 100},
]


@pytest.mark.parametrize("plan", PLANS, ids=[f"{p['order']}-{p['block_threads']}-{p['unit_paths']}" for p in PLANS])
def test_batch_equals_separate_renders(D, plan):
    """24 media with uneven budgets (2^10..2^16 paths, fewer and more paths
    than the 32x32x128 cells), under each work decomposition."""
    ws = W.batched(24, seed=0x5EED, lo_log2=10, hi_log2=16)
    items = items_of(D, ws)
    b = D.Batch(items, plan)
    assert b.plan == plan
    hi, lo = b.empty()
    b.render(hi, lo)
    assert_same(batch_images(D, b, hi, lo), separate(D, items))


def test_batch_ragged_ranges_and_modes(D):
    """Path ranges that start and end inside the cell map, a scene without
    paths, and the uniform and DA-only strategies in one batch."""
    ws = small(W.batched(5, seed=0xAB, lo_log2=9, hi_log2=13), width=4, n_bins=16)
    ws[0]["params"]["path_offset"] = 77
    ws[1]["params"]["path_offset"] = 3 * 256 + 5
    ws[1]["params"]["n_paths"] = 5000
    ws[2]["params"]["n_paths"] = 0
    modes = ["darts", "darts", "darts", "uniform", "da_only"]
    items = [items_of(D, [w], m)[0] for w, m in zip(ws, modes)]
    for plan in PLANS:
        b = D.Batch(items, plan)
        hi, lo = b.empty()
        b.render(hi, lo)
        got = batch_images(D, b, hi, lo)
        assert_same(got, separate(D, items))
        assert np.all(got[2] == 0)


def test_batch_repeats_and_accumulates(D):
    """The unit counter rewinds at the end of every launch: a second launch
    into the same images doubles them, and a launch into fresh images
    reproduces the first."""
    ws = W.batched(12, seed=0x77, lo_log2=10, hi_log2=14)
    b = D.Batch(items_of(D, ws), {"order": "ids", "unit_paths": 512})
    hi1, lo1 = b.empty()
    b.render(hi1, lo1)
    first = batch_images(D, b, hi1, lo1)
    b.render(hi1, lo1)
    twice = batch_images(D, b, hi1, lo1)
    hi2, lo2 = b.empty()
    b.render(hi2, lo2)
    again = batch_images(D, b, hi2, lo2)
    assert_same(again, first)
    assert_same([x / 2 for x in twice], first)


def test_batch_graph_replays(D):
    """The captured graph (clear + batch launch) replayed several times, with
    other device work and synchronisations in between, gives the eager
    result every time."""
    ws = W.batched(16, seed=0x9A, lo_log2=10, hi_log2=15)
    items = items_of(D, ws)
    b = D.Batch(items, {"order": "tiles", "unit_paths": 1024})
    hi, lo = b.empty()
    b.render(hi, lo)
    eager = batch_images(D, b, hi, lo)
    ghi, glo = b.empty()
    for r in range(4):
        ghi.fill_(123.0)      # stale contents: the graph clears them
        b.graph_launch(ghi, glo)
        assert_same(batch_images(D, b, ghi, glo), eager)
        sc, p, mode, t = items[r]
        D.render_transient(sc, p, mode, t)   # unrelated eager work between replays
        torch.cuda.synchronize()


def test_batch_autotune(D):
    """The autotuner times its candidate plans, keeps the fastest and leaves
    the batch producing the same images."""
    ws = W.batched(16, seed=0x31, lo_log2=10, hi_log2=14)
    items = items_of(D, ws)
    b = D.Batch(items)
    hi, lo = b.empty()
    plan, ms = b.autotune(hi, lo, reps=1)
    assert ms > 0 and b.plan == plan
    assert plan["order"] in ("tiles", "ids") and plan["block_threads"] in (64, 256)
    hi, lo = b.empty()
    b.render(hi, lo)
    assert_same(batch_images(D, b, hi, lo), separate(D, items))


def test_batch_compensated_global_atomics(D):
    """Id-order units add every finished path's sum to its cell with a global
    compensated atomic pair: two infinite-medium scenes with 1024 paths per
    cell from different waves; hi + lo equals the exact sum of the per-path
    values to 1e-9 of the sum of their magnitudes."""
    items, exact, scale = [], [], []
    for seed in (0xA1, 0xB2):
        w = W.infinite_point()
        sc, pr, dm = w["scene"], dict(w["params"], seed=seed), w["dims"]
        t = D.build_da_tables(sc["medium"], dm)
        vals = D.render_paths(sc, pr, "darts", t).cpu().numpy().astype(np.float64)
        idx = np.arange(pr["n_paths"]) % 64
        exact.append(np.bincount(idx, weights=vals, minlength=64))
        scale.append(np.bincount(idx, weights=np.abs(vals), minlength=64))
        items.append((sc, pr, "darts", t))
    b = D.Batch(items, {"order": "ids", "block_threads": 64, "waves_per_cu": 16, "unit_paths": 64})
    hi, lo = b.empty()
    b.render(hi, lo)
    for h, l, e, sc_ in zip(b.images(hi), b.images(lo), exact, scale):
        tot = (h.double() + l.double()).cpu().numpy().ravel()
        err = np.abs(tot - e) / np.maximum(sc_, 1e-300)
        assert err.max() <= 1e-9, err.max()


def test_batch_vs_oracle(D, oracle):
    """Four media of the batched sweep on an 8x8 sensor, 32 bins over
    [0, 10), 2^15 paths each: batch images against the FP64 oracle with the
    image bar (relative L2 <= 1%, |delta|/sigma <= 4 on 99.9% of cells)."""
    from test_gpu_render import compare_images
    ws = small(W.batched(4, seed=0xC3))
    for w in ws:
        w["params"]["n_paths"] = 1 << 15
    items = items_of(D, ws)
    b = D.Batch(items, {"order": "ids", "unit_paths": 4096})
    hi, lo = b.empty()
    b.render(hi, lo)
    got = batch_images(D, b, hi, lo)
    for w, g in zip(ws, got):
        sc, pr, dm = w["scene"], w["params"], w["dims"]
        _, cdf = oracle.build_table(sc["medium"], dm)
        img_o, m2_o, _ = oracle.render(sc, pr, "darts", cdf, dm)
        n = oracle.paths_per_cell(sc, pr, "darts")
        rel, frac = compare_images(g, m2_o, img_o, m2_o, n)
        print(f"{sc['medium']}: rel L2 {rel:.2e}, within 4 sigma {frac:.5f}")
        assert rel <= 0.01, rel
        assert frac >= 0.999, frac


def test_batch_with_floor_scenes(D):
    """Media over a Lambertian floor and plain boxes in one batch (the batch
    then runs the floor kernel for every scene) equal their separate renders."""
    ws = W.batched(6, seed=0xF1, lo_log2=10, hi_log2=14)
    fl = W.fog_slab_small()
    fl["params"]["n_paths"] = 1 << 14
    fl2 = W.box_floor_point()
    fl2["params"]["n_paths"] = 1 << 13
    items = items_of(D, ws) + items_of(D, [fl, fl2])
    for plan in PLANS[:3]:
        b = D.Batch(items, plan)
        hi, lo = b.empty()
        b.render(hi, lo)
        assert_same(batch_images(D, b, hi, lo), separate(D, items))
