"""GPU renders of media over an opaque Lambertian floor (surface events and
case II floor connections, Section V-B) against the FP64 oracle on the same
Philox streams, with the bars of test_gpu_render: per path 1e-3 relative on
>= 99% of paths; images relative L2 <= 1% and |delta|/sigma <= 4 on >= 99.9%
of cells; gradients within 2e-3 of the oracle's."""
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


def setup(D, oracle, w):
    sc, dm = w["scene"], w["dims"]
    return D.build_da_tables(sc["medium"], dm), oracle.build_table(sc["medium"], dm)[1]


@pytest.mark.parametrize("wname,mode", [("fog_slab_small", "darts"), ("fog_slab_small", "uniform"),
                                        ("fog_slab_small", "da_only"), ("box_floor_point", "darts"),
                                        ("box_floor_point", "eda_only")])
def test_floor_per_path_parity(D, oracle, wname, mode):
    w = getattr(W, wname)()
    sc, pr, dm = w["scene"], w["params"], w["dims"]
    t, cdf = setup(D, oracle, w)
    g = D.render_paths(sc, pr, mode, t).cpu().numpy().astype(np.float64)
    o, cells = oracle.render_paths(sc, pr, mode, cdf, dm)
    close = np.abs(g - o) <= 1e-3 * np.abs(o) + 1e-30
    print(f"{wname}/{mode}: {close.mean():.5f} of paths agree, nonzero {np.mean(o != 0):.3f}")
    assert close.mean() >= 0.99


@pytest.mark.parametrize("wname,mode", [("fog_slab_small", "darts"), ("fog_slab_small", "vanilla"),
                                        ("box_floor_point", "darts"), ("box_floor_point", "uniform"),
                                        ("box_floor_point", "vanilla")])
def test_floor_image_parity(D, oracle, wname, mode):
    from test_gpu_render import compare_images
    w = getattr(W, wname)()
    sc, pr, dm = w["scene"], dict(w["params"], n_paths=1 << 18), w["dims"]
    t, cdf = setup(D, oracle, w)
    hi, lo, m2, st = D.render_transient(sc, pr, mode, t, want_m2=True, want_stats=True)
    torch.cuda.synchronize()
    img_g = hi.double().cpu().numpy() + lo.double().cpu().numpy()
    img_o, m2_o, st_o = oracle.render(sc, pr, mode, cdf, dm)
    n = oracle.paths_per_cell(sc, pr, mode)
    rel, frac = compare_images(img_g, m2.double().cpu().numpy(), img_o, m2_o, n)
    sg = D.stats_dict(st)
    print(f"{wname}/{mode}: rel L2 {rel:.2e}, within 4 sigma {frac:.5f}; samples {sg['samples']}/{st_o['samples']}"
          f" rejected {sg['rejected']}/{st_o['rejected']}")
    assert rel <= 0.01, rel
    assert frac >= 0.999, frac
    assert abs(sg["samples"] - st_o["samples"]) <= 0.005 * st_o["samples"]


@pytest.mark.parametrize("mode", ["darts", "da_only"])
def test_floor_gradient_matches_oracle(D, oracle, mode):
    w = W.box_floor_point()
    sc, pr, dm = w["scene"], dict(w["params"], n_paths=1 << 18), w["dims"]
    t, cdf = setup(D, oracle, w)
    gimg = np.random.default_rng(3).random(oracle.image_shape(sc)).astype(np.float32)
    g = D.render_transient_backward(sc, pr, mode, t, torch.from_numpy(gimg).cuda())
    torch.cuda.synchronize()
    g = g.cpu().numpy()
    go = oracle.render_gradient(sc, pr, mode, gimg.astype(np.float64), cdf, dm)
    print(mode, g, go)
    assert np.max(np.abs(g - go)) <= 2e-3 * np.max(np.abs(go)), (g, go)


def test_fog_slab_full_size_sampled_cells(D, oracle):
    """The fog layer at its full size (256x256 pixels x 1024 bins, 2^28
    paths, 4 per cell): cells of both emitters' arrival times recomputed by
    the oracle path by path."""
    w = W.fog_slab()
    sc, pr, dm = w["scene"], w["params"], w["dims"]
    t, cdf = setup(D, oracle, w)
    hi, lo, _, _ = D.render_transient(sc, pr, "darts", t)
    torch.cuda.synchronize()
    npix = 256 * 256
    nc = npix * 1024
    rng = np.random.default_rng(11)
    cells = []
    for b in rng.choice(np.arange(150, 500), 32, replace=False):
        px, py = rng.integers(96, 160, 2)
        cells.append(int(b) * npix + int(py) * 256 + int(px))
    img = (hi.double() + lo.double()).cpu().numpy().ravel()
    del hi, lo
    ids = np.concatenate([np.arange(4, dtype=np.uint64) * np.uint64(nc) + np.uint64(c) for c in cells])
    vals = oracle.render_path_list(sc, pr, "darts", ids, cdf, dm).reshape(len(cells), 4)
    agree = 0
    for k, c in enumerate(cells):
        s = vals[k].sum()
        agree += abs(img[c] - s) <= 1e-3 * abs(s) + 1e-12
    print("cells agreeing path by path:", agree, "of", len(cells))
    assert agree >= len(cells) - 2
