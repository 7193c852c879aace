"""GPU sensor-response renders (a general W over the path-length bins,
Eq. (4); Section V-B) against the FP64 oracle on the same Philox streams.
Bars as for the time-resolved renders: per path 1e-3 relative on >= 99% of
paths; per-pixel images relative L2 <= 1% and |delta|/sigma <= 4 on >= 99.9%
of pixels; the rejected-sample counters agree with the oracle's to 0.5%."""
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


def case(D, oracle, wname="box_hg_small", n_paths=1 << 16):
    w = {"box_hg_small": W.box_hg_small, "box_hg": W.box_hg}[wname]()
    sc, pr, dm = w["scene"], dict(w["params"], n_paths=n_paths), w["dims"]
    resp = W.two_peak_response(sc["bins"])
    t = D.build_da_tables(sc["medium"], dm)
    _, cdf = oracle.build_table(sc["medium"], dm)
    return sc, pr, dm, resp, D.build_response(resp), t, cdf


def test_response_table_layout(D, oracle):
    sc, pr, dm, resp, R, t, cdf = case(D, oracle)
    tab = R.table.cpu().numpy()
    n = len(resp)
    w = np.asarray(resp, np.float64)
    run = np.cumsum(w) / w.sum()
    want = np.concatenate([[0.0], run.astype(np.float32)[:-1], [1.0]]).astype(np.float32)
    assert np.array_equal(tab[:n + 1], want)
    assert np.array_equal(tab[n + 1:], np.asarray(resp, np.float32))


@pytest.mark.parametrize("mode", ["darts", "uniform", "da_only"])
def test_response_per_path_parity(D, oracle, mode):
    sc, pr, dm, resp, R, t, cdf = case(D, oracle)
    g = D.render_paths(sc, pr, mode, t, response=R).cpu().numpy().astype(np.float64)
    o, pix = oracle.render_response_paths(sc, pr, mode, resp, cdf, dm)
    assert np.array_equal(pix, np.arange(pr["n_paths"]) % 64)
    close = np.abs(g - o) <= 1e-3 * np.abs(o) + 1e-30
    print(f"{mode}: {close.mean():.5f} of paths agree")
    assert close.mean() >= 0.99


@pytest.mark.parametrize("wname,mode", [("box_hg_small", "darts"), ("box_hg_small", "vanilla"),
                                        ("box_hg", "darts"), ("box_hg", "vanilla"), ("box_hg", "uniform")])
def test_response_image_parity(D, oracle, wname, mode):
    from test_gpu_render import compare_images
    sc, pr, dm, resp, R, t, cdf = case(D, oracle, wname, 1 << 18)
    hi, lo, m2, st = D.render_transient(sc, pr, mode, t, want_m2=True, want_stats=True, response=R)
    torch.cuda.synchronize()
    img_g = hi.double().cpu().numpy() + lo.double().cpu().numpy()
    img_o, m2_o, st_o = oracle.render_response(sc, pr, mode, resp, cdf, dm)
    n = oracle.paths_per_pixel(sc, pr)
    assert np.array_equal(n, D.paths_per_cell(sc, pr, mode, response=R).numpy())
    rel, frac = compare_images(img_g, m2.double().cpu().numpy(), img_o, m2_o, n)
    sg = D.stats_dict(st)
    print(f"{wname}/{mode}: rel L2 {rel:.2e}, within 4 sigma {frac:.5f}; samples {sg['samples']} / "
          f"{st_o['samples']}, rejected {sg['rejected']} / {st_o['rejected']}")
    assert rel <= 0.01, rel
    assert frac >= 0.999, frac
    assert abs(sg["samples"] - st_o["samples"]) <= 0.005 * st_o["samples"]
    assert abs(sg["rejected"] - st_o["rejected"]) <= 0.005 * max(st_o["rejected"], 200)
    if mode != "vanilla":
        assert sg["rejected"] == 0


@pytest.mark.parametrize("mode", ["vanilla", "darts"])
def test_response_second_moments_match_oracle(D, oracle, mode):
    """Per-pixel sums of squares under the two-peak response against the
    oracle's on the same paths: with a response every contribution of a
    path goes to its pixel, and the path's total is squared once."""
    sc, pr, dm, resp, R, t, cdf = case(D, oracle, "box_hg_small", 1 << 16)
    _, _, m2, _ = D.render_transient(sc, pr, mode, t, want_m2=True, response=R)
    torch.cuda.synchronize()
    m2_g = m2.double().cpu().numpy()
    _, m2_o, _ = oracle.render_response(sc, pr, mode, resp, cdf, dm)
    tot = abs(m2_g.sum() - m2_o.sum()) / m2_o.sum()
    rel = np.linalg.norm(m2_g - m2_o) / np.linalg.norm(m2_o)
    print(f"{mode}: m2 total {tot:.2e}, relative L2 {rel:.2e}")
    assert tot <= 2e-4 and rel <= 5e-4, (tot, rel)


def test_vanilla_response_is_weighted_transient_on_gpu(D, oracle):
    """Same paths: the vanilla response image equals the W-weighted sum of
    the vanilla time-resolved image up to the order of the additions."""
    sc, pr, dm, resp, R, t, cdf = case(D, oracle, "box_hg", 1 << 18)
    hi, lo, _, _ = D.render_transient(sc, pr, "vanilla", None, response=R)
    ht, lt, _, _ = D.render_transient(sc, pr, "vanilla", None)
    torch.cuda.synchronize()
    img = (hi.double() + lo.double()).cpu().numpy()
    want = np.tensordot(np.asarray(resp, np.float64), (ht.double() + lt.double()).cpu().numpy(), axes=(0, 0))
    assert np.abs(img - want).max() <= 1e-5 * np.abs(want).max()


def test_response_in_a_batch(D, oracle):
    """Scenes with and without a sensor response in one batched launch give
    the separate renders."""
    sc, pr, dm, resp, R, t, cdf = case(D, oracle, "box_hg_small", 1 << 15)
    items = [(sc, pr, "darts", t, R), (sc, pr, "darts", t), (sc, dict(pr, seed=9), "uniform", None, R)]
    for plan in [{"order": "tiles"}, {"order": "ids", "unit_paths": 1000}]:
        b = D.Batch(items, plan)
        hi, lo = b.empty()
        b.render(hi, lo)
        torch.cuda.synchronize()
        for (it, h, l) in zip(items, b.images(hi), b.images(lo)):
            it = tuple(it) + (None,) * (5 - len(it))
            eh, el, _, _ = D.render_transient(it[0], it[1], it[2], it[3], response=it[4])
            got = (h.double() + l.double()).cpu().numpy()
            want = (eh.double() + el.double()).cpu().numpy()
            assert got.shape == want.shape
            assert np.abs(got - want).max() <= 1e-6 * max(np.abs(want).max(), 1e-30)
