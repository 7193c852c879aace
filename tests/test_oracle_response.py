"""CPU pins of the sensor-response estimators (Eq. (4) with a general W,
the path-length control of Section V-B) in the FP64 oracle.

- Vanilla weights each shadow connection by W of its length, so on the same
  paths its response image is exactly the W-weighted sum of its time-resolved
  image (an identity, checked to rounding).
- The DARTS family draws each path's target segment with probability
  proportional to W and divides by it; its response image must agree with the
  independent vanilla estimate, and with W concentrated on one segment with
  the time-gated estimate of that segment.
- Vanilla produces samples whose length the sensor ignores (rejections); the
  DARTS family produces none.
- A planted mistake (the W / probability weight dropped) fails the
  agreement test."""
import numpy as np
import pytest

from paper_2402_03106_amd import workloads as W


def setup(oracle, n_paths):
    w = W.box_hg_small()
    sc, pr, dm = w["scene"], dict(w["params"], n_paths=n_paths), w["dims"]
    _, cdf = oracle.build_table(sc["medium"], dm)
    return sc, pr, dm, cdf


def z_per_pixel(a, b):
    """z-scores of the difference of two independent per-pixel estimates
    given as (estimate, variance of the estimate)."""
    return (a[0] - b[0]) / np.sqrt(np.maximum(a[1] + b[1], 1e-300))


def estimate(img, m2, n):
    mean = img / n
    var = np.maximum(m2 / n - mean ** 2, 0) / n
    return mean, var


def test_vanilla_response_is_weighted_transient(oracle):
    sc, pr, dm, cdf = setup(oracle, 1 << 16)
    resp = W.two_peak_response(sc["bins"])
    img_r, _, st = oracle.render_response(sc, pr, "vanilla", resp, cdf, dm)
    img_t, _, _ = oracle.render(sc, pr, "vanilla", cdf, dm)
    want = np.tensordot(np.asarray(resp), img_t, axes=(0, 0))
    assert np.allclose(img_r, want, rtol=1e-12, atol=0), np.abs(img_r - want).max()
    assert st["samples"] > 0


def test_response_estimators_agree(oracle):
    """DARTS, uniform-S and vanilla response images of the two-peak W: total
    within 4 combined standard errors and per pixel |z| <= 5.5.  At the
    paper's alpha = 0.5 the DARTS estimator is heavy-tailed on this g = 0.7
    medium, so the sample variance under-reads its spread: over five seeds
    the largest of the 64 per-pixel |z| of DARTS against vanilla ranged over
    3.8-5.1 (and the mean per-pixel z over -0.5 to -0.9, the skew of such an
    estimator), while the totals stayed within 3 standard errors."""
    sc, pr, dm, cdf = setup(oracle, 1 << 20)
    resp = W.two_peak_response(sc["bins"])
    n = oracle.paths_per_pixel(sc, pr)
    est = {}
    for mode in ["darts", "uniform", "vanilla"]:
        img, m2, _ = oracle.render_response(sc, pr, mode, resp, cdf, dm)
        est[mode] = estimate(img, m2, n)
    for mode in ["darts", "uniform"]:
        z = z_per_pixel(est[mode], est["vanilla"])
        tot = (est[mode][0].sum() - est["vanilla"][0].sum()) / np.sqrt(est[mode][1].sum() + est["vanilla"][1].sum())
        print(mode, "total z", tot, "max |z|", np.abs(z).max())
        assert abs(tot) < 4.0, (mode, tot)
        assert np.abs(z).max() < 5.5, (mode, np.abs(z).max())


def test_response_planted_mistake_is_caught(oracle):
    sc, pr, dm, cdf = setup(oracle, 1 << 18)
    resp = W.two_peak_response(sc["bins"])
    n = oracle.paths_per_pixel(sc, pr)
    good = estimate(*oracle.render_response(sc, pr, "vanilla", resp, cdf, dm)[:2], n)
    bad = estimate(*oracle.render_response(sc, pr, "darts", resp, cdf, dm, mutation="response_unweighted")[:2], n)
    tot = (bad[0].sum() - good[0].sum()) / np.sqrt(bad[1].sum() + good[1].sum())
    assert abs(tot) > 6.0, tot


def test_one_segment_response_is_the_gated_image(oracle):
    """W = 1 on segment b only: every DARTS path targets b, so the response
    image estimates the time-gated image of bin b."""
    sc, pr, dm, cdf = setup(oracle, 1 << 19)
    b = 12
    resp = [0.0] * sc["bins"]["n_bins"]
    resp[b] = 1.0
    n = oracle.paths_per_pixel(sc, pr)
    r = estimate(*oracle.render_response(sc, pr, "darts", resp, cdf, dm)[:2], n)
    prt = dict(pr, seed=pr["seed"] + 1, n_paths=1 << 22)   # 2048 paths per cell of bin b
    img, m2, _ = oracle.render(sc, prt, "darts", cdf, dm)
    nc = np.maximum(oracle.paths_per_cell(sc, prt, "darts"), 1)
    g = estimate(img[b], m2[b], nc[b])
    z = z_per_pixel(r, g)
    print("max |z|", np.abs(z).max())
    assert np.abs(z).max() < 4.5


def test_rejected_samples(oracle):
    """Vanilla's connections whose length has W = 0 are rejected samples;
    DARTS and uniform-S only sample lengths inside the chosen segment."""
    sc, pr, dm, cdf = setup(oracle, 1 << 16)
    resp = W.two_peak_response(sc["bins"])
    _, _, sv = oracle.render_response(sc, pr, "vanilla", resp, cdf, dm)
    assert 0.05 < sv["rejected"] / sv["samples"] < 0.95
    for mode in ["darts", "uniform"]:
        _, _, sd = oracle.render_response(sc, pr, mode, resp, cdf, dm)
        assert sd["samples"] > 0 and sd["rejected"] == 0


def test_response_segment_frequencies(oracle):
    """The DARTS family's segment choice follows W: with W nonzero on two
    segments only, each path's value is its gated estimate for the segment it
    chose (the same random numbers otherwise) times W_k / P(k) = sum W, so
    matching it against the two one-segment renders tells which segment each
    path chose; the fraction choosing segment 5 must be P(5) = W_5 / sum W."""
    sc, pr, dm, cdf = setup(oracle, 1 << 16)
    resp = [0.0] * sc["bins"]["n_bins"]
    resp[5], resp[20] = 1.0, 3.0
    vals, pix = oracle.render_response_paths(sc, pr, "darts", resp, cdf, dm)
    assert np.array_equal(pix, np.arange(pr["n_paths"]) % 64)
    # the same paths with W = 1 on one segment give the unscaled gated values
    v5, _ = oracle.render_response_paths(sc, pr, "darts", [1.0 if k == 5 else 0.0 for k in range(32)], cdf, dm)
    v20, _ = oracle.render_response_paths(sc, pr, "darts", [1.0 if k == 20 else 0.0 for k in range(32)], cdf, dm)
    # sum W = 4: a path that chose segment k carries 4 * (its one-segment value)
    # identifiable (and independent of the segment draw): both values nonzero and distinct
    ident = (v5 != 0) & (v20 != 0) & ~np.isclose(v5, v20, rtol=1e-9, atol=0)
    took5 = ident & np.isclose(vals, 4.0 * v5, rtol=1e-12, atol=0)
    took20 = ident & np.isclose(vals, 4.0 * v20, rtol=1e-12, atol=0)
    assert not np.any(took5 & took20)
    decided = took5 | took20
    assert decided.sum() == ident.sum()
    assert decided.sum() > 1000
    frac5 = took5.sum() / decided.sum()
    print("fraction choosing segment 5:", frac5)
    assert abs(frac5 - 0.25) < 0.05
