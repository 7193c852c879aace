"""CPU pins of the opaque Lambertian floor (Section V-B, case II: surface
events in the walk and surface points as connection vertices) in the FP64
oracle.

- Single bounce off the floor through a nearly transparent layer: every
  estimator's cell value is the pixel average of albedo/pi * cos * I / r^2
  over the floor points whose path length falls in the bin, computed here by
  quadrature over the pixel.
- All orders, bounded weights: DARTS, uniform-S and both ablation arms
  against vanilla path tracing (which reaches the floor through its own
  shadow connections).
- A planted mistake (the floor cosine dropped) fails the single-bounce pin."""
import numpy as np
import pytest

from paper_2402_03106_amd import workloads as W


def thin_layer():
    """Layer z in [0, 1] over [-2, 2]^2 with a floor of albedo 0.7, a nearly
    transparent medium, emitter (0.3, -0.2, 1.6) above it, 4x4 orthographic
    pixels over [-1, 1]^2 at z = 1 looking down, 16 bins over [2, 4)."""
    w = W.box_hg_small()
    sc = w["scene"]
    sc["medium"] = {"sigma_s": 1e-7, "sigma_a": 0.0, "g": 0.0}
    sc["geometry"] = {"kind": 2, "lo": (-2.0, -2.0, 0.0), "hi": (2.0, 2.0, 1.0), "floor_albedo": 0.7}
    sc["emitters"] = [{"pos": (0.3, -0.2, 1.6), "start": 0.0, "power": 2.0}]
    sc["sensor"].update({"origin": (-1.0, -1.0, 1.0), "du": (2.0, 0.0, 0.0), "dv": (0.0, 2.0, 0.0),
                         "width": 4, "height": 4})
    sc["bins"] = {"l_lo": 2.0, "l_hi": 4.0, "n_bins": 16}
    w["params"]["max_bounces"] = 4
    w["dims"] = {"n_cs": 8, "n_s": 8, "n_cos": 8, "s_max": 4.0}
    return w


def single_bounce_quadrature(sc, q=256):
    """Cell means: average over a q x q grid of each pixel of the floor term
    (albedo/pi) cos I / r^2, binned by the length 1 + r (camera at z = 1)."""
    s, b, e = sc["sensor"], sc["bins"], sc["emitters"][0]
    rho = sc["geometry"]["floor_albedo"]
    H, Wd, nb = s["height"], s["width"], b["n_bins"]
    out = np.zeros((nb, H, Wd))
    f = (np.arange(q) + 0.5) / q
    for py in range(H):
        for px in range(Wd):
            X = s["origin"][0] + (px + f[None, :]) / Wd * s["du"][0]
            Y = s["origin"][1] + (py + f[:, None]) / H * s["dv"][1]
            dx, dy, dz = e["pos"][0] - X, e["pos"][1] - Y, e["pos"][2]
            r = np.sqrt(dx * dx + dy * dy + dz * dz)
            val = rho / np.pi * (dz / r) * (e["power"] / (4 * np.pi)) / r ** 2
            L = 1.0 + r
            k = np.floor((L - b["l_lo"]) / (b["l_hi"] - b["l_lo"]) * nb).astype(int)
            for kk in range(nb):
                out[kk, py, px] = np.where(k == kk, val, 0.0).mean()
    return out


@pytest.mark.parametrize("mode", ["darts", "uniform", "vanilla"])
def test_single_floor_bounce_closed_form(oracle, mode):
    w = thin_layer()
    sc, dm = w["scene"], w["dims"]
    p = dict(w["params"], n_paths=1 << 20)
    _, cdf = oracle.build_table(sc["medium"], dm)
    img, m2, _ = oracle.render(sc, p, mode, cdf, dm)
    n = np.maximum(oracle.paths_per_cell(sc, p, mode), 1)
    est = img / n
    se = np.sqrt(np.maximum(m2 / n - est ** 2, 0) / n)
    want = single_bounce_quadrature(sc)
    z = (est - want) / np.maximum(se, 1e-3 * want.max())
    print(mode, "max |z|", np.abs(z).max(), "total", est.sum(), want.sum())
    assert np.abs(z).max() < 4.5
    assert abs(est.sum() / want.sum() - 1) < 0.01


def test_floor_planted_mistake_is_caught(oracle):
    w = thin_layer()
    sc, dm = w["scene"], w["dims"]
    p = dict(w["params"], n_paths=1 << 18)
    _, cdf = oracle.build_table(sc["medium"], dm)
    img, _, _ = oracle.render(sc, p, "darts", cdf, dm, mutation="floor_no_cosine")
    n = np.maximum(oracle.paths_per_cell(sc, p, "darts"), 1)
    assert abs((img / n).sum() / single_bounce_quadrature(sc).sum() - 1) > 0.05


def test_floor_estimators_agree(oracle):
    """Medium over the floor, all scattering orders, bounded weights: per-bin
    |z| <= 4.5 against vanilla for every DARTS-family arm."""
    w = W.box_floor_point()
    sc, dm = w["scene"], w["dims"]
    p = dict(w["params"], n_paths=1 << 22)
    _, cdf = oracle.build_table(sc["medium"], dm)
    est = {}
    for mode in ["vanilla", "darts", "uniform", "da_only", "eda_only"]:
        img, m2, _ = oracle.render(sc, p, mode, cdf, dm)
        n = np.maximum(oracle.paths_per_cell(sc, p, mode), 1)
        e = (img / n).ravel()
        est[mode] = (e, (np.maximum(m2 / n - (img / n) ** 2, 0) / n).ravel())
    for mode in ["darts", "uniform", "da_only", "eda_only"]:
        v = est[mode][1] + est["vanilla"][1]
        ok = v > 0
        z = (est[mode][0] - est["vanilla"][0])[ok] / np.sqrt(v[ok])
        print(mode, "max |z|", np.abs(z).max())
        assert np.abs(z).max() < 4.5, mode
        assert np.all(est[mode][0][~ok] == est["vanilla"][0][~ok])


def test_zero_albedo_floor_is_an_open_face(oracle):
    """A black floor (albedo 0) absorbs what reaches it, as the open face of
    kind 1 lets it leave: per-path values are identical."""
    w = W.box_floor_point()
    sc, dm = w["scene"], w["dims"]
    p = dict(w["params"], n_paths=1 << 14)
    _, cdf = oracle.build_table(sc["medium"], dm)
    sc0 = dict(sc, geometry=dict(sc["geometry"], floor_albedo=0.0))
    sc1 = dict(sc, geometry=dict(sc["geometry"], kind=1))
    v0, _ = oracle.render_paths(sc0, p, "darts", cdf, dm)
    v1, _ = oracle.render_paths(sc1, p, "darts", cdf, dm)
    assert np.array_equal(v0, v1)
