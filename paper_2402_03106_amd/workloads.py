"""Seeded synthetic workloads (scene descriptions only, no method arithmetic).

The paper's test scenes are triangle meshes that are not available; these
homogeneous media stand in for them (the box medium of ``box_hg`` has a
camera-to-emitter depth of about 3.35 transport mean free paths, inside the
3.2-4.3 range of the paper's scene table, Section VI).  Every value here is
plain data: both the GPU library's binding and the CPU oracle consume the same
dictionaries, so this module is the only thing the two sides share.
"""
from __future__ import annotations

import copy

# Strategy names understood by both sides.
MODES = ("darts", "uniform", "vanilla", "da_only", "eda_only")


def infinite_point() -> dict:
    """Infinite homogeneous medium, isotropic unit-energy pulse at the origin
    (start 0), point fluence detector at distance 1; sigma_s = 1,
    sigma_a = 0.01, isotropic phase; 64 path-length bins over [0, 10);
    2^16 paths, at most 50 bounces; 64x64x32 direction table, S_max = 10."""
    return {
        "name": "infinite_point",
        "scene": {
            "medium": {"sigma_s": 1.0, "sigma_a": 0.01, "g": 0.0},
            "geometry": {"kind": 0, "lo": (0.0, 0.0, 0.0), "hi": (0.0, 0.0, 0.0)},
            "emitters": [{"pos": (0.0, 0.0, 0.0), "start": 0.0, "power": 1.0}],
            "sensor": {"kind": 0, "origin": (1.0, 0.0, 0.0), "dir": (0.0, 0.0, 1.0),
                       "du": (0.0, 0.0, 0.0), "dv": (0.0, 0.0, 0.0), "width": 1, "height": 1},
            "bins": {"l_lo": 0.0, "l_hi": 10.0, "n_bins": 64},
        },
        "params": {"n_paths": 1 << 16, "path_offset": 0, "seed": 0xC1, "max_bounces": 50,
                   "n_ris": 8, "alpha": 0.5},
        "dims": {"n_cs": 64, "n_s": 64, "n_cos": 32, "s_max": 10.0},
    }


def box_hg() -> dict:
    """Box medium [-1,1]^3 with index-matched boundary, sigma_t = 5, albedo
    0.95 (sigma_s = 4.75, sigma_a = 0.25), Henyey-Greenstein g = 0.7; one
    pulsed point emitter at (0, 0, 1.5) with start 0; 64x64 orthographic
    radiance sensor on the plane z = +1 over [-1,1]^2 looking along -z; 256
    bins over path length [0, 40); 2^20 paths; 64x64x32 FP32 direction table
    with S_max = 40; at most 256 bounces."""
    return {
        "name": "box_hg",
        "scene": {
            "medium": {"sigma_s": 4.75, "sigma_a": 0.25, "g": 0.7},
            "geometry": {"kind": 1, "lo": (-1.0, -1.0, -1.0), "hi": (1.0, 1.0, 1.0)},
            "emitters": [{"pos": (0.0, 0.0, 1.5), "start": 0.0, "power": 1.0}],
            "sensor": {"kind": 1, "origin": (-1.0, -1.0, 1.0), "dir": (0.0, 0.0, -1.0),
                       "du": (2.0, 0.0, 0.0), "dv": (0.0, 2.0, 0.0), "width": 64, "height": 64},
            "bins": {"l_lo": 0.0, "l_hi": 40.0, "n_bins": 256},
        },
        "params": {"n_paths": 1 << 20, "path_offset": 0, "seed": 0xC2, "max_bounces": 256,
                   "n_ris": 8, "alpha": 0.5},
        "dims": {"n_cs": 64, "n_s": 64, "n_cos": 32, "s_max": 40.0},
    }


def box_hg_small() -> dict:
    """The box medium of ``box_hg`` with an 8x8 sensor and 32 bins over
    [0, 10): a size the oracle finishes in seconds, for CPU pins."""
    w = box_hg()
    w["name"] = "box_hg_small"
    w["scene"]["sensor"]["width"] = 8
    w["scene"]["sensor"]["height"] = 8
    w["scene"]["bins"] = {"l_lo": 0.0, "l_hi": 10.0, "n_bins": 32}
    w["params"]["n_paths"] = 1 << 16
    w["dims"] = {"n_cs": 32, "n_s": 32, "n_cos": 32, "s_max": 10.0}
    return w


def box_point() -> dict:
    """Box medium [-1,1]^3 (sigma_s = 2, sigma_a = 0.1, g = 0.5) lit by a
    pulse at (0, 0, 1.5) and seen by a point fluence detector at (1.5, 0, 0),
    both outside the medium so that every estimator has bounded weights; 32
    bins over [0, 16).  Used to check independent estimators against each
    other at all scattering orders."""
    return {
        "name": "box_point",
        "scene": {
            "medium": {"sigma_s": 2.0, "sigma_a": 0.1, "g": 0.5},
            "geometry": {"kind": 1, "lo": (-1.0, -1.0, -1.0), "hi": (1.0, 1.0, 1.0)},
            "emitters": [{"pos": (0.0, 0.0, 1.5), "start": 0.0, "power": 1.0}],
            "sensor": {"kind": 0, "origin": (1.5, 0.0, 0.0), "dir": (0.0, 0.0, 1.0),
                       "du": (0.0, 0.0, 0.0), "dv": (0.0, 0.0, 0.0), "width": 1, "height": 1},
            "bins": {"l_lo": 0.0, "l_hi": 16.0, "n_bins": 32},
        },
        "params": {"n_paths": 1 << 18, "path_offset": 0, "seed": 0xB0, "max_bounces": 128,
                   "n_ris": 8, "alpha": 0.5},
        "dims": {"n_cs": 32, "n_s": 32, "n_cos": 32, "s_max": 16.0},
    }


def box_floor_point() -> dict:
    """The medium of ``box_point`` as a layer z in [0, 1] over [-1, 1]^2
    whose bottom face is an opaque Lambertian floor of albedo 0.5; pulse at
    (0, 0, 1.5) and point fluence detector at (0.8, 0, 1.5), both above the
    layer, so every estimator has bounded weights; 32 bins over [0, 16)."""
    w = box_point()
    w["name"] = "box_floor_point"
    w["scene"]["geometry"] = {"kind": 2, "lo": (-1.0, -1.0, 0.0), "hi": (1.0, 1.0, 1.0), "floor_albedo": 0.5}
    w["scene"]["sensor"]["origin"] = (0.8, 0.0, 1.5)
    return w


def box_hg_grad() -> dict:
    """Differentiable rendering workload: the box geometry of ``box_hg`` at
    sigma_s = 8, sigma_a = 0.2, g = 0.5 with a 128x128 sensor and 512 bins
    over [0, 40); an L2 loss against a target rendered at sigma_s = 10,
    sigma_a = 0.1, g = 0.6; gradients from 2^22 replayed paths."""
    w = box_hg()
    w["name"] = "box_hg_grad"
    w["scene"]["medium"] = {"sigma_s": 8.0, "sigma_a": 0.2, "g": 0.5}
    w["scene"]["sensor"]["width"] = 128
    w["scene"]["sensor"]["height"] = 128
    w["scene"]["bins"] = {"l_lo": 0.0, "l_hi": 40.0, "n_bins": 512}
    w["params"]["n_paths"] = 1 << 22
    w["params"]["seed"] = 0xC4
    w["target_medium"] = {"sigma_s": 10.0, "sigma_a": 0.1, "g": 0.6}
    return w


def batched(n_media: int = 256, seed: int = 0xC3, lo_log2: int = 12, hi_log2: int = 18) -> list:
    """Batch of independent box media for the many-configuration sweep: the
    geometry, emitter and camera of ``box_hg`` with sigma_s ~ U[0.5, 20],
    albedo ~ U[0.8, 0.999] (sigma_a = sigma_s (1/albedo - 1)),
    g ~ U[-0.3, 0.9], 32x32 sensors, 128 bins over [0, 40), path budgets
    log-uniform in [2^lo_log2, 2^hi_log2] and one Philox key per medium;
    64x64x32 direction tables with S_max = 40.  Drawn from numpy's PCG64
    stream of `seed`; returns a list of workload dictionaries."""
    import numpy as np
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(n_media):
        sigma_s = float(rng.uniform(0.5, 20.0))
        albedo = float(rng.uniform(0.8, 0.999))
        g = float(rng.uniform(-0.3, 0.9))
        n = int(round(2.0 ** rng.uniform(lo_log2, hi_log2)))
        w = box_hg()
        w["name"] = f"batched_{i}"
        w["scene"]["medium"] = {"sigma_s": sigma_s, "sigma_a": sigma_s * (1.0 / albedo - 1.0), "g": g}
        w["scene"]["sensor"]["width"] = 32
        w["scene"]["sensor"]["height"] = 32
        w["scene"]["bins"] = {"l_lo": 0.0, "l_hi": 40.0, "n_bins": 128}
        w["params"]["n_paths"] = n
        w["params"]["seed"] = (seed << 32) | i
        out.append(w)
    return out


def fog_slab() -> dict:
    """Fog layer over a diffuse ground (the set-up of the paper's Fig. 1):
    a slab 10 mean free paths thick (sigma_s = 2, sigma_a = 0.02, g = 0.85,
    so thickness 10 / 2.02) over an opaque Lambertian floor of albedo 0.5 at
    z = 0, laterally 100 units wide (effectively infinite); two pulsed point
    emitters 1 unit above the fog at x = -1.5 and x = +1.5, the second starting
    3 length units later; a 256x256 orthographic sensor on the slab's top face
    over [-4, 4]^2 looking down; 1024 bins over [0, 40); 2^28 paths, at most
    256 bounces; 64x64x32 direction table, S_max = 40.  (Emitters outside the
    medium keep every estimator's variance finite.)"""
    h = 10.0 / 2.02
    return {
        "name": "fog_slab",
        "scene": {
            "medium": {"sigma_s": 2.0, "sigma_a": 0.02, "g": 0.85},
            "geometry": {"kind": 2, "lo": (-50.0, -50.0, 0.0), "hi": (50.0, 50.0, h), "floor_albedo": 0.5},
            "emitters": [{"pos": (-1.5, 0.0, h + 1.0), "start": 0.0, "power": 1.0},
                         {"pos": (1.5, 0.0, h + 1.0), "start": 3.0, "power": 1.0}],
            "sensor": {"kind": 1, "origin": (-4.0, -4.0, h), "dir": (0.0, 0.0, -1.0),
                       "du": (8.0, 0.0, 0.0), "dv": (0.0, 8.0, 0.0), "width": 256, "height": 256},
            "bins": {"l_lo": 0.0, "l_hi": 40.0, "n_bins": 1024},
        },
        "params": {"n_paths": 1 << 28, "path_offset": 0, "seed": 0xC5, "max_bounces": 256,
                   "n_ris": 8, "alpha": 0.5},
        "dims": {"n_cs": 64, "n_s": 64, "n_cos": 32, "s_max": 40.0},
    }


def fog_slab_small() -> dict:
    """``fog_slab`` at oracle scale: 16x16 pixels, 64 bins over [0, 20),
    2^16 paths, 32x32x32 table with S_max = 20."""
    w = fog_slab()
    w["name"] = "fog_slab_small"
    w["scene"]["sensor"]["width"] = w["scene"]["sensor"]["height"] = 16
    w["scene"]["bins"] = {"l_lo": 0.0, "l_hi": 20.0, "n_bins": 64}
    w["params"]["n_paths"] = 1 << 16
    w["dims"] = {"n_cs": 32, "n_s": 32, "n_cos": 32, "s_max": 20.0}
    return w


def fog_slab_fit() -> dict:
    """The inverse problem on the fog layer: the scene of ``fog_slab`` seen by
    a 16x16 sensor (0.5-unit pixels) with 128 bins over [0, 40) (512 paths
    per cell at 2^24 paths per render: the gradient of an L2 loss multiplies
    two independent per-cell estimates, so its noise falls fast with the
    paths per cell); the target is rendered at the true medium
    (sigma_s = 2, g = 0.85) and the fit starts from sigma_s = 1, g = 0.6 with
    sigma_a = 0.02 known."""
    w = fog_slab()
    w["name"] = "fog_slab_fit"
    w["scene"]["sensor"]["width"] = w["scene"]["sensor"]["height"] = 16
    w["scene"]["bins"] = {"l_lo": 0.0, "l_hi": 40.0, "n_bins": 128}
    w["params"]["n_paths"] = 1 << 24
    w["init_medium"] = {"sigma_s": 1.0, "sigma_a": 0.02, "g": 0.6}
    w["target_medium"] = dict(w["scene"]["medium"])
    return w


def two_peak_response(bins: dict, peaks=((3.0, 0.4, 1.0), (5.5, 0.4, 0.6)), cutoff: float = 1e-3) -> list:
    """A sensor response W with two Gaussian peaks over the bins' path-length
    range, sampled at the bin centres and set to zero below `cutoff` (the
    two-peak response of the paper's W study, Section V-B); each peak is
    (centre, width, height).  Values are rounded to float32 so both sides read
    identical numbers."""
    import numpy as np
    n, lo, hi = int(bins["n_bins"]), float(bins["l_lo"]), float(bins["l_hi"])
    c = lo + (np.arange(n) + 0.5) * (hi - lo) / n
    w = sum(h * np.exp(-0.5 * ((c - m) / s) ** 2) for m, s, h in peaks)
    w = np.where(w < cutoff, 0.0, w)
    return [float(x) for x in w.astype(np.float32)]


def with_(w: dict, **changes) -> dict:
    """Copy of a workload with params/scene entries replaced, e.g.
    ``with_(w, n_paths=4096, medium={"sigma_s": 2.0, ...})``."""
    w = copy.deepcopy(w)
    for k, v in changes.items():
        if k in w["params"]:
            w["params"][k] = v
        elif k in w["scene"]:
            w["scene"][k] = v
        elif k in w["dims"]:
            w["dims"][k] = v
        else:
            raise KeyError(k)
    return w
