"""Benchmark: transient paths/s of the DARTS hot path on one MI355X.

A step is one pass of the whole hot path over one frame of synthetic input:
build the elliptical-DA direction table for the medium, then render one frame
of the box workload (64x64 sensor x 256 time bins = 2^20 cells) with 2^28
paths (256 per cell).  `value` is DARTS paths/s with everything resident in
HBM.  The line also carries
  - `roofline`: the render kernel's algorithmic FP32 FLOP/s (FLOPs per vertex
    step times the steps of one launch, over the kernel's mean duration timed
    with HIP events on its own stream) against the MI355X vector peak;
  - `cpu_baseline`: the FP64 oracle on the host cores, on a bounded sample
    of the same workload;
  - `uniform`: the temporally uniform baseline (uniform length-sum
    connection, exponential distance, phase sampling) on the same frame;
  - `time_to_mse`: time to reach MSE <= 1e-4 (cells normalised by the 0.95
    quantile, as in the paper's parameter study) for DARTS at three values
    of the EDA preference alpha, DA-only, uniform and vanilla, from per-cell
    variances (all estimators are unbiased, so MSE is their variance, which
    falls as 1/N);
  - `time_gated`: the same for single time-gated frames of the box workload
    at three gates, each normalised by its own 0.95 quantile.

usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "transient paths/s and time-to-MSE 1e-4, DARTS vs uniform sampling, 1×MI355X"
FIT_SETTINGS = {"steps": 200, "mode": "da_only", "lr": 0.05, "lr_final": 0.01, "n_paths": 1 << 26}
PEAK_FP32_TFLOPS = 157.3      # MI355X vector FP32 (256 CU x 2.4 GHz x 256 FLOP/clk)
HBM_PEAK_GBS = 8000.0

# Algorithmic work of the roofline: the per-unit figures of the hot path's
# scope table, about 375 floating-point operations per vertex step (a
# vertex that passed the early-exit test: connection test and connection,
# medium-event draw, 8 RIS candidates with the FP64 normalisation, move,
# direction sample) and about 60 per path (camera ray, medium entry, target
# interval).
FLOPS_PER_VERTEX_STEP = 375
FLOPS_PER_PATH = 60

# Cross-check: floating-point operations per part of a vertex step, counted
# op by op from the algorithm as the kernel evaluates it.  Counted: FP32 and
# FP64 add, subtract, multiply (1 each), fused multiply-add (2), and each
# exp, log, sqrt, rsqrt, reciprocal, sin, cos (1).  Not counted: compares,
# min/max, selects, conversions, integer and RNG work.
FLOPS = {
    "setup": 47,            # pixel jitter, camera ray, emitter and target interval, slab entry, C, early exit
    "connect_test": 23,     # residual range above C, exit length d_m + |x + w d_m - x_e| (every step)
    "connect_texp": 103,    # focal term, truncated-exponential S, t(S), p(t), control vertex, exit toward
                            # the emitter, phase function, transmittance
    "connect_uniform": 86,  # the same with S uniform
    "flight_test": 4,       # medium-event probability
    "ris": 222,             # 8 candidates (distance without cancellation, residual, validity, DA
                            # fluence exponent), FP64 weights and pick, weight factor, b = w.(x_e - x)
    "exp_distance": 8,      # plain exponential distance
    "move": 18,             # advance, throughput, distance to the emitter, early-exit test
    "direction": 69,        # uniforms, axis to the emitter, frame, phase pdf, MIS weight, boundary distance
    "direction_eda": 13,    # gamma, table cell, EDA pdf, mixture pdf (EDA enabled)
    "eda_branch": 7,        # cos inside the drawn bin and its sine (the bin search is compares only)
    "hg_branch": 20,        # HG inverse CDF without cancellation
    "hg_bin": 8,            # cos-bin of a phase-sampled direction (EDA enabled)
}


def algorithmic_flops(s: dict, paths: int) -> tuple:
    """FLOPs of one DARTS launch from its statistics counters: the per-unit
    figures times vertex steps and paths."""
    steps = s["vertices"] - s["early_exit"]             # vertices that passed the early-exit test
    return float(FLOPS_PER_VERTEX_STEP * steps + FLOPS_PER_PATH * paths), steps


def counted_flops(s: dict, mode: str) -> float:
    """FLOPs of one launch from its statistics counters and the op-by-op part
    counts (the cross-check of the per-unit figures)."""
    steps = s["vertices"] - s["early_exit"]
    flights = steps - s["truncated"]
    draws = flights - s["medium_exit"]
    moves = draws - s["ris_all_invalid"]
    dirs = moves - (s["early_exit"] - s["setup_exit"])
    eda = s["eda_branch"]
    f = s["paths"] * FLOPS["setup"]
    f += steps * FLOPS["connect_test"] + flights * FLOPS["flight_test"] + moves * FLOPS["move"]
    f += dirs * FLOPS["direction"]
    if mode == "darts":
        f += s["connections"] * FLOPS["connect_texp"] + draws * FLOPS["ris"]
        f += dirs * FLOPS["direction_eda"] + eda * FLOPS["eda_branch"] + (dirs - eda) * (FLOPS["hg_branch"] + FLOPS["hg_bin"])
    else:
        f += s["connections"] * FLOPS["connect_uniform"] + draws * FLOPS["exp_distance"] + dirs * FLOPS["hg_branch"]
    return float(f)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--paths-log2", type=int, default=28)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-mse", action="store_true", help="skip the time-to-MSE measurement")
    ap.add_argument("--no-uniform", action="store_true", help="skip the uniform-baseline throughput")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched many-media launch")
    ap.add_argument("--no-response", action="store_true", help="skip the two-peak sensor-response study")
    ap.add_argument("--no-fog", action="store_true", help="skip the fog-layer render and the Adam fit")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint timing on the differentiable box")
    ap.add_argument("--batched-reps", type=int, default=5, help="timed graph launches of the batch")
    ap.add_argument("--batched-scale", type=int, default=1,
                    help="multiply every medium's path budget of the batched sweep (the default line uses 1)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-converge", action="store_true",
                    help="skip the measured (progressive-launch) time to MSE 1e-4 on three time gates")
    ap.add_argument("--converge-cap-seconds", type=float, default=4.0,
                    help="most seconds of launches per arm and gate in the measured time to MSE")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="after timing, copy this many bytes device-to-device once (a kernel of known "
                         "traffic that calibrates the HBM byte counters of a profiler run)")
    return ap.parse_args()


def kernel_source_hash() -> str:
    """First 16 hex digits of the sha256 of the kernel sources with their
    comments and whitespace removed (an edited comment leaves the kernel, and
    its counter record, as they were), and of the compiler flags they are
    built with."""
    import hashlib
    import re
    from paper_2402_03106_amd import build as B
    h = hashlib.sha256()
    h.update(" ".join(B.HIPCC_FLAGS).encode())
    for f in ["paper_2402_03106_amd/csrc/darts.hip", "paper_2402_03106_amd/csrc/darts_device.hpp"]:
        with open(os.path.join(ROOT, f), encoding="utf-8") as fh:
            text = fh.read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)   # block comments
        text = re.sub(r"//[^\n]*", " ", text)                 # line comments
        h.update(re.sub(r"\s+", "", text).encode())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per render launch from the committed counter profile, if it
    was taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", "render_kernel_box_hg_traffic.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch")


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this implementation runs on one GPU; --gpus must be 1 "
                          "(multi-GPU sharding is not implemented)"}))
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2402_03106_amd import darts
    from paper_2402_03106_amd import workloads as W

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    darts.lib()
    n = 1 << a.paths_log2
    w = W.with_(W.box_hg(), n_paths=n)
    sc, pr, dm = w["scene"], w["params"], w["dims"]
    shape = darts.image_shape(sc)
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    hi = torch.zeros(shape, dtype=torch.float32, device=dev)
    lo = torch.zeros(shape, dtype=torch.float32, device=dev)
    cdf = torch.empty((dm["n_cs"], dm["n_s"], dm["n_cos"] + 1), dtype=torch.float32, device=dev)

    def step(mode, ev=None, params=pr):
        table = darts.build_da_tables(sc["medium"], dm, out=cdf)
        if ev is not None:
            ev[0].record(stream)
        darts.render_transient(sc, params, mode, table, hi, lo)
        if ev is not None:
            ev[1].record(stream)

    def timed(mode, steps, warmup, params=pr):
        # every arm starts from a cleared image (outside the timed region), so
        # its frames accumulate into the same state whatever ran before
        hi.zero_()
        lo.zero_()
        for _ in range(warmup):
            step(mode, None, params)
        torch.cuda.synchronize()
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(steps)]
        t0 = time.perf_counter()
        for i in range(steps):
            step(mode, evs[i], params)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        kern_ms = [e0.elapsed_time(e1) for e0, e1 in evs]
        return wall, kern_ms

    def count_steps(mode):
        table = darts.build_da_tables(sc["medium"], dm, out=cdf)
        h2, l2 = torch.zeros_like(hi), torch.zeros_like(lo)
        _, _, _, st = darts.render_transient(sc, pr, mode, table, h2, l2, want_stats=True)
        torch.cuda.synchronize()
        s = darts.stats_dict(st)
        flops, steps = algorithmic_flops(s, n)
        return s, steps, flops, counted_flops(s, mode)

    wall, kern_ms = timed("darts", a.steps, a.warmup)
    stats, n_steps, flops, flops_counted = count_steps("darts")
    mean_kern_s = sum(kern_ms) / len(kern_ms) / 1e3
    achieved = flops / mean_kern_s / 1e12
    value = a.steps * n / wall
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "paths/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": wall / a.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "box_hg: box [-1,1]^3, sigma_t=5, albedo 0.95, HG g=0.7, emitter (0,0,1.5); "
                        "64x64 orthographic sensor x 256 bins over [0,40); 64x64x32 FP32 direction table",
            "paths_per_step": n, "paths_per_cell": n >> 20, "mode": "darts (RIS 8 + EDA/MIS + texp ellipse)",
            "alpha": pr["alpha"],
            "step": "build_da_tables + render_transient",
        },
        "render_kernel_ms": mean_kern_s * 1e3,
        "vertex_steps_per_launch": n_steps,
        "mean_steps_per_path": n_steps / n,
        "roofline": {
            "bound": "alu", "achieved": achieved, "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32_TFLOPS, "traffic": measured_traffic(),
            "flops_per_launch": flops, "vertex_steps": n_steps, "paths": n,
            "per_unit": {"vertex_step": FLOPS_PER_VERTEX_STEP, "path": FLOPS_PER_PATH},
            "op_counted_flops_per_launch": flops_counted,
            "op_counted_achieved": flops_counted / mean_kern_s / 1e12,
        },
        "stats": stats,
    }
    print(f"[bench] darts {value:.4g} paths/s, kernel {mean_kern_s*1e3:.2f} ms, "
          f"{achieved:.2f} TFLOP/s algorithmic", file=sys.stderr, flush=True)

    if not a.no_uniform:
        wall_u, kern_u = timed("uniform", max(2, a.steps // 2), 1)
        st_u, n_steps_u, _, flops_u = count_steps("uniform")
        ku = sum(kern_u) / len(kern_u) / 1e3
        out["uniform"] = {"paths_per_s": max(2, a.steps // 2) * n / wall_u, "render_kernel_ms": ku * 1e3,
                          "mean_steps_per_path": n_steps_u / n, "op_counted_tflops": flops_u / ku / 1e12}
        print(f"[bench] uniform {out['uniform']['paths_per_s']:.4g} paths/s", file=sys.stderr, flush=True)

    if not a.no_mse:
        thr = {"darts": value, "uniform": out.get("uniform", {}).get("paths_per_s")}
        for arm, mode, alpha in MSE_ARMS:
            if not thr.get(arm):
                wall_x, _ = timed(mode, 2, 1, dict(pr, alpha=alpha))
                thr[arm] = 2 * n / wall_x
        out["time_to_mse"] = {
            "box_hg": time_to_mse(darts, torch, np, w, thr, 1 << 28, k=64),
            "infinite_point": time_to_mse(darts, torch, np, W.infinite_point(), None, 1 << 24),
        }
        out["time_gated"] = time_gated(darts, torch, np, W)
        print(f"[bench] time to MSE {out['time_to_mse']}", file=sys.stderr, flush=True)
        print(f"[bench] time-gated {out['time_gated']}", file=sys.stderr, flush=True)
    if not a.no_response:
        out["response"] = response_bench(darts, torch, np, W, w)
        print(f"[bench] response {out['response']}", file=sys.stderr, flush=True)
    if not a.no_fog:
        out["fog_slab"] = fog_bench(darts, torch, W)
        print(f"[bench] fog_slab {out['fog_slab']}", file=sys.stderr, flush=True)
    if not a.no_adjoint:
        out["adjoint"] = adjoint_bench(darts, torch, W)
        print(f"[bench] adjoint {out['adjoint']}", file=sys.stderr, flush=True)
    if not a.no_batched:
        out["batched"] = batched_bench(darts, torch, W, a.batched_reps, a.batched_scale)
        print(f"[bench] batched {out['batched']}", file=sys.stderr, flush=True)
    if not a.no_converge:
        out["measured_time_to_mse"] = measured_convergence(darts, torch, np, W, cap_seconds=a.converge_cap_seconds)
        print(f"[bench] measured time to MSE {out['measured_time_to_mse']}", file=sys.stderr, flush=True)
    if a.copy_bytes > 0:
        src = torch.empty(a.copy_bytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = src.numel() * 4

    if not a.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w, a.cpu_seconds)
        print(f"[bench] cpu {out['cpu_baseline']}", file=sys.stderr, flush=True)

    print(json.dumps(out), flush=True)


# Arms of the time-to-MSE study: (name, mode, alpha).  alpha sets the EDA
# probability gamma = kappa / (kappa + alpha) of Eq. (19); 0.5 is the paper's
# usual value, the larger ones bound the one-sample MIS weight
# phase / mixture <= 1 / (1 - gamma) <= 1 + 1/alpha more tightly.
MSE_ARMS = [("darts", "darts", 0.5), ("darts_alpha2", "darts", 2.0), ("darts_alpha4", "darts", 4.0),
            ("da_only", "da_only", 0.5), ("uniform", "uniform", 0.5), ("vanilla", "vanilla", 0.5)]


def time_to_mse(darts, torch, np, w, thr, n0, target=1e-4, k=16):
    """MSE(N) = mean over cells of Var(cell estimate) / q95^2 (q95: 0.95
    quantile of the uniform-sampling image, the paper's normalisation before
    MSE).  All arms are unbiased, so MSE is their variance, which scales as
    1/N.  It is estimated from k independent batches of n0/k paths (seed 0xEF,
    ids disjoint from the timed frames): the per-cell sample variance of the
    batch images times n0/k is the variance of one path's worth of estimate.
    `max_cell_share` (the largest cell's share of the summed variance) flags
    a heavy-tailed arm, whose variance estimate is dominated by a few paths.
    For the arms where a path feeds one cell, the per-path second moments of
    one n0-path render give a second estimate (`mse_times_paths_m2`); vanilla
    feeds one path into many bins, so only the batch estimate applies.  Wall
    time to the target = N* / measured paths/s + one table build, for the
    workload's throughput `thr` (None: the MSE-per-path products only).  The
    times are extrapolated from the variance, not measured to convergence."""
    sc, pr, dm = w["scene"], w["params"], w["dims"]
    nb = n0 // k
    table = darts.build_da_tables(sc["medium"], dm)
    var, m2v, means = {}, {}, {}
    for arm, mode, alpha in MSE_ARMS:
        s1 = s2 = None
        for i in range(k):
            pb = dict(pr, n_paths=nb, path_offset=(1 << 40) + i * nb, seed=0xEF, alpha=alpha)
            hi, lo, _, _ = darts.render_transient(sc, pb, mode, table)
            n = darts.paths_per_cell(sc, pb, mode).numpy()
            x = (hi.double() + lo.double()).cpu().numpy() / np.maximum(n, 1)
            s1 = x if s1 is None else s1 + x
            s2 = x * x if s2 is None else s2 + x * x
        means[arm] = s1 / k
        # variance of one batch image x paths per batch
        var[arm] = np.maximum(s2 - k * means[arm] ** 2, 0) / (k - 1) * nb
        if mode != "vanilla":
            p0 = dict(pr, n_paths=n0, path_offset=1 << 40, seed=0xEF, alpha=alpha)
            hi, lo, m2, _ = darts.render_transient(sc, p0, mode, table, want_m2=True)
            n = darts.paths_per_cell(sc, p0, mode).numpy()
            mean = (hi.double() + lo.double()).cpu().numpy() / np.maximum(n, 1)
            pv = np.maximum(m2.double().cpu().numpy() / np.maximum(n, 1) - mean ** 2, 0)
            m2v[arm] = pv / np.maximum(n / n0, 1e-300)  # per-path variance / (paths per cell per path)
    torch.cuda.synchronize()
    q95 = float(np.quantile(means["uniform"], 0.95))
    t0 = time.perf_counter()
    darts.build_da_tables(sc["medium"], dm)
    torch.cuda.synchronize()
    t_table = time.perf_counter() - t0
    rep = {"target": target, "q95": q95, "paths_for_variance": n0, "batches": k,
           "note": "extrapolated from measured variance and throughput; vanilla reuses each path for "
                   "every bin of its pixel (temporal reuse), the other arms dedicate each path to one bin"}
    for arm in var:
        mse_times_n = float(np.mean(var[arm])) / q95 ** 2   # MSE x total paths
        r = {"alpha": dict((a, al) for a, _, al in MSE_ARMS)[arm], "mse_times_paths": mse_times_n,
             "paths_needed": mse_times_n / target,
             "max_cell_share": float(var[arm].max() / max(float(var[arm].sum()), 1e-300))}
        if arm in m2v:
            r["mse_times_paths_m2"] = float(np.mean(m2v[arm])) / q95 ** 2
        if thr and thr.get(arm):
            r["paths_per_s"] = thr[arm]
            r["seconds"] = r["paths_needed"] / thr[arm] + t_table
        rep[arm] = r
    for arm in var:
        if arm == "uniform":
            continue
        if "seconds" in rep[arm] and "seconds" in rep["uniform"]:
            rep[f"uniform_over_{arm}_time"] = rep["uniform"]["seconds"] / rep[arm]["seconds"]
        rep[f"uniform_over_{arm}_mse_per_path"] = rep["uniform"]["mse_times_paths"] / rep[arm]["mse_times_paths"]
    return rep


GATES = (3.0, 6.0, 10.0)


def time_gated(darts, torch, np, W, gates=GATES, width=0.15625, n_thr=1 << 26, k=32, nb=1 << 22, target=1e-4):
    """Time-gated frames of the box workload, the form of the paper's
    evaluation (Section VI-B): one frame per gate [L0, L0 + width) (64x64
    pixels, one bin, every path of the DARTS family dedicated to it), each
    normalised by its own 0.95 quantile (of the uniform-sampling frame)
    before MSE.  Per arm: throughput on that frame, MSE x paths from k
    independent batches of nb paths, the largest pixel's share of the
    variance, and time to MSE `target` (extrapolated)."""
    rep = {"width": width, "batches": k, "paths_for_variance": k * nb, "target": target}
    for L0 in gates:
        w = W.box_hg()
        w["scene"]["bins"] = {"l_lo": L0, "l_hi": L0 + width, "n_bins": 1}
        sc, pr, dm = w["scene"], w["params"], w["dims"]
        table = darts.build_da_tables(sc["medium"], dm)
        stream = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        arms, means = {}, {}
        for arm, mode, alpha in MSE_ARMS:
            p = dict(pr, n_paths=n_thr, alpha=alpha)
            hi, lo, _, _ = darts.render_transient(sc, p, mode, table)
            torch.cuda.synchronize()
            e0.record(stream)
            darts.render_transient(sc, p, mode, table, hi, lo)
            e1.record(stream)
            torch.cuda.synchronize()
            thr = n_thr / (e0.elapsed_time(e1) / 1e3)
            s1 = s2 = None
            for i in range(k):
                pb = dict(pr, n_paths=nb, path_offset=(1 << 40) + i * nb, seed=0xEF, alpha=alpha)
                h, l, _, _ = darts.render_transient(sc, pb, mode, table)
                n = darts.paths_per_cell(sc, pb, mode).numpy()
                x = (h.double() + l.double()).cpu().numpy() / np.maximum(n, 1)
                s1 = x if s1 is None else s1 + x
                s2 = x * x if s2 is None else s2 + x * x
            means[arm] = s1 / k
            v = np.maximum(s2 - k * means[arm] ** 2, 0) / (k - 1) * nb
            arms[arm] = {"alpha": alpha, "paths_per_s": thr, "var": float(v.mean()),
                         "max_cell_share": float(v.max() / max(float(v.sum()), 1e-300))}
        q95 = float(np.quantile(means["uniform"], 0.95))
        g = {"q95": q95}
        for arm, r in arms.items():
            mse_n = r.pop("var") / q95 ** 2
            r["mse_times_paths"] = mse_n
            r["seconds_to_target"] = mse_n / target / r["paths_per_s"]
            g[arm] = r
        for arm in arms:
            if arm != "uniform":
                g[f"uniform_over_{arm}_time"] = g["uniform"]["seconds_to_target"] / g[arm]["seconds_to_target"]
        rep[f"gate_{L0:g}"] = g
    return rep


MEASURED_ARMS = (("darts", "darts", 0.5), ("darts_alpha2", "darts", 2.0), ("darts_alpha4", "darts", 4.0),
                 ("da_only", "da_only", 0.5), ("uniform", "uniform", 0.5), ("vanilla", "vanilla", 0.5))


def measured_convergence(darts, torch, np, W, gates=(3.0, 6.0, 10.0), width=0.15625, q95_log2=32,
                         arms=MEASURED_ARMS, target=1e-4, cap_seconds=4.0):
    """Time to MSE `target` measured, not extrapolated, on time-gated frames
    of the box workload (one gate [L0, L0 + width) per frame, the form of the
    paper's comparison).  Each arm renders two independent replicas (seeds
    0xC0 and 0xC1, disjoint path ids) by progressive launches, each doubling
    the path count (N = 2^20, 2^21, ...; every launch adds as many new paths
    as the frame already holds).  Both replicas are unbiased and independent,
    so half the mean squared difference of their images is the MSE of one
    replica at N paths; no reference image enters.  The MSE is normalised by
    the 0.95 quantile of the frame (from 2^q95_log2 paths each of DARTS at
    alpha = 4 and uniform sampling).  Wall time is that of one replica's
    launches plus one table build, accumulated until the MSE reaches the
    target (`reached`, and `seconds_at_crossing` placed between the last two
    doublings with MSE ~ 1/N) or until the launches have taken `cap_seconds`
    (then `extrapolated_seconds` continues MSE ~ 1/N from the last doubling).
    `time_ratio_vs_uniform`: uniform sampling's time over the arm's (above 1:
    the arm is faster), from the crossings or the extrapolations."""
    out = {}
    for L0 in gates:
        w = W.box_hg()
        w["scene"]["bins"] = {"l_lo": L0, "l_hi": L0 + width, "n_bins": 1}
        sc, pr, dm = w["scene"], w["params"], w["dims"]
        t0 = time.perf_counter()
        table = darts.build_da_tables(sc["medium"], dm)
        torch.cuda.synchronize()
        t_table = time.perf_counter() - t0
        shape = darts.image_shape(sc)
        img = torch.zeros(shape, dtype=torch.float64, device="cuda")
        for mode, alpha in (("darts", 4.0), ("uniform", 0.5)):
            pq = dict(pr, n_paths=1 << q95_log2, path_offset=1 << 45, seed=0x5EF, alpha=alpha)
            hi, lo, _, _ = darts.render_transient(sc, pq, mode, table)
            n = darts.paths_per_cell(sc, pq, mode).to("cuda")
            img += (hi.double() + lo.double()) / n.clamp(min=1) / 2
        q95 = float(np.quantile(img.cpu().numpy(), 0.95))
        rep = {"gate": [L0, L0 + width], "target": target, "q95": q95, "q95_paths": 2 << q95_log2,
               "table_build_s": t_table, "cap_seconds": cap_seconds}
        for arm, mode, alpha in arms:
            imgs = [[torch.zeros(shape, dtype=torch.float32, device="cuda") for _ in range(2)] for _ in range(2)]
            total, wall, hist = 0, t_table, []
            while True:
                add = (1 << 20) if total == 0 else total
                for rpl, seed in enumerate((0xC0, 0xC1)):
                    pc = dict(pr, n_paths=add, path_offset=(1 << 44) + total, seed=seed, alpha=alpha)
                    torch.cuda.synchronize()
                    t1 = time.perf_counter()
                    darts.render_transient(sc, pc, mode, table, imgs[rpl][0], imgs[rpl][1])
                    torch.cuda.synchronize()
                    if rpl == 0:
                        wall += time.perf_counter() - t1
                total += add
                pall = dict(pr, n_paths=total, path_offset=1 << 44, alpha=alpha)
                n = darts.paths_per_cell(sc, pall, mode).to("cuda").clamp(min=1)
                a = (imgs[0][0].double() + imgs[0][1].double()) / n
                b = (imgs[1][0].double() + imgs[1][1].double()) / n
                mse = float(((a - b) ** 2).mean()) / 2 / q95 ** 2
                hist.append((total, wall, mse))
                if mse <= target or wall - t_table >= cap_seconds or total >= (1 << 40):
                    break
            mse_last = hist[-1][2]
            reached = mse_last <= target
            frac = mse_last / target   # MSE ~ 1/N and launch time ~ N
            r = {"alpha": alpha, "paths": total, "seconds": wall, "mse": mse_last, "reached": reached,
                 "history": [{"paths": x, "seconds": y, "mse": z} for x, y, z in hist]}
            if reached:
                r["seconds_at_crossing"] = t_table + (wall - t_table) * min(1.0, frac)
                r["paths_at_crossing"] = total * min(1.0, frac)
            else:
                r["extrapolated_seconds"] = t_table + (wall - t_table) * frac
            rep[arm] = r
        tu = rep["uniform"].get("seconds_at_crossing", rep["uniform"].get("extrapolated_seconds")) \
            if "uniform" in rep else None
        for arm, _, _ in arms:
            ta = rep[arm].get("seconds_at_crossing", rep[arm].get("extrapolated_seconds"))
            if tu and ta:
                rep[arm]["time_ratio_vs_uniform"] = tu / ta
        out[f"L0={L0:g}"] = rep
    return out


def response_bench(darts, torch, np, W, w, n_thr=1 << 26, n_var=1 << 26, k=64, target=1e-4):
    """Two-peak sensor response W on the box workload (one value per pixel,
    Eq. (4)): throughput of each arm of the time-to-MSE study, the fraction
    of full path samples the sensor rejects (W = 0 at their length), and time
    to MSE `target` (normalised by the 0.95 quantile of the uniform-sampling
    image, variance from k independent batches, extrapolated at the measured
    throughput; `max_cell_share` as in time_to_mse)."""
    sc, pr, dm = w["scene"], w["params"], w["dims"]
    resp = W.two_peak_response(sc["bins"])
    R = darts.build_response(resp)
    table = darts.build_da_tables(sc["medium"], dm)
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    rep = {"response": "two Gaussian peaks at L = 3.0 and 5.5 (width 0.4, heights 1 and 0.6), zero below 1e-3",
           "target": target, "batches": k, "paths_for_variance": n_var}
    thr, var, means = {}, {}, {}
    for arm, mode, alpha in MSE_ARMS:
        p = dict(pr, n_paths=n_thr, alpha=alpha)
        hi, lo, _, st = darts.render_transient(sc, p, mode, table, want_stats=True, response=R)
        torch.cuda.synchronize()
        s = darts.stats_dict(st)
        e0.record(stream)
        darts.render_transient(sc, p, mode, table, hi, lo, response=R)
        e1.record(stream)
        torch.cuda.synchronize()
        thr[arm] = n_thr / (e0.elapsed_time(e1) / 1e3)
        s1 = s2 = None
        nb = n_var // k
        for i in range(k):
            pb = dict(pr, n_paths=nb, path_offset=(1 << 40) + i * nb, seed=0xEF, alpha=alpha)
            h, l, _, _ = darts.render_transient(sc, pb, mode, table, response=R)
            n = darts.paths_per_cell(sc, pb, mode, response=R).numpy()
            x = (h.double() + l.double()).cpu().numpy() / np.maximum(n, 1)
            s1 = x if s1 is None else s1 + x
            s2 = x * x if s2 is None else s2 + x * x
        means[arm] = s1 / k
        var[arm] = np.maximum(s2 - k * means[arm] ** 2, 0) / (k - 1) * nb
        rep[arm] = {"alpha": alpha, "paths_per_s": thr[arm], "samples": s["samples"], "rejected": s["rejected"],
                    "rejected_fraction": s["rejected"] / max(s["samples"], 1),
                    "max_cell_share": float(var[arm].max() / max(float(var[arm].sum()), 1e-300))}
    q95 = float(np.quantile(means["uniform"], 0.95))
    rep["q95"] = q95
    for arm in var:
        mse_n = float(np.mean(var[arm])) / q95 ** 2
        rep[arm]["mse_times_paths"] = mse_n
        rep[arm]["seconds_to_target"] = mse_n / target / thr[arm]
    for arm in var:
        if arm != "uniform":
            rep[f"uniform_over_{arm}_time"] = rep["uniform"]["seconds_to_target"] / rep[arm]["seconds_to_target"]
            rep[f"uniform_over_{arm}_mse_per_path"] = rep["uniform"]["mse_times_paths"] / rep[arm]["mse_times_paths"]
    return rep


def fog_bench(darts, torch, W, reps=2):
    """Fog layer over a Lambertian floor, two emitters 3 length units apart:
    the full 256x256 x 1024-bin DARTS render at 2^28 paths (HIP-event timed),
    then 200 Adam steps recovering (sigma_s, g) from a synthetic target with
    the adjoint kernel (on the 16x16 x 128-bin version of the scene)."""
    from paper_2402_03106_amd import inverse
    w = W.fog_slab()
    sc, pr, dm = w["scene"], w["params"], w["dims"]
    table = darts.build_da_tables(sc["medium"], dm)
    hi, lo, _, _ = darts.render_transient(sc, pr, "darts", table)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        darts.render_transient(sc, pr, "darts", table, hi, lo)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    n = int(pr["n_paths"])
    del hi, lo
    torch.cuda.empty_cache()
    fw = W.fog_slab_fit()
    fit = inverse.fit_medium(fw, fw["target_medium"], fw["init_medium"], **FIT_SETTINGS)
    tm, im = fw["target_medium"], fw["init_medium"]
    # what the fit's target image determines: Gauss-Newton geometry of the L2
    # fit from forward-mode derivative images (the target of 2^27 paths the
    # fit uses; Jacobians from 2^31 paths each, uniform sampling for the
    # lightest-tailed estimate)
    info = inverse.fit_information(fw, tm, "uniform", target_paths=1 << 27, jac_paths=1 << 31)
    return {
        "render": {"paths": n, "cells": 256 * 256 * 1024, "render_ms": ms, "paths_per_s": n / ms * 1e3},
        "fit": {"target": {"sigma_s": tm["sigma_s"], "g": tm["g"]}, "init": {"sigma_s": im["sigma_s"], "g": im["g"]},
                "estimate": {"sigma_s": fit["sigma_s"], "g": fit["g"]},
                "rel_error": {"sigma_s": fit["sigma_s"] / tm["sigma_s"] - 1, "g": fit["g"] / tm["g"] - 1,
                              "reduced_sigma_s": fit["sigma_s"] * (1 - fit["g"]) / (tm["sigma_s"] * (1 - tm["g"])) - 1},
                "steps": fit["steps"], "seconds": fit["seconds"], "ms_per_step": fit["seconds"] / fit["steps"] * 1e3,
                "paths_per_render": fit["paths_per_render"], "mode": fit["mode"],
                "image": "16x16 x 128 bins over [0,40)"},
        "fit_information": info,
    }


def adjoint_bench(darts, torch, W, reps=3):
    """The differentiable box (sigma_s = 8, sigma_a = 0.2, g = 0.5; 128x128
    pixels x 512 bins, 2^22 paths): forward render and adjoint replay
    (darts_render_transient_backward) of the L2 loss against a target
    rendered at sigma_s = 10, sigma_a = 0.1, g = 0.6 (2^24 paths, other
    ids), each launch timed with HIP events on its stream; the gradient
    d loss / d(sigma_s, sigma_a, g) it gives is reported alongside."""
    w = W.box_hg_grad()
    sc, pr, dm = w["scene"], w["params"], w["dims"]
    tsc = dict(sc, medium=w["target_medium"])
    stream = torch.cuda.current_stream()
    ttab = darts.build_da_tables(tsc["medium"], dm)
    tp = dict(pr, n_paths=1 << 24, path_offset=1 << 42)
    th, tl, _, _ = darts.render_transient(tsc, tp, "darts", ttab)
    T = (th.double() + tl.double()) / darts.paths_per_cell(tsc, tp, "darts").to("cuda").clamp(min=1)
    table = darts.build_da_tables(sc["medium"], dm)
    n = darts.paths_per_cell(sc, pr, "darts").to("cuda").clamp(min=1)
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    fwd, bwd = [], []
    for _ in range(reps + 1):
        hi = torch.zeros_like(th)
        lo = torch.zeros_like(tl)
        e0.record(stream)
        darts.render_transient(sc, pr, "darts", table, hi, lo)
        e1.record(stream)
        I = (hi.double() + lo.double()) / n
        gimg = (2.0 * (I - T) / n).float()
        e2.record(stream)
        g = darts.render_transient_backward(sc, pr, "darts", table, gimg)
        e3 = torch.cuda.Event(enable_timing=True)
        e3.record(stream)
        torch.cuda.synchronize()
        fwd.append(e0.elapsed_time(e1))
        bwd.append(e2.elapsed_time(e3))
    fwd, bwd = fwd[1:], bwd[1:]      # the first pass warms up
    paths = int(pr["n_paths"])
    return {"workload": "box_hg_grad: 128x128 x 512 bins, 2^22 paths, L2 loss vs the target medium",
            "forward_ms": min(fwd), "backward_ms": min(bwd), "backward_paths_per_s": paths / min(bwd) * 1e3,
            "cells": int(n.numel()), "grad": [float(x) for x in g.cpu()]}


def batched_bench(darts, torch, W, reps, scale=1):
    """The many-media sweep: 256 box media with uneven budgets in one
    persistent launch (plan chosen by the autotuner), replayed as a captured
    graph (clear + launch), against one render call per medium on the same
    paths.  Tables are built once, outside the timed region.  `scale`
    multiplies every medium's budget (how the launch's tail weighs)."""
    ws = W.batched()
    for w in ws:
        w["params"]["n_paths"] = int(w["params"]["n_paths"]) * int(scale)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tables = [darts.build_da_tables(w["scene"]["medium"], w["dims"]) for w in ws]
    torch.cuda.synchronize()
    t_tables = time.perf_counter() - t0
    items = [(w["scene"], w["params"], "darts", t) for w, t in zip(ws, tables)]
    n_paths = sum(int(w["params"]["n_paths"]) for w in ws)
    b = darts.Batch(items)
    hi, lo = b.empty()
    t0 = time.perf_counter()
    plan, tuned_ms = b.autotune(hi, lo, reps=2)
    t_tune = time.perf_counter() - t0
    stream = torch.cuda.current_stream()
    b.graph_launch(hi, lo)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        b.graph_launch(hi, lo)
    e1.record(stream)
    torch.cuda.synchronize()
    graph_ms = e0.elapsed_time(e1) / reps
    # one render call per medium, same paths, into the same batch images
    views_hi, views_lo = b.images(hi), b.images(lo)
    seq = []
    for r in range(2):
        e0.record(stream)
        for (sc, p, mode, t), h, l in zip(items, views_hi, views_lo):
            darts.render_transient(sc, p, mode, t, h, l)
        e1.record(stream)
        torch.cuda.synchronize()
        seq.append(e0.elapsed_time(e1))
    seq_ms = min(seq)
    # the batch's work: the same paths rendered one medium at a time with the
    # statistics counters (vertex steps), priced at the per-unit figures
    steps = 0
    for sc, p, mode, t in items:
        _, _, _, st = darts.render_transient(sc, p, mode, t, want_stats=True)
        s_ = darts.stats_dict(st)
        steps += s_["vertices"] - s_["early_exit"]
    torch.cuda.synchronize()
    flops = FLOPS_PER_VERTEX_STEP * steps + FLOPS_PER_PATH * n_paths
    return {"media": len(ws), "budget_scale": int(scale), "paths": n_paths, "plan": plan, "autotune_s": t_tune, "tuned_launch_ms": tuned_ms,
            "graph_launch_ms": graph_ms, "paths_per_s": n_paths / graph_ms * 1e3,
            "vertex_steps": steps, "mean_steps_per_path": steps / n_paths,
            "algorithmic_tflops": flops / graph_ms / 1e9, "vertex_steps_per_s": steps / graph_ms * 1e3,
            "separate_calls_ms": seq_ms, "speedup_vs_separate_calls": seq_ms / graph_ms,
            "table_build_s": t_tables,
            "workload": "256 box media, sigma_s~U[0.5,20], albedo~U[0.8,0.999], g~U[-0.3,0.9], 32x32 x 128 bins "
                        f"over [0,40), budgets log-uniform in [2^12,2^18]{'' if scale == 1 else f' x {scale}'}, "
                        "64x64x32 tables"}


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def _oracle_rate(ref, w, mode, cdf, threads, seconds):
    """Paths/s of the oracle on workload w, doubling the sample from 2^12
    until about `seconds` of work."""
    sc, pr, dm = w["scene"], w["params"], w["dims"]
    n = 1 << 12
    while True:
        p = dict(pr, n_paths=n)
        t0 = time.perf_counter()
        ref.render(sc, p, mode, cdf, dm, n_threads=threads)
        dt = time.perf_counter() - t0
        if dt >= seconds or n >= (1 << 26):
            return n, dt
        n = n * 2 if dt * 2.5 < seconds else max(n + 1, int(n * seconds / max(dt, 1e-3)))


def cpu_baseline(w, seconds):
    """The oracle as it stands on the host cores: DARTS on the same box
    workload (`value`, about `seconds` of work on all threads, plus a quarter
    of that work on one thread), and the planned grid: DARTS, uniform and
    vanilla on the box workload and on the infinite-medium workload, each on
    all threads and on one thread (about seconds/16 each)."""
    from oracle import ref
    from paper_2402_03106_amd import workloads as W
    sc, pr, dm = w["scene"], w["params"], w["dims"]
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count()
    _, cdf = ref.build_table(sc["medium"], dm, n_threads=threads)
    n, dt = _oracle_rate(ref, w, "darts", cdf, threads, seconds)
    # one thread on about a quarter of that work: the per-core rate
    n1 = max(1 << 12, int(n / max(threads, 1) / 4))
    t0 = time.perf_counter()
    ref.render(sc, dict(pr, n_paths=n1), "darts", cdf, dm, n_threads=1)
    dt1 = time.perf_counter() - t0
    grid = {}
    for wname, wk in (("box_hg", w), ("infinite_point", W.infinite_point())):
        _, cdf_k = ref.build_table(wk["scene"]["medium"], wk["dims"], n_threads=threads)
        for mode in ("darts", "uniform", "vanilla"):
            e = {}
            for label, th in (("all_threads", threads), ("one_thread", 1)):
                nk, dk = _oracle_rate(ref, wk, mode, cdf_k if mode == "darts" else None, th, seconds / 16)
                e[label] = {"paths_per_s": nk / dk, "paths": nk, "seconds": dk}
            grid[f"{wname}/{mode}"] = e
    return {"value": n / dt, "unit": "paths/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"{n} DARTS paths of the box workload (ids 0..{n - 1}), FP64, {dt:.1f} s",
            "single_thread_value": n1 / dt1,
            "single_thread_sample": f"{n1} paths (ids 0..{n1 - 1}) on one thread, {dt1:.1f} s",
            "grid": grid}


if __name__ == "__main__":
    main()
