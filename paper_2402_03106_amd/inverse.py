"""Recovering medium parameters from a time-resolved image with the adjoint
kernel: Adam on (sigma_s, g) with sigma_a held fixed.

Each step renders the current medium twice with independent path ids: the
first render gives the residual r = I - T against the target T, the second is
differentiated (path replay, darts_render_transient_backward) with the
adjoint image 2 r, which makes the step's gradient an unbiased estimate of
the gradient of the L2 loss sum (I - T)^2.

The diffuse part of a time-resolved image depends on sigma_s and g mostly
through the reduced scattering coefficient sigma_s (1 - g), so the loss has a
long shallow valley along sigma_s (1 - g) = const.  The optimiser's
coordinates are therefore log(sigma_s (1 - g)) and atanh(g / 0.99): the valley
runs along the second axis, where Adam's per-coordinate step normalisation
keeps moving, and every step stays a valid medium.
"""
from __future__ import annotations

import math
import time

import torch

from . import darts


def _theta(log_sr, atanh_g, sigma_a):
    g = 0.99 * torch.tanh(atanh_g)
    return torch.stack([torch.exp(log_sr) / (1.0 - g), torch.as_tensor(sigma_a, dtype=log_sr.dtype), g])


def fit_medium(w: dict, target_medium: dict, init_medium: dict, steps: int = 200, lr: float = 0.05,
               lr_final: float = 0.005, n_paths: int = 1 << 24, target_paths: int = 1 << 27,
               mode: str = "darts", seed: int = 0xADA0, target_image: torch.Tensor | None = None,
               average_last: int = 20, relative: bool = False, rel_floor: float = 1e-2) -> dict:
    """Fit (sigma_s, g) of workload `w` (its scene, bins and table dims) to a
    target rendered at `target_medium` (or given as `target_image`, the
    per-cell estimates [n_bins, H, W]), starting from `init_medium`.  The
    learning rate decays from `lr` to `lr_final` on a cosine schedule; the
    estimate is the mean of the last `average_last` iterates (the single
    iterates carry the noise of the stochastic gradient).  Returns the
    trajectory and the estimate.

    With `relative` the loss is sum_c (I_c - T_c)^2 / (T_c^2 + e^2) with e =
    rel_floor * max T: every cell counts by its relative error, so the dim
    early (single-scattering) and late cells, which separate sigma_s from g,
    weigh as much as the bright diffuse ones (a plain L2 loss only sees the
    reduced scattering coefficient sigma_s (1 - g))."""
    sc, dm, pr = w["scene"], w["dims"], w["params"]
    sigma_a = float(target_medium["sigma_a"])
    if target_image is None:
        t_true = torch.tensor([target_medium["sigma_s"], sigma_a, target_medium["g"]], dtype=torch.float64)
        with torch.no_grad():
            target_image = darts.transient_image(t_true, sc, dict(pr, n_paths=target_paths, seed=seed), mode, dm)
    T = target_image.detach()
    if relative:
        wgt = 1.0 / (T * T + (rel_floor * float(T.max())) ** 2)
    else:
        wgt = torch.ones_like(T)
    log_s = torch.tensor(math.log(init_medium["sigma_s"] * (1.0 - init_medium["g"])), dtype=torch.float64,
                         requires_grad=True)
    atanh_g = torch.tensor(math.atanh(init_medium["g"] / 0.99), dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([log_s, atanh_g], lr=lr)
    sched = torch.optim.lr_scheduler.CosineAnnealingLR(opt, T_max=max(steps, 1), eta_min=lr_final)
    hist = []
    t0 = time.perf_counter()
    for it in range(steps):
        theta = _theta(log_s, atanh_g, sigma_a)
        with torch.no_grad():
            I1 = darts.transient_image(theta.detach(), sc, dict(pr, n_paths=n_paths, seed=seed + 2 * it + 1), mode, dm)
        I2 = darts.transient_image(theta, sc, dict(pr, n_paths=n_paths, seed=seed + 2 * it + 2), mode, dm)
        r = (I1 - T).detach()
        surrogate = (2.0 * wgt * r * I2).sum()
        opt.zero_grad()
        surrogate.backward()
        opt.step()
        sched.step()
        th = theta.detach()
        hist.append({"step": it, "loss": float((wgt * r * r).sum()), "sigma_s": float(th[0]), "g": float(th[2])})
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    tail = hist[-max(1, min(average_last, len(hist))):]
    return {"sigma_s": sum(h["sigma_s"] for h in tail) / len(tail), "sigma_a": sigma_a,
            "g": sum(h["g"] for h in tail) / len(tail), "history": hist, "seconds": elapsed, "steps": steps,
            "paths_per_render": n_paths, "mode": mode}
