"""Recovering medium parameters from a time-resolved image with the adjoint
kernel: Adam on (sigma_s, g) with sigma_a held fixed.

Each step renders the current medium twice with independent path ids: the
first render gives the residual r = I - T against the target T, the second is
differentiated (path replay, darts_render_transient_backward) with the
adjoint image 2 r, which makes the step's gradient an unbiased estimate of
the gradient of the L2 loss sum (I - T)^2.

The optimiser's coordinates are log(sigma_s (1 - g)) and atanh(g / 0.99):
every step stays a valid medium, and the direction along which a
time-resolved image of a forward-scattering layer changes least (constant
reduced scattering coefficient sigma_s (1 - g)) is one coordinate axis.
How well an image determines sigma_s and g at all is measured by
`fisher_information`.
"""
from __future__ import annotations

import math
import time

import torch

from . import darts


def _image_stats(w: dict, medium: dict, mode: str, n_paths: int, seed: int, offset: int = 0):
    """Per-cell estimates and per-cell variances of the estimate of one
    render of n_paths paths (from the second moments of the same render)."""
    sc, dm, pr = dict(w["scene"], medium=medium), w["dims"], w["params"]
    p = dict(pr, n_paths=n_paths, seed=seed, path_offset=offset)
    flags = darts.MODES[mode]
    table = darts.build_da_tables(medium, dm) if flags & darts.EDA_DIR else None
    hi, lo, m2, _ = darts.render_transient(sc, p, mode, table, want_m2=True)
    n = darts.paths_per_cell(sc, p, mode).to(hi.device).clamp(min=1)
    mean = (hi.double() + lo.double()) / n
    var = torch.clamp(m2.double() / n - mean * mean, min=0) / n
    return mean, var


def tangent_image(w: dict, medium: dict, mode: str, n_paths: int, seed: int, offset: int = 0) -> torch.Tensor:
    """Per-cell derivatives of the per-cell estimates with respect to
    (sigma_s, sigma_a, g), [3, n_bins, H, W] (forward-mode derivative images
    of one render of n_paths paths)."""
    sc, dm, pr = dict(w["scene"], medium=medium), w["dims"], w["params"]
    p = dict(pr, n_paths=n_paths, seed=seed, path_offset=offset)
    flags = darts.MODES[mode]
    table = darts.build_da_tables(medium, dm) if flags & darts.EDA_DIR else None
    t = darts.render_transient_tangent(sc, p, mode, table)
    n = darts.paths_per_cell(sc, p, mode).to(t.device).clamp(min=1)
    return t.double() / n


def fit_information(w: dict, medium: dict, mode: str = "da_only", target_paths: int = 1 << 27,
                    jac_paths: int = 1 << 29, seed: int = 0xF15) -> dict:
    """How well the L2 fit of `fit_medium` can determine (sigma_s, g), with
    sigma_a known, from a target image of workload `w` with `target_paths`
    paths at `medium`.

    J: the per-cell derivatives dI_c/dtheta of the image's expectation,
    theta = (sigma_s, g), from the forward-mode derivative images
    (darts_render_transient_tangent) of two independent renders of jac_paths
    paths; the Gauss-Newton matrix J^T J of the L2 loss is formed as
    J_a^T J_b (symmetrised), an unbiased estimate (the noise of the estimates
    does not square).  Returned, in relative units (theta scaled by its
    values): the matrix, its condition number, the cosine of the angle
    between the columns of J (|cos| -> 1: to first order the image changes
    with sigma_s and g only through one combination of them), the direction
    in (log sigma_s, log g) along which the image changes least and its
    cosine with the direction of constant sigma_s (1 - g).  When the matrix
    is positive definite, also the standard deviations that the target's own
    noise (per-cell variance var_c from the second moments of a third render,
    scaled to target_paths) leaves in the fit's estimate near the optimum,
    covariance (J^T J)^-1 (J^T diag(var) J) (J^T J)^-1, for sigma_s, g and
    sigma_s (1 - g), and the correlation of the sigma_s and g estimates."""
    import numpy as np
    th = np.array([medium["sigma_s"], medium["g"]], dtype=np.float64)
    jac = []
    for rep in range(2):
        t = tangent_image(w, medium, mode, jac_paths, seed + rep)
        jac.append(torch.stack([t[0].reshape(-1), t[2].reshape(-1)], 1))
    Ja, Jb = jac
    sym = lambda m: 0.5 * (m + m.T)
    G = sym(Ja.T @ Jb).cpu().numpy()
    D = np.diag(th)
    Grel = D @ G @ D
    ev, evec = np.linalg.eigh(Grel)
    weak = evec[:, 0] / np.linalg.norm(evec[:, 0])            # least-changing direction, relative units
    # sigma_s (1 - g) is constant along d log sigma_s = g / (1 - g) d log g
    const_red = np.array([th[1] / (1.0 - th[1]), 1.0])
    const_red /= np.linalg.norm(const_red)
    out = {"gauss_newton_relative": Grel.tolist(),
           "condition_number": float(ev.max() / ev.min()) if ev.min() > 0 else float("inf"),
           "column_cosine": float(G[0, 1] / np.sqrt(G[0, 0] * G[1, 1])),
           "weak_direction_rel": weak.tolist(), "constant_reduced_direction_rel": const_red.tolist(),
           "weak_vs_constant_reduced_cosine": float(abs(weak @ const_red)),
           "target_paths": target_paths, "jac_paths": jac_paths, "mode": mode}
    if ev.min() > 0:
        _, var = _image_stats(w, medium, mode, jac_paths, seed + 99, offset=1 << 40)
        var = (var * (jac_paths / target_paths)).reshape(-1)
        V = sym((Ja * var[:, None]).T @ Jb).cpu().numpy()
        Gi = np.linalg.inv(G)
        cov = Gi @ V @ Gi
        sd = np.sqrt(np.maximum(np.diag(cov), 0.0))
        gv = np.array([1.0 - th[1], -th[0]])                  # gradient of sigma_s (1 - g)
        red = th[0] * (1.0 - th[1])
        out["fit_rel_std"] = {"sigma_s": float(sd[0] / th[0]), "g": float(sd[1] / abs(th[1])),
                              "reduced_sigma_s": float(np.sqrt(max(gv @ cov @ gv, 0.0))) / red}
        out["correlation"] = float(cov[0, 1] / (sd[0] * sd[1])) if sd[0] > 0 and sd[1] > 0 else float("nan")
    return out

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
    iterates carry the noise of the stochastic gradient), taken in the
    coordinates Adam works in, log sigma_s (1 - g) and atanh(g / 0.99), and
    mapped back, so that the estimate's sigma_s (1 - g) is the geometric mean
    of the iterates' (averaging sigma_s and g separately would bias it where
    g is near 1 and sigma_s = sigma_s (1 - g) / (1 - g) swings between
    iterates).  Returns the trajectory and the estimate.

    With `relative` the loss is sum_c (I_c - T_c)^2 / (T_c^2 + e^2) with e =
    rel_floor * max T: every cell counts by its relative error, so the dim
    early (single-scattering) and late cells, which separate sigma_s from g,
    weigh as much as the bright diffuse ones (to first order a plain L2 loss
    on the fog layer's view changes only with sigma_s (1 - g): see
    fit_information)."""
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
        coords = (float(log_s), float(atanh_g))
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
        hist.append({"step": it, "loss": float((wgt * r * r).sum()), "sigma_s": float(th[0]), "g": float(th[2]),
                     "log_reduced": coords[0], "atanh_g": coords[1]})
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    tail = hist[-max(1, min(average_last, len(hist))):]
    reduced = math.exp(sum(h["log_reduced"] for h in tail) / len(tail))
    g = 0.99 * math.tanh(sum(h["atanh_g"] for h in tail) / len(tail))
    return {"sigma_s": reduced / (1.0 - g), "sigma_a": sigma_a, "g": g, "reduced_sigma_s": reduced,
            "history": hist, "seconds": elapsed, "steps": steps, "paths_per_render": n_paths, "mode": mode}
