"""GPU building blocks vs the FP64 oracle, one item per thread through
darts_debug_pointwise.  Bar: bit-exact for integer work (Philox, candidate
uniforms); relative 1e-5 (absolute floor 1e-6 for unit-bounded quantities)
for the FP32 samplers and densities; discrete choices (RIS pick, MIS branch,
cos-bin) may flip only where FP32 rounding sits on a decision boundary."""
import ctypes as C
import math

import numpy as np
import pytest
import torch

from paper_2402_03106_amd import workloads as W

pytestmark = pytest.mark.gpu
F32 = np.float32


@pytest.fixture(scope="module")
def D():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2402_03106_amd import darts
    darts.lib()
    return darts


class Bits(int):
    """A 32-bit integer argument, passed to the kernel by bit pattern."""


def run(D, fn, rows, med=None, table=None):
    """rows: lists of floats and Bits.  Returns (out float64 [n, 8],
    float inputs as float64 [n, 16], integer inputs as uint32 [n, 16])."""
    inp = np.zeros((len(rows), D.PW_IN), F32)
    ib = inp.view(np.uint32)
    for i, r in enumerate(rows):
        for j, v in enumerate(r):
            if isinstance(v, Bits):
                ib[i, j] = int(v) & 0xFFFFFFFF
            else:
                inp[i, j] = v
    x = torch.from_numpy(inp.copy()).cuda()
    out = D.debug_pointwise(fn, x, med, table)
    torch.cuda.synchronize()
    fl = np.where(np.isfinite(inp), inp, np.where(np.isinf(inp), inp, 0)).astype(np.float64)
    return out.cpu().numpy().astype(np.float64), fl, ib.copy()


def ubits(v):
    return Bits(int(v))


def rel_ok(a, b, rtol=1e-5, atol=0.0):
    return np.abs(a - b) <= rtol * np.abs(b) + atol


def test_philox_bit_exact(D, oracle):
    rng = np.random.default_rng(10)
    rows, refs = [], []
    kat = [([0, 0, 0, 0], [0, 0]), ([0xFFFFFFFF] * 4, [0xFFFFFFFF] * 2),
           ([0x243f6a88, 0x85a308d3, 0x13198a2e, 0x03707344], [0xa4093822, 0x299f31d0])]
    for _ in range(2000):
        kat.append((list(rng.integers(0, 2 ** 32, 4)), list(rng.integers(0, 2 ** 32, 2))))
    for ctr, key in kat:
        rows.append([int(v) for v in ctr + key])
        refs.append(oracle.philox(ctr, key))
    inp = np.zeros((len(rows), D.PW_IN), np.uint32)
    inp[:, :6] = np.array(rows, np.uint64).astype(np.uint32)
    out = D.debug_pointwise("philox", torch.from_numpy(inp.view(F32).copy()).cuda())
    torch.cuda.synchronize()
    got = out.cpu().numpy()[:, :4].view(np.uint32)
    assert np.array_equal(got, np.array(refs, np.uint32))


def test_sobol_bit_exact(D, oracle):
    L = oracle.lib()
    rng = np.random.default_rng(11)
    rows, ref = [], []
    for _ in range(3000):
        r, c, e = int(rng.integers(32)), int(rng.integers(8)), int(rng.integers(0, 2 ** 32))
        rows.append([ubits(r), ubits(c), ubits(e)])
        ref.append(L.ref_sobol_u(r, c, e))
    out, _, _ = run(D, "sobol", rows)
    assert np.array_equal(out[:, 0], np.array(ref))


def test_hg_pdf(D, oracle):
    L = oracle.lib()
    rng = np.random.default_rng(12)
    gs = np.concatenate([[-0.95, -0.3, 0.0, 1e-4, 0.5, 0.7, 0.95], rng.uniform(-0.95, 0.95, 40)]).astype(F32)
    mus = np.concatenate([[-1, -0.5, 0, 0.5, 0.999, 1], rng.uniform(-1, 1, 40)]).astype(F32)
    rows = [[m, g] for g in gs for m in mus]
    out, inp, _ = run(D, "hg_pdf", rows)
    ref = np.array([L.ref_hg_pdf(m, g) for m, g in inp[:, :2]])
    assert np.all(rel_ok(out[:, 0], ref)), np.max(np.abs(out[:, 0] / ref - 1))


def test_hg_sample(D, oracle):
    L = oracle.lib()
    rng = np.random.default_rng(13)
    gs = np.concatenate([[-0.95, -0.3, 0.0, 1e-6, 1e-3, 0.5, 0.7, 0.95], rng.uniform(-0.95, 0.95, 30)]).astype(F32)
    xis = np.concatenate([[0.0, 1e-7, 0.5, 1 - 2 ** -24], rng.random(60)]).astype(F32)
    rows = [[x, g] for g in gs for x in xis]
    out, inp, _ = run(D, "hg_sample", rows)
    mu_ref = np.array([L.ref_hg_sample_mu(x, g) for x, g in inp[:, :2]])
    sin_ref = np.sqrt(np.maximum((1 - mu_ref) * (1 + mu_ref), 0))
    assert np.all(rel_ok(out[:, 0], mu_ref, 1e-5, 1e-6)), np.max(np.abs(out[:, 0] - mu_ref))
    assert np.all(rel_ok(out[:, 1], sin_ref, 1e-5, 1e-6)), np.max(np.abs(out[:, 1] - sin_ref))


@pytest.mark.parametrize("med", [dict(sigma_s=1.0, sigma_a=0.01, g=0.0), dict(sigma_s=4.75, sigma_a=0.25, g=0.7)])
def test_da_log_phi(D, oracle, med):
    L = oracle.lib()
    m = C.byref(oracle.medium(med))
    rng = np.random.default_rng(14)
    rows = [[r, s] for r, s in zip(rng.uniform(0, 10, 3000).astype(F32), rng.uniform(1e-3, 40, 3000).astype(F32))]
    out, inp, _ = run(D, "da_logphi", rows, med)
    D_ = 1.0 / (3 * (med["sigma_a"] + med["sigma_s"] * (1 - med["g"])))
    ref = np.array([L.ref_da_log_phi(m, r, s) for r, s in inp[:, :2]]) + 1.5 * math.log(4 * math.pi * D_)
    assert np.all(rel_ok(out[:, 0], ref, 1e-5, 1e-5)), np.max(np.abs(out[:, 0] - ref) / np.maximum(np.abs(ref), 1))


def test_truncated_exponential(D, oracle):
    L = oracle.lib()
    rng = np.random.default_rng(15)
    rows = []
    for _ in range(3000):
        rows.append([rng.random(), rng.uniform(0.01, 20), rng.choice([rng.uniform(1e-3, 5), np.inf])])
    rows += [[0.0, 5.0, 2.0], [1 - 2 ** -24, 5.0, 2.0], [1e-7, 0.1, 1e-3]]
    rows = [[F32(a) for a in r] for r in rows]
    out, inp, _ = run(D, "texp", rows)
    xr = np.array([L.ref_texp_sample(u, s, w) for u, s, w in inp[:, :3]])
    pr = np.array([L.ref_texp_pdf(x, s, w) for x, (u, s, w) in zip(xr, inp[:, :3])])
    assert np.all(rel_ok(out[:, 0], xr, 1e-5, 1e-12)), np.max(np.abs(out[:, 0] / np.maximum(xr, 1e-30) - 1))
    assert np.all(rel_ok(out[:, 1], pr, 1e-5)), np.max(np.abs(out[:, 1] / pr - 1))


def test_ellipse(D, oracle):
    L = oracle.lib()
    rng = np.random.default_rng(16)
    rows = []
    for _ in range(4000):
        Cd = rng.uniform(1e-3, 10)
        S = Cd * (1 + 10 ** rng.uniform(-4, 1))
        mu = rng.choice([rng.uniform(-1, 1), 1 - 10 ** rng.uniform(-7, -1)])
        rows.append([F32(S), F32(Cd), F32(mu), F32(rng.uniform(0.1, 3))])
    out, inp, _ = run(D, "ellipse", rows)
    t = np.array([L.ref_ell_t(S, Cd, mu) for S, Cd, mu in inp[:, :3]])
    r = inp[:, 0] - t
    pt = np.array([L.ref_ell_pdf_t(pS, S, Cd, mu, tt, 0) for (S, Cd, mu, pS), tt in zip(inp[:, :4], t)])
    # t, r and p_t of the FP64 oracle use the plain formulas (r = S - t);
    # the kernel's cancellation-free forms agree to FP32 rounding
    assert np.all(rel_ok(out[:, 0], t, 1e-5)), np.max(np.abs(out[:, 0] / t - 1))
    assert np.all(rel_ok(out[:, 1], r, 1e-5)), np.max(np.abs(out[:, 1] / r - 1))
    assert np.all(rel_ok(out[:, 2], pt, 1e-5)), np.max(np.abs(out[:, 2] / pt - 1))


def test_onb(D, oracle):
    L = oracle.lib()
    rng = np.random.default_rng(17)
    ns = [[0, 0, 1], [0, 0, -1], [1, 0, 0], [0, 1, 0]]
    for v in rng.normal(size=(2000, 3)):
        ns.append(list(v / np.linalg.norm(v)))
    rows = [[F32(a) for a in n] for n in ns]
    out, inp, _ = run(D, "onb", rows)
    for o, n in zip(out, inp[:, :3]):
        b1 = (C.c_double * 3)()
        b2 = (C.c_double * 3)()
        L.ref_onb((C.c_double * 3)(*n), b1, b2)
        assert np.allclose(o[:3], b1[:], atol=2e-6) and np.allclose(o[3:6], b2[:], atol=2e-6)


def test_box_exit(D, oracle):
    L = oracle.lib()
    rng = np.random.default_rng(18)
    rows = []
    for _ in range(3000):
        x = rng.uniform(-0.999, 0.999, 3)
        w = rng.normal(size=3)
        w /= np.linalg.norm(w)
        rows.append([*x, *w, -1, -1, -1, 1, 1, 1])
    rows.append([0, 0, 0, 0, 0, 1, -1, -1, -1, 1, 1, 1])
    rows = [[F32(a) for a in r] for r in rows]
    out, inp, _ = run(D, "box_exit", rows)
    g = oracle.geometry({"kind": 1, "lo": (-1, -1, -1), "hi": (1, 1, 1)})
    ref = np.array([L.ref_box_exit(C.byref(g), (C.c_double * 3)(*r[:3]), (C.c_double * 3)(*r[3:6])) for r in inp])
    assert np.all(rel_ok(out[:, 0], ref, 1e-5, 1e-6))


def test_exit_length(D, oracle):
    """Largest length sum of a connection (boundary clipping, Section V-B)
    against the FP64 oracle on the same float inputs.  General rays: S_exit
    to FP32 rounding of its terms.  Rays aimed within 1e-6..1e-2 rad of an
    emitter beyond the boundary: the excess S_exit - C, which d_m + |b| - C
    loses to cancellation in FP32, to within what FP32 rounding of the unit
    vector a to the emitter allows (a few ulp; the bar allows 16 eps on
    |w - a|, hence C |w - a| 16 eps on C (1 - mu) = C |w - a|^2 / 2); the
    plain FP32 sum is shown to miss that bar, so the test sees the
    difference."""
    L = oracle.lib()
    eps = float(np.finfo(np.float32).eps)
    rng = np.random.default_rng(22)
    rows, kind = [], []
    for _ in range(2000):
        x, xe = rng.uniform(-1, 1, 3), rng.normal(size=3) * 2
        w = rng.normal(size=3)
        w /= np.linalg.norm(w)
        rows.append([*x, *w, *xe, rng.uniform(0.01, 3)])
        kind.append(0)
    for eta in [0.0, 1e-6, 1e-5, 1e-4, 1e-3, 1e-2]:
        for _ in range(300):
            x = rng.uniform(-1, 1, 3)
            xe = x + rng.normal(size=3) * rng.uniform(0.5, 3)
            a = (xe - x) / np.linalg.norm(xe - x)
            n = np.cross(a, rng.normal(size=3))
            w = a * math.cos(eta) + n / np.linalg.norm(n) * math.sin(eta)
            rows.append([*x, *(w / np.linalg.norm(w)), *xe, np.linalg.norm(xe - x) * rng.uniform(0.05, 0.95)])
            kind.append(1)
    rows = [[F32(v) for v in r] for r in rows]
    kind = np.array(kind)
    out, inp, _ = run(D, "exit_length", rows)
    x, w32, xe, dm = inp[:, 0:3], inp[:, 3:6], inp[:, 6:9], inp[:, 9]
    # S_exit is defined for a unit direction: the float inputs stand for w / |w|
    w = w32 / np.linalg.norm(w32, axis=1)[:, None]
    ref = np.array([L.ref_exit_length(_v(a), _v(b), _v(c), d) for a, b, c, d in zip(x, w, xe, dm)])
    Cd = np.linalg.norm(xe - x, axis=1)
    bl = np.linalg.norm(x + w * dm[:, None] - xe, axis=1)
    g = kind == 0
    assert np.all(np.abs(out[g, 0] - ref[g]) <= 4 * eps * (dm[g] + bl[g] + Cd[g]))
    # aimed rays: the oracle's plain sum d_m + |b| rounds once per term in FP64;
    # cross-checked against the cancellation-free law-of-cosines excess
    eps64 = float(np.finfo(np.float64).eps)
    a_hat = (xe - x) / Cd[:, None]
    wa = np.linalg.norm(w - a_hat, axis=1)
    ex_ref = 2 * dm * (0.5 * Cd * wa * wa) / (bl + Cd - dm)
    h = kind == 1
    round64 = 4 * eps64 * (dm + bl + Cd)
    assert np.all(np.abs(ref[h] - (Cd[h] + ex_ref[h])) <= round64[h])
    delta = 16 * eps
    tol = 2 * dm * 0.5 * Cd * (2 * wa * delta + delta * delta) / (bl + Cd - dm) + 1e-5 * ex_ref + round64
    err = np.abs(out[:, 1] - (ref - Cd))
    assert np.all(err[h] <= tol[h]), np.max(err[h] / tol[h])
    assert np.all(out[h, 0] >= Cd[h] * (1 - 4 * eps))
    # the plain FP32 sum d_m + |b| - C fails the same bar on most aimed rays within 1e-3 rad
    x32, xe32, dm32 = (v.astype(np.float32) for v in (x, xe, dm))
    b32 = np.linalg.norm(x32 + w32 * dm32[:, None] - xe32, axis=1).astype(np.float32)
    plain = (dm32 + b32).astype(np.float32) - np.linalg.norm(xe32 - x32, axis=1).astype(np.float32)
    tight = h & (wa < 1.5e-3)
    assert np.mean(np.abs(plain[tight] - ex_ref[tight]) > tol[tight]) > 0.5


def _v(x):
    return (C.c_double * 3)(*x)


def test_ris_step(D, oracle):
    """Whole RIS free-flight step (Section IV-C) against the oracle on the same
    inputs.  Items whose discrete decisions agree (validity of each of the 8
    candidates, the selected candidate) match in the distance and in the
    weight factor to 1e-5 relative, every one of them.  An item may decide
    otherwise only where the oracle's decision sits within FP32 rounding of
    its boundary (a candidate on the residual-time ellipsoid or at zero
    residual, or a running weight sum at u times the total): such items are
    counted and each one's decision margin is bounded."""
    L = oracle.lib()
    med = dict(sigma_s=4.75, sigma_a=0.25, g=0.7)
    m = C.byref(oracle.medium(med))
    rng = np.random.default_rng(19)
    rows = []
    xe = np.array([0, 0, 1.5])
    for _ in range(4000):
        x = rng.uniform(-1, 1, 3)
        w = rng.normal(size=3)
        w /= np.linalg.norm(w)
        Cd = np.linalg.norm(xe - x)
        R_hi = Cd + rng.choice([rng.uniform(0, 0.3), rng.uniform(0, 20)])
        d_m = rng.choice([rng.uniform(0.01, 3), np.inf])
        rows.append([*x, *w, *xe, R_hi, d_m, ubits(int(rng.integers(32))), ubits(int(rng.integers(0, 2 ** 32))),
                     rng.random()])
    out, inp, ib = run(D, "ris", rows, med)
    errs, flips, n_ok = [], [], 0
    for o, r, rb in zip(out, inp, ib):
        row, eps = int(rb[11]), int(rb[12])
        d, fac, det = C.c_double(), C.c_double(), oracle.RisDetail()
        # the step is defined for a unit direction: the float input stands for w / |w|
        wu = r[3:6] / np.linalg.norm(r[3:6])
        okr = L.ref_ris_step_detail(m, 8, (C.c_double * 3)(*r[0:3]), (C.c_double * 3)(*wu),
                                    (C.c_double * 3)(*r[6:9]), r[9], r[10], row, eps, r[13], C.byref(d),
                                    C.byref(fac), C.byref(det), 0)
        same = okr == int(o[0]) and int(o[4]) == det.mask and (okr == 0 or int(o[3]) == det.sel)
        if not same:
            flips.append(min(det.valid_margin, det.pick_margin))
            continue
        n_ok += 1
        if okr:
            errs.append((abs(o[1] - d.value) / d.value, abs(o[2] - fac.value) / fac.value))
    errs = np.array(errs)
    print(f"RIS: {n_ok} agree ({len(errs)} with a selection), max rel. error d {errs[:, 0].max():.2e}, "
          f"factor {errs[:, 1].max():.2e}; {len(flips)} flipped, margins {sorted(flips)[-3:]}")
    assert len(errs) > 2000
    assert errs[:, 0].max() <= 1e-5 and errs[:, 1].max() <= 1e-5
    assert len(flips) <= 0.002 * len(rows)
    assert all(mg <= 1e-5 for mg in flips), flips


@pytest.mark.parametrize("n_cos", [32, 256])
def test_direction_sampling(D, oracle, n_cos):
    """EDA/HG mixture with its MIS weight (Section V-A, Eq. (19)) on a real
    table (the small box's 32 cos-bins, and the paper's 256).  Items whose
    discrete decisions agree (MIS branch, table row, cos-bin) match the
    oracle's direction to 1e-5 and the oracle's weight function at the
    sampled direction to 1e-5 relative, every one of them.  An item may
    decide otherwise only within FP32 rounding of a decision boundary (u0 at
    gamma, C/S or S at a table cell edge, a phase-sampled direction at a
    cos-bin edge): such items are counted and each one's margin is bounded."""
    L = oracle.lib()
    w = W.box_hg_small()
    med, dims = w["scene"]["medium"], dict(w["dims"], n_cos=n_cos)
    table = D.build_da_tables(med, dims)
    _, cdf = oracle.build_table(med, dims)
    torch.cuda.synchronize()
    rng = np.random.default_rng(20)
    rows = []
    xe = np.array([0, 0, 1.5])
    alpha = 0.5
    for _ in range(4000):
        x = rng.uniform(-1, 1, 3)
        wp = rng.normal(size=3)
        wp /= np.linalg.norm(wp)
        Cd = np.linalg.norm(xe - x)
        S = Cd * (1 + 10 ** rng.uniform(-3, 1))
        u = rng.integers(0, 2 ** 32, 4)
        rows.append([*x, *xe, *wp, S, *[ubits(int(v)) for v in u], 1.0, alpha])
    out, inp, ib = run(D, "direction", rows, med, table)
    mm, dd = C.byref(oracle.medium(med)), C.byref(oracle.dims(dims))
    cp = np.ascontiguousarray(cdf).ctypes.data_as(C.POINTER(C.c_float))
    v3 = lambda a: (C.c_double * 3)(*a)
    dir_err, wt_err, flips = [], [], []
    for o, r, rb in zip(out, inp, ib):
        u = [L.ref_u01(int(v)) for v in rb[10:14]]
        x, xe_, S = r[0:3], r[3:6], r[9]
        wp = r[6:9] / np.linalg.norm(r[6:9])
        wo, wt, eb, k = (C.c_double * 3)(), C.c_double(), C.c_int(), C.c_int()
        L.ref_sample_direction(mm, dd, cp, alpha, 1, v3(x), v3(xe_), v3(wp), S, (C.c_double * 4)(*u), wo,
                               C.byref(wt), C.byref(eb), C.byref(k), 0)
        Cd = float(np.linalg.norm(xe_ - x))
        row = L.ref_table_row(dd, Cd, S, 0)
        if int(o[4]) == eb.value and int(o[5]) == row and int(o[6]) == k.value:
            wg = o[0:3]
            dir_err.append(np.linalg.norm(wg - np.array(wo[:])))
            wr = L.ref_direction_weight(mm, dd, cp, alpha, 1, v3(x), v3(xe_), v3(wp), S, v3(wg / np.linalg.norm(wg)),
                                        k.value)
            wt_err.append(abs(o[3] - wr) / wr)
            continue
        # decision margins, from the oracle's FP64 quantities
        kappa = Cd / S
        gam = L.ref_gamma(kappa, alpha)
        cell = lambda t: abs(t - round(t))
        a = (xe_ - x) / Cd
        bin_pos = (np.dot(np.array(wo[:]), a) + 1) * 0.5 * n_cos
        flips.append(min(abs(u[0] - gam), cell(kappa * dims["n_cs"]), cell(S / dims["s_max"] * dims["n_s"]),
                         cell(bin_pos) if not eb.value else np.inf))
    dir_err, wt_err = np.array(dir_err), np.array(wt_err)
    print(f"direction ({n_cos} bins): {len(dir_err)} agree, max |w - w_ref| {dir_err.max():.2e}, "
          f"max rel. weight error {wt_err.max():.2e}; {len(flips)} flipped, margins {sorted(flips)[-3:]}")
    assert dir_err.max() <= 1e-5 and wt_err.max() <= 1e-5
    assert len(flips) <= 0.002 * len(rows)
    assert all(mg <= 1e-5 for mg in flips), flips


def test_connection_matches_oracle(D, oracle):
    """One elliptical connection (Section V-B, Eq. (20)-(22)): range test,
    sampled length sum, control vertex, phase function, transmittance and
    Jacobian together, against the oracle on the same float inputs, with
    truncated-exponential and uniform S, in the box and in an infinite
    medium.  General rays: whether the length-sum range is empty agrees
    except within 1e-5 (relative) of its ends, and the contribution agrees to
    2e-5 plus what FP32 rounding of the range's ends allows: an end set by
    R_lo or R_hi carries the rounding of C (a few 1e-7 C), i.e. 8e-7 C / W
    of a range of width W.  Rays aimed within 1e-4..1e-2 rad of an emitter
    beyond the boundary, with the range [C, S_exit) clipped by it to a few
    ulps of C and up: the contribution is proportional to S_exit - C, known
    to FP32 rounding of the direction to the emitter, so the bar adds
    1e-6 / theta (theta the angle, about 4 eps on |w - a| twice); a width
    formed as (C + (S_exit - C)) - C would carry half an ulp of C and miss
    it."""
    L = oracle.lib()
    med = W.box_hg()["scene"]["medium"]
    mm = C.byref(oracle.medium(med))
    box = oracle.geometry({"kind": 1, "lo": (-1, -1, -1), "hi": (1, 1, 1)})
    inf = oracle.geometry({"kind": 0})
    rng = np.random.default_rng(31)
    rows, kind = [], []

    def exit_dist(x, w):
        t = np.where(w > 0, (1 - x) / np.where(w > 0, w, 1), np.where(w < 0, (-1 - x) / np.where(w < 0, w, 1), np.inf))
        return float(t.min())

    for _ in range(3000):
        in_box = rng.uniform() < 0.7
        x = rng.uniform(-0.95, 0.95, 3)
        w = rng.normal(size=3)
        w /= np.linalg.norm(w)
        if in_box:
            d = rng.normal(size=3)
            xe = d / np.linalg.norm(d) * rng.uniform(1.8, 3.0)
        else:
            xe = rng.uniform(-1, 1, 3)
        Cd = np.linalg.norm(xe - x)
        R_lo = Cd * (1 + rng.uniform(-0.3, 0.5))
        R_hi = R_lo + 10 ** rng.uniform(-3, 0.5)
        dm = exit_dist(x, w) if in_box else np.inf
        rows.append([*x, *w, *xe, R_lo, R_hi, dm, rng.uniform(), float(rng.uniform() < 0.5), float(in_box)])
        kind.append(0)
    for theta in [1e-4, 3e-4, 1e-3, 3e-3, 1e-2]:
        for _ in range(200):
            x = rng.uniform(-0.9, 0.9, 3)
            d = rng.normal(size=3)
            xe = d / np.linalg.norm(d) * rng.uniform(1.8, 3.0)
            a = (xe - x) / np.linalg.norm(xe - x)
            n = np.cross(a, rng.normal(size=3))
            w = a * math.cos(theta) + n / np.linalg.norm(n) * math.sin(theta)
            Cd = np.linalg.norm(xe - x)
            rows.append([*x, *w, *xe, Cd * 0.9, Cd * 1.5, exit_dist(x, w), rng.uniform(), float(rng.uniform() < 0.5), 1.0])
            kind.append(1)
    rows = [[F32(v) for v in r] for r in rows]
    kind = np.array(kind)
    out, inp, _ = run(D, "connect", rows, med)
    v3 = lambda a: (C.c_double * 3)(*a)
    n_cmp, flips, worst = 0, [], []
    for o, r, k in zip(out, inp, kind):
        x, w32, xe = r[0:3], r[3:6], r[6:9]
        w = w32 / np.linalg.norm(w32)
        R_lo, R_hi, dm, u, texp, in_box = r[9], r[10], r[11], r[12], int(r[13]), r[14] != 0
        t, rin, mu, re = C.c_double(), C.c_double(), C.c_double(), C.c_int()
        c = L.ref_connect(mm, C.byref(box if in_box else inf), v3(x), v3(w), v3(xe), R_lo, R_hi,
                          dm if in_box else np.inf, u, texp, C.byref(t), C.byref(rin), C.byref(mu), C.byref(re))
        Cd = float(np.linalg.norm(xe - x))
        s_exit = L.ref_exit_length(v3(x), v3(w), v3(xe), dm) if in_box else np.inf
        lo_end, hi_end = max(R_lo, Cd), min(R_hi, s_exit)
        if int(o[4]) != re.value:
            flips.append(abs(hi_end - lo_end) / Cd)
            continue
        if not re.value:
            assert o[0] == 0.0
            continue
        width = hi_end - lo_end
        r_set = R_lo > Cd or R_hi < s_exit          # an end of the range set by R_lo or R_hi
        theta = float(np.linalg.norm(w - (xe - x) / Cd))
        bar = 2e-5 + (8e-7 * Cd / width if r_set else 0.0) + 1e-6 / theta
        err = abs(o[0] - c) / c
        worst.append(err / bar)
        n_cmp += 1
        assert err <= bar, (k, r, o[0], c, err, bar)
    print(f"connections: {n_cmp} compared (max error / bar {max(worst):.3f}), {len(flips)} range flips "
          f"(margins {sorted(flips)[-3:]})")
    assert n_cmp >= 2000 and np.sum(kind == 1) >= 1000
    assert len(flips) <= 5 and all(f <= 1e-5 for f in flips)


def test_direction_near_the_emitter_axis(D, oracle):
    """EDA directions in the table's last cos-bin, within 4e-9..2e-4 of
    cos(theta) = 1 about the axis to the emitter (alpha = 0, so every
    direction comes from the table; u3 = 1 - m 2^-24).  Such rays put the
    connection's control vertex next to the emitter, where the contribution
    goes as the inverse squared distance, so the angle matters, not just the
    vector: |w - a|^2 = 2 (1 - cos theta) from the GPU's FP32 direction
    (evaluated in FP64) must equal the oracle's to what FP32 rounding of the
    components of w and a allows (each within 2^-24 of its value, so |w - a|
    within about 1.04e-7: a relative bar of 4.2e-7 / |w - a|, twice that
    bound, plus 1e-5).  A cos(theta) rounded to FP32 before sin(theta) is
    formed moves in steps of 2^-24 and fails this by orders of magnitude."""
    L = oracle.lib()
    w = W.box_hg_small()
    med, dims = w["scene"]["medium"], w["dims"]
    n_cos = dims["n_cos"]
    table = D.build_da_tables(med, dims)
    _, cdf = oracle.build_table(med, dims)
    torch.cuda.synchronize()
    rng = np.random.default_rng(23)
    rows = []
    xe = np.array([0, 0, 1.5])
    for _ in range(2000):
        x = rng.uniform(-1, 1, 3)
        wp = rng.normal(size=3)
        wp /= np.linalg.norm(wp)
        Cd = np.linalg.norm(xe - x)
        S = Cd * (1 + 10 ** rng.uniform(-3, 1))
        m = int(2 ** rng.uniform(0, 16))
        u = [0, 0xFFFFFF00, int(rng.integers(0, 2 ** 32)), ((1 << 24) - m) << 8]
        rows.append([*x, *xe, *wp, S, *[ubits(v) for v in u], 1.0, 0.0])
    out, inp, ib = run(D, "direction", rows, med, table)
    mm, dd = C.byref(oracle.medium(med)), C.byref(oracle.dims(dims))
    cp = np.ascontiguousarray(cdf).ctypes.data_as(C.POINTER(C.c_float))
    v3 = lambda a: (C.c_double * 3)(*a)
    rel, bar, n_last = [], [], 0
    for o, r, rb in zip(out, inp, ib):
        u = [L.ref_u01(int(v)) for v in rb[10:14]]
        x, xe_, S = r[0:3], r[3:6], r[9]
        wp = r[6:9] / np.linalg.norm(r[6:9])
        wo, wt, eb, k = (C.c_double * 3)(), C.c_double(), C.c_int(), C.c_int()
        L.ref_sample_direction(mm, dd, cp, 0.0, 1, v3(x), v3(xe_), v3(wp), S, (C.c_double * 4)(*u), wo,
                               C.byref(wt), C.byref(eb), C.byref(k), 0)
        assert eb.value == 1 and int(o[4]) == 1
        if k.value != n_cos - 1 or int(o[6]) != k.value:
            continue
        n_last += 1
        a = (xe_ - x) / np.linalg.norm(xe_ - x)
        d_o = float(np.sum((np.array(wo[:]) - a) ** 2))
        d_g = float(np.sum((o[0:3] - a) ** 2))
        rel.append(abs(d_g - d_o) / d_o)
        bar.append(4.2e-7 / math.sqrt(d_o) + 1e-5)
    rel, bar = np.array(rel), np.array(bar)
    print(f"near-axis EDA directions: {n_last} in the last cos-bin, max relative error of |w - a|^2 "
          f"{rel.max():.2e}, max error / bar {np.max(rel / bar):.3f}")
    assert n_last >= 1000
    assert np.all(rel <= bar)


TABLE_CASES = [("box_hg_small", None), ("infinite_point", None), ("box_hg", None),
               ("box_hg", {"n_cs": 16, "n_s": 16, "n_cos": 256, "s_max": 40.0}),
               ("box_hg", {"n_cs": 8, "n_s": 8, "n_cos": 1024, "s_max": 40.0}),
               ("box_hg", {"n_cs": 3, "n_s": 5, "n_cos": 7, "s_max": 13.0})]


@pytest.mark.parametrize("wname,dims_", TABLE_CASES,
                         ids=[f"{c[0]}-{'own' if c[1] is None else c[1]['n_cos']}" for c in TABLE_CASES])
def test_table_matches_oracle(D, oracle, wname, dims_):
    """The elliptical-DA table against the oracle's: the workloads' own
    dimensions, the paper's 256 cos-bins, the largest allowed count (1024,
    more bins than a wave has lanes) and a ragged odd-sized table."""
    for w in [getattr(W, wname)()]:
        med, dims = w["scene"]["medium"], dims_ or w["dims"]
        t = D.build_da_tables(med, dims)
        torch.cuda.synchronize()
        _, cdf = oracle.build_table(med, dims)
        got = t.cdf.cpu().numpy()
        assert got.shape == cdf.shape
        assert np.max(np.abs(got.astype(np.float64) - cdf)) <= 1e-6
        assert np.all(got[..., 0] == 0) and np.all(got[..., -1] == 1)


def test_hardware_transcendentals(D):
    """Accuracy of the transcendental-unit instructions the kernels rely on,
    over the argument ranges they see: relative error of rcp / rsqrt, absolute
    error of log2 (never used on arguments near 1 where only absolute accuracy
    would be available), relative error of exp2 on (-127, 0], absolute error
    of sin/cos of 2 pi u on [0, 1)."""
    rng = np.random.default_rng(21)
    pos = np.concatenate([10 ** rng.uniform(-6, 6, 20000), rng.uniform(0.5, 2, 20000)]).astype(F32)
    out, inp, _ = run(D, "math", [[x] for x in pos])
    x = inp[:, 0]
    rel = lambda a, b: np.max(np.abs(a / b - 1))
    print("rcp", rel(out[:, 0], 1 / x), "rsq", rel(out[:, 1], 1 / np.sqrt(x)),
          "log2 abs", np.max(np.abs(out[:, 2] - np.log2(x))))
    assert rel(out[:, 0], 1 / x) < 3e-7
    assert rel(out[:, 1], 1 / np.sqrt(x)) < 3e-7
    assert np.max(np.abs(out[:, 2] - np.log2(x))) < 2e-6
    far = np.abs(np.log2(x)) > 0.25
    assert np.max(np.abs(out[far, 2] / np.log2(x[far]) - 1)) < 2e-6
    neg = (-rng.uniform(0, 126, 20000)).astype(F32)
    out, inp, _ = run(D, "math", [[x] for x in neg])
    assert rel(out[:, 3], 2.0 ** inp[:, 0]) < 2e-6
    u = rng.random(20000).astype(F32)
    out, inp, _ = run(D, "math", [[x] for x in u])
    assert np.max(np.abs(out[:, 4] - np.sin(2 * np.pi * inp[:, 0]))) < 2e-6
    assert np.max(np.abs(out[:, 5] - np.cos(2 * np.pi * inp[:, 0]))) < 2e-6
