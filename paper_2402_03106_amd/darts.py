"""Python binding of libdarts (include/darts.h): argument marshalling only.

Every step of the path runs in the HIP kernels of ``csrc/darts.hip``; torch
provides device memory and the stream.  The functions keep the C names:
``table_bytes``, ``build_da_tables``, ``render_transient``, ``render_paths``,
``render_transient_backward``, ``debug_pointwise``, ``last_error``.  Scenes
are the plain dictionaries of ``paper_2402_03106_amd.workloads``.

There is no CPU fallback: if ``libdarts.so`` is missing or no GPU is visible
the calls raise.
"""
from __future__ import annotations

import ctypes as C
import math
import os
from dataclasses import dataclass

import torch

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libdarts.so")

OK, ERR_INVALID_ARG, ERR_DEVICE, ERR_UNSUPPORTED, ERR_TABLE_MISMATCH = 0, -1, -2, -3, -4
RIS_DIST, EDA_DIR, ELL_TEXP, ELL_UNIFORM, DIRECT_REUSE = 0x1, 0x2, 0x4, 0x8, 0x10
MODES = {
    "darts": RIS_DIST | EDA_DIR | ELL_TEXP,
    "uniform": ELL_UNIFORM,
    "vanilla": DIRECT_REUSE,
    "da_only": RIS_DIST | ELL_UNIFORM,
    "eda_only": EDA_DIR | ELL_TEXP,
    "texp_only": ELL_TEXP,
}
MAX_EMITTERS = 8
ST_NAMES = ["paths", "vertices", "connections", "early_exit", "medium_exit", "ris_all_invalid",
            "eda_branch", "truncated", "zero_paths", "setup_exit", "samples", "rejected"]
ST_COUNT = 16
PW_IN, PW_OUT = 16, 8
PW = {name: i for i, name in enumerate(
    ["philox", "hg_pdf", "hg_sample", "da_logphi", "texp", "ellipse", "sobol", "onb", "box_exit",
     "ris", "direction", "math", "exit_length", "connect"])}


class DartsError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libdarts error {code}: {msg}")
        self.code = code


class _Medium(C.Structure):
    _fields_ = [("sigma_s", C.c_double), ("sigma_a", C.c_double), ("g", C.c_double)]


class _Emitter(C.Structure):
    _fields_ = [("pos", C.c_float * 3), ("start", C.c_float), ("power", C.c_float)]


class _Sensor(C.Structure):
    _fields_ = [("kind", C.c_int), ("origin", C.c_float * 3), ("dir", C.c_float * 3),
                ("du", C.c_float * 3), ("dv", C.c_float * 3), ("width", C.c_int), ("height", C.c_int)]


class _Geometry(C.Structure):
    _fields_ = [("kind", C.c_int), ("lo", C.c_float * 3), ("hi", C.c_float * 3), ("floor_albedo", C.c_float)]


class _Bins(C.Structure):
    _fields_ = [("l_lo", C.c_float), ("l_hi", C.c_float), ("n_bins", C.c_int)]


class _Scene(C.Structure):
    _fields_ = [("medium", _Medium), ("geom", _Geometry), ("emitters", C.POINTER(_Emitter)),
                ("n_emitters", C.c_int), ("sensor", _Sensor), ("bins", _Bins), ("response_dev", C.c_void_p)]


class _Dims(C.Structure):
    _fields_ = [("n_cs", C.c_int), ("n_s", C.c_int), ("n_cos", C.c_int), ("s_max", C.c_float)]


class _Table(C.Structure):
    _fields_ = [("medium", _Medium), ("dims", _Dims), ("cdf_dev", C.c_void_p)]


class _Params(C.Structure):
    _fields_ = [("n_paths", C.c_uint64), ("path_offset", C.c_uint64), ("seed", C.c_uint64),
                ("max_bounces", C.c_int), ("n_ris", C.c_int), ("alpha", C.c_float), ("flags", C.c_uint)]


class _BatchItem(C.Structure):
    _fields_ = [("scene", _Scene), ("params", _Params), ("table", C.POINTER(_Table))]


class _BatchPlan(C.Structure):
    _fields_ = [("order", C.c_int), ("block_threads", C.c_int), ("waves_per_cu", C.c_int),
                ("unit_paths", C.c_int64)]


_lib = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
        L = C.CDLL(LIB_PATH)
        vp, i64 = C.c_void_p, C.c_int64
        L.darts_last_error.restype = C.c_char_p
        L.darts_abi_version.restype = C.c_int
        L.darts_table_bytes.argtypes = [C.POINTER(_Dims), C.POINTER(C.c_size_t)]
        L.darts_build_da_tables.argtypes = [C.POINTER(_Medium), C.POINTER(_Dims), vp, vp]
        L.darts_render_transient.argtypes = [C.POINTER(_Scene), C.POINTER(_Params), C.POINTER(_Table),
                                             vp, vp, vp, vp, vp]
        L.darts_render_paths.argtypes = [C.POINTER(_Scene), C.POINTER(_Params), C.POINTER(_Table), vp, vp]
        L.darts_render_transient_backward.argtypes = [C.POINTER(_Scene), C.POINTER(_Params), C.POINTER(_Table),
                                                      vp, vp, vp]
        L.darts_render_transient_tangent.argtypes = [C.POINTER(_Scene), C.POINTER(_Params), C.POINTER(_Table),
                                                     vp, vp]
        L.darts_debug_pointwise.argtypes = [C.c_int, vp, vp, i64, C.POINTER(_Medium), C.POINTER(_Table), vp]
        L.darts_set_target_waves.argtypes = [i64]
        L.darts_set_ids_max_reps.argtypes = [i64]
        L.darts_set_vanilla_privatised.argtypes = [C.c_int]
        L.darts_response_bytes.argtypes = [C.c_int, C.POINTER(C.c_size_t)]
        L.darts_build_response.argtypes = [C.POINTER(C.c_float), C.c_int, vp, vp]
        pp = C.POINTER(C.c_void_p)
        L.darts_batch_default_plan.argtypes = [C.POINTER(_BatchPlan)]
        L.darts_batch_create.argtypes = [C.POINTER(_BatchItem), C.c_int, C.POINTER(_BatchPlan), pp]
        L.darts_batch_image_offsets.argtypes = [vp, C.POINTER(C.c_int64)]
        L.darts_batch_set_plan.argtypes = [vp, C.POINTER(_BatchPlan)]
        L.darts_batch_get_plan.argtypes = [vp, C.POINTER(_BatchPlan)]
        L.darts_batch_render.argtypes = [vp, vp, vp, vp]
        L.darts_batch_graph_launch.argtypes = [vp, vp, vp, vp]
        L.darts_batch_autotune.argtypes = [vp, vp, vp, C.c_int, C.POINTER(_BatchPlan), C.POINTER(C.c_double), vp]
        L.darts_batch_destroy.argtypes = [vp]
        L.darts_batch_render_noalloc.argtypes = [C.POINTER(_BatchItem), C.c_int, C.POINTER(_BatchPlan), vp, vp,
                                                 C.c_int64, vp]
        _lib = L
    return _lib


def last_error() -> str:
    return lib().darts_last_error().decode()


def _check(rc: int):
    if rc != OK:
        raise DartsError(rc, last_error())


def _stream(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("device tensor expected")
    if not t.is_contiguous():
        raise ValueError("contiguous tensor expected")
    return C.c_void_p(t.data_ptr())


def _hold(t: torch.Tensor, stream) -> torch.Tensor:
    """A contiguous tensor whose memory stays reserved for work queued on
    `stream` (the caching allocator otherwise only orders reuse against the
    stream the tensor was allocated on)."""
    c = t.contiguous()
    if stream is not None and stream != torch.cuda.current_stream(c.device):
        c.record_stream(stream)
    return c


def _f3(v):
    return (C.c_float * 3)(*[float(x) for x in v])


def medium(m: dict) -> _Medium:
    return _Medium(float(m["sigma_s"]), float(m["sigma_a"]), float(m["g"]))


def dims(d: dict) -> _Dims:
    return _Dims(int(d["n_cs"]), int(d["n_s"]), int(d["n_cos"]), float(d["s_max"]))


class _SceneHolder:
    def __init__(self, sc: dict, response=None):
        ems = sc["emitters"]
        self.em = (_Emitter * len(ems))(*[_Emitter(_f3(e["pos"]), float(e.get("start", 0.0)),
                                                   float(e.get("power", 1.0))) for e in ems])
        s, g, b = sc["sensor"], sc["geometry"], sc["bins"]
        self.c = _Scene(medium(sc["medium"]),
                        _Geometry(int(g["kind"]), _f3(g.get("lo", (0, 0, 0))), _f3(g.get("hi", (0, 0, 0))),
                                  float(g.get("floor_albedo", 0.0))),
                        C.cast(self.em, C.POINTER(_Emitter)), len(ems),
                        _Sensor(int(s["kind"]), _f3(s["origin"]), _f3(s.get("dir", (0, 0, -1))),
                                _f3(s.get("du", (0, 0, 0))), _f3(s.get("dv", (0, 0, 0))),
                                int(s.get("width", 1)), int(s.get("height", 1))),
                        _Bins(float(b["l_lo"]), float(b["l_hi"]), int(b["n_bins"])),
                        C.c_void_p(response.table.data_ptr()) if response is not None else None)
        if response is not None and response.n_bins != int(b["n_bins"]):
            raise ValueError("the response table has a different number of segments than the scene's bins")


def params(p: dict, mode) -> _Params:
    flags = MODES[mode] if isinstance(mode, str) else int(mode)
    return _Params(int(p["n_paths"]), int(p.get("path_offset", 0)), int(p["seed"]), int(p["max_bounces"]),
                   int(p.get("n_ris", 8)), float(p.get("alpha", 0.5)), flags)


def image_shape(sc: dict, response=None):
    """[n_bins, H, W], or [H, W] with a sensor response."""
    s = sc["sensor"]
    if response is not None:
        return (int(s.get("height", 1)), int(s.get("width", 1)))
    return (int(sc["bins"]["n_bins"]), int(s.get("height", 1)), int(s.get("width", 1)))


@dataclass
class Response:
    """A built sensor-response table (device float[2 n_bins + 1]) and the W
    values it holds."""
    table: torch.Tensor
    w: tuple

    @property
    def n_bins(self) -> int:
        return len(self.w)


def build_response(w, stream=None, device="cuda") -> Response:
    """Device table of a piecewise-constant sensor response W over the
    scene's bins (darts_build_response)."""
    wf = [float(x) for x in w]
    n = len(wf)
    nbytes = C.c_size_t()
    _check(lib().darts_response_bytes(n, C.byref(nbytes)))
    out = torch.empty(int(nbytes.value) // 4, dtype=torch.float32, device=device)
    arr = (C.c_float * n)(*wf)
    _check(lib().darts_build_response(arr, n, _ptr(out), _stream(stream)))
    return Response(out, tuple(C.c_float(x).value for x in wf))


# --------------------------------------------------------------------------
# Tables
# --------------------------------------------------------------------------
@dataclass
class Table:
    """A built direction table: device float tensor [n_cs, n_s, n_cos + 1]
    plus the medium and dims it was built for."""
    cdf: torch.Tensor
    medium: dict
    dims: dict

    def c_struct(self) -> _Table:
        return _Table(medium(self.medium), dims(self.dims), C.c_void_p(self.cdf.data_ptr()))


def table_bytes(d: dict) -> int:
    n = C.c_size_t()
    _check(lib().darts_table_bytes(C.byref(dims(d)), C.byref(n)))
    return int(n.value)


def build_da_tables(med: dict, d: dict, out: torch.Tensor | None = None, stream=None,
                    device="cuda") -> Table:
    nbytes = table_bytes(d)
    shape = (int(d["n_cs"]), int(d["n_s"]), int(d["n_cos"]) + 1)
    if out is None:
        out = torch.empty(shape, dtype=torch.float32, device=device)
    if out.numel() * 4 != nbytes or out.dtype != torch.float32:
        raise ValueError("table tensor has the wrong size or dtype")
    _check(lib().darts_build_da_tables(C.byref(medium(med)), C.byref(dims(d)), _ptr(out), _stream(stream)))
    return Table(out, dict(med), dict(d))


# --------------------------------------------------------------------------
# Render
# --------------------------------------------------------------------------
def render_transient(sc: dict, p: dict, mode, table: Table | None = None, image_hi=None, image_lo=None,
                     image_m2=None, stats=None, want_m2: bool = False, want_stats: bool = False,
                     stream=None, device="cuda", response: Response | None = None):
    """Accumulate raw sums into (image_hi, image_lo[, image_m2]); allocates
    zeroed outputs when none are given.  Returns (hi, lo, m2, stats).  With a
    sensor response the images are per pixel [H, W]."""
    shape = image_shape(sc, response)
    if image_hi is None:
        image_hi = torch.zeros(shape, dtype=torch.float32, device=device)
    if image_lo is None:
        image_lo = torch.zeros(shape, dtype=torch.float32, device=device)
    if want_m2 and image_m2 is None:
        image_m2 = torch.zeros(shape, dtype=torch.float32, device=device)
    if want_stats and stats is None:
        stats = torch.zeros(ST_COUNT, dtype=torch.int64, device=device)
    for t in (image_hi, image_lo, image_m2):
        if t is not None and (tuple(t.shape) != shape or t.dtype != torch.float32):
            raise ValueError(f"image tensors must be float32 {shape}")
    h = _SceneHolder(sc, response)
    tb = C.byref(table.c_struct()) if table is not None else None
    _check(lib().darts_render_transient(C.byref(h.c), C.byref(params(p, mode)), tb, _ptr(image_hi),
                                        _ptr(image_lo), _ptr(image_m2), _ptr(stats), _stream(stream)))
    return image_hi, image_lo, image_m2, stats


def render_paths(sc: dict, p: dict, mode, table: Table | None = None, out=None, stream=None, device="cuda",
                 response: Response | None = None):
    n = int(p["n_paths"])
    if out is None:
        out = torch.empty(n, dtype=torch.float32, device=device)
    h = _SceneHolder(sc, response)
    tb = C.byref(table.c_struct()) if table is not None else None
    _check(lib().darts_render_paths(C.byref(h.c), C.byref(params(p, mode)), tb, _ptr(out), _stream(stream)))
    return out


def render_transient_backward(sc: dict, p: dict, mode, table: Table | None, grad_image: torch.Tensor,
                              grad_out=None, stream=None, response: Response | None = None):
    if grad_out is None:
        grad_out = torch.zeros(3, dtype=torch.float64, device=grad_image.device)
    h = _SceneHolder(sc, response)
    tb = C.byref(table.c_struct()) if table is not None else None
    gi = _hold(grad_image, stream)
    _check(lib().darts_render_transient_backward(C.byref(h.c), C.byref(params(p, mode)), tb,
                                                 _ptr(gi), _ptr(grad_out), _stream(stream)))
    return grad_out


def render_transient_tangent(sc: dict, p: dict, mode, table: Table | None, out=None, stream=None,
                             device="cuda", response: Response | None = None) -> torch.Tensor:
    """Per-cell derivative images of the raw sums, [3, *image_shape] for
    (sigma_s, sigma_a, g) (darts_render_transient_tangent), accumulated into
    `out` (zeros by default)."""
    shape = (3,) + tuple(image_shape(sc, response))
    if out is None:
        out = torch.zeros(shape, dtype=torch.float32, device=device)
    h = _SceneHolder(sc, response)
    tb = C.byref(table.c_struct()) if table is not None else None
    _check(lib().darts_render_transient_tangent(C.byref(h.c), C.byref(params(p, mode)), tb, _ptr(out),
                                                _stream(stream)))
    return out


def debug_pointwise(fn: str, inputs: torch.Tensor, med: dict | None = None, table: Table | None = None,
                    stream=None) -> torch.Tensor:
    if inputs.dtype != torch.float32 or inputs.dim() != 2 or inputs.shape[1] != PW_IN:
        raise ValueError(f"inputs must be float32 [n, {PW_IN}]")
    out = torch.zeros((inputs.shape[0], PW_OUT), dtype=torch.float32, device=inputs.device)
    m = C.byref(medium(med)) if med is not None else None
    tb = C.byref(table.c_struct()) if table is not None else None
    x = _hold(inputs, stream)
    _check(lib().darts_debug_pointwise(PW[fn], _ptr(x), _ptr(out), inputs.shape[0], m, tb, _stream(stream)))
    return out


# --------------------------------------------------------------------------
# Batched persistent render
# --------------------------------------------------------------------------
BATCH_ORDERS = {"tiles": 0, "ids": 1}


def _plan_dict(pl: _BatchPlan) -> dict:
    return {"order": {v: k for k, v in BATCH_ORDERS.items()}[pl.order], "block_threads": pl.block_threads,
            "waves_per_cu": pl.waves_per_cu, "unit_paths": int(pl.unit_paths)}


def _plan_struct(plan: dict | None) -> _BatchPlan:
    pl = _BatchPlan()
    _check(lib().darts_batch_default_plan(C.byref(pl)))
    if plan:
        if "order" in plan:
            pl.order = BATCH_ORDERS[plan["order"]] if isinstance(plan["order"], str) else int(plan["order"])
        for k in ("block_threads", "waves_per_cu", "unit_paths"):
            if k in plan:
                setattr(pl, k, int(plan[k]))
    return pl


class _BatchItems:
    """The C array of batch items for a list of (scene dict, params dict,
    mode, Table or None[, Response]) with everything it points to kept
    alive."""

    def __init__(self, items):
        items = [tuple(it) + (None,) * (5 - len(it)) for it in items]   # (scene, params, mode, table[, response])
        self.holders = [_SceneHolder(it[0], it[4]) for it in items]
        self.tables = [it[3] for it in items]
        self.responses = [it[4] for it in items]
        self.tstructs = [t.c_struct() if t is not None else None for t in self.tables]
        self.arr = (_BatchItem * len(items))()
        for i, (sc, p, mode, t, _) in enumerate(items):
            self.arr[i].scene = self.holders[i].c
            self.arr[i].params = params(p, mode)
            self.arr[i].table = C.pointer(self.tstructs[i]) if t is not None else None
        self.shapes = [image_shape(it[0], it[4]) for it in items]
        self.offsets = [0]
        for sh in self.shapes:
            self.offsets.append(self.offsets[-1] + math.prod(sh))


class Batch:
    """Many scenes rendered by one persistent launch (darts_batch_*).  items:
    list of (scene dict, params dict, mode, Table or None).  The tables must
    stay alive as long as the batch; the Batch keeps references to them."""

    def __init__(self, items, plan: dict | None = None):
        self._h = C.c_void_p()
        self._items = _BatchItems(items)
        self.shapes = self._items.shapes
        pl = _plan_struct(plan)
        _check(lib().darts_batch_create(self._items.arr, len(self.shapes), C.byref(pl), C.byref(self._h)))
        offs = (C.c_int64 * (len(self.shapes) + 1))()
        _check(lib().darts_batch_image_offsets(self._h, offs))
        self.offsets = [int(x) for x in offs]

    @property
    def numel(self) -> int:
        return self.offsets[-1]

    def images(self, flat: torch.Tensor):
        """Per-scene views [n_bins, height, width] of a flat batch image."""
        return [flat[self.offsets[i]:self.offsets[i + 1]].view(self.shapes[i]) for i in range(len(self.shapes))]

    def empty(self, device="cuda"):
        z = lambda: torch.zeros(self.numel, dtype=torch.float32, device=device)
        return z(), z()

    def _out(self, hi, lo):
        for t in (hi, lo):
            if t is None or t.dtype != torch.float32 or t.numel() != self.numel:
                raise ValueError(f"batch images must be float32 with {self.numel} elements")
        return _ptr(hi), _ptr(lo)

    def render(self, hi, lo, stream=None):
        """One launch accumulating into (hi, lo)."""
        _check(lib().darts_batch_render(self._h, *self._out(hi, lo), _stream(stream)))
        return hi, lo

    def graph_launch(self, hi, lo, stream=None):
        """Clear (hi, lo) and render, as one captured graph."""
        _check(lib().darts_batch_graph_launch(self._h, *self._out(hi, lo), _stream(stream)))
        return hi, lo

    def autotune(self, hi, lo, reps: int = 2, stream=None):
        pl, ms = _BatchPlan(), C.c_double()
        _check(lib().darts_batch_autotune(self._h, *self._out(hi, lo), int(reps), C.byref(pl), C.byref(ms),
                                          _stream(stream)))
        return _plan_dict(pl), float(ms.value)

    @property
    def plan(self) -> dict:
        pl = _BatchPlan()
        _check(lib().darts_batch_get_plan(self._h, C.byref(pl)))
        return _plan_dict(pl)

    @plan.setter
    def plan(self, plan: dict):
        _check(lib().darts_batch_set_plan(self._h, C.byref(_plan_struct(plan))))

    def close(self):
        if self._h:
            lib().darts_batch_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch_render_noalloc(items, hi: torch.Tensor, lo: torch.Tensor, plan: dict | None = None, stream=None):
    """darts_batch_render_noalloc: render the batch `items` (as for Batch)
    in one call that allocates no memory, accumulating into the flat images
    (hi, lo) (float32, at least as many elements as the scenes' images
    together).  Returns the per-scene image offsets."""
    its = _BatchItems(items)
    for t in (hi, lo):
        if t is None or t.dtype != torch.float32:
            raise ValueError("batch images must be float32")
    n = min(hi.numel(), lo.numel())
    _check(lib().darts_batch_render_noalloc(its.arr, len(its.shapes), C.byref(_plan_struct(plan)), _ptr(hi),
                                            _ptr(lo), n, _stream(stream)))
    return its.offsets


def set_ids_max_reps(n: int):
    """Tuning knob: renders whose cells hold at most n repetitions take
    consecutive path ids per wave instead of tiles of cells (-1: never)."""
    _check(lib().darts_set_ids_max_reps(int(n)))


def set_vanilla_privatised(on: bool):
    """Tuning knob: vanilla renders histogram per pixel in LDS when it fits
    (default True); False: a global atomic pair per contribution."""
    _check(lib().darts_set_vanilla_privatised(1 if on else 0))


def set_target_waves(n: int):
    """Tuning knob: the number of waves a tile-decomposed render aims for
    (default 65536); results change only in the order of the additions."""
    _check(lib().darts_set_target_waves(int(n)))


def stats_dict(stats: torch.Tensor) -> dict:
    s = stats.cpu().tolist()
    return {k: int(s[i]) for i, k in enumerate(ST_NAMES)}


def paths_per_cell(sc: dict, p: dict, mode, response: Response | None = None) -> torch.Tensor:
    """Paths mapped to each cell by the stratified map (path id i lands in
    cell i mod n_cells); vanilla reuses a path for all bins of its pixel.
    With a sensor response the cells are the pixels."""
    shape = image_shape(sc, response)
    if response is not None:
        npix = shape[0] * shape[1]
        n, off = int(p["n_paths"]), int(p.get("path_offset", 0))
        ids = torch.arange(npix, dtype=torch.int64)
        first = (ids - off) % npix
        cnt = torch.where(first < n, (n - 1 - first) // npix + 1, torch.zeros_like(first)).to(torch.float64)
        return cnt.reshape(shape)
    nc = shape[0] * shape[1] * shape[2]
    n, off = int(p["n_paths"]), int(p.get("path_offset", 0))
    ids = torch.arange(nc, dtype=torch.int64)
    first = (ids - off) % nc
    cnt = torch.where(first < n, (n - 1 - first) // nc + 1, torch.zeros_like(first)).to(torch.float64)
    cnt = cnt.reshape(shape)
    if (MODES[mode] if isinstance(mode, str) else int(mode)) & DIRECT_REUSE:
        cnt = cnt.sum(0, keepdim=True).expand(shape).clone()
    return cnt


# --------------------------------------------------------------------------
# Differentiable rendering
# --------------------------------------------------------------------------
class TransientRender(torch.autograd.Function):
    """Per-cell estimates I(theta) (raw sums / paths per cell) of a render as a
    differentiable function of theta = (sigma_s, sigma_a, g).  The backward
    pass replays the same paths (same ids, seed and tables) through
    darts_render_transient_backward; nothing is stored between the passes
    except the table and the per-cell path counts."""

    @staticmethod
    def forward(ctx, theta, scene, params_, mode, dims_):
        vals = [float(v) for v in theta.detach().cpu().tolist()]
        med = {"sigma_s": vals[0], "sigma_a": vals[1], "g": vals[2]}
        sc = dict(scene, medium=med)
        flags = MODES[mode] if isinstance(mode, str) else int(mode)
        table = build_da_tables(med, dims_) if flags & EDA_DIR else None
        hi, lo, _, _ = render_transient(sc, params_, mode, table)
        n = paths_per_cell(sc, params_, mode).to(hi.device)
        img = (hi.double() + lo.double()) / n.clamp(min=1)
        ctx.sc, ctx.params, ctx.mode, ctx.table = sc, params_, mode, table
        ctx.save_for_backward(n, theta)
        return img

    @staticmethod
    def backward(ctx, grad_img):
        n, theta = ctx.saved_tensors
        grad_raw = (grad_img / n.clamp(min=1)).float().contiguous()
        g = render_transient_backward(ctx.sc, ctx.params, ctx.mode, ctx.table, grad_raw)
        return g.to(device=theta.device, dtype=theta.dtype), None, None, None, None


def transient_image(theta: torch.Tensor, scene: dict, params_: dict, mode, dims_: dict) -> torch.Tensor:
    """Differentiable per-cell image (float64, [n_bins, H, W]) of the medium
    theta = tensor([sigma_s, sigma_a, g])."""
    return TransientRender.apply(theta, scene, params_, mode, dims_)
