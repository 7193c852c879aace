"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every function include/darts.h declares, and rejects bad arguments before
touching the device."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "darts.h")


@pytest.fixture(scope="module")
def D():
    from paper_2402_03106_amd import build as B
    from paper_2402_03106_amd import darts
    if not os.path.exists(darts.LIB_PATH):
        B.build_library()
    darts.lib()
    return darts


def declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:int|const char \*)\s*(darts_\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ["darts_build_da_tables", "darts_render_transient", "darts_render_transient_backward",
                     "darts_table_bytes", "darts_last_error"]:
        assert required in names


def test_library_exports_every_declared_symbol(D):
    L = D.lib()
    for name in declared_functions():
        assert hasattr(L, name), name
    assert L.darts_abi_version() == 2


def test_library_has_no_torch_dependency(D):
    """The boundary is plain C: the shared library must not link torch."""
    maps = open(f"/proc/{os.getpid()}/maps").read()
    assert D.LIB_PATH in maps, [l for l in maps.splitlines() if "darts" in l]
    import subprocess
    out = subprocess.run(["ldd", D.LIB_PATH], capture_output=True, text=True).stdout
    # library names only: the load addresses ldd prints are random hex
    names = [ln.split()[0] for ln in out.splitlines() if ln.strip()]
    assert not [n for n in names if "torch" in n or n.startswith("libc10")], names


def test_pointwise_ids_match_header(D):
    """The binding's diagnostic ids follow the header's enum order."""
    src = open(HEADER).read()
    block = re.search(r"enum\s*\{([^}]*DARTS_PW_COUNT[^}]*)\}", src, flags=re.S).group(1)
    block = re.sub(r"/\*.*?\*/", "", block, flags=re.S)
    names = re.findall(r"DARTS_PW_(\w+)", block)
    assert names[-1] == "COUNT"
    assert [n.lower() for n in names[:-1]] == sorted(D.PW, key=D.PW.get)


def test_table_bytes(D):
    assert D.table_bytes(dict(n_cs=64, n_s=64, n_cos=32, s_max=40.0)) == 64 * 64 * 33 * 4
    for bad in [dict(n_cs=0, n_s=4, n_cos=4, s_max=1.0), dict(n_cs=4, n_s=4, n_cos=4, s_max=0.0),
                dict(n_cs=4, n_s=4, n_cos=2048, s_max=1.0)]:
        with pytest.raises(D.DartsError) as e:
            D.table_bytes(bad)
        assert e.value.code == D.ERR_INVALID_ARG
    L = D.lib()
    assert L.darts_table_bytes(C.byref(D.dims(dict(n_cs=1, n_s=1, n_cos=1, s_max=1.0))), None) == D.ERR_INVALID_ARG


def _scene():
    from paper_2402_03106_amd import workloads as W
    return W.box_hg_small()


def _render_rc(D, sc, p, flags, table=None, hi=1, lo=1):
    h = D._SceneHolder(sc)
    tb = C.byref(table) if table is not None else None
    fake = C.c_void_p(0x1000) if hi else None
    fake_lo = C.c_void_p(0x2000) if lo else None
    return D.lib().darts_render_transient(C.byref(h.c), C.byref(D.params(p, flags)), tb, fake, fake_lo,
                                         None, None, None)


def test_render_rejects_bad_arguments_before_launch(D):
    w = _scene()
    sc, p = w["scene"], w["params"]
    table = D._Table(D.medium(sc["medium"]), D.dims(w["dims"]), C.c_void_p(0x3000))
    cases = []
    bad_medium = dict(sc, medium=dict(sigma_s=-1.0, sigma_a=0.1, g=0.0))
    cases.append((bad_medium, p, "uniform", None, D.ERR_INVALID_ARG))
    cases.append((dict(sc, medium=dict(sigma_s=1.0, sigma_a=0.1, g=1.0)), p, "uniform", None, D.ERR_INVALID_ARG))
    cases.append((dict(sc, bins=dict(l_lo=1.0, l_hi=1.0, n_bins=4)), p, "uniform", None, D.ERR_INVALID_ARG))
    cases.append((dict(sc, emitters=[]), p, "uniform", None, D.ERR_INVALID_ARG))
    cases.append((sc, dict(p, max_bounces=0), "uniform", None, D.ERR_INVALID_ARG))
    cases.append((sc, dict(p, n_ris=4), "darts", table, D.ERR_UNSUPPORTED))
    cases.append((sc, p, D.ELL_TEXP | D.ELL_UNIFORM, None, D.ERR_INVALID_ARG))
    cases.append((sc, p, D.RIS_DIST, None, D.ERR_INVALID_ARG))
    cases.append((sc, p, D.DIRECT_REUSE | D.RIS_DIST, None, D.ERR_INVALID_ARG))
    cases.append((sc, p, 0x400, None, D.ERR_INVALID_ARG))
    cases.append((sc, p, "darts", None, D.ERR_INVALID_ARG))          # EDA needs a table
    other = D._Table(D.medium(dict(sigma_s=1.0, sigma_a=0.1, g=0.0)), D.dims(w["dims"]), C.c_void_p(0x3000))
    cases.append((sc, p, "darts", other, D.ERR_TABLE_MISMATCH))
    for scn, pp, flags, tb, code in cases:
        assert _render_rc(D, scn, pp, flags, tb) == code, (flags, code, D.last_error())
        assert D.last_error() != ""
    assert _render_rc(D, sc, p, "uniform", None, hi=0) == D.ERR_INVALID_ARG


def test_pointwise_rejects_unknown_function(D):
    assert D.lib().darts_debug_pointwise(99, None, None, 0, None, None, None) == D.ERR_INVALID_ARG
    assert D.lib().darts_debug_pointwise(0, None, None, -1, None, None, None) == D.ERR_INVALID_ARG


def test_paths_per_cell_counts(D):
    import torch
    sc = dict(sensor=dict(kind=1, width=2, height=1, origin=(0, 0, 0)), bins=dict(l_lo=0, l_hi=1, n_bins=3))
    c = D.paths_per_cell(sc, dict(n_paths=7, path_offset=5), "darts").reshape(-1)
    ids = torch.arange(5, 12) % 6
    ref = torch.bincount(ids, minlength=6).double()
    assert torch.equal(c, ref)


def _batch_item(D, flags, table=None, n_paths=1024):
    from paper_2402_03106_amd import workloads as W
    w = W.batched(1, seed=1)[0]
    h = D._SceneHolder(w["scene"])
    it = D._BatchItem()
    it.scene = h.c
    p = dict(w["params"], n_paths=n_paths)
    it.params = D.params(p, flags)
    it.table = table
    return it, h


def test_batch_create_validates_before_the_device(D):
    """darts_batch_create rejects bad requests before any device call."""
    import ctypes as C
    L = D.lib()
    out = C.c_void_p()
    arr = (D._BatchItem * 1)()
    assert L.darts_batch_create(arr, 0, None, C.byref(out)) == D.ERR_INVALID_ARG
    it, h = _batch_item(D, "vanilla")
    arr[0] = it
    assert L.darts_batch_create(arr, 1, None, C.byref(out)) == D.ERR_UNSUPPORTED
    it, h = _batch_item(D, "darts")          # EDA needs a table
    arr[0] = it
    assert L.darts_batch_create(arr, 1, None, C.byref(out)) == D.ERR_INVALID_ARG
    assert "item 0" in D.last_error()
    it, h = _batch_item(D, "uniform")
    arr[0] = it
    bad = D._plan_struct({"block_threads": 96})
    assert L.darts_batch_create(arr, 1, C.byref(bad), C.byref(out)) == D.ERR_INVALID_ARG
    bad = D._plan_struct({"unit_paths": 8})
    assert L.darts_batch_create(arr, 1, C.byref(bad), C.byref(out)) == D.ERR_INVALID_ARG
    assert not out.value
    assert L.darts_batch_render(None, None, None, None) == D.ERR_INVALID_ARG
    assert L.darts_batch_destroy(None) == D.OK


def test_response_table_validation(D):
    import ctypes as C
    L = D.lib()
    n = C.c_size_t()
    assert L.darts_response_bytes(0, C.byref(n)) == D.ERR_INVALID_ARG
    assert L.darts_response_bytes(32, C.byref(n)) == D.OK and n.value == 65 * 4
    dummy = C.c_void_p(16)   # never dereferenced: validation fails first
    for bad in ([0.0, 0.0], [1.0, -1.0], [1.0, float("nan")], [float("inf"), 1.0]):
        arr = (C.c_float * len(bad))(*bad)
        assert L.darts_build_response(arr, len(bad), dummy, None) == D.ERR_INVALID_ARG
