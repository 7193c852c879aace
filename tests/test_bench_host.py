"""Host logic of bench.py (no GPU): the one-GPU guard, the rule that the HBM
traffic of the counter profile is reported only for the kernel source it was
measured on, and the FLOP accounting's bookkeeping."""
import importlib.util
import json
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def test_traffic_follows_the_kernel_source(bench, tmp_path, monkeypatch):
    src = tmp_path / "paper_2402_03106_amd" / "csrc"
    src.mkdir(parents=True)
    for f in ["darts.hip", "darts_device.hpp"]:
        shutil.copy(os.path.join(ROOT, "paper_2402_03106_amd", "csrc", f), src / f)
    (tmp_path / "profiles").mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    rec = tmp_path / "profiles" / "render_kernel_box_hg_traffic.json"
    rec.write_text(json.dumps({"kernel_source_hash": bench.kernel_source_hash(), "bytes_per_launch": 1234}))
    assert bench.measured_traffic() == 1234
    with open(src / "darts.hip", "a") as f:   # an edited comment leaves the record valid
        f.write("\n// a comment\n")
    assert bench.measured_traffic() == 1234
    with open(src / "darts.hip", "a") as f:   # any change to the code voids it
        f.write("static int extra_symbol = 1;\n")
    assert bench.measured_traffic() is None
    rec.unlink()
    assert bench.measured_traffic() is None


def test_flop_accounting(bench):
    """The roofline's FLOPs are the per-unit figures (375 per vertex step, 60
    per path) times the launch's counted units; the op-by-op part counts are
    pinned here and, on a launch with the box workload's mix of events,
    land within 10% of the per-unit figures."""
    s = {"paths": 100, "vertices": 1000, "early_exit": 100, "setup_exit": 40, "truncated": 0,
         "medium_exit": 100, "ris_all_invalid": 10, "connections": 270, "eda_branch": 120}
    f, steps = bench.algorithmic_flops(s, 100)
    assert steps == 900
    assert f == 375 * 900 + 60 * 100
    F = bench.FLOPS
    assert F == {"setup": 47, "connect_test": 23, "connect_texp": 103, "connect_uniform": 86, "flight_test": 4,
                 "ris": 222, "exp_distance": 8, "move": 18, "direction": 69, "direction_eda": 13,
                 "eda_branch": 7, "hg_branch": 20, "hg_bin": 8}
    fc = bench.counted_flops(s, "darts")
    fu = bench.counted_flops(s, "uniform")
    moves = 900 - 100 - 10
    dirs = moves - (100 - 40)
    # what DARTS adds over uniform sampling on the same counts
    extra = (270 * (F["connect_texp"] - F["connect_uniform"]) + 800 * (F["ris"] - F["exp_distance"]) +
             dirs * F["direction_eda"] + 120 * F["eda_branch"] + (dirs - 120) * F["hg_bin"] - 120 * F["hg_branch"])
    assert fc - fu == extra
    assert abs(fc / f - 1) < 0.1, fc / f
