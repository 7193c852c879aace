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
    with open(src / "darts.hip", "a") as f:   # any change to the kernel source voids the record
        f.write("\n")
    assert bench.measured_traffic() is None
    rec.unlink()
    assert bench.measured_traffic() is None


def test_flop_accounting(bench):
    # a launch in which every vertex step moves on, no path is truncated and
    # the direction counts follow from the step counts
    s = {"vertices": 1000, "early_exit": 100, "setup_exit": 40, "truncated": 0, "medium_exit": 150,
         "ris_all_invalid": 10, "connections": 60, "eda_branch": 200}
    f_d, steps = bench.algorithmic_flops(s, "darts")
    f_u, steps_u = bench.algorithmic_flops(s, "uniform")
    assert steps == steps_u == 900
    F = bench.FLOPS
    moves = 900 - 150 - 10
    dirs = moves - (100 - 40)
    # what DARTS adds over uniform sampling on the same counts
    extra = (60 * (F["connect_texp"] - F["connect_uniform"]) + 750 * (F["ris"] - F["exp_distance"]) +
             dirs * F["direction_eda"] + 200 * F["eda_branch"] + (dirs - 200) * F["hg_bin"] - 200 * F["hg_branch"])
    assert f_d - f_u == extra
    assert 300 < f_d / steps < 600
