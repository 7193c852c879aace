"""Register, LDS and scratch budget of the timed render kernel, read from the
gfx950 assembly the build's own compiler flags produce (CPU only: hipcc
cross-compiles).  The frame's HBM traffic stays near its algorithmic bytes
only while the DARTS image kernel keeps all path state in registers and LDS:
no scratch (spill) memory, and it runs at 5 resident waves per SIMD only
with at most 96 VGPRs (512 per SIMD lane, in granules of 8) and 32 KiB of LDS
per 256-thread block (5 blocks of a CU's 160 KiB)."""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
TIMED = "_ZN12_GLOBAL__N_113render_kernelILi0ELi0ELb0ELb0ELi0EEEvNS_7KParamsE"


@pytest.fixture(scope="module")
def kernels(tmp_path_factory):
    if not (os.path.exists(HIPCC) or shutil.which(HIPCC)):
        pytest.skip("hipcc not available")
    from paper_2402_03106_amd import build as B
    out = tmp_path_factory.mktemp("isa") / "darts.s"
    flags = [f for f in B.HIPCC_FLAGS if f not in ("-shared", "-fPIC")]
    cmd = [HIPCC, *flags, "--cuda-device-only", "-S", "-I", os.path.join(ROOT, "include"), B.SRC, "-o", str(out)]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-2000:]
    s = out.read_text()
    res = {}
    for m in re.finditer(r"\.amdhsa_kernel (\S+)", s):
        blk = s[m.start():s.find(".end_amdhsa_kernel", m.start())]
        res[m.group(1)] = {k: int(re.search(r"\.amdhsa_" + k + r"\s+(\d+)", blk).group(1))
                           for k in ("next_free_vgpr", "private_segment_fixed_size", "group_segment_fixed_size")}
    return res


def test_timed_kernel_has_no_scratch_and_fits_five_waves(kernels):
    k = kernels[TIMED]
    assert k["private_segment_fixed_size"] == 0, k
    assert k["next_free_vgpr"] <= 96, k
    assert k["group_segment_fixed_size"] <= 32 * 1024, k


def test_image_kernels_without_statistics_have_no_scratch(kernels):
    """Every image-output render kernel without statistics counters (DARTS
    family and vanilla, with and without the floor, the tile and id-range
    decompositions, and vanilla's pixel decomposition)."""
    names = [n for n in kernels if re.search(r"render_kernelILi[01]ELi0ELb0E", n)]
    assert len(names) == 10, names
    for n in names:
        assert kernels[n]["private_segment_fixed_size"] == 0, (n, kernels[n])
