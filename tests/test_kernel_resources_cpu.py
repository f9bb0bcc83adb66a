"""Register budget of the sweep kernels, read from the compiler's resource remarks (gfx950
cross-compile, no GPU).  Every single-step sweep must keep 4 wavefronts per SIMD and use no
scratch memory: one vector register past 128 drops a sweep to 3 waves and costs about a
quarter of its speed, and spilled vector registers turn into memory traffic.  The two-step
forward sweep (16-wave blocks, one per compute unit) must keep its 4 waves per SIMD; it may
spill a few registers (the code path of tiles that meet all three PML slabs needs more than
128; the one- and two-slab paths need 118-119)."""

import os
import re
import shutil
import subprocess
import tempfile
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2603_24027_amd", "csrc")


def _remarks(src):
    from paper_2603_24027_amd import build
    with tempfile.TemporaryDirectory() as d:
        cmd = [build.hipcc(), *build.HIPCC_FLAGS, "-Rpass-analysis=kernel-resource-usage", "-c",
               os.path.join(CSRC, src), "-o", os.path.join(d, "k.o")]
        r = subprocess.run(cmd, capture_output=True, text=True, timeout=600)
        assert r.returncode == 0, r.stderr[-2000:]
        return r.stderr


@pytest.fixture(scope="module")
def usage():
    if not (os.environ.get("HIPCC") or os.path.exists("/opt/rocm/bin/hipcc") or shutil.which("hipcc")):
        pytest.skip("hipcc not available")
    import sys
    sys.path.insert(0, ROOT)
    with ThreadPoolExecutor(4) as ex:
        texts = list(ex.map(_remarks, ["forward.hip", "reverse.hip", "forward2.hip", "reverse2.hip"]))
    out = {}
    for text in texts:
        for block in re.split(r"remark: Function Name: ", text)[1:]:
            name = block.split()[0]
            out[name] = {k: int(re.search(pat, block).group(1)) for k, pat in
                         (("occupancy", r"Occupancy \[waves/SIMD\]: (\d+)"), ("vgprs", r"VGPRs: (\d+)"),
                          ("scratch", r"ScratchSize \[bytes/lane\]: (\d+)"))}
    return out


@pytest.mark.parametrize("kernel", ["k_fwd_step", "k_prim_rev", "k_adj_step"])
def test_sweeps_keep_four_waves_and_no_scratch(usage, kernel):
    found = {n: u for n, u in usage.items() if kernel in n}
    assert found, "no %s instantiation in the remarks" % kernel
    for name, u in found.items():
        assert u["occupancy"] >= 4, (name, u)
        assert u["scratch"] == 0, (name, u)


def test_two_step_sweep_keeps_four_waves(usage):
    found = {n: u for n, u in usage.items() if "k_fwd2_step" in n}
    assert found, "no k_fwd2_step instantiation in the remarks"
    for name, u in found.items():
        assert u["occupancy"] >= 4, (name, u)
        assert u["scratch"] <= 128, (name, u)


def test_two_step_reversal_keeps_four_waves_and_no_scratch(usage):
    found = {n: u for n, u in usage.items() if "k_rev2" in n}
    assert found, "no k_rev2 instantiation in the remarks"
    for name, u in found.items():
        assert u["occupancy"] >= 4, (name, u)
        assert u["scratch"] == 0, (name, u)
