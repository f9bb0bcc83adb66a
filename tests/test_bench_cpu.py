"""Host logic of bench.py: the one-GPU guard, the algorithmic byte counts, the counter
summaries it reads and its agreement metrics (no GPU needed)."""

import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench            # noqa: E402
import workloads as w   # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_algorithmic_bytes_at_128_cube():
    # 128^3, P = 10, 32^3 design: counted by hand from the per-cell figures
    prob = w.c2()
    N, NI = 128 ** 3, 108 ** 3
    S = 2 * 10 * 3 * 128 ** 2            # PML slab cells summed over the three axes
    shell = 2 * 3 * 108 ** 2             # interior face cells (low and high faces)
    ab = bench.algorithmic_bytes(prob, 32 ** 3)
    assert ab["fwd_step"] == 52 * N + 32 * S == 140_509_184
    assert ab["adj_step"] == 52 * N + 32 * S + 16 * shell == 141_628_928
    assert ab["prim_rev"] == 52 * NI + 28 * 32 ** 3 == 66_422_528


def test_algorithmic_bytes_without_pml_has_no_shell():
    from dataclasses import replace
    prob = replace(w.tiny(n=(14, 13, 12), steps=5), pml=0)
    ab = bench.algorithmic_bytes(prob, 1)
    N = 14 * 13 * 12
    assert ab["fwd_step"] == ab["adj_step"] == 52 * N


def test_counter_summary_is_used_only_for_the_current_kernel_sources(tmp_path, monkeypatch):
    prof = tmp_path / "profiles"
    prof.mkdir()
    rec = {"kernel": "adj_step", "workload": "demo", "hbm_bytes_per_launch": 123456789,
           "kernel_source_hash": bench.kernel_source_hash()}
    (prof / "adj_step_demo_pmc.txt").write_text("header\njson: " + json.dumps(rec) + "\n")
    stale = dict(rec, kernel_source_hash="0" * 16)
    (prof / "fwd_step_demo_pmc.txt").write_text("json: " + json.dumps(stale) + "\n")
    for rel in bench.KERNEL_SOURCES:              # the hash reads the sources under ROOT
        os.makedirs(tmp_path / os.path.dirname(rel), exist_ok=True)
        with open(os.path.join(ROOT, rel), "rb") as f, open(tmp_path / rel, "wb") as g:
            g.write(f.read())
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.read_traffic("adj_step", "demo") == 123456789
    assert bench.read_traffic("fwd_step", "demo") is None       # other sources: not used
    assert bench.read_traffic("prim_rev", "demo") is None       # no summary at all


def test_agreement_metrics():
    a = np.array([1.0, 2.0, -3.0])
    assert bench.cosine(a, 2 * a) == pytest.approx(1.0, abs=1e-15)
    assert bench.cosine(a, -a) == pytest.approx(-1.0, abs=1e-15)
    assert bench.rel_l2(a, a) == 0.0
    assert bench.rel_l2(1.1 * a, a) == pytest.approx(0.1, rel=1e-12)


def test_every_workload_and_crop_resolves():
    for name, (preset, kw, dtype, k) in bench.WORKLOADS.items():
        prob = w.make(preset, **kw)
        assert prob.cells == prob.nx * prob.ny * prob.nz and prob.steps > 0, name
        assert dtype in ("fp32", "fp16", "bf16", "fp8_e4m3_scaled") and k >= 1
    for name, crop in bench.CROPS.items():
        big, small = w.make(bench.WORKLOADS[name][0]), w.make(crop)
        assert (small.nx, small.ny, small.nz) == (128, 128, 128) and small.pml == big.pml


def test_default_workload_is_hbm_bound_with_both_forms_and_a_crop():
    # the headline runs the 256x256x128 slab (working set far above the 256 MB Infinity Cache),
    # times FP32 every step beside FP8 k = 16 (exactly 64x: 16 divides 4000) and reports the
    # gradient errors on the oracle-checked 128^3 crop of the same recipe
    name = bench.DEFAULT_WORKLOAD
    assert name not in bench.CACHE_RESIDENT
    prob = w.make(bench.WORKLOADS[name][0])
    per_step = 52 * prob.cells            # both field buffers and eps touched by one forward step
    assert per_step > 1.5 * 256e6
    assert bench.COMPRESSED[name][0] == ("fp8_e4m3_scaled", 16, "linear") and prob.steps % 16 == 0
    crop = w.make(bench.CROPS[name])
    assert crop.steps % 16 == 0 and crop.wavelength == prob.wavelength
    assert crop.design_shape == prob.design_shape and crop.pml == prob.pml


def test_cpu_sample_is_bounded_and_host_is_described():
    for preset in ("c2", "c4", "c5"):
        p = w.make(preset)
        steps = bench.cpu_sample_steps(p.cells)
        assert 1 <= steps and p.cells * steps <= 7e7
    model, ncpu, usable = bench.host_description()
    assert isinstance(model, str) and model and ncpu >= 1 and 1 <= usable <= ncpu
