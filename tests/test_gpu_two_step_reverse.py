"""Two reverse primal steps per sweep (temporal blocking of the reversal) against the FP64
oracle and against the single-step reversal (needs an MI355X).

The two-step reversal is forced with FDTD_REV_STEPS=2 and its tile depth chosen with
FDTD_REV2_TILE_Z (16 or 8 planes of 60 x 12 interior columns).  It takes the interface
shell of its first step from a buffer laid out as one kept step and applies its second
step's loss seed and gradient term after the first step's transpose, so these tests cover
every path of that bookkeeping.  Bars, as for the single-step reversal:
  * gradient with FP32 storage at every step against the oracle's FP64 gradient: relative
    L2 <= 1e-4 and every design cell within 1e-4 of the largest, on every grid of the
    single-step parity tests (ragged, kappa > 1 with alpha > 0, periodic without PML,
    zero boundary without PML), both tile depths, odd and even step counts (odd: one single
    step first), T = 1, 2, 3;
  * compressed storage and the cubic reconstruction against the oracle running the same
    codec and rule: cosine >= 0.9999, relative L2 <= 1e-2;
  * the flux objectives (whose seeds reach the adjoint H as well);
  * against the single-step reversal on the same input: relative L2 <= 1e-6 (the same FP32
    arithmetic, up to contraction into fused multiply-adds), bitwise repeatable;
  * at 128^3 and 256x256x128 against the single-step reversal: relative L2 <= 1e-5.
"""

import contextlib
import os
from dataclasses import replace

import numpy as np
import pytest

import workloads as w
from oracle import adjoint, metrics

from gpu_helpers import gpu_run, rel, require_gpu, say
from test_gpu_parity import CASES, FLUX_CASES, ORACLE_MODE

pytestmark = pytest.mark.gpu


@contextlib.contextmanager
def two_step_reverse(cz=16):
    keys = ("FDTD_REV_STEPS", "FDTD_REV2_TILE_Z")
    old = {k: os.environ.get(k) for k in keys}
    os.environ.update({"FDTD_REV_STEPS": "2", "FDTD_REV2_TILE_Z": str(cz)})
    try:
        yield
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def _check_grad(out, g, tol=1e-4):
    r = rel(out["grad"], g)
    cos = metrics.cosine_similarity(out["grad"], g)
    cell = float(np.max(np.abs(out["grad"] - g)) / np.max(np.abs(g)))
    say("  rel-L2 %.3e cosine %.12f per-cell max|d|/max|g| %.3e" % (r, cos, cell))
    assert r <= tol and cos >= 1 - 1e-8
    assert cell <= tol


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("cz", [16, 8])
def test_two_step_reverse_gradient_fp32(case, cz):
    require_gpu()
    prob = CASES[case]()
    say("two-step reversal, gradient fp32 k=1", case, prob.steps, "depth", cz)
    with two_step_reverse(cz):
        out = gpu_run(prob, keep_fields=False)
    L, g = adjoint.grad_time_reversal(prob, "fp64", 1, match_fp32=True)
    assert abs(out["loss"] - L) <= 1e-5 * abs(L)
    _check_grad(out, g)


@pytest.mark.parametrize("steps", [77, 1, 2, 3])
def test_two_step_reverse_odd_and_short_runs(steps):
    require_gpu()
    prob = w.c1(steps=steps)
    say("two-step reversal, c1 steps", steps)
    with two_step_reverse():
        out = gpu_run(prob, keep_fields=False)
    _, g = adjoint.grad_time_reversal(prob, "fp64", 1, match_fp32=True)
    if np.any(g != 0.0):
        _check_grad(out, g)
    else:
        assert not np.any(out["grad"] != 0.0)


@pytest.mark.parametrize("dtype,k", [("fp8_e4m3_scaled", 3), ("fp8_e4m3_scaled", 16), ("bf16", 4), ("fp16", 1)])
def test_two_step_reverse_compressed(dtype, k):
    require_gpu()
    prob = w.c1()
    say("two-step reversal, gradient", dtype, "k", k)
    with two_step_reverse():
        out = gpu_run(prob, dtype, k, keep_fields=False)
    _, g = adjoint.grad_time_reversal(prob, ORACLE_MODE[dtype], k, match_fp32=True)
    r = rel(out["grad"], g)
    cos = metrics.cosine_similarity(out["grad"], g)
    say("  vs oracle same codec: rel-L2 %.3e cosine %.9f" % (r, cos))
    assert cos >= 0.9999 and r <= 1e-2


@pytest.mark.parametrize("dtype,k,case", [("fp32", 3, "c1"), ("fp8_e4m3_scaled", 16, "c1"), ("bf16", 5, "ragged")])
def test_two_step_reverse_cubic(dtype, k, case):
    require_gpu()
    prob = CASES[case]()
    say("two-step reversal, cubic", dtype, k, case)
    with two_step_reverse():
        out = gpu_run(prob, dtype, k, keep_fields=False, interp="cubic")
    _, g = adjoint.grad_time_reversal(prob, ORACLE_MODE[dtype], k, match_fp32=True, interp=3)
    r = rel(out["grad"], g)
    cos = metrics.cosine_similarity(out["grad"], g)
    say("  vs oracle same codec and rule: rel-L2 %.3e cosine %.9f" % (r, cos))
    assert cos >= 0.9999 and r <= 1e-2


@pytest.mark.parametrize("case", list(FLUX_CASES))
def test_two_step_reverse_flux(case):
    require_gpu()
    prob = FLUX_CASES[case]()
    say("two-step reversal, flux objective", case)
    with two_step_reverse():
        out = gpu_run(prob, keep_fields=False)
    _, g = adjoint.grad_time_reversal(prob, "fp64", 1, match_fp32=True)
    r = rel(out["grad"], g)
    cos = metrics.cosine_similarity(out["grad"], g)
    say("  rel-L2 %.3e cosine %.12f" % (r, cos))
    assert r <= 1e-4 and cos >= 1 - 1e-8


@pytest.mark.parametrize("case", ["c1", "ragged", "kappa"])
def test_two_step_reverse_matches_single_step(case):
    require_gpu()
    prob = CASES[case]()
    say("two-step vs single-step reversal", case)
    one = gpu_run(prob, keep_fields=False)
    with two_step_reverse():
        two = gpu_run(prob, keep_fields=False)
        again = gpu_run(prob, keep_fields=False)
    say("  rel-L2 %.3e" % rel(two["grad"], one["grad"]))
    assert rel(two["grad"], one["grad"]) <= 1e-6
    assert np.array_equal(two["grad"], again["grad"])


@pytest.mark.parametrize("preset", ["c2", "c4"])
def test_two_step_reverse_benchmark_size(preset):
    require_gpu()
    prob = w.make(preset)
    say("two-step vs single-step reversal at", prob.name)
    one = gpu_run(prob, keep_fields=False)
    with two_step_reverse():
        two = gpu_run(prob, keep_fields=False)
    say("  rel-L2 %.3e" % rel(two["grad"], one["grad"]))
    assert rel(two["grad"], one["grad"]) <= 1e-5
