"""Two forward steps per sweep (temporal blocking) against the FP64 oracle and against the
single-step sweep (needs an MI355X).

The two-step sweep is forced with FDTD_FWD_STEPS=2 (the library picks it by itself only
where most of its tiles carry no PML, i.e. at 512x512x256 among the presets) and its tile
depth with FDTD_FWD2_TILE_Z (16 or 8 planes of 60 x 12 columns).  Bars:
  * fields and loss vs the oracle: the single-step sweep's (relative L2 <= 1e-5, element by
    element <= 3e-5 of each component's largest magnitude on the interior and on the PML,
    per-step loss terms <= 1e-4 relative), on every grid of the single-step parity tests
    (ragged, kappa > 1 with alpha > 0, periodic, no PML), even and odd step counts, and
    every tile shape;
  * against the single-step sweep on the same input: both evaluate the same FP32
    arithmetic; round-off differs only where the compiler contracted a product into a
    fused multiply-add differently, so relative L2 <= 1e-6 over a few hundred steps;
  * the recorder: the FP32 store holds the oracle's interface values (3e-5 of each block's
    largest magnitude over the run), also on the steps whose values the sweep keeps only
    in its intermediate buffer; every code of an FP8 recording equals the oracle codec's
    encoding of the FP32 store's values, bit for bit;
  * the gradient after a two-step forward: per cell within 1e-4 of the oracle gradient's
    largest magnitude;
  * at 256x256x128 (4000 steps), against the single-step sweep: relative L2 <= 1e-5.
"""

import contextlib
import os
from dataclasses import replace

import numpy as np
import pytest
import torch

import workloads as w
import paper_2603_24027_amd as pk
from oracle import adjoint, codec, yee

from gpu_helpers import gpu_run, rel, require_gpu, say, store_slice
from test_gpu_parity import CASES, assert_fields_elementwise

pytestmark = pytest.mark.gpu

SHAPES = [16, 8]     # tile depths


@contextlib.contextmanager
def two_step(cz=16):
    keys = ("FDTD_FWD_STEPS", "FDTD_FWD2_TILE_Z")
    old = {k: os.environ.get(k) for k in keys}
    os.environ.update({"FDTD_FWD_STEPS": "2", "FDTD_FWD2_TILE_Z": str(cz)})
    try:
        yield
    finally:
        for k, v in old.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def _oracle(prob):
    return yee.run_forward(yee.Solver(prob, match_fp32=True))


def _check_forward(prob, out, st, losses):
    assert rel(out["E"], st.E) <= 1e-5
    assert rel(out["H"], st.H) <= 1e-5
    assert_fields_elementwise(prob, out["E"], out["H"], st)
    assert abs(out["loss"] - losses.sum()) <= 1e-5 * abs(losses.sum())
    big = losses > 1e-6 * losses.max()
    assert np.max(np.abs(out["series"][big] - losses[big]) / losses[big]) <= 1e-4


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("shape", SHAPES)
def test_two_step_fields_and_loss(case, shape):
    require_gpu()
    prob = CASES[case]()
    say("two-step forward", case, prob.shape, prob.steps, "tile", shape)
    with two_step(shape):
        out = gpu_run(prob, series=True, backward=False)
    st, losses, _ = _oracle(prob)
    _check_forward(prob, out, st, losses)


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("steps", [77, 1, 2])
def test_two_step_odd_and_short_runs(shape, steps):
    # odd T: one single step, then pairs; T = 1: no pair at all; T = 2: one pair
    require_gpu()
    prob = w.c1(steps=steps)
    say("two-step forward c1 steps", steps, "tile", shape)
    with two_step(shape):
        out = gpu_run(prob, series=True, backward=False)
    st, losses, _ = _oracle(prob)
    for got, ref in ((out["E"], st.E), (out["H"], st.H)):
        if np.any(ref != 0.0):
            assert rel(got, ref) <= 1e-5
        else:   # H^{1/2} after one step from rest
            assert not np.any(got != 0.0)
    assert abs(out["loss"] - losses.sum()) <= 1e-5 * abs(losses.sum())


@pytest.mark.parametrize("case", ["c1", "ragged", "kappa"])
def test_two_step_matches_single_step(case):
    require_gpu()
    prob = CASES[case]()
    say("two-step vs single-step", case)
    one = gpu_run(prob, series=True, backward=False)
    with two_step():
        two = gpu_run(prob, series=True, backward=False)
        again = gpu_run(prob, series=True, backward=False)
    assert rel(two["E"], one["E"]) <= 1e-6 and rel(two["H"], one["H"]) <= 1e-6
    assert abs(two["loss"] - one["loss"]) <= 1e-6 * abs(one["loss"])
    # bitwise repeatable
    assert np.array_equal(two["E"], again["E"]) and np.array_equal(two["H"], again["H"])
    assert two["loss"] == again["loss"]


def _forward(prob, dtype, k):
    obj = pk.Gradient(prob, dtype, k, with_backward=False)
    obj.forward(torch.from_numpy(np.ascontiguousarray(prob.eps, np.float32)).cuda())
    torch.cuda.synchronize()
    return obj


@pytest.mark.parametrize("case,steps", [("c1", None), ("ragged", None), ("kappa", None), ("c1", 77)])
def test_two_step_fp32_store_holds_oracle_interface_values(case, steps):
    require_gpu()
    prob = CASES[case]()
    if steps is not None:
        prob = replace(prob, steps=steps, src_wave=prob.src_wave[:steps])
    say("two-step FP32 store vs oracle interface values,", case, prob.steps)
    with two_step():
        ref = _forward(prob, "fp32", 1)
    solver = yee.Solver(prob, match_fp32=True)
    _, _, _, kept_H, kept_E = adjoint.record_forward(solver, "fp64", 1)
    T = prob.steps
    scale = np.zeros(12)
    for n in kept_H:
        for b, want in enumerate(kept_H[n] + kept_E[n]):
            scale[b] = max(scale[b], float(np.max(np.abs(want))))
    for j in range(int(ref.info.slices)):
        n = T - 1 - j
        blocks, _ = store_slice(ref, j)
        for b, want in enumerate(kept_H[n] + kept_E[n]):
            got = blocks[b].astype(np.float64)
            err = np.max(np.abs(got - np.asarray(want, np.float64).ravel())) / max(scale[b], 1e-30)
            assert err <= 3e-5, (case, n, b, err)


@pytest.mark.parametrize("dtype,k", [("fp8_e4m3_scaled", 3), ("fp8_e4m3_scaled", 16), ("bf16", 1)])
def test_two_step_store_codes_bit_exact(dtype, k):
    require_gpu()
    prob = w.c1()
    say("two-step store codes vs oracle codec, c1", dtype, k)
    with two_step():
        ref = _forward(prob, "fp32", 1)
        obj = _forward(prob, dtype, k)
    for a, b in zip(obj.fields(), ref.fields()):
        assert torch.equal(a, b)
    mode = "fp8_e4m3fn_scaled" if dtype == "fp8_e4m3_scaled" else dtype
    for j in range(int(obj.info.slices)):
        blocks, scales = store_slice(obj, j)
        ref_blocks, _ = store_slice(ref, j * k)
        for b in range(12):
            codes, s = codec.encode_block(ref_blocks[b], mode)
            assert np.array_equal(blocks[b].astype(np.int64), codes), (dtype, k, j, b)
            if scales is not None:
                assert float(scales[b]) == s, (dtype, k, j, b)


@pytest.mark.parametrize("case", ["c1", "ragged"])
def test_two_step_gradient_against_oracle(case):
    require_gpu()
    prob = CASES[case]()
    say("gradient after a two-step forward,", case)
    with two_step():
        out = gpu_run(prob, backward=True, keep_fields=False)
    ref = adjoint.grad_time_reversal(prob, "fp64", 1, match_fp32=True)[1]
    g = out["grad"].ravel()
    r = np.asarray(ref, np.float64).ravel()
    assert rel(g, r) <= 1e-4
    assert np.max(np.abs(g - r)) <= 1e-4 * np.max(np.abs(r))


@pytest.mark.parametrize("preset", ["c2", "c4"])
def test_two_step_benchmark_size_against_single_step(preset):
    require_gpu()
    prob = w.make(preset)
    say("two-step vs single-step at", prob.name, prob.steps, "steps")
    one = gpu_run(prob, backward=False)
    with two_step():
        two = gpu_run(prob, backward=False)
    say("  rel L2 E %.2e H %.2e, loss %.3e vs %.3e" % (rel(two["E"], one["E"]), rel(two["H"], one["H"]),
                                                       two["loss"], one["loss"]))
    assert rel(two["E"], one["E"]) <= 1e-5 and rel(two["H"], one["H"]) <= 1e-5
    assert abs(two["loss"] - one["loss"]) <= 1e-5 * abs(one["loss"])
