"""Store-level parity of the interface recorder and the autograd binding (needs an MI355X).

Recorder (Section 2: interface slices, bit-width reduction, subsampling):
  * the FP32 store of every kept step holds the oracle's interface values, element by
    element, to 3e-5 of the block's largest magnitude over the run (FP32 against FP64
    arithmetic);
  * the forward does not depend on the storage type (final fields bitwise equal), so the
    FP32 store of the same problem holds exactly the values every other recorder
    quantised: each code, and each FP8 scale, must equal what the oracle's codec gives
    for those values, bit for bit; checked at 32^3 for every type and at the 128^3 and
    256x256x128 benchmark sizes on sampled kept steps.
Binding: a non-finite loss raises FDTD_ENONFINITE; a backward after a later forward on
the same Gradient raises FDTD_ESTATE; the returned gradient is not the library's buffer;
at 128^3 the gradient returned through FDTDGrad matches the FP64 oracle's exact gradient
per cell and central differences of the GPU loss on 16 seeded design cells.
"""

import numpy as np
import pytest
import torch

import workloads as w
import paper_2603_24027_amd as pk
from oracle import adjoint, codec, yee

from gpu_helpers import gpu_run, require_gpu, say, store_slice

pytestmark = pytest.mark.gpu

ORACLE_MODE = {"fp32": "fp32", "fp16": "fp16", "bf16": "bf16", "fp8_e4m3_scaled": "fp8_e4m3fn_scaled",
               **{m: m for m in ("fp8_e4m3b11fnuz", "fp8_e5m2fnuz", "fp8_e4m3fnuz", "fp8_e4m3", "fp8_e3m4",
                                 "fp8_e4m3fn")}}
LOSSY = [t for t in ORACLE_MODE if t != "fp32"]


def _forward(prob, dtype, k):
    obj = pk.Gradient(prob, dtype, k, with_backward=False)
    obj.forward(torch.from_numpy(np.ascontiguousarray(prob.eps, np.float32)).cuda())
    torch.cuda.synchronize()
    return obj


def _codes_match_fp32_store(prob, ref, dtype, k, kept):
    """Every block of the kept steps `kept` of a (dtype, k) recording equals the oracle's
    encoding of the FP32 (k = 1) store's values of the same time step."""
    obj = _forward(prob, dtype, k)
    for a, b in zip(obj.fields(), ref.fields()):
        assert torch.equal(a, b), "the forward must not depend on the storage type"
    mode = ORACLE_MODE[dtype]
    for j in kept:
        blocks, scales = store_slice(obj, j)
        ref_blocks, _ = store_slice(ref, j * k)          # time step T-1-j*k in the k = 1 store
        for b in range(12):
            codes, s = codec.encode_block(ref_blocks[b], mode)
            assert np.array_equal(blocks[b].astype(np.int64), codes), (prob.name, dtype, k, j, b)
            if scales is not None:
                assert float(scales[b]) == s, (prob.name, dtype, k, j, b, float(scales[b]), s)
    del obj


@pytest.mark.parametrize("case", ["c1", "ragged", "kappa"])
def test_fp32_store_holds_oracle_interface_values(case):
    require_gpu()
    from test_gpu_parity import CASES
    prob = CASES[case]()
    say("FP32 store vs oracle interface values,", case)
    ref = _forward(prob, "fp32", 1)
    solver = yee.Solver(prob, match_fp32=True)
    _, _, _, kept_H, kept_E = adjoint.record_forward(solver, "fp64", 1)
    T = prob.steps
    # each block's largest magnitude over the run (late, decayed steps are not normalised by
    # their own small values)
    scale = np.zeros(12)
    for n in kept_H:
        for b, want in enumerate(kept_H[n] + kept_E[n]):
            scale[b] = max(scale[b], float(np.max(np.abs(want))))
    worst = 0.0
    for j in range(int(ref.info.slices)):
        n = T - 1 - j
        blocks, _ = store_slice(ref, j)
        for b, want in enumerate(kept_H[n] + kept_E[n]):
            want = np.asarray(want, np.float64).ravel()
            got = blocks[b].astype(np.float64)
            err = np.max(np.abs(got - want)) / max(scale[b], 1e-30)
            worst = max(worst, err)
            assert err <= 3e-5, (case, n, b, err)
    say("  worst block max|d| / max over the run of |ref| %.3e" % worst)


@pytest.mark.parametrize("k", [1, 3])
def test_store_codes_bit_exact_every_type_c1(k):
    require_gpu()
    prob = w.c1()
    say("store codes vs oracle codec, c1, every type, k", k)
    ref = _forward(prob, "fp32", 1)
    slices = int(np.ceil(prob.steps / k))
    for dtype in LOSSY:
        _codes_match_fp32_store(prob, ref, dtype, k, range(slices))


@pytest.mark.parametrize("preset", ["c2", "c4"])
def test_store_codes_bit_exact_benchmark_size(preset):
    # sampled kept steps of the FP8 (k = 16, 64x) and BF16 (k = 4) recorders at full size
    require_gpu()
    prob = w.make(preset)
    say("store codes vs oracle codec,", prob.name)
    ref = _forward(prob, "fp32", 1)
    for dtype, k in [("fp8_e4m3_scaled", 16), ("bf16", 4), ("fp8_e4m3b11fnuz", 16)]:
        slices = int(np.ceil(prob.steps / k))
        kept = sorted(set(np.linspace(0, slices - 1, 7).astype(int).tolist()))
        _codes_match_fp32_store(prob, ref, dtype, k, kept)
        say("  %s k=%d: kept steps %s bit-exact" % (dtype, k, kept))


# --------------------------------------------------------------------------- binding

def test_nonfinite_loss_raises():
    require_gpu()
    prob = w.tiny()
    gobj = pk.Gradient(prob, "fp32", 1)
    bg = torch.from_numpy(prob.eps).cuda()
    design = torch.from_numpy(prob.design_eps()).cuda()
    design[1, 1, 1] = float("nan")
    with pytest.raises(pk.FdtdError) as e:
        pk.FDTDGrad.apply(design.requires_grad_(True), gobj, bg)
    assert e.value.code == pk._lib.FDTD_ENONFINITE
    # a finite design on the same object works afterwards
    ok = torch.from_numpy(prob.design_eps()).cuda().requires_grad_(True)
    loss = pk.FDTDGrad.apply(ok, gobj, bg)
    assert np.isfinite(float(loss.item()))


def test_backward_after_a_later_forward_raises_and_grad_is_a_copy():
    require_gpu()
    prob = w.tiny()
    gobj = pk.Gradient(prob, "fp32", 1)
    bg = torch.from_numpy(prob.eps).cuda()
    d1 = torch.from_numpy(prob.design_eps()).cuda().requires_grad_(True)
    # a float64 design: its gradient is returned in float64, the library buffer's own type
    d2 = (torch.from_numpy(prob.design_eps()).cuda().double() * 1.01).requires_grad_(True)
    l1 = pk.FDTDGrad.apply(d1, gobj, bg)
    l2 = pk.FDTDGrad.apply(d2, gobj, bg)
    with pytest.raises(pk.FdtdError) as e:
        l1.backward()
    assert e.value.code == pk._lib.FDTD_ESTATE
    l2.backward()
    d2_32 = d2.detach().float().cpu().numpy()
    _, g2 = adjoint.grad_time_reversal(prob.with_design(d2_32), "fp64", 1, match_fp32=True)
    got = d2.grad.double().cpu().numpy()
    assert np.linalg.norm(got - g2) <= 1e-4 * np.linalg.norm(g2)
    # the caller owns its gradient: the library's next backward does not overwrite it
    keep = d2.grad.clone()
    l3 = pk.FDTDGrad.apply(d1, gobj, bg)
    l3.backward()
    assert torch.equal(d2.grad, keep)


def test_c2_autograd_gradient_per_cell_and_finite_differences():
    # 128^3 through the torch.autograd.Function: 16 seeded design cells against the FP64 oracle's
    # exact gradient (stored) and against central differences of the GPU loss
    require_gpu()
    import os
    prob = w.c2(seed=0)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "oracle_grad_%s_seed0.npy" % prob.name)
    exact = np.load(path)
    gobj = pk.Gradient(prob, "fp32", 1)
    bg = torch.from_numpy(prob.eps).cuda()
    design = torch.from_numpy(prob.design_eps()).cuda().requires_grad_(True)
    pk.FDTDGrad.apply(design, gobj, bg).backward()
    g = design.grad.double().cpu().numpy().ravel()
    scale = np.max(np.abs(exact))
    cells = w.fd_cells(prob, 16, seed=0)
    err = np.abs(g[cells] - exact.ravel()[cells]) / scale
    say("c2 FDTDGrad vs FP64 oracle on 16 cells: max |d| / max|g| %.3e" % err.max())
    assert err.max() <= 1e-5
    # central differences of the GPU loss (fourth order in h: the truncation error is far below
    # the FP32 rounding of the loss, which the tolerance bounds)
    fwd = pk.Gradient(prob, "fp32", 1, with_backward=False)
    base = prob.design_eps().ravel().astype(np.float64)
    h = 0.05

    def loss_at(cell, delta):
        d = base.copy()
        d[cell] += delta
        eps = prob.eps.copy()
        eps[prob.design_slices()] = d.reshape(prob.design_shape).astype(np.float32)
        fwd.forward(torch.from_numpy(eps).cuda())
        return fwd.loss_value()

    worst = 0.0
    for c in cells:
        fd = (8 * (loss_at(c, h) - loss_at(c, -h)) - (loss_at(c, 2 * h) - loss_at(c, -2 * h))) / (12 * h)
        e = abs(fd - g[c]) / scale
        worst = max(worst, e)
        say("  cell %6d: adjoint %+.6e  central difference %+.6e  |d|/max|g| %.2e" % (c, g[c], fd, e))
    assert worst <= 2e-2
