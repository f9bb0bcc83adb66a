"""Checks at the benchmark's full size, in the launch configuration bench.py times (needs an MI355X).

The FP64 oracle would need tens of minutes for one 128^3 x 1000-step gradient,
so at full size the checks use properties that hold at any size:
  * the gradient is the derivative of the loss: a directional central
    difference of the GPU loss along a random design perturbation matches
    <grad, direction> (the sum over 32768 cells averages FP32 noise away);
  * time reversal returns the interior to the initial (zero) state;
  * repeat runs are bitwise identical;
  * the storage accounting of the compressed recorder (Fig. 3 caption).
Oracle parity at every tile and ragged-tail shape is covered on smaller grids
in test_gpu_parity.py.
"""

import numpy as np
import pytest
import torch

import workloads as w
import paper_2603_24027_amd as pk
from oracle import metrics

from gpu_helpers import gpu_run, require_gpu, say

pytestmark = pytest.mark.gpu


def _loss(gobj, prob, design):
    eps = prob.eps.copy()
    eps[prob.design_slices()] = design.astype(np.float32)
    t = torch.from_numpy(eps).cuda()
    return float(gobj.forward(t).item())


def test_c2_fp32_gradient_is_derivative_of_loss():
    require_gpu()
    prob = w.c2()
    say("c2 full size: fp32 k=1 gradient, directional derivative, reversal, determinism")
    out = gpu_run(prob, "fp32", 1, keep_fields=False)
    g = out["grad"]
    assert np.all(np.isfinite(g)) and np.linalg.norm(g) > 0
    # reversal: the interior is back at the zero initial state
    gobj = out["obj"]
    E, H = gobj.fields()
    P = prob.pml
    I = (slice(None), slice(P, prob.nz - P), slice(P, prob.ny - P), slice(P, prob.nx - P))
    resid = float(max(E[I].abs().max().item(), H[I].abs().max().item()))
    peak_run = gpu_run(w.c2(steps=130), "fp32", 1, backward=False)
    peak = float(max(np.abs(peak_run["E"]).max(), np.abs(peak_run["H"]).max()))
    say("  reversal residual %.3e of peak %.3e" % (resid, peak))
    assert resid <= 1e-3 * peak
    # directional derivative with the GPU forward
    rng = np.random.default_rng(7)
    d = rng.standard_normal(prob.design_shape)
    base = prob.design_eps().astype(np.float64)
    h = 2e-3
    fwd = pk.Gradient(prob, "fp32", 1, with_backward=False)
    lp = _loss(fwd, prob, base + h * d)
    lm = _loss(fwd, prob, base - h * d)
    fd = (lp - lm) / (2 * h)
    ad = float(np.sum(g * d))
    say("  directional: adjoint %.6e  central difference %.6e" % (ad, fd))
    assert abs(fd - ad) <= 5e-3 * abs(ad)
    # determinism
    again = gpu_run(prob, "fp32", 1, keep_fields=False)
    assert again["loss"] == out["loss"] and np.array_equal(again["grad"], g)


def _directional_check(prob, h, tol, seed=7):
    """Adjoint directional derivative <grad, d> against a central difference of the GPU
    forward loss along a random design direction d; returns the FP32 k=1 run."""
    out = gpu_run(prob, "fp32", 1, keep_fields=False)
    g = out["grad"]
    assert np.all(np.isfinite(g)) and np.linalg.norm(g) > 0
    rng = np.random.default_rng(seed)
    d = rng.standard_normal(prob.design_shape)
    base = prob.design_eps().astype(np.float64)
    fwd = pk.Gradient(prob, "fp32", 1, with_backward=False)
    fd = (_loss(fwd, prob, base + h * d) - _loss(fwd, prob, base - h * d)) / (2 * h)
    ad = float(np.sum(g * d))
    say("  %s directional: adjoint %.6e  central difference %.6e" % (prob.name, ad, fd))
    assert abs(fd - ad) <= tol * abs(ad)
    del fwd
    return out


def test_c4_waveguide_gradient_is_derivative_of_loss():
    # 256x256x128, 12-cell CPML, 4000 steps, plane source in a silicon slab
    require_gpu()
    prob = w.c4()
    out = _directional_check(prob, 2e-3, 1e-2)
    gobj = out["obj"]
    E, H = gobj.fields()
    P = prob.pml
    I = (slice(None), slice(P, prob.nz - P), slice(P, prob.ny - P), slice(P, prob.nx - P))
    resid = float(max(E[I].abs().max().item(), H[I].abs().max().item()))
    say("  reversal residual %.3e" % resid)
    assert np.isfinite(resid)
    del out, gobj, E, H
    ref = gpu_run(prob, "fp32", 1, keep_fields=False)
    for dtype, k, ratio_expected in [("bf16", 4, 8.0), ("fp8_e4m3_scaled", 16, 64.0)]:
        c = gpu_run(prob, dtype, k, keep_fields=False)
        ratio = ref["info"].payload_bytes / c["info"].payload_bytes
        cos = metrics.cosine_similarity(c["grad"], ref["grad"])
        say("  c4 %s k=%d: storage ratio %.2f, cosine vs fp32 k=1 %.6f" % (dtype, k, ratio, cos))
        assert ratio == ratio_expected                  # 16 divides 4000: exactly 64x (Fig. 3 caption)
        assert c["loss"] == pytest.approx(ref["loss"], rel=1e-12)
        # a 30-cell wavelength spans about 52 steps: k = 16 keeps 3.3 samples per period and the
        # linear interpolation bounds the agreement (0.97 on the oracle-checked 128^3 crop)
        assert cos >= (0.999 if k == 4 else 0.9)


def test_c5_memory_scale_gradient_is_derivative_of_loss():
    # 512x512x256, 16-cell CPML, 8000 steps, FP32 store of every step (57 GB) in HBM
    require_gpu()
    prob = w.c5()
    out = _directional_check(prob, 2e-3, 1e-2)
    m = (480, 480, 224)                                   # interior extents
    values = 2 * 2 * (m[1] * m[2] + m[0] * m[2] + m[0] * m[1])   # two sides, two components per face
    assert out["info"].payload_bytes == values * 4 * 8000 == 57_016_320_000


def test_c2_compressed_storage_and_agreement():
    require_gpu()
    prob = w.c2()
    ref = gpu_run(prob, "fp32", 1, keep_fields=False)
    for dtype, k in [("bf16", 4), ("fp8_e4m3_scaled", 16)]:
        out = gpu_run(prob, dtype, k, keep_fields=False)
        ratio = ref["info"].payload_bytes / out["info"].payload_bytes
        cos = metrics.cosine_similarity(out["grad"], ref["grad"])
        say("  c2 %s k=%d: storage ratio %.2f, cosine vs fp32 k=1 %.6f, rel-L2 %.3e"
            % (dtype, k, ratio, cos, metrics.rel_l2(out["grad"], ref["grad"])))
        assert ratio == pytest.approx(32 / pk.STORAGE_BITS[dtype] * k * (1000 / 16) / np.ceil(1000 / 16)
                                      if k == 16 else 32 / pk.STORAGE_BITS[dtype] * k, rel=1e-12)
        assert out["loss"] == pytest.approx(ref["loss"], rel=1e-12)   # the forward does not depend on storage
        assert np.all(np.isfinite(out["grad"]))
        assert cos > 0.5


def test_paper_regime_fp8_k16_keeps_gradient_direction():
    """At ~136 steps per period (the paper's Section 2 example), FP8 with k = 16 (63.5x here:
    16 does not divide 1000) keeps the direction of the full-FP32-storage gradient to cosine
    >= 0.99 (0.9986 measured, limited by the linear interpolation in time; Section 3).  This
    bar is a regression check, not the 0.999 accuracy target, which this setting misses."""
    require_gpu()
    prob = w.c3p()
    say("c3p (lambda 77.5 cells): fp8 k=16 vs fp32 k=1")
    ref = gpu_run(prob, "fp32", 1, keep_fields=False)
    out = gpu_run(prob, "fp8_e4m3_scaled", 16, keep_fields=False)
    cos = metrics.cosine_similarity(out["grad"], ref["grad"])
    say("  cosine %.6f rel-L2 %.3e" % (cos, metrics.rel_l2(out["grad"], ref["grad"])))
    assert cos >= 0.99


def _oracle_gradient(name, seed):
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                        "oracle_grad_%s_seed%d.npy" % (name, seed))
    if not os.path.exists(path):
        pytest.skip("stored oracle gradient %s not present (tests/golden/make_oracle_grads.py)" % path)
    return np.load(path)


def test_c2_fp32_gradient_matches_fp64_oracle():
    # parity at the benchmark size against the oracle's exact gradient (stored by the oracle script)
    require_gpu()
    prob = w.c2(seed=0)
    exact = _oracle_gradient(prob.name, 0)
    g = gpu_run(prob, "fp32", 1, keep_fields=False)["grad"]
    r, c = metrics.rel_l2(g, exact), metrics.cosine_similarity(g, exact)
    say("c2 fp32 k=1 vs FP64 oracle: rel-L2 %.3e cosine %.12f" % (r, c))
    assert r <= 1e-5 and c >= 1 - 1e-9


@pytest.mark.parametrize("dtype,k,cos_min", [("fp8_e4m3_scaled", 8, 0.999), ("fp8_e4m3_scaled", 16, 0.998),
                                             ("bf16", 4, 0.9999), ("fp8_e5m2fnuz", 4, 0.999)])
def test_c3p_compressed_gradient_vs_fp64_oracle(dtype, k, cos_min):
    # the paper's sampling (about 136 steps per period): compressed storage against the exact gradient
    require_gpu()
    prob = w.c3p(seed=0)
    exact = _oracle_gradient(prob.name, 0)
    g = gpu_run(prob, dtype, k, keep_fields=False)["grad"]
    c = metrics.cosine_similarity(g, exact)
    say("c3p %s k=%d vs FP64 oracle: cosine %.6f rel-L2 %.3e" % (dtype, k, c, metrics.rel_l2(g, exact)))
    assert c >= cos_min


def test_c2pw_fp32_gradient_matches_fp64_oracle():
    # plane-wave source (magnetic-current sheet) and flux objective at the benchmark size
    require_gpu()
    prob = w.c2pw(seed=0)
    exact = _oracle_gradient(prob.name, 0)
    g = gpu_run(prob, "fp32", 1, keep_fields=False)["grad"]
    r, c = metrics.rel_l2(g, exact), metrics.cosine_similarity(g, exact)
    say("c2pw fp32 k=1 vs FP64 oracle: rel-L2 %.3e cosine %.12f" % (r, c))
    assert r <= 1e-5 and c >= 1 - 1e-9


# The slab-waveguide recipes of the 256x256x128 (c4, c4p) and 512x512x256 (c5) problems on
# 128^3 crops, against the exact gradient.  At a 30-cell wavelength a period spans about 52
# steps: k = 16 keeps about 3.3 samples per period and the linear-in-time interpolation, not
# the FP8 rounding, bounds the agreement (cosine 0.97 measured on c5crop; 0.95 is the bar).
# At 77.5 cells (c4pcrop, ~136 steps per period, the paper's sampling) the bar is the
# measured value rounded down: it is below the 0.999 target, which linear interpolation
# at k = 16 does not reach.
# The cubic option (interp "cubic") rebuilds the skipped steps from four kept ones instead of two.
CROP_CASES = [("c5crop", "fp32", 1, "linear", 1 - 1e-9), ("c5crop", "bf16", 4, "linear", 0.999),
              ("c5crop", "fp8_e4m3_scaled", 16, "linear", 0.95),
              ("c4crop", "fp32", 1, "linear", 1 - 1e-9), ("c4crop", "bf16", 4, "linear", 0.999),
              ("c4crop", "fp8_e4m3_scaled", 16, "linear", 0.98), ("c4crop", "fp8_e4m3_scaled", 16, "cubic", 0.98),
              ("c4pcrop", "fp32", 1, "linear", 1 - 1e-9), ("c4pcrop", "fp8_e4m3_scaled", 8, "linear", 0.9999),
              ("c4pcrop", "fp8_e4m3_scaled", 16, "linear", 0.9985), ("c4pcrop", "fp8_e4m3_scaled", 16, "cubic", 0.999)]


@pytest.mark.parametrize("preset,dtype,k,interp,cos_min", CROP_CASES)
def test_crop_gradient_vs_fp64_oracle(preset, dtype, k, interp, cos_min):
    require_gpu()
    prob = w.make(preset, seed=0)
    exact = _oracle_gradient(prob.name, 0)
    out = gpu_run(prob, dtype, k, keep_fields=False, interp=interp)
    g = out["grad"]
    r, c = metrics.rel_l2(g, exact), metrics.cosine_similarity(g, exact)
    ratio = 32 / pk.STORAGE_BITS[dtype] * k
    say("%s %s k=%d %s (%.0fx smaller) vs FP64 oracle: cosine %.9f rel-L2 %.3e"
        % (preset, dtype, k, interp, ratio, c, r))
    if k > 1:
        assert prob.steps % k == 0
        assert out["info"].payload_bytes * ratio == store_fp32_bytes(prob)
    assert c >= cos_min
    if dtype == "fp32":
        assert r <= 1e-5
        cell = float(np.max(np.abs(g - exact)) / np.max(np.abs(exact)))
        say("  per-cell max|d|/max|g| %.3e" % cell)
        assert cell <= 1e-5


def store_fp32_bytes(prob):
    P = prob.pml
    m = (prob.nx - 2 * P, prob.ny - 2 * P, prob.nz - 2 * P)
    return 4 * (m[1] * m[2] + m[0] * m[2] + m[0] * m[1]) * 4 * prob.steps

