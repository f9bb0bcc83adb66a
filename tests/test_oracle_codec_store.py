"""Pins of the oracle's codec (against library casts), subsampling/interpolation (closed forms),
storage accounting and the paper's worked numbers (CPU only)."""

import json
import math
import os

import numpy as np
import pytest
import torch

from oracle import codec, metrics, store, yee

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "paper_worked_numbers.json")

_TORCH = {"fp16": (torch.float16, torch.int16, codec.FP16),
          "bf16": (torch.bfloat16, torch.int16, codec.BF16),
          "fp8_e4m3fn": (torch.float8_e4m3fn, torch.uint8, codec.FP8_E4M3FN)}


def _torch_codes(x32: np.ndarray, name: str) -> np.ndarray:
    dt, it, fmt = _TORCH[name]
    t = torch.from_numpy(np.ascontiguousarray(x32, np.float32)).to(dt).view(it)
    mask = (1 << fmt.bits) - 1
    return t.numpy().astype(np.int64) & mask


def _probe_values(fmt, rng):
    """All finite values, all midpoints, midpoints +- one float32 ulp, and random values."""
    codes, vals, _, ov = codec._table(fmt)
    mids = (vals[:-1] + vals[1:]) / 2
    mids32 = mids.astype(np.float32)
    lo = np.nextafter(mids32, np.float32(-np.inf))
    hi = np.nextafter(mids32, np.float32(np.inf))
    top = float(np.log2(min(vals[-1], 3e38)))
    rnd = (2.0 ** rng.uniform(-40 if fmt.exp_bits < 8 else -140, top, 200000)).astype(np.float32)
    allv = np.concatenate([vals.astype(np.float32), mids32, lo, hi, rnd])
    allv = allv[np.isfinite(allv) & (np.abs(allv.astype(np.float64)) < ov)]
    return np.concatenate([allv, -allv, np.array([0.0, -0.0], np.float32)])


@pytest.mark.parametrize("name", ["fp16", "bf16", "fp8_e4m3fn"])
def test_encode_matches_library_cast(name):
    rng = np.random.default_rng(0)
    fmt = _TORCH[name][2]
    x = _probe_values(fmt, rng)
    mine = codec.encode(x, fmt)
    ref = _torch_codes(x, name)
    bad = np.nonzero(mine != ref)[0]
    assert bad.size == 0, (x[bad[:5]], mine[bad[:5]], ref[bad[:5]])


@pytest.mark.parametrize("name", ["fp16", "bf16", "fp8_e4m3fn"])
def test_decode_matches_library_cast(name):
    dt, it, fmt = _TORCH[name]
    codes = np.arange(1 << fmt.bits)
    mine = codec.decode(codes, fmt)
    signed = codes.astype(np.int64)
    if it == torch.int16:
        signed = np.where(signed >= 32768, signed - 65536, signed)
        t = torch.tensor(signed, dtype=torch.int16)
    else:
        t = torch.tensor(signed, dtype=torch.uint8)
    ref = t.view(dt).to(torch.float64).numpy()
    fin = np.isfinite(ref)
    assert np.array_equal(np.isfinite(mine), fin)
    assert np.array_equal(mine[fin], ref[fin])


def test_fp8_overflow_rule_matches_library():
    x = np.array([448.0, 463.9, 464.0, 464.1, 479.0, 1e4], np.float32)
    assert np.array_equal(codec.encode(x, codec.FP8_E4M3FN), _torch_codes(x, "fp8_e4m3fn"))


def test_fp8_scale_exponent_definition():
    for m, e in [(448.0, 0), (449.0, 1), (224.0, -1), (224.0001, 0), (1.0, -8), (0.875, -9), (0.8751, -8),
                 (896.0, 1), (0.0, 0), (1e-45, -126), (3e38, 120)]:
        got = codec.fp8_scale_exponent(m)
        assert got == e, (m, got, e)
        if m and -126 < e < 127:
            assert codec.FP8_MAX * 2.0 ** e >= m > codec.FP8_MAX * 2.0 ** (e - 1)


def test_fp8_scaled_block_never_saturates_and_is_tight():
    rng = np.random.default_rng(1)
    for scale in (1e-30, 1e-6, 1.0, 3.0, 1e6):
        x = (rng.standard_normal(4096) * scale).astype(np.float32)
        codes, s = codec.encode_block(x, "fp8_e4m3fn_scaled")
        assert math.log2(s) == int(math.log2(s))
        v = codec.decode(codes, codec.FP8_E4M3FN)
        assert np.all(np.isfinite(v))
        assert np.max(np.abs(v)) <= 448.0
        assert np.max(np.abs(x)) / s > 224.0     # the largest value lands in the top binade
        rt = codec.decode_block(codes, s, "fp8_e4m3fn_scaled")
        # 3 mantissa bits: relative error <= 2^-4 for values in the normal range of the block
        big = np.abs(x) > np.max(np.abs(x)) * 2.0 ** -6
        assert np.all(np.abs(rt[big] - x[big]) <= 2.0 ** -4 * np.abs(x[big]))


def test_roundtrip_fp32_and_fp64_modes():
    x = np.random.default_rng(2).standard_normal(100)
    assert np.array_equal(codec.roundtrip_block(x, "fp64"), x)
    assert np.array_equal(codec.roundtrip_block(x, "fp32"), x.astype(np.float32).astype(np.float64))


# -- subsampling and interpolation --------------------------------------------

def test_kept_steps_and_brackets():
    assert store.kept_steps(10, 1) == list(range(9, -1, -1))
    assert store.kept_steps(10, 4) == [9, 5, 1]
    assert store.kept_steps(16, 4) == [15, 11, 7, 3]
    assert store.kept_steps(5, 8) == [4]
    assert store.bracket(9, 10, 4) == (9, 9, 0.0)
    assert store.bracket(8, 10, 4) == (5, 9, 0.75)
    assert store.bracket(0, 10, 4) == (-1, 1, 0.5)
    assert store.bracket(2, 5, 8) == (-1, 4, 0.6)
    for T, k in [(1000, 16), (37, 5), (8, 8), (3, 1)]:
        assert len(store.kept_steps(T, k)) == math.ceil(T / k)


@pytest.mark.parametrize("T,k", [(64, 4), (100, 16), (37, 5), (20, 1)])
def test_interpolation_exact_for_linear_signals(T, k):
    """A signal linear in n that vanishes at the anchor n = -1 is reproduced exactly."""
    kept = {n: np.array([3.0 * (n + 1), -0.5 * (n + 1)]) for n in store.kept_steps(T, k)}
    for n in range(T):
        v = store.interpolate(n, T, k, kept, np.zeros(2))
        assert np.allclose(v, [3.0 * (n + 1), -0.5 * (n + 1)], rtol=0, atol=1e-12)


@pytest.mark.parametrize("k,factor", [(8, 0.983), (16, 0.932), (32, 0.739)])
def test_interpolation_sine_midpoint_factor(k, factor):
    """Fig. 1b analogue: 136 steps per period; mid-interval the interpolant is cos(pi k / 136) of the sine."""
    Ps = 136.0
    T = 40 * k
    f = lambda n: np.sin(2 * np.pi * (n + 1) / Ps + 0.3)
    kept = {n: np.array([f(n)]) for n in store.kept_steps(T, k)}
    for n1 in store.kept_steps(T, k)[:-1]:
        mid = n1 - k // 2
        v = store.interpolate(mid, T, k, kept, np.zeros(1))[0]
        assert v == pytest.approx(math.cos(math.pi * k / Ps) * f(mid), abs=1e-12)
    assert math.cos(math.pi * k / Ps) == pytest.approx(factor, abs=5e-4)


def test_storage_bytes_closed_form():
    # 128^3 with a 10-cell PML: 12 blocks of 108 x 108 per kept step
    assert store.shell_values_per_step(128, 128, 128, 10) == 12 * 108 * 108
    assert store.storage_bytes(128, 128, 128, 10, 1000, 1, "fp32") == (12 * 108 * 108 * 1000 * 4, 0)
    pay, sc = store.storage_bytes(256, 256, 128, 12, 4000, 16, "fp8_e4m3fn_scaled")
    full, _ = store.storage_bytes(256, 256, 128, 12, 4000, 1, "fp32")
    assert full / pay == 64.0 and sc == 250 * 48
    assert store.shell_values_per_step(20, 20, 20, 0) == 0


# -- the paper's worked numbers --------------------------------------------

def test_paper_eq1_time_step():
    e = json.load(open(GOLDEN))["entries"][0]
    dt = yee.courant_time_step(e["courant"], e["dx_m"], e["c_m_per_s"])
    assert float(f"{dt:.{e['printed_digits']}g}") == e["dt_s"]


def test_paper_period_and_steps_per_period():
    ents = json.load(open(GOLDEN))["entries"]
    period = ents[1]["wavelength_m"] / yee.SPEED_OF_LIGHT
    assert float(f"{period:.3g}") == ents[1]["period_s"]
    dt = yee.courant_time_step(0.99, 20e-9, yee.SPEED_OF_LIGHT)
    assert round(period / dt) == ents[2]["steps_per_period"]


def test_paper_compression_factor():
    e = json.load(open(GOLDEN))["entries"][3]
    assert store.compression_factor("fp8_e4m3fn_scaled", e["k"]) == e["factor"]
    assert codec.STORAGE_BITS["fp8_e4m3fn_scaled"] == e["bits"]
    assert store.compression_factor("fp32", 1) == 1.0
    assert store.compression_factor("bf16", 4) == 8.0


def test_cosine_similarity_eq2():
    x = np.array([1.0, 2.0, -3.0])
    assert metrics.cosine_similarity(x, 5 * x) == pytest.approx(1.0, abs=1e-15)
    assert metrics.cosine_similarity(x, -x) == pytest.approx(-1.0, abs=1e-15)
    assert metrics.cosine_similarity([1, 0], [0, 2]) == 0.0
    assert metrics.cosine_similarity([1, 1], [1, 0]) == pytest.approx(1 / math.sqrt(2), rel=1e-15)
    assert metrics.rel_l2([1.1, 2.0], [1.0, 2.0]) == pytest.approx(0.1 / math.sqrt(5), rel=1e-12)


# -- the unscaled 8-bit family of Section 3 (Fig. 3) ----------------------------

_TORCH_FNUZ = {"fp8_e4m3fnuz": torch.float8_e4m3fnuz, "fp8_e5m2fnuz": torch.float8_e5m2fnuz}


def _lib_codes(x32, dt):
    return torch.from_numpy(np.ascontiguousarray(x32, np.float32)).to(dt).view(torch.uint8).numpy().astype(np.int64)


@pytest.mark.parametrize("name", ["fp8_e4m3fnuz", "fp8_e5m2fnuz"])
def test_fnuz_encode_decode_match_library(name):
    fmt = codec.UNSCALED_FP8[name]
    rng = np.random.default_rng(3)
    x = _probe_values(fmt, rng)
    assert np.array_equal(codec.encode(x, fmt), _lib_codes(x, _TORCH_FNUZ[name]))
    # overflow and the sign of zero
    edge = np.array([1e9, -1e9, -0.0, -1e-30, np.nan], np.float32)
    assert np.array_equal(codec.encode(edge, fmt), _lib_codes(edge, _TORCH_FNUZ[name]))
    codes = np.arange(256)
    ref = torch.tensor(codes, dtype=torch.uint8).view(_TORCH_FNUZ[name]).to(torch.float64).numpy()
    mine = codec.decode(codes, fmt)
    assert np.array_equal(np.isnan(mine), np.isnan(ref))
    fin = ~np.isnan(ref)
    assert np.array_equal(mine[fin], ref[fin])


def test_e4m3b11fnuz_is_e4m3fnuz_scaled_by_eight():
    """Bias 11 vs bias 8 with identical fields: code(x) in b11 == code(8 x) in fnuz, value / 8."""
    fmt = codec.FP8_E4M3B11FNUZ
    rng = np.random.default_rng(4)
    x = _probe_values(fmt, rng)
    assert np.array_equal(codec.encode(x, fmt), _lib_codes(8.0 * x.astype(np.float64), torch.float8_e4m3fnuz))
    codes = np.arange(256)
    ref = torch.tensor(codes, dtype=torch.uint8).view(torch.float8_e4m3fnuz).to(torch.float64).numpy() / 8.0
    mine = codec.decode(codes, fmt)
    fin = ~np.isnan(ref)
    assert np.array_equal(mine[fin], ref[fin]) and np.isnan(mine[~fin]).all()
    assert np.max(mine[fin]) == 30.0 and np.min(mine[fin & (mine > 0)]) == 2.0 ** -13


def test_ieee_e4m3_agrees_with_e4m3fn_below_its_overflow():
    """IEEE-style e4m3 shares bias and fields with e4m3fn for exponent fields below 15 (max 240)."""
    fmt = codec.FP8_E4M3
    rng = np.random.default_rng(5)
    x = _probe_values(fmt, rng)
    x = x[np.abs(x.astype(np.float64)) < 248.0]
    assert np.array_equal(codec.encode(x, fmt), _lib_codes(x, torch.float8_e4m3fn))
    assert codec.decode(codec.encode(np.array([248.0, -1e3]), fmt), fmt).tolist() == [np.inf, -np.inf]
    assert codec.decode(np.array([0x78, 0x7f]), fmt)[0] == np.inf and np.isnan(codec.decode([0x7f], fmt)[0])


def test_e3m4_definition_constants():
    """No library cast exists for e3m4; its table comes from the generic field decoder pinned
    above on six formats.  Check the constants its definition fixes (bias 3, IEEE specials)."""
    fmt = codec.FP8_E3M4
    vals = codec.decode(np.arange(128), fmt)
    fin = vals[np.isfinite(vals)]
    assert fin.max() == 15.5 and fin[fin > 0].min() == 2.0 ** -6
    assert codec.decode([0x10], fmt)[0] == 0.25          # smallest normal 2^(1-3)
    assert codec.decode([0x70], fmt)[0] == np.inf
    assert codec.encode(np.array([15.75, 15.7]), fmt).tolist() == [0x70, 0x6F]   # tie to even -> inf


# --------------------------------------------------------------------------- cubic reconstruction option

@pytest.mark.parametrize("T,k", [(37, 5), (64, 16), (10, 4), (1000, 16), (9, 3)])
def test_cubic_reproduces_cubic_polynomials_through_the_anchor(T, k):
    # degree-3 Lagrange interpolation is exact for cubics; the zero anchor at -1 is a node,
    # so the polynomial must vanish there
    p = lambda t: (t + 1.0) * (0.3 * t * t - 2.0 * t + 5.0)
    kept = {n: np.array([p(n)]) for n in store.kept_steps(T, k)}
    for n in range(T):
        got = store.interpolate_cubic(n, T, k, kept, np.zeros(1))
        assert abs(float(got[0]) - p(n)) <= 1e-9 * max(1.0, abs(p(n))), (T, k, n)


def test_cubic_weights_partition_of_unity_and_kept_steps_exact():
    for T, k in [(37, 5), (100, 8), (17, 16)]:
        K = set(store.kept_steps(T, k))
        for n in range(T):
            nodes = store.cubic_nodes(n, T, k)
            assert abs(sum(w for _, w in nodes) - 1.0) < 1e-12
            if n in K:
                assert nodes == [(n, 1.0)]
            else:
                assert all(a in K or a == -1 for a, _ in nodes)
                assert min(a for a, _ in nodes) < n < max(a for a, _ in nodes)


def test_cubic_midpoint_factor_closed_form():
    # equally spaced nodes, n in the middle of the middle interval: weights (-1, 9, 9, -1)/16,
    # so a cosine centred there comes back scaled by (9 cos(th/2) - cos(3 th/2)) / 8, th = w k
    T, k, period = 1601, 16, 136.0
    w = 2.0 * math.pi / period
    n = T - 1 - 5 * k - k // 2                    # midway between kept steps, far from both ends
    kept = {m: np.array([math.cos(w * (m - n))]) for m in store.kept_steps(T, k)}
    got = float(store.interpolate_cubic(n, T, k, kept, np.zeros(1))[0])
    th = w * k
    assert abs(got - (9.0 * math.cos(th / 2) - math.cos(3 * th / 2)) / 8.0) < 1e-12
    lin = float(store.interpolate(n, T, k, kept, np.zeros(1))[0])
    assert abs(lin - math.cos(th / 2)) < 1e-12                 # the linear rule's factor
    assert abs(1 - got) < 0.1 * abs(1 - lin)                    # an order of magnitude closer at 8.5 samples/period


def test_cubic_falls_back_to_linear_with_few_nodes():
    T, k = 9, 4                                                 # kept steps 8, 4, 0 plus the anchor: 4 nodes
    assert len(store.cubic_nodes(2, T, k)) == 4
    T, k = 5, 3                                                 # kept 4, 1 plus the anchor: 3 nodes -> linear
    for n in range(T):
        a = store.interpolate_cubic(n, T, k, {m: np.array([m * 1.0 + 1]) for m in store.kept_steps(T, k)}, np.zeros(1))
        b = store.interpolate(n, T, k, {m: np.array([m * 1.0 + 1]) for m in store.kept_steps(T, k)}, np.zeros(1))
        assert np.array_equal(a, b)
