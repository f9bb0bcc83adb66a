"""HIP path vs FP64 oracle on the same seeded inputs (needs an MI355X).

Tolerances:
  * fields and loss, FP32 storage k = 1: relative L2 <= 1e-5 (all six components,
    final state), and element by element, per component, max |d| <= 3e-5 of the
    component's largest magnitude, on the interior and on the PML slabs separately;
    per-step loss terms <= 1e-5 relative;
  * gradient, FP32 k = 1: relative L2 <= 1e-4 against the oracle's FP64 gradient
    (FP32 round-off accumulated over the forward and the reversed sweep), and every
    design cell within 1e-4 of the gradient's largest magnitude;
  * compressed storage: against the oracle running the same codec and
    interpolation, cosine >= 0.9999 and relative L2 <= 1e-2 (codes may differ
    where the FP32 and FP64 recorded values straddle a rounding boundary);
  * the codec on its own: bit-exact codes, scales and decoded values.
"""

from dataclasses import replace

import numpy as np
import pytest
import torch

import workloads as w
import paper_2603_24027_amd as pk
from oracle import adjoint, codec, metrics, yee

from gpu_helpers import gpu_run, rel, require_gpu, say

pytestmark = pytest.mark.gpu

ORACLE_MODE = {"fp32": "fp32", "fp16": "fp16", "bf16": "bf16", "fp8_e4m3_scaled": "fp8_e4m3fn_scaled",
               **{m: m for m in ("fp8_e4m3b11fnuz", "fp8_e5m2fnuz", "fp8_e4m3fnuz", "fp8_e4m3", "fp8_e3m4",
                                 "fp8_e4m3fn")}}


def _periodic_problem():
    n = (24, 20, 16)
    p = w.dipole_problem("periodic", n, 0, 80, (12, 10, 8), 10.0, (8, 6, 5), (14, 12, 9), (2, 2, 12), (22, 18, 13))
    return replace(p, boundary=1, name="periodic_24x20x16")


CASES = {
    "tiny": lambda: w.tiny(),
    "c1": lambda: w.c1(),
    "ragged": lambda: w.ragged(),
    "kappa": lambda: replace(w.tiny(n=(20, 18, 16), pml=4, steps=70), pml_kappa_max=3.0, pml_alpha_max=0.15),
    "periodic": _periodic_problem,
    "nopml_zero_boundary": lambda: replace(w.tiny(n=(14, 13, 12), steps=50), pml=0),
}


# --------------------------------------------------------------------------- codec

@pytest.mark.parametrize("dtype", list(ORACLE_MODE))
def test_codec_bit_exact(dtype):
    require_gpu()
    say("codec", dtype)
    rng = np.random.default_rng(42)
    blocks = []
    for b, scale in enumerate([1e-30, 1e-8, 3e-5, 1e-3, 0.02, 1.0, 7.5, 300.0, 1e5, 0.0, 1e-40, 2.0]):
        x = rng.standard_normal(4099) * scale
        x[:8] = [0.0, -0.0, scale, -scale, scale * 0.5, 1e-45, -1e-41, scale * (1 + 2 ** -12)]
        blocks.append(x.astype(np.float32))
    vals = np.stack(blocks)
    vals[9] = 0.0                                   # an all-zero block
    if dtype in ("fp16",):
        vals = np.clip(vals, -60000, 60000).astype(np.float32)
    t = torch.from_numpy(vals.ravel().copy()).cuda()
    codes, scales, dec = pk.codec_roundtrip(t, dtype, vals.shape[0])
    torch.cuda.synchronize()
    codes = codes.cpu().numpy()
    dec = dec.cpu().numpy().reshape(vals.shape)
    mode = ORACLE_MODE[dtype]
    for b in range(vals.shape[0]):
        ref_codes, ref_s = codec.encode_block(vals[b], mode)
        ref_dec = codec.decode_block(ref_codes, ref_s, mode).astype(np.float32)
        got = codes.reshape(vals.shape)[b]
        if dtype == "fp32":
            assert np.array_equal(got.view(np.float32), ref_codes.astype(np.float32))
        else:
            mask = (1 << (8 * got.itemsize)) - 1
            assert np.array_equal(got.astype(np.int64) & mask, ref_codes), (dtype, b)
        if dtype == "fp8_e4m3_scaled":
            assert float(scales[b].item()) == ref_s, (b, float(scales[b].item()), ref_s)
        nan = np.isnan(ref_dec)
        assert np.array_equal(np.isnan(dec[b]), nan), (dtype, b)
        assert np.array_equal(dec[b][~nan].view(np.uint32), ref_dec[~nan].view(np.uint32)), (dtype, b)


# --------------------------------------------------------------------------- forward

def assert_fields_elementwise(prob, E, H, st, tol=3e-5):
    """Per component: max |d| / max |ref| on the interior and on the PML slabs (each <= tol of
    the component's largest magnitude); the region-normalised figure is printed as well."""
    P = prob.pml
    interior = np.zeros(prob.shape, bool)
    interior[P:prob.nz - P, P:prob.ny - P, P:prob.nx - P] = True
    names = ("Ex", "Ey", "Ez", "Hx", "Hy", "Hz")
    for c in range(6):
        got = (E if c < 3 else H)[c % 3]
        ref = (st.E if c < 3 else st.H)[c % 3]
        scale = np.max(np.abs(ref))
        if scale == 0.0:
            assert np.max(np.abs(got)) == 0.0
            continue
        d = np.abs(got - ref)
        for region, mask in (("interior", interior), ("pml", ~interior)):
            if not mask.any():
                continue
            err = float(d[mask].max()) / scale
            own = float(d[mask].max()) / max(float(np.abs(ref[mask]).max()), 1e-300)
            say("  %s %-8s max|d|/max|ref| %.2e (of the region's own max %.2e)" % (names[c], region, err, own))
            assert err <= tol, (names[c], region, err)


@pytest.mark.parametrize("case", list(CASES))
def test_forward_fields_and_loss(case):
    require_gpu()
    prob = CASES[case]()
    say("forward", case, prob.shape, prob.steps)
    out = gpu_run(prob, series=True, backward=False)
    s = yee.Solver(prob, match_fp32=True)
    st, losses, _ = yee.run_forward(s)
    assert rel(out["E"], st.E) <= 1e-5
    assert rel(out["H"], st.H) <= 1e-5
    assert_fields_elementwise(prob, out["E"], out["H"], st)
    assert abs(out["loss"] - losses.sum()) <= 1e-5 * abs(losses.sum())
    big = losses > 1e-6 * losses.max()
    assert np.max(np.abs(out["series"][big] - losses[big]) / losses[big]) <= 1e-4
    assert abs(out["series"].sum() - out["loss"]) <= 1e-12 * out["loss"]


@pytest.mark.parametrize("frac", [4, 2])
def test_forward_fields_at_partial_horizon(frac):
    require_gpu()
    prob = w.c1(steps=200 // frac)
    say("forward c1 steps", prob.steps)
    out = gpu_run(prob, backward=False)
    st, _, _ = yee.run_forward(yee.Solver(prob, match_fp32=True))
    assert rel(out["E"], st.E) <= 1e-5 and rel(out["H"], st.H) <= 1e-5


# --------------------------------------------------------------------------- gradient

@pytest.mark.parametrize("case", list(CASES))
def test_gradient_fp32_full_storage(case):
    require_gpu()
    prob = CASES[case]()
    say("gradient fp32 k=1", case)
    out = gpu_run(prob)
    L, g = adjoint.grad_time_reversal(prob, "fp64", 1, match_fp32=True)
    assert abs(out["loss"] - L) <= 1e-5 * abs(L)
    r = rel(out["grad"], g)
    cos = metrics.cosine_similarity(out["grad"], g)
    cell = float(np.max(np.abs(out["grad"] - g)) / np.max(np.abs(g)))
    say("  rel-L2 %.3e cosine %.12f per-cell max|d|/max|g| %.3e" % (r, cos, cell))
    assert r <= 1e-4 and cos >= 1 - 1e-8
    assert cell <= 1e-4


def test_gradient_against_finite_differences():
    require_gpu()
    prob = w.tiny()
    say("gradient vs FD, tiny, all design cells")
    out = gpu_run(prob)
    fd = adjoint.grad_finite_difference(prob, np.arange(out["grad"].size), h=1e-4)
    g = out["grad"].ravel()
    assert np.all(np.abs(g - fd) <= 1e-4 * np.max(np.abs(fd)) + 1e-4 * np.abs(fd))
    prob = w.c1()
    cells = w.fd_cells(prob, 3, seed=0)
    say("gradient vs FD, c1, cells", cells)
    out = gpu_run(prob)
    fd = adjoint.grad_finite_difference(prob, cells, h=1e-4)
    g = out["grad"].ravel()[cells]
    scale = np.max(np.abs(out["grad"]))
    assert np.all(np.abs(g - fd) <= 1e-3 * scale + 1e-3 * np.abs(fd)), (g, fd)


@pytest.mark.parametrize("dtype", ["fp32", "fp16", "bf16", "fp8_e4m3_scaled"])
@pytest.mark.parametrize("k", [1, 3, 16])
def test_gradient_compressed_against_oracle_compressed(dtype, k):
    require_gpu()
    prob = w.c1()
    say("gradient", dtype, "k", k, "c1")
    out = gpu_run(prob, dtype, k)
    _, g = adjoint.grad_time_reversal(prob, ORACLE_MODE[dtype], k, match_fp32=True)
    r = rel(out["grad"], g)
    cos = metrics.cosine_similarity(out["grad"], g)
    say("  vs oracle same codec: rel-L2 %.3e cosine %.9f" % (r, cos))
    assert cos >= 0.9999 and r <= 1e-2
    if dtype in ("fp32", "fp16", "bf16") and k in (1, 3):
        assert r <= 1e-3


@pytest.mark.parametrize("dtype,k,case", [("fp32", 3, "c1"), ("fp32", 16, "c1"), ("fp8_e4m3_scaled", 16, "c1"),
                                          ("bf16", 5, "ragged"), ("fp16", 4, "kappa")])
def test_gradient_cubic_reconstruction_against_oracle(dtype, k, case):
    """The cubic option of the reinjection (four nodes, zero anchor, shifted at the ends)
    against the oracle running the same rule."""
    require_gpu()
    prob = CASES[case]()
    say("gradient cubic", dtype, "k", k, case)
    out = gpu_run(prob, dtype, k, interp="cubic")
    _, g = adjoint.grad_time_reversal(prob, ORACLE_MODE[dtype], k, match_fp32=True, interp=3)
    r = rel(out["grad"], g)
    cos = metrics.cosine_similarity(out["grad"], g)
    say("  vs oracle same codec and rule: rel-L2 %.3e cosine %.9f" % (r, cos))
    assert cos >= 0.9999 and r <= 1e-2
    if dtype == "fp32":
        assert r <= 1e-3


@pytest.mark.parametrize("dtype", ["fp8_e4m3b11fnuz", "fp8_e5m2fnuz", "fp8_e4m3fnuz", "fp8_e4m3", "fp8_e3m4",
                                   "fp8_e4m3fn"])
def test_gradient_unscaled_fp8_against_oracle(dtype):
    """The unscaled 8-bit types of Section 3 through the whole path (k = 4)."""
    require_gpu()
    prob = w.c1()
    say("gradient", dtype, "k 4 c1")
    out = gpu_run(prob, dtype, 4)
    _, g = adjoint.grad_time_reversal(prob, ORACLE_MODE[dtype], 4, match_fp32=True)
    cos = metrics.cosine_similarity(out["grad"], g)
    say("  vs oracle same codec: rel-L2 %.3e cosine %.9f" % (rel(out["grad"], g), cos))
    assert cos >= 0.999


def test_gradient_ragged_compressed_k_not_dividing_T():
    require_gpu()
    prob = w.ragged(steps=37)
    say("gradient ragged fp8 k=5 (5 does not divide 37)")
    out = gpu_run(prob, "fp8_e4m3_scaled", 5)
    _, g = adjoint.grad_time_reversal(prob, "fp8_e4m3fn_scaled", 5, match_fp32=True)
    assert metrics.cosine_similarity(out["grad"], g) >= 0.9999


def test_single_step_and_k_beyond_T():
    require_gpu()
    for steps, k in [(1, 1), (6, 10)]:
        prob = w.tiny(steps=steps)
        say("gradient tiny steps", steps, "k", k)
        out = gpu_run(prob, "fp16", k)
        L, g = adjoint.grad_time_reversal(prob, "fp16", k, match_fp32=True)
        assert abs(out["loss"] - L) <= 1e-5 * abs(L) + 1e-30
        if np.linalg.norm(g) > 0:
            assert metrics.cosine_similarity(out["grad"], g) >= 0.9999


# --------------------------------------------------------------------------- binding

def test_autograd_function_and_double_backward():
    require_gpu()
    prob = w.tiny()
    say("autograd tiny")
    gobj = pk.Gradient(prob, "fp32", 1)
    bg = torch.from_numpy(prob.eps).cuda()
    design = torch.from_numpy(prob.design_eps()).cuda().requires_grad_(True)
    loss = pk.FDTDGrad.apply(design, gobj, bg)
    (3.0 * loss).backward()
    _, g = adjoint.grad_time_reversal(prob, "fp64", 1, match_fp32=True)
    assert rel(design.grad.double().cpu().numpy(), 3.0 * g) <= 1e-4
    with pytest.raises(pk.FdtdError) as e:
        gobj.backward()
    assert e.value.code == -5


def test_deterministic_repeat():
    require_gpu()
    prob = w.c1()
    say("determinism c1 fp8 k=4")
    a = gpu_run(prob, "fp8_e4m3_scaled", 4)
    b = gpu_run(prob, "fp8_e4m3_scaled", 4)
    assert a["loss"] == b["loss"]
    assert np.array_equal(a["grad"], b["grad"])


def test_graph_replay_matches_eager():
    """Repeated calls replay the captured launch sequence; every replay equals the eager run
    bitwise, with unrelated eager work and synchronisations between replays."""
    require_gpu()
    prob = w.c1()
    say("graph replay vs eager, c1 fp8 k=4 and fp32 k=1")
    for dtype, k in [("fp8_e4m3_scaled", 4), ("fp32", 1)]:
        pk.set_graphs(False)
        try:
            ref = gpu_run(prob, dtype, k, series=True)
        finally:
            pk.set_graphs(True)
        gobj = pk.Gradient(prob, dtype, k, series=True)
        eps = torch.from_numpy(prob.eps).cuda()
        for rep in range(4):
            loss = float(gobj.forward(eps).item())
            series = gobj.buf.series.cpu().numpy()
            grad = gobj.backward().cpu().numpy()
            torch.cuda.synchronize()
            junk = torch.arange(4096, device="cuda", dtype=torch.float32)
            assert float((junk * 2).sum().item()) == 4095.0 * 4096.0
            assert loss == ref["loss"], (dtype, rep)
            assert np.array_equal(series, ref["series"]), (dtype, rep)
            assert np.array_equal(grad, ref["grad"]), (dtype, rep)


# --------------------------------------------------------------------------- Poynting-flux objective

FLUX_CASES = {
    "tiny_flux_z": lambda: replace(w.tiny(), loss=3),
    "c1_flux_z": lambda: replace(w.c1(), loss=3),
    "ragged_flux_x": lambda: replace(w.ragged(), loss=1, pml_kappa_max=3.0),
    "periodic_flux_y": lambda: replace(_periodic_problem(), loss=2),
}


@pytest.mark.parametrize("case", list(FLUX_CASES))
def test_flux_objective_forward_and_gradient(case):
    require_gpu()
    prob = FLUX_CASES[case]()
    say("flux objective", case, "loss kind", prob.loss)
    out = gpu_run(prob, series=True)
    _, losses, _ = yee.run_forward(yee.Solver(prob, match_fp32=True))
    scale = np.sum(np.abs(losses))          # the flux changes sign: compare against the size of its terms
    assert abs(out["loss"] - losses.sum()) <= 1e-5 * scale
    assert np.max(np.abs(out["series"] - losses)) <= 1e-4 * np.max(np.abs(losses))
    L, g = adjoint.grad_time_reversal(prob, "fp64", 1, match_fp32=True)
    r = rel(out["grad"], g)
    cos = metrics.cosine_similarity(out["grad"], g)
    say("  rel-L2 %.3e cosine %.12f" % (r, cos))
    assert r <= 1e-4 and cos >= 1 - 1e-8


def test_flux_gradient_against_finite_differences():
    require_gpu()
    prob = replace(w.tiny(), loss=3)
    out = gpu_run(prob)
    fd = adjoint.grad_finite_difference(prob, np.arange(out["grad"].size), h=1e-4)
    g = out["grad"].ravel()
    assert np.all(np.abs(g - fd) <= 1e-4 * np.max(np.abs(fd)) + 1e-4 * np.abs(fd))


def test_flux_compressed_against_oracle_compressed():
    require_gpu()
    prob = replace(w.c1(), loss=3)
    out = gpu_run(prob, "fp8_e4m3_scaled", 4)
    _, g = adjoint.grad_time_reversal(prob, ORACLE_MODE["fp8_e4m3_scaled"], 4, match_fp32=True)
    cos = metrics.cosine_similarity(out["grad"], g)
    say("  fp8 k=4 flux: cosine vs oracle-compressed %.8f" % cos)
    assert cos >= 0.9999


# --------------------------------------------------------------------------- plane-wave (TFSF) source

TFSF_CASES = {
    "tiny_pw_flux": lambda: w.tiny_pw(),
    "c1_pw_energy": lambda: w.with_tfsf_plane_wave(w.c1(), 10, 20.0),
    "periodic_pw_flux": lambda: replace(w.with_tfsf_plane_wave(_periodic_problem(), 4, 10.0, 0.6), loss=3),
}


@pytest.mark.parametrize("case", list(TFSF_CASES))
def test_tfsf_forward_and_gradient(case):
    require_gpu()
    prob = TFSF_CASES[case]()
    say("plane-wave source", case)
    out = gpu_run(prob)
    st, losses, _ = yee.run_forward(yee.Solver(prob, match_fp32=True))
    assert rel(out["E"], st.E) <= 1e-5 and rel(out["H"], st.H) <= 1e-5
    assert abs(out["loss"] - losses.sum()) <= 1e-5 * np.sum(np.abs(losses))
    L, g = adjoint.grad_time_reversal(prob, "fp64", 1, match_fp32=True)
    r = rel(out["grad"], g)
    cos = metrics.cosine_similarity(out["grad"], g)
    say("  rel-L2 %.3e cosine %.12f" % (r, cos))
    assert r <= 1e-4 and cos >= 1 - 1e-8


def test_tfsf_compressed_against_oracle_compressed():
    require_gpu()
    prob = w.with_tfsf_plane_wave(w.c1(), 10, 20.0)
    out = gpu_run(prob, "bf16", 3)
    _, g = adjoint.grad_time_reversal(prob, ORACLE_MODE["bf16"], 3, match_fp32=True)
    cos = metrics.cosine_similarity(out["grad"], g)
    say("  bf16 k=3 plane wave: cosine vs oracle-compressed %.8f" % cos)
    assert cos >= 0.9999


# --------------------------------------------------------------------------- tile shapes

TILES = {
    "fwd8x4": {"FDTD_TILE_Y": "8", "FDTD_TILE_Z": "4"},
    "fwd8x8": {"FDTD_TILE_Y": "8", "FDTD_TILE_Z": "8"},
    "adj4x8": {"FDTD_ADJ_TILE_Y": "4", "FDTD_ADJ_TILE_Z": "8"},   # the large-grid default
    "adj4x4_rev8x8": {"FDTD_ADJ_TILE_Y": "4", "FDTD_ADJ_TILE_Z": "4", "FDTD_REV_TILE_Y": "8",
                      "FDTD_REV_TILE_Z": "8"},
    "rev4x5": {"FDTD_REV_TILE_Z": "5"},
    "rev4x6": {"FDTD_REV_TILE_Z": "6"},
    "adj8x4_rev4x8_fwd4x4": {"FDTD_ADJ_TILE_Y": "8", "FDTD_ADJ_TILE_Z": "4", "FDTD_REV_TILE_Y": "4",
                             "FDTD_REV_TILE_Z": "8", "FDTD_TILE_Y": "4", "FDTD_TILE_Z": "4"},
}


@pytest.mark.parametrize("tiles", list(TILES))
@pytest.mark.parametrize("case", ["ragged", "kappa"])
def test_every_tile_shape_against_oracle(tiles, case, monkeypatch):
    # every instantiated sweep shape, including the ones only large grids select by default
    require_gpu()
    for name, value in TILES[tiles].items():
        monkeypatch.setenv(name, value)
    prob = CASES[case]()
    say("tile shapes", tiles, case)
    out = gpu_run(prob, "fp16", 3)
    L, g = adjoint.grad_time_reversal(prob, "fp16", 3, match_fp32=True)
    assert abs(out["loss"] - L) <= 1e-5 * abs(L)
    r = rel(out["grad"], g)
    cos = metrics.cosine_similarity(out["grad"], g)
    say("  rel-L2 %.3e cosine %.12f" % (r, cos))
    assert cos >= 0.9999 and r <= 1e-2


@pytest.mark.parametrize("case,steps", [("ragged", 1), ("kappa", 1), ("c1", 1), ("periodic", 1), ("ragged", 2),
                                        ("kappa", 2)])
def test_launch_orders_give_the_same_bits(case, steps, monkeypatch):
    # the order table only decides where each tile's workgroup runs (loss partials are
    # indexed by tile), so the default and the octant orders agree bit for bit, with one
    # or two steps per forward and per reverse primal sweep; the octant order is checked
    # against the oracle
    require_gpu()
    prob = CASES[case]()
    monkeypatch.setenv("FDTD_FWD_STEPS", str(steps))
    monkeypatch.setenv("FDTD_REV_STEPS", str(steps))
    say("launch orders", case, "steps per sweep", steps)
    outs = []
    for order in ("1", "2"):
        monkeypatch.setenv("FDTD_TILE_ORDER", order)
        outs.append(gpu_run(prob, keep_fields=False))
    assert outs[0]["loss"] == outs[1]["loss"]
    assert np.array_equal(outs[0]["grad"], outs[1]["grad"])
    L, g = adjoint.grad_time_reversal(prob, "fp64", 1, match_fp32=True)
    r = rel(outs[1]["grad"], g)
    say("  octant order vs oracle: rel-L2 %.3e" % r)
    assert abs(outs[1]["loss"] - L) <= 1e-5 * abs(L) and r <= 1e-4


SHELL_GRIDS = {
    # the one-step reversal puts the x-face shell cells into row 0 of their plane when
    # P >= 2 and the face's rows fit in one grid row; these grids take either path
    "pml2_rows_fit": lambda: w.tiny(n=(20, 18, 16), pml=2, steps=50),
    "pml1_in_place": lambda: w.tiny(n=(14, 13, 12), pml=1, steps=50),
    "tall_in_place": lambda: w.tiny(n=(16, 40, 16), pml=3, steps=50),
}


@pytest.mark.parametrize("case", list(SHELL_GRIDS))
@pytest.mark.parametrize("dtype,k", [("fp32", 1), ("fp16", 3)])
def test_interface_shell_layouts_against_oracle(case, dtype, k):
    require_gpu()
    prob = SHELL_GRIDS[case]()
    say("interface shell layout", case, dtype, "k", k)
    out = gpu_run(prob, dtype, k, keep_fields=False)
    L, g = adjoint.grad_time_reversal(prob, ORACLE_MODE[dtype], k, match_fp32=True)
    assert abs(out["loss"] - L) <= 1e-5 * abs(L)
    r = rel(out["grad"], g)
    cos = metrics.cosine_similarity(out["grad"], g)
    cell = float(np.max(np.abs(out["grad"] - g)) / np.max(np.abs(g)))
    say("  rel-L2 %.3e cosine %.12f per-cell %.3e" % (r, cos, cell))
    if dtype == "fp32":
        assert r <= 1e-4 and cell <= 1e-4
    else:
        assert cos >= 0.9999 and r <= 1e-2


def test_graph_cache_eviction_with_calls_in_flight():
    """More distinct calls than the graph cache keeps, enqueued without synchronising:
    evicting a graph waits for its last launch, and every result equals the eager one."""
    require_gpu()
    prob = w.tiny(steps=40)
    pk.set_graphs(False)
    try:
        ref = gpu_run(prob, "fp16", 2, keep_fields=False)
    finally:
        pk.set_graphs(True)
    eps = torch.from_numpy(prob.eps).cuda()
    objs, outs = [], []
    for i in range(12):                       # 24 distinct calls (forward and backward each)
        g = pk.Gradient(prob, "fp16", 2)
        loss = g.forward(eps)
        outs.append((loss, g.backward()))
        objs.append(g)
    torch.cuda.synchronize()
    for loss, grad in outs:
        assert float(loss.item()) == ref["loss"]
        assert np.array_equal(grad.cpu().numpy(), ref["grad"])
