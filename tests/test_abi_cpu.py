"""The C-ABI library loads, exports every declared symbol, and validates arguments before any
HIP call (so these run on a machine without a GPU: every call here fails validation or is
host-only)."""

import ctypes
import os
import re
import subprocess
from dataclasses import replace

import numpy as np
import pytest

import workloads as w
import paper_2603_24027_amd as pk
from paper_2603_24027_amd import _lib
from oracle import store as ostore

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fdtd.h")


def test_every_declared_symbol_is_exported():
    decl = set(re.findall(r"FDTD_API\s+[\w\s\*]+?\b(\w+)\s*\(", open(HEADER).read()))
    assert decl == set(_lib.EXPORTS)
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True, text=True,
                         check=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if " T " in ln}
    assert decl <= exported
    lib = pk.load()
    for name in decl:
        assert hasattr(lib, name)


def test_struct_layout_matches_header():
    # offsets of the ctypes mirror against the C layout rules for this header
    assert ctypes.sizeof(_lib.FdtdStoreCfg) == 12
    assert ctypes.sizeof(_lib.FdtdStoreInfo) == 11 * 8
    assert ctypes.sizeof(_lib.FdtdRecord) == 24
    assert _lib.FdtdProblem.courant.offset == 24
    assert _lib.FdtdProblem.src_wave.offset % 8 == 0
    # the loss kind and the magnetic current follow the design box (pointers 8-byte aligned)
    P_ = _lib.FdtdProblem
    assert P_.loss.offset == P_.des_hi.offset + 12
    assert P_.msrc_comp.offset == P_.loss.offset + 4 and P_.msrc_hi.offset == P_.msrc_lo.offset + 12
    assert P_.msrc_wave.offset == (P_.msrc_hi.offset + 12 + 7) // 8 * 8
    assert P_.msrc_profile.offset == P_.msrc_wave.offset + 8
    assert ctypes.sizeof(P_) == P_.msrc_profile.offset + 8


@pytest.mark.parametrize("name", ["c1", "c2", "c4", "c5", "tiny", "ragged"])
def test_store_config_matches_closed_form(name):
    kw = {"steps": 8} if name in ("c4", "c5") else {}
    prob = w.make(name, **kw)
    p = pk.Problem(prob)
    modes = [("fp32", "fp32"), ("fp16", "fp16"), ("bf16", "bf16"), ("fp8_e4m3_scaled", "fp8_e4m3fn_scaled")]
    modes += [(m, m) for m in ("fp8_e4m3b11fnuz", "fp8_e5m2fnuz", "fp8_e4m3fnuz", "fp8_e4m3", "fp8_e3m4", "fp8_e4m3fn")]
    for dtype, mode in modes:
        for k in (1, 3, 16):
            info = pk.store_config(p, dtype, k)
            pay, sc = ostore.storage_bytes(prob.nx, prob.ny, prob.nz, prob.pml, prob.steps, k, mode)
            assert info.payload_bytes == pay and info.scale_bytes == sc
            assert info.values_per_slice == ostore.shell_values_per_step(prob.nx, prob.ny, prob.nz, prob.pml)
            assert info.slices == len(ostore.kept_steps(prob.steps, k))
            assert info.store_bytes >= pay + sc
            stride = info.fields_bytes // 24          # floats between components: >= cells, whole lines
            assert info.fields_bytes == 24 * stride and stride >= prob.cells and stride % 32 == 0
            assert info.design_cells == int(np.prod(prob.design_shape))


def test_compression_factor_64x_on_slab_config():
    p = pk.Problem(w.c4(steps=4000))
    full = pk.store_config(p, "fp32", 1).payload_bytes
    small = pk.store_config(p, "fp8_e4m3_scaled", 16).payload_bytes
    assert full / small == 64.0


@pytest.mark.parametrize("name", ["c1", "c4", "c5", "ragged"])
def test_workspace_does_not_depend_on_the_sweep_choice(name, monkeypatch):
    # the caller sizes the workspace from store_config once; one or two steps per sweep
    # (forward or reverse) and the launch order must all fit that same size
    kw = {"steps": 9} if name in ("c4", "c5") else {}
    p = pk.Problem(w.make(name, **kw))
    ref = pk.store_config(p, "fp8_e4m3_scaled", 4).workspace_bytes
    for env in ({"FDTD_FWD_STEPS": "1"}, {"FDTD_FWD_STEPS": "2"}, {"FDTD_REV_STEPS": "1"}, {"FDTD_REV_STEPS": "2"},
                {"FDTD_TILE_ORDER": "1"}, {"FDTD_TILE_ORDER": "2"}):
        for key, value in env.items():
            monkeypatch.setenv(key, value)
        assert pk.store_config(p, "fp8_e4m3_scaled", 4).workspace_bytes == ref, env
        for key in env:
            monkeypatch.delenv(key)


def _call_forward(prob, dtype="fp32", k=1, interp=1):
    lib = pk.load()
    p = pk.Problem(prob)
    cfg = _lib.FdtdStoreCfg(pk.STORE_DTYPES[dtype], k, interp)
    rec = _lib.FdtdRecord()
    return lib.fdtd_forward(ctypes.byref(p.c), ctypes.byref(cfg), None, None, None, None, None, None, None,
                            ctypes.byref(rec), None)


def test_validation_errors_before_any_device_work():
    base = w.tiny()
    assert _call_forward(base) == _lib.FDTD_EINVAL                       # NULL device buffers
    assert "NULL" in pk.load().fdtd_last_error().decode()
    assert _call_forward(replace(base, courant=1.01)) == _lib.FDTD_ECFL
    assert _call_forward(replace(base, courant=0.0)) == _lib.FDTD_ECFL
    assert _call_forward(replace(base, courant=float("nan"))) == _lib.FDTD_ECFL
    assert _call_forward(replace(base, des_lo=(2, 5, 5))) == _lib.FDTD_EREGION    # into the PML
    assert _call_forward(replace(base, det_hi=(8, 8, 10))) == _lib.FDTD_EREGION
    assert _call_forward(replace(base, src_lo=(6, 6, 6), src_hi=(6, 7, 7))) == _lib.FDTD_EREGION  # empty
    assert _call_forward(replace(base, pml=6)) == _lib.FDTD_EINVAL       # 2P >= n
    assert _call_forward(replace(base, boundary=1)) == _lib.FDTD_EINVAL  # periodic with a PML
    assert _call_forward(replace(base, steps=0)) == _lib.FDTD_EINVAL
    assert _call_forward(replace(base, loss=4)) == _lib.FDTD_EINVAL       # unknown loss kind
    assert _call_forward(replace(base, loss=-1)) == _lib.FDTD_EINVAL
    pw = w.with_tfsf_plane_wave(base, 5, 8.0)
    assert _call_forward(replace(pw, msrc_lo=(0, 3, 4))) == _lib.FDTD_EREGION   # sheet into the PML
    assert _call_forward(replace(pw, msrc_comp=3)) == _lib.FDTD_EINVAL
    assert _call_forward(base, k=0) == _lib.FDTD_ESTORE
    assert _call_forward(base, interp=2) == _lib.FDTD_ESTORE               # only linear (0, 1) or cubic (3)
    assert _call_forward(base, interp=3) == _lib.FDTD_EINVAL               # valid: fails on the NULL buffers
    assert _call_forward(base, dtype="fp8_e4m3_scaled", k=4) == _lib.FDTD_EINVAL


def test_backward_record_checks():
    lib = pk.load()
    prob = w.tiny()
    p = pk.Problem(prob)
    cfg = _lib.FdtdStoreCfg(0, 1)
    rec = _lib.FdtdRecord(problem_hash=123, dtype=0, k=1, steps=prob.steps, consumed=0)
    args = (None,) * 8
    rc = lib.fdtd_backward(ctypes.byref(p.c), ctypes.byref(cfg), *args, ctypes.byref(rec), None)
    assert rc == _lib.FDTD_ESTORE                                         # record of another problem
    assert "different problem" in lib.fdtd_last_error().decode()
    rec2 = _lib.FdtdRecord(problem_hash=123, dtype=0, k=2, steps=prob.steps, consumed=1)
    assert lib.fdtd_backward(ctypes.byref(p.c), ctypes.byref(cfg), *args, ctypes.byref(rec2), None) \
        == _lib.FDTD_ESTORE
    assert lib.fdtd_backward(ctypes.byref(p.c), ctypes.byref(cfg), *args, None, None) == _lib.FDTD_EINVAL
    with pytest.raises(pk.FdtdError) as e:
        _lib.check(_lib.FDTD_ESTATE)
    assert e.value.code == _lib.FDTD_ESTATE


def test_codec_entry_validation():
    lib = pk.load()
    assert lib.fdtd_codec_roundtrip(10, None, 1, 1, None, None, None, None) == _lib.FDTD_ESTORE
    assert lib.fdtd_codec_roundtrip(-1, None, 1, 1, None, None, None, None) == _lib.FDTD_ESTORE
    assert lib.fdtd_codec_roundtrip(0, None, -1, 1, None, None, None, None) == _lib.FDTD_EINVAL
    assert lib.fdtd_codec_roundtrip(3, None, 1, 4, None, None, None, None) == _lib.FDTD_EINVAL
    assert lib.fdtd_codec_roundtrip(0, None, 0, 4, None, None, None, None) == _lib.FDTD_OK


def test_strerror_table():
    lib = pk.load()
    for code in range(0, -8, -1):
        assert lib.fdtd_strerror(code)
    assert lib.fdtd_strerror(-99) == b"unknown error"


def test_noalloc_forward_validates_before_device_work():
    # NULL buffers, then a problem whose workspace exceeds the library's array: both refused
    # before any HIP call (non-NULL stand-in pointers are never dereferenced on this path)
    lib = pk.load()
    fake = ctypes.c_void_p(0x1000)
    for prob, want in [(w.tiny(), None), (w.c4(steps=8), _lib.FDTD_EINVAL)]:
        p = pk.Problem(prob)
        cfg = _lib.FdtdStoreCfg(0, 1)
        rec = _lib.FdtdRecord()
        assert lib.fdtd_forward_noalloc(ctypes.byref(p.c), ctypes.byref(cfg), None, None, None, None, None, None,
                                        ctypes.byref(rec), None) == _lib.FDTD_EINVAL
        if want is not None:
            info = pk.store_config(p, "fp32", 1)
            assert info.workspace_bytes - info.fields_bytes > _lib.NOALLOC_SCRATCH_BYTES
            rc = lib.fdtd_forward_noalloc(ctypes.byref(p.c), ctypes.byref(cfg), fake, fake, fake, fake, fake, None,
                                          ctypes.byref(rec), None)
            assert rc == want
            assert "FDTD_NOALLOC_SCRATCH_BYTES" in lib.fdtd_last_error().decode()


def test_noalloc_limit_matches_header():
    text = open(HEADER).read()
    m = re.search(r"#define FDTD_NOALLOC_SCRATCH_BYTES \((\d+)u << (\d+)\)", text)
    assert m and int(m.group(1)) << int(m.group(2)) == _lib.NOALLOC_SCRATCH_BYTES
    # a 128^3 problem fits (the header's claim), for every storage type
    p = pk.Problem(w.c2())
    for dtype in pk.STORE_DTYPES:
        info = pk.store_config(p, dtype, 1)
        assert info.workspace_bytes - info.fields_bytes <= _lib.NOALLOC_SCRATCH_BYTES
