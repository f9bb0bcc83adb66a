"""Python binding of the HIP FDTD gradient library: buffers, calls, and a torch.autograd.Function.

Every step of the method runs in the library's kernels; this module only
builds the C structs, allocates device memory through torch, and passes
pointers and the current HIP stream.
"""

from __future__ import annotations

import ctypes
from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch

from . import _lib
from ._lib import FDTD_ENONFINITE, FDTD_ESTATE, FdtdError, FdtdProblem, FdtdRecord, FdtdStoreCfg, FdtdStoreInfo, \
    check, load

STORE_DTYPES = {
    "fp32": _lib.STORE_FP32,
    "fp16": _lib.STORE_FP16,
    "bf16": _lib.STORE_BF16,
    "fp8_e4m3_scaled": _lib.STORE_FP8_E4M3_SCALED,
    "fp8_e4m3b11fnuz": _lib.STORE_FP8_E4M3B11FNUZ,
    "fp8_e5m2fnuz": _lib.STORE_FP8_E5M2FNUZ,
    "fp8_e4m3fnuz": _lib.STORE_FP8_E4M3FNUZ,
    "fp8_e4m3": _lib.STORE_FP8_E4M3,
    "fp8_e3m4": _lib.STORE_FP8_E3M4,
    "fp8_e4m3fn": _lib.STORE_FP8_E4M3FN,
}
STORAGE_BITS = {name: (32 if name == "fp32" else 16 if name in ("fp16", "bf16") else 8) for name in STORE_DTYPES}


def _i3(v):
    return _lib.I3(*[int(x) for x in v])


def _stream_handle(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


class Problem:
    """C-struct view of a problem description (grid, PML, source, detector, design box, eps).

    ``desc`` is any object with the fields of ``workloads.Problem``.
    """

    def __init__(self, desc):
        self.desc = desc
        self._wave = np.ascontiguousarray(desc.src_wave, np.float32)
        self._profile = np.ascontiguousarray(desc.src_profile, np.float32)
        self._mwave = np.ascontiguousarray(getattr(desc, "msrc_wave", np.zeros(0)), np.float32)
        self._mprofile = np.ascontiguousarray(getattr(desc, "msrc_profile", np.zeros(0)), np.float32)
        has_m = self._mwave.size > 0 and self._mprofile.size > 0
        fp = ctypes.POINTER(ctypes.c_float)
        self.c = FdtdProblem(
            nx=desc.nx, ny=desc.ny, nz=desc.nz, pml=desc.pml, steps=desc.steps, boundary=desc.boundary,
            courant=desc.courant, pml_order=desc.pml_order, pml_sigma_scale=desc.pml_sigma_scale,
            pml_kappa_max=desc.pml_kappa_max, pml_alpha_max=desc.pml_alpha_max, src_comp=desc.src_comp,
            src_lo=_i3(desc.src_lo), src_hi=_i3(desc.src_hi),
            src_wave=self._wave.ctypes.data_as(fp), src_profile=self._profile.ctypes.data_as(fp),
            det_lo=_i3(desc.det_lo), det_hi=_i3(desc.det_hi), des_lo=_i3(desc.des_lo), des_hi=_i3(desc.des_hi),
            loss=int(getattr(desc, "loss", 0)),
            msrc_comp=int(getattr(desc, "msrc_comp", 0)),
            msrc_lo=_i3(getattr(desc, "msrc_lo", (0, 0, 0)) if has_m else (0, 0, 0)),
            msrc_hi=_i3(getattr(desc, "msrc_hi", (0, 0, 0)) if has_m else (0, 0, 0)),
            msrc_wave=self._mwave.ctypes.data_as(fp) if has_m else None,
            msrc_profile=self._mprofile.ctypes.data_as(fp) if has_m else None)

    @property
    def shape(self):
        return (self.desc.nz, self.desc.ny, self.desc.nx)

    @property
    def design_shape(self):
        lo, hi = self.desc.des_lo, self.desc.des_hi
        return (hi[2] - lo[2], hi[1] - lo[1], hi[0] - lo[0])

    def design_slices(self):
        lo, hi = self.desc.des_lo, self.desc.des_hi
        return (slice(lo[2], hi[2]), slice(lo[1], hi[1]), slice(lo[0], hi[0]))


def store_config(problem: Problem, dtype: str = "fp32", k: int = 1) -> FdtdStoreInfo:
    lib = load()
    cfg = FdtdStoreCfg(STORE_DTYPES[dtype], int(k), _lib.INTERP_LINEAR)
    info = FdtdStoreInfo()
    check(lib.store_config(ctypes.byref(problem.c), ctypes.byref(cfg), ctypes.byref(info)))
    return info


@dataclass
class Buffers:
    fields: torch.Tensor
    psi: torch.Tensor
    store: torch.Tensor
    workspace: torch.Tensor
    loss: torch.Tensor
    series: Optional[torch.Tensor]
    adj_fields: Optional[torch.Tensor] = None
    adj_psi: Optional[torch.Tensor] = None
    grad: Optional[torch.Tensor] = None


def _bytes(n, device):
    return torch.empty(max(int(n), 1), dtype=torch.uint8, device=device)


class Gradient:
    """One problem + recorder configuration with its device buffers.

    forward(eps) records and returns the loss; backward() runs the time-reversed
    pass and returns dL/deps on the design box (float64, [z][y][x]).  interp picks
    how the backward rebuilds the steps between kept ones: "linear" (the paper's)
    or "cubic" (see include/fdtd.h).
    """

    def __init__(self, problem, dtype: str = "fp32", k: int = 1, device="cuda", series: bool = False,
                 with_backward: bool = True, interp: str = "linear"):
        self.problem = problem if isinstance(problem, Problem) else Problem(problem)
        self.dtype = dtype
        self.k = int(k)
        self.interp = interp
        self.device = torch.device(device)
        self.cfg = FdtdStoreCfg(STORE_DTYPES[dtype], self.k,
                                {"linear": _lib.INTERP_LINEAR, "cubic": _lib.INTERP_CUBIC}[interp])
        self.info = store_config(self.problem, dtype, k)
        i = self.info
        dev = self.device
        self.stride = int(i.fields_bytes) // 24          # floats between field components
        self.buf = Buffers(
            fields=torch.empty(6 * self.stride, dtype=torch.float32, device=dev),
            psi=_bytes(i.psi_bytes, dev),
            store=_bytes(i.store_bytes, dev),
            workspace=_bytes(i.workspace_bytes, dev),
            loss=torch.zeros((), dtype=torch.float64, device=dev),
            series=torch.zeros(self.problem.desc.steps, dtype=torch.float64, device=dev) if series else None)
        if with_backward:
            self.buf.adj_fields = torch.empty(6 * self.stride, dtype=torch.float32, device=dev)
            self.buf.adj_psi = _bytes(i.adj_psi_bytes, dev)
            self.buf.grad = torch.empty(self.problem.design_shape, dtype=torch.float64, device=dev)
        self.record = FdtdRecord()
        self.eps = None
        self.generation = 0              # forward calls so far (FDTDGrad ties a backward to its forward)
        # persistent buffers of FDTDGrad: the full eps map and the upstream gradient scale keep
        # their device addresses across iterations, so repeated calls replay the same graphs
        self.eps_buf = None
        self.scale_buf = torch.ones((), dtype=torch.float64, device=dev) if with_backward else None

    @property
    def storage_bytes(self) -> int:
        return int(self.info.payload_bytes)

    def forward(self, eps: torch.Tensor) -> torch.Tensor:
        """eps: float32 [nz, ny, nx] on the device.  Returns the loss (0-d float64 tensor)."""
        assert eps.dtype == torch.float32 and eps.is_contiguous() and eps.device.type == "cuda"
        assert tuple(eps.shape) == self.problem.shape
        self.eps = eps
        self.generation += 1
        b = self.buf
        check(load().fdtd_forward(
            ctypes.byref(self.problem.c), ctypes.byref(self.cfg), eps.data_ptr(), b.fields.data_ptr(),
            b.psi.data_ptr(), b.store.data_ptr(), b.workspace.data_ptr(), b.loss.data_ptr(),
            b.series.data_ptr() if b.series is not None else None, ctypes.byref(self.record),
            _stream_handle(self.device)))
        return b.loss

    def forward_noalloc(self, eps: torch.Tensor) -> torch.Tensor:
        """forward() through fdtd_forward_noalloc: the library's own device array serves as
        the workspace (the problem must fit in it; see include/fdtd.h)."""
        assert eps.dtype == torch.float32 and eps.is_contiguous() and eps.device.type == "cuda"
        assert tuple(eps.shape) == self.problem.shape
        self.eps = eps
        self.generation += 1
        b = self.buf
        check(load().fdtd_forward_noalloc(
            ctypes.byref(self.problem.c), ctypes.byref(self.cfg), eps.data_ptr(), b.fields.data_ptr(),
            b.psi.data_ptr(), b.store.data_ptr(), b.loss.data_ptr(),
            b.series.data_ptr() if b.series is not None else None, ctypes.byref(self.record),
            _stream_handle(self.device)))
        return b.loss

    def loss_value(self) -> float:
        """The loss of the last forward call as a Python float (waits for the device).
        Raises FdtdError(FDTD_ENONFINITE) when it is NaN or infinite, e.g. after a
        non-finite or non-positive eps."""
        v = float(self.buf.loss.item())
        if not np.isfinite(v):
            raise FdtdError(FDTD_ENONFINITE, "loss of %s is %r (check eps: finite and > 0)"
                            % (getattr(self.problem.desc, "name", "problem"), v))
        return v

    def backward(self, grad_scale: Optional[torch.Tensor] = None) -> torch.Tensor:
        b = self.buf
        if b.grad is None:
            raise RuntimeError("constructed without backward buffers")
        check(load().fdtd_backward(
            ctypes.byref(self.problem.c), ctypes.byref(self.cfg), self.eps.data_ptr(), b.fields.data_ptr(),
            b.store.data_ptr(), b.workspace.data_ptr(), b.adj_fields.data_ptr(), b.adj_psi.data_ptr(),
            grad_scale.data_ptr() if grad_scale is not None else None, b.grad.data_ptr(),
            ctypes.byref(self.record), _stream_handle(self.device)))
        return b.grad

    def fields(self):
        """(E, H) views of the field buffer, each [3, nz, ny, nx]."""
        n = int(self.info.cells)
        f = self.buf.fields.view(6, self.stride)[:, :n].unflatten(1, self.problem.shape)
        return f[:3], f[3:]


class FDTDGrad(torch.autograd.Function):
    """loss = FDTDGrad.apply(eps_design, grad_obj, eps_background).

    eps_design: float32 design-box tensor [dz, dy, dx]; eps_background: float32
    full map [nz, ny, nx] (its design box is overwritten by eps_design).
    The forward reads the loss back and raises FdtdError(FDTD_ENONFINITE) when it
    is not finite.  The backward runs the library's time-reversed pass; it raises
    FdtdError(FDTD_ESTATE) when called a second time on the same forward (the
    fields were reversed) or after a later forward on the same grad_obj (its
    fields, store and eps now belong to that call).
    """

    @staticmethod
    def forward(ctx, eps_design, grad_obj: Gradient, eps_background):
        if grad_obj.eps_buf is None:
            grad_obj.eps_buf = torch.empty(grad_obj.problem.shape, dtype=torch.float32, device=grad_obj.device)
        eps = grad_obj.eps_buf
        eps.copy_(eps_background.detach())
        eps[grad_obj.problem.design_slices()] = eps_design.detach().to(torch.float32)
        loss = grad_obj.forward(eps).clone()
        grad_obj.loss_value()                      # raises on a non-finite loss
        ctx.grad_obj = grad_obj
        ctx.generation = grad_obj.generation
        ctx.in_dtype = eps_design.dtype
        return loss

    @staticmethod
    def backward(ctx, grad_loss):
        gobj = ctx.grad_obj
        if gobj.generation != ctx.generation:
            raise FdtdError(FDTD_ESTATE, "a later forward on the same Gradient replaced this loss's fields and store")
        gobj.scale_buf.copy_(grad_loss.detach().reshape(()))
        g = gobj.backward(grad_scale=gobj.scale_buf)
        return g.to(ctx.in_dtype, copy=True), None, None


def codec_roundtrip(values: torch.Tensor, dtype: str, n_blocks: int):
    """Encode/decode float32 blocks with the recorder's codec.  Returns (codes, scales, decoded)."""
    assert values.dtype == torch.float32 and values.is_cuda and values.is_contiguous()
    block_len = values.numel() // n_blocks
    assert block_len * n_blocks == values.numel()
    nbytes = STORAGE_BITS[dtype] // 8
    code_dtype = {4: torch.int32, 2: torch.int16, 1: torch.uint8}[nbytes]
    codes = torch.empty(values.numel(), dtype=code_dtype, device=values.device)
    scales = torch.empty(max(n_blocks, 1), dtype=torch.float32, device=values.device)
    decoded = torch.empty_like(values)
    check(load().fdtd_codec_roundtrip(STORE_DTYPES[dtype], values.data_ptr(), n_blocks, block_len,
                                      codes.data_ptr(), scales.data_ptr(), decoded.data_ptr(),
                                      _stream_handle(values.device)))
    return codes, scales[:n_blocks], decoded


def set_graphs(on: bool = True):
    """Replay repeated forward/backward calls as HIP graphs (default) or enqueue every launch."""
    check(load().fdtd_set_graphs(1 if on else 0))


def timing_enable(on: bool = True):
    check(load().fdtd_timing_enable(1 if on else 0))


def timing_read():
    """{kernel name: (launches, total_ms)} for the launches since timing_enable(True)."""
    arr = (_lib.FdtdKernelTime * 16)()
    n = check(load().fdtd_timing_read(arr, 16))
    return {arr[i].name.decode(): (int(arr[i].launches), float(arr[i].total_ms)) for i in range(n)}
