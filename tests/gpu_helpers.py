"""Shared helpers of the GPU parity tests: run the HIP path and the oracle on the same seeded input."""

import numpy as np
import torch

import paper_2603_24027_amd as pk


def require_gpu():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    pk.load()


def say(*a):
    print(*a, flush=True)


def gpu_run(prob, dtype="fp32", k=1, series=False, backward=True, keep_fields=True, interp="linear"):
    """Forward (+ backward) through the C ABI.  Returns dict with loss, series, E, H, grad, info."""
    g = pk.Gradient(prob, dtype, k, device="cuda", series=series, with_backward=backward, interp=interp)
    eps = torch.from_numpy(np.ascontiguousarray(prob.eps, np.float32)).cuda()
    loss = g.forward(eps)
    out = {"info": g.info, "obj": g}
    if keep_fields:
        E, H = g.fields()
        out["E"] = E.double().cpu().numpy()
        out["H"] = H.double().cpu().numpy()
    if series:
        out["series"] = g.buf.series.cpu().numpy()
    out["loss"] = float(loss.item())
    if backward:
        out["grad"] = g.backward().cpu().numpy()
        torch.cuda.synchronize()
    return out


def rel(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


STORE_BYTES = {"fp32": 4, "fp16": 2, "bf16": 2}


def store_layout(gobj):
    """(bytes per value, bytes between kept steps, byte offset of the FP8 scale table) of the
    interface store, as include/fdtd.h lays it out."""
    nb = STORE_BYTES.get(gobj.dtype, 1)
    vps = int(gobj.info.values_per_slice)
    stride = (vps * nb + 255) // 256 * 256
    return nb, stride, int(gobj.info.slices) * stride


def block_lengths(prob):
    """Values of the 12 (face, component) blocks of one kept step, in store order."""
    P = prob.pml
    mx, my, mz = prob.nx - 2 * P, prob.ny - 2 * P, prob.nz - 2 * P
    ax, ay, az = my * mz, mx * mz, mx * my
    return [ax, ax, ay, ay, az, az] * 2


def store_slice(gobj, j):
    """The 12 blocks of kept step j (the j-th kept step counted back from the last time step)
    as numpy arrays of raw codes (float32 for FP32, uint16 for 16-bit, uint8 for 8-bit types),
    and the 12 FP8 scales (None for the other types)."""
    nb, stride, scale_off = store_layout(gobj)
    vps = int(gobj.info.values_per_slice)
    raw = gobj.buf.store[j * stride: j * stride + vps * nb].cpu().numpy()
    view = {4: np.float32, 2: np.uint16, 1: np.uint8}[nb]
    vals = raw.view(view)
    out, o = [], 0
    for n in block_lengths(gobj.problem.desc):
        out.append(vals[o:o + n])
        o += n
    scales = None
    if gobj.dtype == "fp8_e4m3_scaled":
        scales = gobj.buf.store[scale_off + j * 48: scale_off + (j + 1) * 48].cpu().numpy().view(np.float32)
    return out, scales
