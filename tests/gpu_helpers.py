"""Shared helpers of the GPU parity tests: run the HIP path and the oracle on the same seeded input."""

import numpy as np
import torch

import paper_2603_24027_amd as pk


def require_gpu():
    assert torch.cuda.is_available(), "GPU tests need an MI355X"
    pk.load()


def say(*a):
    print(*a, flush=True)


def gpu_run(prob, dtype="fp32", k=1, series=False, backward=True, keep_fields=True):
    """Forward (+ backward) through the C ABI.  Returns dict with loss, series, E, H, grad, info."""
    g = pk.Gradient(prob, dtype, k, device="cuda", series=series, with_backward=backward)
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
