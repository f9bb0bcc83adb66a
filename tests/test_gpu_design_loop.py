"""The inverse-design loop on the HIP gradient (needs an MI355X).

The chain rho -> filter -> projection -> eps -> detector energy is differentiated
by torch autograd around FDTDGrad; its directional derivative must match a
central difference of the library's forward loss, and a few NAdam iterations
must raise the objective, with full and with compressed interface storage.
"""

import numpy as np
import pytest
import torch

import workloads as w
import paper_2603_24027_amd as pk
from paper_2603_24027_amd.optimize import DesignLoop

from gpu_helpers import require_gpu, say

pytestmark = pytest.mark.gpu


def test_design_chain_directional_derivative():
    require_gpu()
    prob = w.tiny(steps=60)
    loop = DesignLoop(prob, "fp32", 1, sigma=0.8, beta=4.0, seed=3)
    rho = loop.rho
    eps_d = loop.design_eps().to(torch.float32)
    loss = pk.FDTDGrad.apply(eps_d, loop.grad, loop.background)
    loss.backward()
    g = rho.grad.detach().clone()
    d = torch.from_numpy(np.random.default_rng(5).standard_normal(tuple(rho.shape))).to(rho.device)
    h = 1e-3

    def value(r):
        with torch.no_grad():
            loop.rho.copy_(r)
            e = loop.design_eps().to(torch.float32)
        return float(pk.FDTDGrad.apply(e, loop.grad, loop.background).item())

    r0 = rho.detach().clone()
    fd = (value(r0 + h * d) - value(r0 - h * d)) / (2 * h)
    ad = float(torch.sum(g * d))
    say("design chain: autograd %.6e  central difference %.6e" % (ad, fd))
    assert abs(fd - ad) <= 2e-3 * abs(ad)


@pytest.mark.parametrize("dtype,k", [("fp32", 1), ("fp8_e4m3_scaled", 4), ("bf16", 2)])
def test_design_loop_improves_objective(dtype, k):
    require_gpu()
    prob = w.tiny(steps=60)
    loop = DesignLoop(prob, dtype, k, sigma=0.8, beta=4.0, lr=0.3, warmup=2, seed=1)
    hist = loop.run(6)
    say("%s k=%d objective %s" % (dtype, k, " ".join("%.4e" % v for v in hist)))
    assert all(np.isfinite(hist))
    assert hist[-1] > hist[0]
