"""A synthetic inverse-design loop on the gradient library (the paper's Section 3 / Fig. 4 setting).

The paper optimises a filtered and projected design with an adaptive first-order
method and compares the trajectories obtained with full and compressed interface
storage.  This module builds the same kind of loop around ``FDTDGrad``:

    rho (free variables, design box)
      -> s = sigmoid(rho)                               in (0, 1)
      -> f = GaussianBlur_sigma(s)                      minimum feature size (edges replicated)
      -> p = projection of f at level eta, sharpness beta (below)
      -> eps = eps_lo + (eps_hi - eps_lo) p             written into the design box
      -> L = the library's loss (detector energy or flux), maximised

with NAdam (Adam with Nesterov momentum) and a linear learning-rate warm-up.
The paper's schedule keeps beta = 1 for the first 40 iterations and then
projects at beta = infinity with a subpixel-smoothed projection, whose
gradient does not vanish at the material interface (Section 3).  Finite beta
uses the tanh projection
      p = (tanh(beta eta) + tanh(beta (f - eta))) / (tanh(beta eta) + tanh(beta (1 - eta)));
beta = infinity uses the fill fraction of each cell by the region f > eta with
the interface taken as the plane through the cell that the filtered field's
local gradient gives: signed distance d = (f - eta) / |grad f| (cells), and
      p = clamp(1/2 + d, 0, 1),
a one-cell linear ramp across the interface (exact for interfaces normal to an
axis), binary away from it.  The filter, projection and optimiser are small
torch operations on the design box; every forward and gradient evaluation of
the field problem runs in the HIP library.
"""

from __future__ import annotations

import math
from typing import List, Optional

import torch

from .solver import FDTDGrad, Gradient


def gaussian_taps(sigma: float, device=None) -> torch.Tensor:
    """Normalised 1-D Gaussian taps exp(-i^2 / (2 sigma^2)), i in [-r, r], r = ceil(3 sigma)."""
    r = max(1, int(math.ceil(3.0 * sigma)))
    i = torch.arange(-r, r + 1, dtype=torch.float64, device=device)
    w = torch.exp(-(i * i) / (2.0 * sigma * sigma))
    return w / w.sum()


def blur3d(x: torch.Tensor, sigma: float) -> torch.Tensor:
    """Separable Gaussian blur of a [z, y, x] tensor with replicated edges; sigma <= 0 is the identity."""
    if sigma <= 0:
        return x
    taps = gaussian_taps(sigma, x.device).to(x.dtype)
    r = (taps.numel() - 1) // 2
    y = x[None, None]
    for axis in range(3):
        shape = [1, 1, 1, 1, 1]
        shape[2 + axis] = taps.numel()
        pad = [0, 0, 0, 0, 0, 0]
        pad[2 * (2 - axis)] = r          # F.pad orders pads from the last dimension
        pad[2 * (2 - axis) + 1] = r
        y = torch.nn.functional.pad(y, pad, mode="replicate")
        y = torch.nn.functional.conv3d(y, taps.view(shape))
    return y[0, 0]


def project(f: torch.Tensor, beta: float, eta: float = 0.5) -> torch.Tensor:
    """Threshold projection of f in [0, 1] at level eta: tanh with sharpness beta (maps 0->0,
    1->1), or for beta = infinity the subpixel-smoothed fill fraction (module docstring)."""
    if math.isinf(beta):
        return project_subpixel(f, eta)
    a = math.tanh(beta * eta)
    return (a + torch.tanh(beta * (f - eta))) / (a + math.tanh(beta * (1.0 - eta)))


def project_subpixel(f: torch.Tensor, eta: float = 0.5) -> torch.Tensor:
    """beta = infinity: fill fraction clamp(1/2 + (f - eta) / |grad f|, 0, 1) of each cell, the
    gradient by central differences (one-sided at the box edges, unit cell size)."""
    grads = torch.gradient(f, spacing=1.0, edge_order=1)
    norm = torch.sqrt(sum(g * g for g in grads) + 1e-12)
    return torch.clamp(0.5 + (f - eta) / norm, 0.0, 1.0)


class DesignLoop:
    """Maximise the detector energy of ``problem`` over its design box.

    ``dtype`` and ``k`` select the interface storage of every gradient (as in
    ``Gradient``).  ``step()`` performs one forward + time-reversed gradient and
    one optimiser update and returns the objective before the update.
    """

    def __init__(self, problem, dtype: str = "fp32", k: int = 1, sigma: float = 3.0, beta: float = 8.0,
                 eta: float = 0.5, eps_range=(1.0, 12.25), lr: float = 0.1, warmup: int = 10, seed: int = 0,
                 device="cuda", rho0: Optional[torch.Tensor] = None, beta_after: Optional[float] = None,
                 switch_at: int = 40):
        self.device = torch.device(device)
        self.grad = Gradient(problem, dtype, k, device=self.device)
        self.background = torch.from_numpy(problem.eps).to(self.device)
        shape = self.grad.problem.design_shape
        if rho0 is None:
            g = torch.Generator(device="cpu").manual_seed(seed)
            rho0 = 0.1 * torch.randn(shape, generator=g, dtype=torch.float64)
        self.rho = rho0.to(self.device, torch.float64).clone().requires_grad_(True)
        self.sigma, self.beta, self.eta = sigma, beta, eta
        # schedule: `beta` for the first `switch_at` iterations, then `beta_after` (if given)
        self.beta_first, self.beta_after, self.switch_at = beta, beta_after, int(switch_at)
        self.lo, self.hi = float(eps_range[0]), float(eps_range[1])
        self.opt = torch.optim.NAdam([self.rho], lr=lr)
        self.warmup = max(1, int(warmup))
        self.lr = lr
        self.iteration = 0
        self.history: List[float] = []

    def design_eps(self) -> torch.Tensor:
        s = torch.sigmoid(self.rho)
        p = project(blur3d(s, self.sigma), self.beta, self.eta)
        return self.lo + (self.hi - self.lo) * p

    def beta_at(self, iteration: int) -> float:
        if self.beta_after is None or iteration < self.switch_at:
            return self.beta_first
        return self.beta_after

    def step(self) -> float:
        self.beta = self.beta_at(self.iteration)
        for group in self.opt.param_groups:
            group["lr"] = self.lr * min(1.0, (self.iteration + 1) / self.warmup)
        self.opt.zero_grad(set_to_none=True)
        eps_d = self.design_eps().to(torch.float32)
        loss = FDTDGrad.apply(eps_d, self.grad, self.background)
        (-loss).backward()                       # maximise the detector energy
        self.opt.step()
        self.iteration += 1
        value = float(loss.item())
        self.history.append(value)
        return value

    def run(self, iterations: int) -> List[float]:
        for _ in range(iterations):
            self.step()
        return self.history
