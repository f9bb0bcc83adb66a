"""Pins of the oracle's Poynting-flux objective (the paper's transmission metric; CPU only).

The loss term of step n is sum_D (E^{n+1} x H^{n+1/2})_axis at the same cell
index.  Pinned by: the sign and size of the flux of travelling discrete plane
waves, finite differences of the per-step term against its seeds, and finite
differences of the whole gradient (time reversal and full storage).
"""

import math
from dataclasses import replace

import numpy as np
import pytest

import workloads as w
from oracle import adjoint, metrics, yee

from test_oracle_physics import _blank, _plane_wave


@pytest.mark.parametrize("direction", [+1, -1])
def test_flux_of_a_travelling_plane_wave(direction):
    # a z-travelling x-polarised discrete eigenmode of a periodic box: over one period the
    # z-flux through a full plane has the sign of the direction of travel and, for a long
    # wavelength, about half the plane's area (|E| = |H| = 1 in these units)
    n = (8, 6, 48)
    p = replace(_blank(n, boundary=1), det_lo=(0, 0, 20), det_hi=(8, 6, 21), loss=3)
    s_ = yee.Solver(p)
    dt = s_.dt
    m = (0, 0, direction)
    st = yee.State(s_.shape)
    st.E[...], st.H[...] = _plane_wave(n, m, dt, 0.0, -0.5 * dt, (0, 1.0, 0))
    k = 2 * math.pi / n[2]
    omega = 2.0 / dt * math.asin(2 * math.sin(k / 2) * dt / 2)
    period = int(round(2 * math.pi / omega / dt))
    total = 0.0
    for step in range(period):
        s_.step(st, step)
        total += s_.detector_loss(st)
    avg = total / period / (n[0] * n[1])
    assert direction * avg > 0.45 and abs(avg) <= 0.5 + 1e-9
    # the other two axes see nothing
    assert abs(s_.detector_flux(st, 0)) < 1e-12 and abs(s_.detector_flux(st, 1)) < 1e-12


@pytest.mark.parametrize("loss", [0, 1, 2, 3])
def test_seeds_are_the_derivative_of_the_step_loss(loss):
    p = replace(w.tiny(), loss=loss)
    s_ = yee.Solver(p)
    rng = np.random.default_rng(loss)
    st = yee.State(s_.shape)
    st.E[...] = rng.standard_normal(st.E.shape)
    st.H[...] = rng.standard_normal(st.H.shape)
    D = (slice(None),) + s_.det_sl
    gE, gH = s_.loss_seeds(st.E[D], st.H[D])
    h = 1e-6
    for field, grad in ((st.E, gE), (st.H, gH)):
        for _ in range(12):
            c = rng.integers(3)
            idx = tuple(int(rng.integers(sl.start, sl.stop)) for sl in s_.det_sl)
            old = field[(c,) + idx]
            field[(c,) + idx] = old + h
            lp = s_.detector_loss(st)
            field[(c,) + idx] = old - h
            lm = s_.detector_loss(st)
            field[(c,) + idx] = old
            loc = tuple(i - sl.start for i, sl in zip(idx, s_.det_sl))
            assert abs((lp - lm) / (2 * h) - grad[(c,) + loc]) < 1e-6


def test_flux_gradient_finite_difference_tiny_all_cells():
    p = replace(w.tiny(), loss=3)
    L, g = adjoint.grad_time_reversal(p, "fp64", 1)
    fd = adjoint.grad_finite_difference(p, np.arange(g.size), h=1e-4)
    assert np.max(np.abs(fd - g.ravel())) <= 1e-6 * np.max(np.abs(g))
    Lf, gf = adjoint.grad_full_storage(p)
    assert abs(L - Lf) <= 1e-13 * abs(L)
    assert metrics.rel_l2(g, gf) < 1e-10


def test_flux_gradient_finite_difference_ragged_x_normal():
    # x-flux through a thick detector on the odd grid (plane Ex source, kappa_max > 1)
    p = replace(w.ragged(steps=30), pml_kappa_max=3.0, loss=1)
    L, g = adjoint.grad_time_reversal(p, "fp64", 1)
    _, gf = adjoint.grad_full_storage(p)
    assert metrics.rel_l2(g, gf) < 1e-10
    cells = w.fd_cells(p, 6, seed=1)
    fd = adjoint.grad_finite_difference(p, cells, h=1e-4)
    assert np.max(np.abs(fd - g.ravel()[cells])) <= 1e-6 * np.max(np.abs(g))


def test_dropping_the_h_seed_breaks_the_flux_gradient():
    # the H-side seed matters: without it the gradient is measurably wrong
    p = replace(w.tiny(), loss=3)
    _, g = adjoint.grad_time_reversal(p, "fp64", 1)
    orig = yee.Solver.loss_seeds
    try:
        yee.Solver.loss_seeds = lambda self, E, H: (orig(self, E, H)[0], np.zeros_like(H))
        _, g_bad = adjoint.grad_time_reversal(p, "fp64", 1)
    finally:
        yee.Solver.loss_seeds = orig
    assert metrics.rel_l2(g_bad, g) > 1e-3
