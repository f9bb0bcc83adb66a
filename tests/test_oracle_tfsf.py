"""Pins of the total-field/scattered-field plane-wave source (CPU only).

With periodic x and y the x-polarised plane wave is exactly one-dimensional,
so the 3-D grid must reproduce the 1-D incident line at the sheet and emit
nothing into the scattered-field side, up to the FP32 rounding of the sheet
signals (the sources are FP32 inputs); the gradient with the
sheet present (the magnetic current enters the H update and its inverse) is
pinned by finite differences.
"""

import numpy as np
from dataclasses import replace

import workloads as w
from oracle import adjoint, metrics, yee

from test_oracle_physics import _blank


def test_tfsf_sheet_is_one_sided_and_reproduces_the_incident_wave():
    n, z0, T = (8, 6, 400), 40, 200
    p = replace(_blank(n, boundary=1, steps=T), det_lo=(0, 0, 100), det_hi=(8, 6, 101))
    p = w.with_tfsf_plane_wave(p, z0, 20.0)
    ex_inc, _ = w.incident_line(T, p.courant, 1.0, 20.0)
    s_ = yee.Solver(p)
    st = yee.State(s_.shape)
    ex_sheet = np.zeros(T)
    for step in range(T):
        ex_sheet[step] = st.E[0, z0, 3, 4]           # E^n at the sheet, before step n
        s_.step(st, step)
    peak = np.max(np.abs(st.E[:, z0:]))
    assert peak > 0.05
    # total field at the sheet = incident field (no scatterer), any x, y
    assert np.max(np.abs(ex_sheet - ex_inc)) <= 1e-6 * np.max(np.abs(ex_inc))
    assert np.max(np.abs(st.E[0, z0] - st.E[0, z0, 0, 0])) <= 1e-14
    # nothing on the scattered-field side (z < z0 for E, z < z0 - 1 for H)
    assert np.max(np.abs(st.E[:, :z0])) <= 1e-6 * peak
    assert np.max(np.abs(st.H[:, :z0 - 1])) <= 1e-6 * peak


def test_tfsf_without_magnetic_sheet_leaks():
    # dropping the M sheet turns it into a two-sided current sheet: the pin above is sharp
    n, z0, T = (8, 6, 400), 40, 200
    p = w.with_tfsf_plane_wave(_blank(n, boundary=1, steps=T), z0, 20.0)
    p = replace(p, msrc_wave=np.zeros(0, np.float32))
    s_ = yee.Solver(p)
    st = yee.State(s_.shape)
    for step in range(T):
        s_.step(st, step)
    assert np.max(np.abs(st.E[:, :z0])) > 0.1 * np.max(np.abs(st.E[:, z0:]))


def test_tfsf_flux_gradient_finite_difference():
    p = w.tiny_pw()
    L, g = adjoint.grad_time_reversal(p, "fp64", 1)
    assert abs(L) > 0
    fd = adjoint.grad_finite_difference(p, np.arange(g.size), h=1e-4)
    assert np.max(np.abs(fd - g.ravel())) <= 1e-6 * np.max(np.abs(g))
    Lf, gf = adjoint.grad_full_storage(p)
    assert abs(L - Lf) <= 1e-12 * abs(L)
    assert metrics.rel_l2(g, gf) < 1e-10
