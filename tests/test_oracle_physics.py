"""Pins of the oracle's Yee / CPML model against closed forms and invariants (CPU only)."""

import math
from dataclasses import replace

import numpy as np
import pytest

import workloads as w
from oracle import yee


def _blank(n, pml=0, boundary=0, steps=1, **kw):
    nx, ny, nz = n
    return w.Problem(name="blank", nx=nx, ny=ny, nz=nz, pml=pml, steps=steps, boundary=boundary,
                     src_comp=2, src_lo=(0, 0, 0), src_hi=(1, 1, 1),
                     src_wave=np.zeros(steps, np.float32), src_profile=np.zeros((1, 1, 1), np.float32),
                     det_lo=(0, 0, 0), det_hi=(1, 1, 1), des_lo=(0, 0, 0), des_hi=(1, 1, 1),
                     eps=np.ones((nz, ny, nx), np.float32), **kw)


# positions of the six components in units of the cell (x, y, z offsets)
E_OFF = ((0.5, 0, 0), (0, 0.5, 0), (0, 0, 0.5))
H_OFF = ((0, 0.5, 0.5), (0.5, 0, 0.5), (0.5, 0.5, 0))


def _plane_wave(n, m, dt, t_E, t_H, pol):
    """Closed-form discrete eigenmode of the periodic Yee grid.

    k_d = 2 pi m_d / N_d, K_d = 2 sin(k_d / 2); dispersion
    (2/dt) sin(w dt / 2) = |K|; E-hat perpendicular to K; H-hat = K x E-hat / |K|.
    Each component is evaluated at its own staggered position.
    """
    nx, ny, nz = n
    k = np.array([2 * math.pi * m[0] / nx, 2 * math.pi * m[1] / ny, 2 * math.pi * m[2] / nz])
    K = 2 * np.sin(k / 2)
    Om = np.linalg.norm(K)
    omega = 2.0 / dt * math.asin(Om * dt / 2)
    Ehat = np.cross(K, pol)
    Ehat /= np.linalg.norm(Ehat)
    Hhat = np.cross(K, Ehat) / Om
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    E = np.zeros((3, nz, ny, nx))
    H = np.zeros((3, nz, ny, nx))
    for c in range(3):
        ph = k[0] * (x + E_OFF[c][0]) + k[1] * (y + E_OFF[c][1]) + k[2] * (z + E_OFF[c][2])
        E[c] = Ehat[c] * np.cos(ph - omega * t_E)
        ph = k[0] * (x + H_OFF[c][0]) + k[1] * (y + H_OFF[c][1]) + k[2] * (z + H_OFF[c][2])
        H[c] = Hhat[c] * np.cos(ph - omega * t_H)
    return E, H


@pytest.mark.parametrize("m,pol", [((1, 0, 0), (0, 0, 1.0)), ((1, 2, 3), (1.0, 0, 0)), ((2, -1, 1), (0, 1.0, 0))])
def test_plane_wave_eigenmode(m, pol):
    n = (16, 12, 10)
    steps = 400
    p = _blank(n, boundary=1, steps=steps)
    s_ = yee.Solver(p)
    dt = s_.dt
    st = yee.State(s_.shape)
    st.E[...], st.H[...] = _plane_wave(n, m, dt, 0.0, -0.5 * dt, pol)
    for step in range(steps):
        s_.step(st, step)
    E_ref, H_ref = _plane_wave(n, m, dt, steps * dt, (steps - 0.5) * dt, pol)
    assert np.max(np.abs(st.E - E_ref)) < 1e-11
    assert np.max(np.abs(st.H - H_ref)) < 1e-11


def test_eigenmode_detects_wrong_dispersion():
    """The closed form is sharp: the continuum frequency (|k| instead of the Yee one) is far off."""
    n, m = (16, 12, 10), (1, 2, 3)
    p = _blank(n, boundary=1)
    dt = yee.Solver(p).dt
    E0, _ = _plane_wave(n, m, dt, 100 * dt, 0, (1.0, 0, 0))
    k = np.array([2 * math.pi * m[0] / 16, 2 * math.pi * m[1] / 12, 2 * math.pi * m[2] / 10])
    K = 2 * np.sin(k / 2)
    w_yee = 2.0 / dt * math.asin(np.linalg.norm(K) * dt / 2)
    assert abs(w_yee - np.linalg.norm(k)) > 1e-3


@pytest.mark.parametrize("boundary", [0, 1])
def test_discrete_energy_conserved(boundary):
    """W^n = sum eps |E^n|^2 + sum H^{n-1/2} . H^{n+1/2} is exactly invariant without PML or source."""
    n = (11, 9, 8)
    p = _blank(n, boundary=boundary)
    rng = np.random.default_rng(5)
    p = replace(p, eps=rng.uniform(1.0, 12.25, (8, 9, 11)).astype(np.float32))
    s_ = yee.Solver(p)
    st = yee.State(s_.shape)
    st.E[...] = rng.uniform(-1, 1, st.E.shape)
    st.H[...] = rng.uniform(-1, 1, st.H.shape)
    W = []
    for step in range(300):
        H_old = st.H.copy()
        s_.h_update(st)
        W.append(np.sum(s_.eps * st.E ** 2) + np.sum(H_old * st.H))
        s_.e_update(st, step)
    W = np.array(W)
    assert np.max(np.abs(W - W[0])) / abs(W[0]) < 1e-12
    # and the plain sum of squares is NOT invariant (the pin is not vacuous)
    assert abs(np.sum(st.E ** 2) + np.sum(st.H ** 2) - W[0]) / abs(W[0]) > 1e-6


def test_reversal_without_pml_is_exact():
    n = (10, 9, 7)
    p = _blank(n, steps=200)
    rng = np.random.default_rng(7)
    p = replace(p, eps=rng.uniform(1.0, 12.25, (7, 9, 10)).astype(np.float32))
    s_ = yee.Solver(p)
    st = yee.State(s_.shape)
    st.E[...] = rng.uniform(-1, 1, st.E.shape)
    st.H[...] = rng.uniform(-1, 1, st.H.shape)
    E0, H0 = st.E.copy(), st.H.copy()
    for step in range(200):
        s_.step(st, step)
    assert np.max(np.abs(st.E - E0)) > 0.1
    for step in range(199, -1, -1):
        s_.e_inverse(st, step)
        s_.h_inverse(st)
    assert np.max(np.abs(st.E - E0)) < 200 * 1e-14
    assert np.max(np.abs(st.H - H0)) < 200 * 1e-14


def test_cpml_without_loss_is_plain_yee():
    """sigma = alpha = 0, kappa = 1 gives a = 0, b = 1: bitwise the grid without PML."""
    prob = w.tiny(steps=40)
    lossless = replace(prob, pml_sigma_scale=0.0, pml_alpha_max=0.0, pml_kappa_max=1.0)
    plain = replace(prob, pml=0)
    a = yee.run_forward(yee.Solver(lossless))[0]
    b = yee.run_forward(yee.Solver(plain))[0]
    assert np.array_equal(a.E, b.E) and np.array_equal(a.H, b.H)


def test_cpml_profile_shape():
    dt = yee.courant_time_step(0.99)
    for node in ("E", "H"):
        b, a, kinv = yee.cpml_profile(30, 6, dt, node, kappa_max=3.0)
        inside = slice(6, 24)
        assert np.all(a[inside] == 0) and np.all(kinv[inside] == 1)
        assert np.count_nonzero(a[:6]) == 6 and np.count_nonzero(a[24:]) == 6
        assert np.all(a[:6] < 0) and np.all((b[:6] > 0) & (b[:6] < 1))
        assert np.all(kinv[:6] < 1)
    # mirror symmetry: E nodes on the low side match H nodes on the high side
    bE, aE, kE = yee.cpml_profile(30, 6, dt, "E")
    bH, aH, kH = yee.cpml_profile(30, 6, dt, "H")
    assert np.allclose(aE[:6], aH[::-1][:6], rtol=0, atol=1e-15)


def test_cpml_absorbs():
    """Reflection from the 8-cell CPML, probed next to the interface, is below 1e-3 of the peak.

    Reference: the same source and probe in a grid large enough that nothing
    reflected from its outer edge reaches the probe within the run.
    """
    steps = 80
    small_n, P = 36, 8
    big_n = 100
    def prob(n, pml):
        c = n // 2
        return w.dipole_problem("refl", (n, n, n), pml, steps, (c, c, c), 12.0, (c, c, c),
                                (c + 1, c + 1, c + 1), (c, c, c), (c + 1, c + 1, c + 1), bandwidth=0.8)
    def probe_series(p, n):
        s_ = yee.Solver(p)
        st = yee.State(s_.shape)
        c = n // 2
        out = []
        for step in range(steps):
            s_.step(st, step)
            out.append(st.E[2][c, c, c + 8 - 0: c + 10].copy())   # up to the interface (index 26 of 36)
        return np.array(out)
    a = probe_series(prob(small_n, P), small_n)
    b = probe_series(prob(big_n, 0), big_n)
    peak = np.max(np.abs(b))
    err = np.max(np.abs(a - b)) / peak
    assert err < 1e-3, err
    # without the PML (hard zero boundary at the same place) the error is large
    c = probe_series(prob(small_n, 0), small_n)
    assert np.max(np.abs(c - b)) / peak > 1e-2


def test_time_step_eq1_normalised():
    assert yee.courant_time_step(0.99) == pytest.approx(0.99 / math.sqrt(3), rel=1e-15)
    assert yee.courant_time_step(1.0) ** 2 * 3 == pytest.approx(1.0, rel=1e-15)
