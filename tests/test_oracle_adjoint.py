"""Pins of the oracle's gradient: transpose identity, finite differences, reconstruction (CPU only)."""

from dataclasses import replace

import numpy as np
import pytest

import workloads as w
from oracle import adjoint, metrics, yee


def _rand_state(shape, rng, psi_in_slabs_only=None):
    st = yee.State(shape)
    st.E[...] = rng.standard_normal(st.E.shape)
    st.H[...] = rng.standard_normal(st.H.shape)
    st.psi_H[...] = rng.standard_normal(st.psi_H.shape)
    st.psi_E[...] = rng.standard_normal(st.psi_E.shape)
    return st


@pytest.mark.parametrize("boundary,pml,kappa", [(0, 3, 1.0), (0, 3, 2.5), (1, 0, 1.0)])
def test_one_step_transpose_identity(boundary, pml, kappa):
    """<A x, y> = <x, A^T y> for one full step (H half then E half), CPML included."""
    rng = np.random.default_rng(11)
    p = w.Problem(name="dot", nx=10, ny=9, nz=8, pml=pml, steps=1, boundary=boundary,
                  pml_kappa_max=kappa, pml_alpha_max=0.1,
                  src_wave=np.zeros(1, np.float32), src_profile=np.zeros((1, 1, 1), np.float32),
                  src_lo=(0, 0, 0), src_hi=(1, 1, 1),
                  eps=rng.uniform(1.0, 12.25, (8, 9, 10)).astype(np.float32))
    s_ = yee.Solver(p)
    x = _rand_state(s_.shape, rng)
    y = _rand_state(s_.shape, rng)
    Ax = x.copy()
    s_.step(Ax, 0)
    a = adjoint.AdjointState(s_.shape)
    a.E[...], a.H[...], a.psi_H[...], a.psi_E[...] = y.E, y.H, y.psi_H, y.psi_E
    adjoint.adjoint_e_half(s_, a)
    adjoint.adjoint_h_half(s_, a)
    lhs = sum(np.sum(u * v) for u, v in ((Ax.E, y.E), (Ax.H, y.H), (Ax.psi_H, y.psi_H), (Ax.psi_E, y.psi_E)))
    rhs = sum(np.sum(u * v) for u, v in ((x.E, a.E), (x.H, a.H), (x.psi_H, a.psi_H), (x.psi_E, a.psi_E)))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1.0)


def test_transpose_identity_catches_a_dropped_term():
    """Sanity of the pin itself: dropping the a*P term of the adjoint PML recursion breaks it."""
    rng = np.random.default_rng(3)
    p = w.Problem(name="dot", nx=10, ny=9, nz=8, pml=3, steps=1, pml_kappa_max=2.0,
                  src_wave=np.zeros(1, np.float32), src_profile=np.zeros((1, 1, 1), np.float32),
                  src_lo=(0, 0, 0), src_hi=(1, 1, 1), eps=np.ones((8, 9, 10), np.float32))
    s_ = yee.Solver(p)
    x = _rand_state(s_.shape, rng)
    y = _rand_state(s_.shape, rng)
    Ax = x.copy()
    s_.step(Ax, 0)
    a = adjoint.AdjointState(s_.shape)
    a.E[...], a.H[...], a.psi_H[...], a.psi_E[...] = y.E, y.H, y.psi_H, y.psi_E
    saved = s_.coef_E
    s_.coef_E = [(b, aa * 0, k) for (b, aa, k) in saved]   # a planted mistake, oracle side only
    adjoint.adjoint_e_half(s_, a)
    s_.coef_E = saved
    adjoint.adjoint_h_half(s_, a)
    lhs = sum(np.sum(u * v) for u, v in ((Ax.E, y.E), (Ax.H, y.H), (Ax.psi_H, y.psi_H), (Ax.psi_E, y.psi_E)))
    rhs = sum(np.sum(u * v) for u, v in ((x.E, a.E), (x.H, a.H), (x.psi_H, a.psi_H), (x.psi_E, a.psi_E)))
    assert abs(lhs - rhs) > 1e-6 * abs(lhs)


def test_gradient_finite_difference_tiny_all_cells():
    """12^3, 3-cell CPML, 60 steps: every design cell against central differences (FP64)."""
    p = w.tiny()
    L, g = adjoint.grad_time_reversal(p, "fp64", 1)
    fd = adjoint.grad_finite_difference(p, np.arange(g.size), h=1e-4)
    assert np.max(np.abs(fd - g.ravel())) <= 1e-6 * np.max(np.abs(g))
    Lf, gf = adjoint.grad_full_storage(p)
    assert abs(L - Lf) <= 1e-13 * abs(L)
    assert metrics.rel_l2(g, gf) < 1e-10


def test_gradient_finite_difference_kappa_and_ragged():
    """Odd grid, plane source, thick detector, kappa_max > 1: sampled cells against FD."""
    p = replace(w.ragged(steps=30), pml_kappa_max=3.0)
    L, g = adjoint.grad_time_reversal(p, "fp64", 1)
    _, gf = adjoint.grad_full_storage(p)
    assert metrics.rel_l2(g, gf) < 1e-10
    cells = w.fd_cells(p, 6, seed=0)
    fd = adjoint.grad_finite_difference(p, cells, h=1e-4)
    ref = g.ravel()[cells]
    assert np.max(np.abs(fd - ref)) <= 1e-6 * np.max(np.abs(g))


def test_time_reversal_reconstructs_interior_history():
    """With the PML and FP64 k = 1 shells, E^n and H^{n-1/2} on I match the forward run at every n."""
    p = w.tiny(steps=50)
    s_ = yee.Solver(p)
    T = p.steps
    _, _, snaps = yee.run_forward(s_, snapshots=tuple(range(T + 1)))
    _, _, trace = adjoint.grad_time_reversal(p, "fp64", 1, return_trace=True)
    I = (slice(None),) + s_.int_sl
    scale = max(np.max(np.abs(snaps[n].E)) for n in snaps)
    for n in range(T):
        E_rec, H_rec = trace[n]
        assert np.max(np.abs(E_rec - snaps[n].E[I])) <= 1e-10 * scale
        assert np.max(np.abs(H_rec - snaps[n].H[I])) <= 1e-10 * scale


def test_wrong_shell_index_is_caught():
    """Reinjecting the shell one cell off (a plausible indexing mistake) gives O(1) gradient error."""
    p = w.tiny(steps=50)
    _, g = adjoint.grad_time_reversal(p, "fp64", 1)
    s_cls = yee.Solver
    orig = s_cls.put_shell_H
    def shifted(self, s, blocks):
        P, (nz, ny, nx) = self.P, self.shape
        ix, iy, iz = slice(P, nx - P), slice(P, ny - P), slice(P, nz - P)
        s.H[1][iz, iy, P - 2], s.H[2][iz, iy, P - 2] = blocks[0], blocks[1]   # planted: P-2
        s.H[2][iz, P - 1, ix], s.H[0][iz, P - 1, ix] = blocks[2], blocks[3]
        s.H[0][P - 1, iy, ix], s.H[1][P - 1, iy, ix] = blocks[4], blocks[5]
    s_cls.put_shell_H = shifted
    try:
        _, g_bad = adjoint.grad_time_reversal(p, "fp64", 1)
    finally:
        s_cls.put_shell_H = orig
    assert metrics.rel_l2(g_bad, g) > 1e-3


def test_compressed_k1_fp32_close_to_exact():
    p = w.tiny(steps=50)
    _, g64 = adjoint.grad_time_reversal(p, "fp64", 1)
    _, g32 = adjoint.grad_time_reversal(p, "fp32", 1)
    assert metrics.rel_l2(g32, g64) < 1e-5
    assert metrics.cosine_similarity(g32, g64) > 1 - 1e-10
