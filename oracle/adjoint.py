"""Reverse-mode gradient dL/deps of the discrete loss, three independent ways.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Loss:  L(eps) = sum_{n=0}^{T-1} sum_{p in D} |E^{n+1}(p)|^2   (detector box D).

The gradient is the exact derivative of the discrete time stepper
(discretise, then differentiate).  The reverse sweep visits n = T-1 .. 0 and,
for each step, undoes the E-half then the H-half of the forward step:

  seed      Ebar[D] += 2 E^{n+1}[D]
  grad      epsbar  -= (dt / eps^2) * sum_c Ebar_c (U_c^n - J_c^n)
  E^T half  v = (dt / eps) Ebar;  for each curl-H term (c, d, s, f):
              P = psibar + s v_c;  gbar = s kinv_E v_c + a_E P;  psibar = b_E P
              Hbar_f += (dminus_d)^T gbar
  H^T half  w = -dt Hbar;        for each curl-E term (c, d, s, f):
              P = psibar + s w_c;  gbar = s kinv_H w_c + a_H P;  psibar = b_H P
              Ebar_f += (dplus_d)^T gbar

(Ebar and Hbar pass through each half unchanged: E^{n+1} = E^n + ..., H' = H - ....)

What each variant needs from the forward run:
  full storage   E^{n+1} on D and U^n - J^n on the design box for every n
                 (the textbook way: keep the history);
  time reversal  only the interface shell of every kept step (Section 1:
                 run the simulation backwards from the final state; Section 2:
                 the PML is not invertible, so the interface fields are
                 recorded and reinjected as sources), optionally compressed
                 by bit-width reduction and k-subsampling;
  finite diff.   nothing (central differences of the forward loss).
"""

from __future__ import annotations

import numpy as np

from . import codec, store
from .yee import E_TERMS, H_TERMS, Solver, State, dminus_T, dplus_T


class AdjointState:
    def __init__(self, shape):
        self.E = np.zeros((3,) + tuple(shape))
        self.H = np.zeros((3,) + tuple(shape))
        self.psi_H = np.zeros((6,) + tuple(shape))
        self.psi_E = np.zeros((6,) + tuple(shape))


def adjoint_e_half(solver: Solver, a: AdjointState):
    """Transpose of the E-half of a step (E += (dt/eps)(U - J), U from H and psi_E)."""
    v = (solver.dt / solver.eps) * a.E
    for t, (c, d, s, f) in enumerate(E_TERMS):
        b, aa, kinv = solver.coef_E[d]
        Pb = a.psi_E[t] + s * v[c]
        gb = s * kinv * v[c] + aa * Pb
        a.psi_E[t] = b * Pb
        a.H[f] += dminus_T(gb, d, solver.periodic)


def adjoint_h_half(solver: Solver, a: AdjointState):
    """Transpose of the H-half of a step (H -= dt s (kinv g + psi_H))."""
    w = -solver.dt * a.H
    for t, (c, d, s, f) in enumerate(H_TERMS):
        b, aa, kinv = solver.coef_H[d]
        Pb = a.psi_H[t] + s * w[c]
        gb = s * kinv * w[c] + aa * Pb
        a.psi_H[t] = b * Pb
        a.E[f] += dplus_T(gb, d, solver.periodic)


def _grad_term(solver: Solver, Ebar: np.ndarray, UJ_design: np.ndarray) -> np.ndarray:
    """-(dt/eps^2) sum_c Ebar_c (U - J)_c on the design box."""
    eps = solver.eps[solver.des_sl]
    Eb = Ebar[(slice(None),) + solver.des_sl]
    return -(solver.dt / eps ** 2) * np.sum(Eb * UJ_design, axis=0)


def loss_and_history(solver: Solver):
    """Forward run keeping E^{n+1}[D], H^{n+1/2}[D] and (U^n - J^n)[design] for every step."""
    T = solver.p.steps
    s = State(solver.shape)
    E_det, H_det, UJ_des = [], [], []
    loss = 0.0
    for n in range(T):
        UJ = solver.step(s, n)
        E_det.append(s.E[(slice(None),) + solver.det_sl].copy())
        H_det.append(s.H[(slice(None),) + solver.det_sl].copy())
        UJ_des.append(UJ[(slice(None),) + solver.des_sl].copy())
        loss += solver.detector_loss(s)
    return loss, E_det, H_det, UJ_des, s


def seed(solver: Solver, a: AdjointState, E_det: np.ndarray, H_det: np.ndarray):
    """Add this step's loss derivatives to the adjoint state (before the step's transpose)."""
    gE, gH = solver.loss_seeds(E_det, H_det)
    a.E[(slice(None),) + solver.det_sl] += gE
    a.H[(slice(None),) + solver.det_sl] += gH


def grad_full_storage(problem, match_fp32: bool = False):
    """(loss, dL/deps on the design box) by the stored-history adjoint."""
    solver = Solver(problem, match_fp32)
    loss, E_det, H_det, UJ_des, _ = loss_and_history(solver)
    a = AdjointState(solver.shape)
    g = np.zeros(problem.design_shape)
    for n in range(problem.steps - 1, -1, -1):
        seed(solver, a, E_det[n], H_det[n])
        g += _grad_term(solver, a.E, UJ_des[n])
        adjoint_e_half(solver, a)
        adjoint_h_half(solver, a)
    return loss, g


def record_forward(solver: Solver, mode: str = "fp64", k: int = 1, steps: int = None):
    """Forward run that keeps the (round-tripped) interface shell of the kept steps.

    Returns (loss, per-step losses, final state, kept_H, kept_E) where kept_X
    maps a step n to the list of 6 blocks the reverse pass will read back.
    """
    T = solver.p.steps if steps is None else steps
    keep = set(store.kept_steps(T, k))
    s = State(solver.shape)
    kept_H, kept_E = {}, {}
    losses = np.zeros(T)
    for n in range(T):
        if n in keep:
            kept_E[n] = [codec.roundtrip_block(b, mode) for b in solver.shell_E(s)]  # E^n
        solver.h_update(s, n)
        if n in keep:
            kept_H[n] = [codec.roundtrip_block(b, mode) for b in solver.shell_H(s)]  # H^{n+1/2}
        solver.e_update(s, n)
        losses[n] = solver.detector_loss(s)
    return float(np.sum(losses)), losses, s, kept_H, kept_E


def shell_at(n: int, T: int, k: int, kept: dict, interp: int = 1):
    """Interpolated list of 6 shell blocks at step n (zero anchor at step -1): linear in
    time (interp 1, Section 2) or the cubic option (interp 3, store.cubic_nodes)."""
    any_blocks = next(iter(kept.values()))
    rule = store.interpolate if interp == 1 else store.interpolate_cubic
    out = []
    for b in range(len(any_blocks)):
        per_step = {m: blocks[b] for m, blocks in kept.items()}
        out.append(rule(n, T, k, per_step, np.zeros_like(any_blocks[b])))
    return out


def grad_time_reversal(problem, mode: str = "fp64", k: int = 1, match_fp32: bool = False,
                       return_trace: bool = False, interp: int = 1):
    """(loss, dL/deps on the design box) by time reversal with (compressed) shell reinjection.

    With return_trace, also returns {n: (E^n, H^{n-1/2}) on the interior} as
    reconstructed by the reverse sweep.
    """
    solver = Solver(problem, match_fp32)
    T = problem.steps
    loss, _, s, kept_H, kept_E = record_forward(solver, mode, k)
    have_shell = solver.P > 0
    a = AdjointState(solver.shape)
    g = np.zeros(problem.design_shape)
    trace = {}
    I = (slice(None),) + solver.int_sl
    for n in range(T - 1, -1, -1):
        seed(solver, a, s.E[(slice(None),) + solver.det_sl], s.H[(slice(None),) + solver.det_sl])
        if have_shell:
            solver.put_shell_H(s, shell_at(n, T, k, kept_H, interp))  # H^{n+1/2} on the low shell
        UJ = solver.e_inverse(s, n)                                     # E^n on I
        g += _grad_term(solver, a.E, UJ[(slice(None),) + solver.des_sl])
        adjoint_e_half(solver, a)
        if have_shell:
            solver.put_shell_E(s, shell_at(n, T, k, kept_E, interp))  # E^n on the high shell
        solver.h_inverse(s, n)                                          # H^{n-1/2} on I
        adjoint_h_half(solver, a)
        if return_trace:
            trace[n] = (s.E[I].copy(), s.H[I].copy())
    if return_trace:
        return loss, g, trace
    return loss, g


def loss_only(problem, match_fp32: bool = False) -> float:
    solver = Solver(problem, match_fp32)
    s = State(solver.shape)
    loss = 0.0
    for n in range(problem.steps):
        solver.step(s, n)
        loss += solver.detector_loss(s)
    return loss


def grad_finite_difference(problem, cells, h: float = 1e-4):
    """Central differences (L(eps + h e_c) - L(eps - h e_c)) / 2h for flat design-box indices."""
    shape = problem.design_shape
    base = problem.design_eps().astype(np.float64)
    out = np.zeros(len(cells))
    for i, c in enumerate(cells):
        idx = np.unravel_index(c, shape)
        vals = []
        for sgn in (+1, -1):
            d = base.copy()
            d[idx] += sgn * h
            p = _with_design64(problem, d)
            vals.append(loss_only(p))
        out[i] = (vals[0] - vals[1]) / (2 * h)
    return out


class _Eps64Problem:
    """Problem view whose eps map is float64 (finite differences need unrounded steps)."""

    def __init__(self, base, eps64):
        self.__dict__.update(base.__dict__)
        self.eps = eps64

    def design_slices(self):
        lo, hi = self.des_lo, self.des_hi
        return (slice(lo[2], hi[2]), slice(lo[1], hi[1]), slice(lo[0], hi[0]))

    @property
    def design_shape(self):
        lo, hi = self.des_lo, self.des_hi
        return (hi[2] - lo[2], hi[1] - lo[1], hi[0] - lo[0])


def _with_design64(problem, design64):
    eps = np.asarray(problem.eps, np.float64).copy()
    eps[problem.design_slices()] = design64
    return _Eps64Problem(problem, eps)
