"""FP64 Yee leapfrog with convolutional PML, forward step and interior inverse.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Normalised units: cell size 1, c = 1, eps0 = mu0 = 1, mu = 1 everywhere.

Staggering (standard Yee cell, integer index (i, j, k) = (x, y, z)):
    Ex (i+1/2, j, k)      Hx (i, j+1/2, k+1/2)
    Ey (i, j+1/2, k)      Hy (i+1/2, j, k+1/2)
    Ez (i, j, k+1/2)      Hz (i+1/2, j+1/2, k)
E^n lives at t = n dt, H^{n+1/2} at t = (n + 1/2) dt.

Arrays are indexed [z, y, x]; grid axis d (0 = x, 1 = y, 2 = z) is numpy
axis 2 - d.  Differences along d:
    dplus  f[i] = f[i+1] - f[i]      (E -> H-update, lands on H positions)
    dminus f[i] = f[i] - f[i-1]      (H -> E-update, lands on E positions)
with values outside the array taken as 0 (boundary 0) or wrapped (boundary 1).

Curl terms are written as (component c, axis d, sign s, source field f):
    curl E: H_c  -=  dt * s * (kinv_H * dplus_d E_f + psi_{c,d})
    curl H: U_c  +=       s * (kinv_E * dminus_d H_f + psi_{c,d})
            E_c  +=  (dt / eps) * (U_c - J_c)
with the convolutional-PML auxiliary recursion psi <- b psi + a g applied to
each difference g (Roden & Gedney's CPML, the absorbing boundary the paper
names in Section 1).  Away from the PML slabs a = 0 and kinv = 1, so psi
stays exactly zero and the update is the plain Yee scheme.
"""

from __future__ import annotations

import math

import numpy as np

# (component, axis, sign, field) for the curl of E (H-update) and of H (E-update)
H_TERMS = ((0, 1, +1, 2), (0, 2, -1, 1), (1, 2, +1, 0), (1, 0, -1, 2), (2, 0, +1, 1), (2, 1, -1, 0))
E_TERMS = ((0, 1, +1, 2), (0, 2, -1, 1), (1, 2, +1, 0), (1, 0, -1, 2), (2, 0, +1, 1), (2, 1, -1, 0))

SPEED_OF_LIGHT = 299792458.0


def courant_time_step(courant: float, dx: float = 1.0, c: float = 1.0) -> float:
    """Eq. 1: the CFL-limited step of a uniform 3-D grid, dt = C dx / (c sqrt(3))."""
    return courant * dx / (c * math.sqrt(3.0))


# ----------------------------------------------------------------------------
# Differences and their transposes
# ----------------------------------------------------------------------------

def _ax(d: int) -> int:
    return 2 - d


def _shift(f: np.ndarray, d: int, offset: int, periodic: bool) -> np.ndarray:
    """g[i] = f[i + offset] along grid axis d, zero (or wrapped) outside."""
    ax = _ax(d)
    if periodic:
        return np.roll(f, -offset, axis=ax)
    g = np.zeros_like(f)
    n = f.shape[ax]
    src = [slice(None)] * 3
    dst = [slice(None)] * 3
    if offset > 0:
        src[ax] = slice(offset, n)
        dst[ax] = slice(0, n - offset)
    else:
        src[ax] = slice(0, n + offset)
        dst[ax] = slice(-offset, n)
    g[tuple(dst)] = f[tuple(src)]
    return g


def dplus(f, d, periodic=False):
    return _shift(f, d, +1, periodic) - f


def dminus(f, d, periodic=False):
    return f - _shift(f, d, -1, periodic)


def dplus_T(g, d, periodic=False):
    """Transpose of dplus: (D+)^T g [i] = g[i-1] - g[i]."""
    return _shift(g, d, -1, periodic) - g


def dminus_T(g, d, periodic=False):
    """Transpose of dminus: (D-)^T g [i] = g[i] - g[i+1]."""
    return g - _shift(g, d, +1, periodic)


# ----------------------------------------------------------------------------
# CPML coefficients
# ----------------------------------------------------------------------------

def cpml_profile(n: int, pml: int, dt: float, node: str, order: int = 3, sigma_scale: float = 1.0,
                 kappa_max: float = 1.0, alpha_max: float = 0.05):
    """(b, a, 1/kappa) along one axis of n cells for E nodes (x = i) or H nodes (x = i + 1/2).

    Depth into the PML is measured from the interior boundary: nodes inside
    [pml, n - pml - 1/2] have depth 0.  With rho = depth / pml:
        sigma = sigma_scale * 0.8 (m + 1) rho^m     (the usual optimum for eta = dx = 1)
        kappa = 1 + (kappa_max - 1) rho^m
        alpha = alpha_max (1 - rho)
        b = exp(-(sigma / kappa + alpha) dt)
        a = sigma (b - 1) / (sigma kappa + kappa^2 alpha)   (0 where sigma = 0)
    """
    x = np.arange(n, dtype=np.float64) + (0.5 if node == "H" else 0.0)
    if pml == 0:
        return np.ones(n), np.zeros(n), np.ones(n)
    depth = np.maximum(np.maximum(pml - x, x - (n - pml - 0.5)), 0.0)
    rho = depth / pml
    sigma = sigma_scale * 0.8 * (order + 1) * rho ** order
    kappa = 1.0 + (kappa_max - 1.0) * rho ** order
    alpha = alpha_max * (1.0 - rho)
    b = np.exp(-(sigma / kappa + alpha) * dt)
    a = np.zeros(n)
    on = sigma > 0
    a[on] = sigma[on] * (b[on] - 1.0) / (sigma[on] * kappa[on] + kappa[on] ** 2 * alpha[on])
    return b, a, 1.0 / kappa


def _along(v: np.ndarray, d: int) -> np.ndarray:
    """Reshape a 1-D per-axis profile so it broadcasts along grid axis d."""
    shape = [1, 1, 1]
    shape[_ax(d)] = v.size
    return v.reshape(shape)


# ----------------------------------------------------------------------------
# Solver
# ----------------------------------------------------------------------------

class State:
    """Fields and PML auxiliaries.  E[c], H[c]: (nz, ny, nx); psi_H[t], psi_E[t]: one per curl term."""

    def __init__(self, shape):
        self.E = np.zeros((3,) + tuple(shape))
        self.H = np.zeros((3,) + tuple(shape))
        self.psi_H = np.zeros((6,) + tuple(shape))
        self.psi_E = np.zeros((6,) + tuple(shape))

    def copy(self):
        s = State(self.E.shape[1:])
        s.E[...] = self.E
        s.H[...] = self.H
        s.psi_H[...] = self.psi_H
        s.psi_E[...] = self.psi_E
        return s


class Solver:
    """FP64 discrete model of one problem.

    match_fp32 rounds the constants the GPU takes in single precision (dt and
    the CPML b, a, 1/kappa) to float32 before use, so that a comparison with
    an FP32 implementation differs only by its arithmetic.  The source signal
    and profile are float32 inputs either way; eps is taken as given (float32
    maps convert exactly; finite differences pass float64 maps).
    """

    def __init__(self, problem, match_fp32: bool = False):
        p = problem
        self.p = p
        self.shape = (p.nz, p.ny, p.nx)
        self.n_axis = (p.nx, p.ny, p.nz)
        self.P = p.pml
        self.periodic = (p.boundary == 1)
        dt = courant_time_step(p.courant)
        r = (lambda v: np.asarray(v, np.float32).astype(np.float64)) if match_fp32 else (lambda v: np.asarray(v, np.float64))
        self.dt = float(r(dt))
        self.coef_E = []
        self.coef_H = []
        for d in range(3):
            for node, dst in (("E", self.coef_E), ("H", self.coef_H)):
                b, a, kinv = cpml_profile(self.n_axis[d], p.pml, dt, node, p.pml_order, p.pml_sigma_scale,
                                          p.pml_kappa_max, p.pml_alpha_max)
                dst.append((_along(r(b), d), _along(r(a), d), _along(r(kinv), d)))
        self.eps = np.asarray(p.eps).astype(np.float64)   # float32 inputs convert exactly
        self.src_comp = p.src_comp
        self.src_sl = (slice(p.src_lo[2], p.src_hi[2]), slice(p.src_lo[1], p.src_hi[1]),
                       slice(p.src_lo[0], p.src_hi[0]))
        self.src_profile = np.asarray(p.src_profile, np.float32).astype(np.float64)
        self.src_wave = np.asarray(p.src_wave, np.float32).astype(np.float64)
        # optional magnetic current sheet (the H half of a total-field/scattered-field source)
        self.msrc_comp = getattr(p, "msrc_comp", 0)
        mlo, mhi = getattr(p, "msrc_lo", (0, 0, 0)), getattr(p, "msrc_hi", (0, 0, 0))
        self.msrc_sl = (slice(mlo[2], mhi[2]), slice(mlo[1], mhi[1]), slice(mlo[0], mhi[0]))
        self.msrc_profile = np.asarray(getattr(p, "msrc_profile", np.zeros((0, 0, 0))), np.float32).astype(np.float64)
        self.msrc_wave = np.asarray(getattr(p, "msrc_wave", np.zeros(0)), np.float32).astype(np.float64)
        self.det_sl = (slice(p.det_lo[2], p.det_hi[2]), slice(p.det_lo[1], p.det_hi[1]),
                       slice(p.det_lo[0], p.det_hi[0]))
        self.des_sl = p.design_slices()
        P = self.P
        self.int_sl = (slice(P, p.nz - P), slice(P, p.ny - P), slice(P, p.nx - P))

    # -- source -------------------------------------------------------------
    def current(self, n: int) -> np.ndarray:
        """J^n on the full grid, (3, nz, ny, nx)."""
        J = np.zeros((3,) + self.shape)
        if n < self.src_wave.size:
            J[self.src_comp][self.src_sl] = self.src_wave[n] * self.src_profile
        return J

    def magnetic_current(self, n: int):
        """M^n on the full grid (enters the H update as dH/dt = -curl E - M), or None."""
        if self.msrc_wave.size == 0 or n is None or n >= self.msrc_wave.size:
            return None
        M = np.zeros((3,) + self.shape)
        M[self.msrc_comp][self.msrc_sl] = self.msrc_wave[n] * self.msrc_profile
        return M

    # -- forward ------------------------------------------------------------
    def h_update(self, s: State, n: int = None):
        """H^{n-1/2} -> H^{n+1/2} from E^n, with the H-side PML recursions and M^n."""
        for t, (c, d, sg, f) in enumerate(H_TERMS):
            b, a, kinv = self.coef_H[d]
            g = dplus(s.E[f], d, self.periodic)
            s.psi_H[t] = b * s.psi_H[t] + a * g
            s.H[c] -= self.dt * sg * (kinv * g + s.psi_H[t])
        M = self.magnetic_current(n)
        if M is not None:
            s.H -= self.dt * M

    def curl_h(self, s: State) -> np.ndarray:
        """U = curl H with the E-side PML recursions applied (updates psi_E)."""
        U = np.zeros((3,) + self.shape)
        for t, (c, d, sg, f) in enumerate(E_TERMS):
            b, a, kinv = self.coef_E[d]
            g = dminus(s.H[f], d, self.periodic)
            s.psi_E[t] = b * s.psi_E[t] + a * g
            U[c] += sg * (kinv * g + s.psi_E[t])
        return U

    def e_update(self, s: State, n: int) -> np.ndarray:
        """E^n -> E^{n+1}; returns U^n - J^n (what the gradient of step n needs)."""
        UJ = self.curl_h(s) - self.current(n)
        s.E += (self.dt / self.eps) * UJ
        return UJ

    def step(self, s: State, n: int) -> np.ndarray:
        self.h_update(s, n)
        return self.e_update(s, n)

    def detector_energy(self, s: State) -> float:
        """sum over the detector box of |E|^2 (all three components, same cell index)."""
        return float(np.sum(s.E[(slice(None),) + self.det_sl] ** 2))

    def detector_flux(self, s: State, axis: int) -> float:
        """sum over the detector box of the Poynting vector component along `axis`,
        (E x H)_axis, from E^{n+1} and H^{n+1/2} at the same cell index."""
        E = s.E[(slice(None),) + self.det_sl]
        H = s.H[(slice(None),) + self.det_sl]
        a, b = (axis + 1) % 3, (axis + 2) % 3
        return float(np.sum(E[a] * H[b] - E[b] * H[a]))

    def detector_loss(self, s: State) -> float:
        """This step's loss term: |E|^2 (loss 0) or the flux along x, y, z (loss 1, 2, 3)."""
        kind = getattr(self.p, "loss", 0)
        return self.detector_energy(s) if kind == 0 else self.detector_flux(s, kind - 1)

    def loss_seeds(self, E_det: np.ndarray, H_det: np.ndarray):
        """(dL/dE^{n+1}, dL/dH^{n+1/2}) of one step's loss term on the detector box."""
        kind = getattr(self.p, "loss", 0)
        if kind == 0:
            return 2.0 * E_det, np.zeros_like(H_det)
        axis = kind - 1
        a, b = (axis + 1) % 3, (axis + 2) % 3
        gE = np.zeros_like(E_det)
        gH = np.zeros_like(H_det)
        gE[a], gE[b] = H_det[b], -H_det[a]       # d/dE_a (E_a H_b - E_b H_a) = H_b, d/dE_b = -H_a
        gH[b], gH[a] = E_det[a], -E_det[b]
        return gE, gH

    # -- interface shell (Section 2: interface slices between volume and PML) -------------
    def shell_H(self, s: State):
        """S_H = H^{n+1/2} at index P-1 on the three low faces (tangential components).

        Returns 6 arrays: (x-low Hy, Hz), (y-low Hz, Hx), (z-low Hx, Hy), each over
        the interior extent of the other two axes ([z][y], [z][x], [y][x] order).
        """
        P, (nz, ny, nx) = self.P, self.shape
        if P == 0:
            return []
        H = s.H
        ix, iy, iz = slice(P, nx - P), slice(P, ny - P), slice(P, nz - P)
        return [H[1][iz, iy, P - 1], H[2][iz, iy, P - 1],
                H[2][iz, P - 1, ix], H[0][iz, P - 1, ix],
                H[0][P - 1, iy, ix], H[1][P - 1, iy, ix]]

    def shell_E(self, s: State):
        """S_E = E^n at index N-P on the three high faces: (x Ey, Ez), (y Ez, Ex), (z Ex, Ey)."""
        P, (nz, ny, nx) = self.P, self.shape
        if P == 0:
            return []
        E = s.E
        ix, iy, iz = slice(P, nx - P), slice(P, ny - P), slice(P, nz - P)
        return [E[1][iz, iy, nx - P], E[2][iz, iy, nx - P],
                E[2][iz, ny - P, ix], E[0][iz, ny - P, ix],
                E[0][nz - P, iy, ix], E[1][nz - P, iy, ix]]

    def put_shell_H(self, s: State, blocks):
        P, (nz, ny, nx) = self.P, self.shape
        if P == 0:
            return
        H = s.H
        ix, iy, iz = slice(P, nx - P), slice(P, ny - P), slice(P, nz - P)
        H[1][iz, iy, P - 1], H[2][iz, iy, P - 1] = blocks[0], blocks[1]
        H[2][iz, P - 1, ix], H[0][iz, P - 1, ix] = blocks[2], blocks[3]
        H[0][P - 1, iy, ix], H[1][P - 1, iy, ix] = blocks[4], blocks[5]

    def put_shell_E(self, s: State, blocks):
        P, (nz, ny, nx) = self.P, self.shape
        if P == 0:
            return
        E = s.E
        ix, iy, iz = slice(P, nx - P), slice(P, ny - P), slice(P, nz - P)
        E[1][iz, iy, nx - P], E[2][iz, iy, nx - P] = blocks[0], blocks[1]
        E[2][iz, ny - P, ix], E[0][iz, ny - P, ix] = blocks[2], blocks[3]
        E[0][nz - P, iy, ix], E[1][nz - P, iy, ix] = blocks[4], blocks[5]

    # -- inverse on the interior (time reversal) ----------------------------------------
    def e_inverse(self, s: State, n: int) -> np.ndarray:
        """E^{n+1} -> E^n on the interior I from H^{n+1/2} (interior + low shell).

        Every interior node has PML depth 0, so U is the plain curl there.
        Returns U^n - J^n (full grid; valid on I only).
        """
        U = np.zeros((3,) + self.shape)
        for (c, d, sg, f) in E_TERMS:
            U[c] += sg * dminus(s.H[f], d, self.periodic)
        UJ = U - self.current(n)
        I = (slice(None),) + self.int_sl
        s.E[I] -= (self.dt / self.eps[self.int_sl]) * UJ[I]
        return UJ

    def h_inverse(self, s: State, n: int = None):
        """H^{n+1/2} -> H^{n-1/2} on I from E^n (interior + high shell) and M^n."""
        dH = np.zeros((3,) + self.shape)
        for (c, d, sg, f) in H_TERMS:
            dH[c] += self.dt * sg * dplus(s.E[f], d, self.periodic)
        M = self.magnetic_current(n)
        if M is not None:
            dH += self.dt * M
        I = (slice(None),) + self.int_sl
        s.H[I] += dH[I]


def run_forward(solver: Solver, steps: int = None, snapshots=()):
    """Plain forward run.  Returns (final state, per-step losses, {n: state copy after n steps})."""
    T = solver.p.steps if steps is None else steps
    s = State(solver.shape)
    losses = np.zeros(T)
    snaps = {}
    if 0 in snapshots:
        snaps[0] = s.copy()
    for n in range(T):
        solver.step(s, n)
        losses[n] = solver.detector_loss(s)
        if (n + 1) in snapshots:
            snaps[n + 1] = s.copy()
    return s, losses, snaps
