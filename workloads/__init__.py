"""Seeded synthetic FDTD problems shared by the oracle, the tests and the benchmark.

This module only *describes* inputs: grid sizes, PML thickness, step count,
Courant number, the permittivity map, the source (a box of cells, a
component, a transverse amplitude profile and a sampled time signal), the
detector box and the design box.  It contains none of the solver's
arithmetic (no Yee update, no PML recursion, no adjoint, no codec), so both
the FP64 oracle and the HIP library can consume it without sharing code.

Conventions (normalised units: cell size 1, c = 1, eps0 = mu0 = 1):
  * arrays are indexed ``[z, y, x]`` (x fastest in memory);
  * boxes are half-open, given as ``(x, y, z)`` tuples ``lo`` / ``hi``;
  * the source current on the source box at step n is
    ``J[n] * profile[z, y, x]`` on component ``src_comp`` (0 = x, 1 = y, 2 = z),
    with ``J[n]`` sampled at t = (n + 1/2) dt (the time of H^{n+1/2}).

The recipes follow the workloads the paper's experiments stand in for: a
free-space dipole with a random high-contrast design block, and a silicon
slab (eps 12.25) in a low-index cladding (eps 2.1) with a Gaussian current
sheet, i.e. the Si / SiO2 material pair of the paper's grating-coupler study
(Section 3).  The paper's own coupler geometry is not specified completely,
so these synthetic grids stand in for it.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import Optional, Tuple

import numpy as np

Box = Tuple[int, int, int]

EPS_SI = 12.25   # silicon at 1550 nm (n ~ 3.5)
EPS_CLAD = 2.1   # silica-like cladding (n ~ 1.45)


@dataclass
class Problem:
    """Complete description of one forward + gradient evaluation."""

    name: str
    nx: int
    ny: int
    nz: int
    pml: int
    steps: int
    courant: float = 0.99
    boundary: int = 0            # 0: zero outside the array, 1: periodic (pml must be 0)
    pml_order: int = 3
    pml_sigma_scale: float = 1.0
    pml_kappa_max: float = 1.0
    pml_alpha_max: float = 0.05
    src_comp: int = 2
    src_lo: Box = (0, 0, 0)
    src_hi: Box = (0, 0, 0)
    src_wave: np.ndarray = field(default_factory=lambda: np.zeros(0, np.float32))
    src_profile: np.ndarray = field(default_factory=lambda: np.zeros((0, 0, 0), np.float32))
    det_lo: Box = (0, 0, 0)
    det_hi: Box = (0, 0, 0)
    des_lo: Box = (0, 0, 0)
    des_hi: Box = (0, 0, 0)
    eps: np.ndarray = field(default_factory=lambda: np.zeros((0, 0, 0), np.float32))
    wavelength: float = 0.0      # informational (cells)
    loss: int = 0                # 0: sum of |E|^2 on the detector; 1, 2, 3: Poynting flux along x, y, z
    # optional magnetic current sheet M (dH/dt = -curl E - M), e.g. the H half of a
    # total-field/scattered-field plane-wave source; empty box = none
    msrc_comp: int = 0
    msrc_lo: Box = (0, 0, 0)
    msrc_hi: Box = (0, 0, 0)
    msrc_wave: np.ndarray = field(default_factory=lambda: np.zeros(0, np.float32))
    msrc_profile: np.ndarray = field(default_factory=lambda: np.zeros((0, 0, 0), np.float32))

    @property
    def shape(self) -> Tuple[int, int, int]:
        return (self.nz, self.ny, self.nx)

    @property
    def cells(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def design_shape(self) -> Tuple[int, int, int]:
        lo, hi = self.des_lo, self.des_hi
        return (hi[2] - lo[2], hi[1] - lo[1], hi[0] - lo[0])

    def design_slices(self):
        lo, hi = self.des_lo, self.des_hi
        return (slice(lo[2], hi[2]), slice(lo[1], hi[1]), slice(lo[0], hi[0]))

    def design_eps(self) -> np.ndarray:
        return self.eps[self.design_slices()].copy()

    def with_design(self, design: np.ndarray) -> "Problem":
        eps = self.eps.copy()
        eps[self.design_slices()] = np.asarray(design, np.float32)
        return replace(self, eps=eps)


# ----------------------------------------------------------------------------
# Source signals
# ----------------------------------------------------------------------------

def gaussian_pulse(steps: int, dt: float, wavelength: float, bandwidth: float = 0.4,
                   amplitude: float = 1.0) -> np.ndarray:
    """Gaussian-modulated sine sampled at t = (n + 1/2) dt, returned as float32.

    Carrier frequency f0 = 1 / wavelength (c = 1).  ``bandwidth`` is the full
    width at half maximum of the amplitude spectrum relative to f0, which fixes
    the envelope width tau = 2 sqrt(2 ln 2) / (2 pi bandwidth f0); the pulse is
    centred at t0 = 3 tau so that it starts from (numerically) zero.
    """
    f0 = 1.0 / wavelength
    tau = 2.0 * math.sqrt(2.0 * math.log(2.0)) / (2.0 * math.pi * bandwidth * f0)
    t0 = 3.0 * tau
    t = (np.arange(steps, dtype=np.float64) + 0.5) * dt
    s = amplitude * np.sin(2.0 * math.pi * f0 * (t - t0)) * np.exp(-((t - t0) ** 2) / (2.0 * tau * tau))
    return s.astype(np.float32)


def time_step(courant: float) -> float:
    """Step size used to *sample* source signals: dt = C / sqrt(3) in cell units.

    Input generation needs the sample times; the solvers compute their own
    step size independently.
    """
    return courant / math.sqrt(3.0)


def incident_line(steps: int, courant: float, eps_bg: float, wavelength: float, bandwidth: float = 0.4,
                  amplitude: float = 1.0, lead: int = 20):
    """Incident plane wave for a total-field/scattered-field sheet, from a 1-D Yee line.

    An x-polarised wave travelling along +z in a uniform medium eps_bg obeys, in
    the 3-D grid, exactly the 1-D recurrence run here (same dt and cell):
        Hy[k] -= dt (Ex[k+1] - Ex[k]);   Ex[k] -= (dt / eps_bg) (Hy[k] - Hy[k-1]) + (dt / eps_bg) J
    driven by a soft current J (the Gaussian pulse) `lead` cells before the sheet.
    Returns (Ex^n at the sheet plane, Hy^{n+1/2} half a cell before it) for n < steps,
    in float64; the line is long enough that nothing returns from its ends.
    """
    dt = time_step(courant)
    half = int(steps * dt / math.sqrt(eps_bg)) + lead + 16
    size = 2 * half + 1
    zs, zi = half, half + lead
    sig = gaussian_pulse(steps, dt, wavelength, bandwidth, amplitude).astype(np.float64)
    ex = np.zeros(size)
    hy = np.zeros(size)
    ex_rec = np.zeros(steps)
    hy_rec = np.zeros(steps)
    c = dt / eps_bg
    for n in range(steps):
        ex_rec[n] = ex[zi]
        hy[:-1] -= dt * (ex[1:] - ex[:-1])
        hy_rec[n] = hy[zi - 1]
        ex[1:] -= c * (hy[1:] - hy[:-1])
        ex[zs] -= c * sig[n]
    return ex_rec, hy_rec


def with_tfsf_plane_wave(p: Problem, z0: int, wavelength: float, bandwidth: float = 0.4,
                         amplitude: float = 1.0) -> Problem:
    """Replace the source of `p` by a total-field/scattered-field sheet at plane z0.

    An x-polarised plane wave enters the total-field region z >= z0 travelling
    along +z over the interior x-y extent: an electric sheet J_x = -Hy_inc(z0 - 1/2)
    on the Ex plane z0 and a magnetic sheet M_y = -Ex_inc(z0) on the Hy plane z0 - 1
    (the corrections of the two updates that straddle the plane).  Nothing is
    emitted into z < z0 where the wave is a plane wave of the background eps at
    the sheet.
    """
    P = p.pml
    lo, hi = (P, P), (p.nx - P, p.ny - P)
    eps_bg = float(p.eps[z0, p.ny // 2, p.nx // 2])
    ex_inc, hy_inc = incident_line(p.steps, p.courant, eps_bg, wavelength, bandwidth, amplitude)
    shape = (1, hi[1] - lo[1], hi[0] - lo[0])
    return replace(p, src_comp=0, src_lo=(lo[0], lo[1], z0), src_hi=(hi[0], hi[1], z0 + 1),
                   src_wave=(-hy_inc).astype(np.float32), src_profile=np.ones(shape, np.float32),
                   msrc_comp=1, msrc_lo=(lo[0], lo[1], z0 - 1), msrc_hi=(hi[0], hi[1], z0),
                   msrc_wave=(-ex_inc).astype(np.float32), msrc_profile=np.ones(shape, np.float32))


# ----------------------------------------------------------------------------
# Presets
# ----------------------------------------------------------------------------

def _point_source(pos: Box):
    lo = tuple(pos)
    hi = (pos[0] + 1, pos[1] + 1, pos[2] + 1)
    return lo, hi, np.ones((1, 1, 1), np.float32)


def _random_design(eps: np.ndarray, lo: Box, hi: Box, lo_val: float, hi_val: float, seed: int):
    rng = np.random.default_rng(seed)
    shape = (hi[2] - lo[2], hi[1] - lo[1], hi[0] - lo[0])
    eps[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]] = rng.uniform(lo_val, hi_val, shape).astype(np.float32)


def dipole_problem(name: str, n: Box, pml: int, steps: int, src: Box, wavelength: float,
                   des_lo: Box, des_hi: Box, det_lo: Box, det_hi: Box, seed: int = 0,
                   eps_range=(1.0, 12.25), bandwidth: float = 0.4, courant: float = 0.99,
                   src_comp: int = 2) -> Problem:
    """Free-space Ez point dipole, random-eps design block, |E|^2 plane detector."""
    nx, ny, nz = n
    eps = np.ones((nz, ny, nx), np.float32)
    _random_design(eps, des_lo, des_hi, eps_range[0], eps_range[1], seed)
    slo, shi, prof = _point_source(src)
    wave = gaussian_pulse(steps, time_step(courant), wavelength, bandwidth)
    return Problem(name=name, nx=nx, ny=ny, nz=nz, pml=pml, steps=steps, courant=courant,
                   src_comp=src_comp, src_lo=slo, src_hi=shi, src_wave=wave, src_profile=prof,
                   det_lo=det_lo, det_hi=det_hi, des_lo=des_lo, des_hi=des_hi, eps=eps,
                   wavelength=wavelength)


def slab_problem(name: str, n: Box, pml: int, steps: int, src_z: int, waist: float,
                 wavelength: float, slab_z: Tuple[int, int], des_lo: Box, des_hi: Box,
                 det_lo: Box, det_hi: Box, seed: int = 0, bandwidth: float = 0.4,
                 courant: float = 0.99) -> Problem:
    """Silicon slab in cladding, Gaussian Jy current sheet, yz-plane output detector."""
    nx, ny, nz = n
    eps = np.full((nz, ny, nx), EPS_CLAD, np.float32)
    eps[slab_z[0]:slab_z[1], :, :] = EPS_SI
    _random_design(eps, des_lo, des_hi, EPS_CLAD, EPS_SI, seed)
    # current sheet over the interior extent of the plane z = src_z
    slo = (pml, pml, src_z)
    shi = (nx - pml, ny - pml, src_z + 1)
    xs = np.arange(slo[0], shi[0], dtype=np.float64)
    ys = np.arange(slo[1], shi[1], dtype=np.float64)
    r2 = (xs[None, :] - nx / 2) ** 2 + (ys[:, None] - ny / 2) ** 2
    prof = np.exp(-r2 / (waist * waist)).astype(np.float32)[None, :, :]
    wave = gaussian_pulse(steps, time_step(courant), wavelength, bandwidth)
    return Problem(name=name, nx=nx, ny=ny, nz=nz, pml=pml, steps=steps, courant=courant,
                   src_comp=1, src_lo=slo, src_hi=shi, src_wave=wave, src_profile=prof,
                   det_lo=det_lo, det_hi=det_hi, des_lo=des_lo, des_hi=des_hi, eps=eps,
                   wavelength=wavelength)


def c1(seed: int = 0, steps: int = 200) -> Problem:
    """32^3, 8-cell CPML, 200 steps, Ez dipole at the centre (lambda 20), 8^3 design."""
    return dipole_problem("c1_32cube", (32, 32, 32), 8, steps, (16, 16, 16), 20.0,
                          (12, 12, 12), (20, 20, 20), (8, 8, 22), (24, 24, 23), seed=seed)


def c2(seed: int = 0, steps: int = 1000, wavelength: float = 20.0) -> Problem:
    """128^3, 10-cell CPML, 1000 steps, Ez dipole (lambda 20), 32^3 design, 64x64 detector."""
    return dipole_problem("c2_128cube", (128, 128, 128), 10, steps, (64, 64, 64), wavelength,
                          (48, 48, 70), (80, 80, 102), (32, 32, 110), (96, 96, 111), seed=seed)


def c3p(seed: int = 0, steps: int = 1000) -> Problem:
    """c2 at lambda 77.5 cells, i.e. ~136 steps per period as in the paper's Section 2 example."""
    p = c2(seed=seed, steps=steps, wavelength=77.5)
    return replace(p, name="c3p_128cube_lambda77")


def c4(seed: int = 0, steps: int = 4000, wavelength: float = 30.0) -> Problem:
    """256x256x128 slab waveguide, 12-cell CPML, 4000 steps, 64x64x8 design."""
    return slab_problem("c4_slab_256x256x128", (256, 256, 128), 12, steps, 100, 16.0, wavelength,
                        (53, 75), (96, 96, 67), (160, 160, 75), (236, 96, 32), (237, 160, 96),
                        seed=seed)


def c4p(seed: int = 0, steps: int = 4000) -> Problem:
    """c4 at lambda 77.5 cells (~136 steps per period, the sampling of the paper's Section 2
    example); 16 divides the 4000 steps, so FP8 with k = 16 stores exactly 1/64 of FP32."""
    return replace(c4(seed=seed, steps=steps, wavelength=77.5), name="c4p_slab_256x256x128_lambda77")


def c4_crop(seed: int = 0, steps: int = 2000, wavelength: float = 30.0) -> Problem:
    """The c4 recipe on a 128^3 grid (x-y cropped to 128 x 128, z kept): 12-cell CPML, the
    same slab, sheet plane, waist and 64x64x8 design box, output plane 20 cells before the
    +x face; 2000 steps (16 divides it)."""
    return slab_problem("c4crop_slab_128cube", (128, 128, 128), 12, steps, 100, 16.0, wavelength,
                        (53, 75), (32, 32, 67), (96, 96, 75), (108, 32, 32), (109, 96, 96),
                        seed=seed)


def c4p_crop(seed: int = 0, steps: int = 2000) -> Problem:
    """c4_crop at lambda 77.5 cells (the 128^3 crop of c4p)."""
    return replace(c4_crop(seed=seed, steps=steps, wavelength=77.5), name="c4pcrop_slab_128cube_lambda77")


def c5(seed: int = 0, steps: int = 8000, wavelength: float = 30.0) -> Problem:
    """512x512x256 slab waveguide, 16-cell CPML, 8000 steps, 128x128x16 design."""
    return slab_problem("c5_slab_512x512x256", (512, 512, 256), 16, steps, 200, 32.0, wavelength,
                        (117, 139), (192, 192, 123), (320, 320, 139), (488, 192, 64),
                        (489, 320, 192), seed=seed)


def c5_crop(seed: int = 0, steps: int = 2000) -> Problem:
    """The c5 recipe instantiated on a 128^3 grid (16-cell CPML), design cropped to 64x64x16."""
    return slab_problem("c5crop_slab_128cube", (128, 128, 128), 16, steps, 100, 32.0, 30.0,
                        (61, 83), (32, 32, 67), (96, 96, 83), (108, 32, 24), (109, 96, 88),
                        seed=seed)


def c2pw(seed: int = 0, steps: int = 1000, wavelength: float = 20.0) -> Problem:
    """c2 driven by a total-field/scattered-field plane wave entering at z = 24, with the
    Poynting flux through the detector plane z = 110 as the objective (transmission)."""
    p = c2(seed=seed, steps=steps, wavelength=wavelength)
    p = with_tfsf_plane_wave(p, 24, wavelength)
    return replace(p, name="c2pw_128cube_tfsf_flux", loss=3)


def tiny_pw(seed: int = 0, steps: int = 60) -> Problem:
    """tiny with a total-field/scattered-field plane wave entering at z = 4 and z-flux objective."""
    p = tiny(seed=seed, steps=steps)
    return replace(with_tfsf_plane_wave(p, 4, 8.0, 0.6), name="tiny_pw", loss=3)


def tiny(seed: int = 0, n: Box = (12, 12, 12), pml: int = 3, steps: int = 60,
         wavelength: float = 8.0) -> Problem:
    """Small grid for brute-force checks: 12^3, 3-cell CPML, 3^3 design around the source."""
    nx, ny, nz = n
    c = (nx // 2, ny // 2, nz // 2)
    return dipole_problem("tiny", n, pml, steps, c, wavelength,
                          (c[0] - 1, c[1] - 1, c[2] - 1), (c[0] + 2, c[1] + 2, c[2] + 2),
                          (pml + 1, pml + 1, nz - pml - 1), (nx - pml - 1, ny - pml - 1, nz - pml),
                          seed=seed, bandwidth=0.6)


def ragged(seed: int = 0, steps: int = 40) -> Problem:
    """Odd-sized grid (not a multiple of any tile) with a plane source and a thick detector box."""
    nx, ny, nz = 70, 37, 29
    pml = 5
    eps = np.full((nz, ny, nx), 1.5, np.float32)
    des_lo, des_hi = (20, 10, 12), (45, 27, 19)
    _random_design(eps, des_lo, des_hi, 1.0, 12.25, seed)
    slo, shi = (pml, pml, 8), (nx - pml, ny - pml, 9)
    rng = np.random.default_rng(seed + 77)
    prof = rng.uniform(0.2, 1.0, (1, shi[1] - slo[1], shi[0] - slo[0])).astype(np.float32)
    wave = gaussian_pulse(steps, time_step(0.99), 10.0, 0.6)
    return Problem(name="ragged_70x37x29", nx=nx, ny=ny, nz=nz, pml=pml, steps=steps,
                   src_comp=0, src_lo=slo, src_hi=shi, src_wave=wave, src_profile=prof,
                   det_lo=(10, 8, 20), det_hi=(60, 30, 23), des_lo=des_lo, des_hi=des_hi,
                   eps=eps, wavelength=10.0)


PRESETS = {
    "c1": c1, "c2": c2, "c3p": c3p, "c4": c4, "c4p": c4p, "c4crop": c4_crop, "c4pcrop": c4p_crop,
    "c5": c5, "c5crop": c5_crop,
    "tiny": tiny, "ragged": ragged, "c2pw": c2pw, "tiny_pw": tiny_pw,
}


def make(name: str, **kw) -> Problem:
    return PRESETS[name](**kw)


def random_fields(shape, seed: int, scale: float = 1.0) -> np.ndarray:
    """Seeded uniform random array in [-scale, scale) as float64 (for state-level tests)."""
    rng = np.random.default_rng(seed)
    return rng.uniform(-scale, scale, shape)


def fd_cells(problem: Problem, count: int, seed: int) -> np.ndarray:
    """Seeded choice of design cells (flat indices into the design box) for finite differences."""
    n = int(np.prod(problem.design_shape))
    rng = np.random.default_rng(1000 + seed)
    return np.sort(rng.choice(n, size=min(count, n), replace=False))
