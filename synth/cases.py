"""Seeded synthetic cases: channel, tube-plus-sac aneurysm, coil, periodic box.

Conventions (all arrays are C-ordered with shape (nz, ny, nx), so the flat box
index is ``x + nx * (y + ny * z)``):

* ``solid`` is ``uint8``: 1 for a solid voxel, 0 for fluid.
* ``phi`` is ``float32`` porosity, in (0, 1] on fluid and 0 on solid voxels.
* ``sac`` is a ``bool`` mask of the aneurysm sac (sphere minus tube).
* ``inlet_shape`` has shape (nz, ny): the normalised Hagen-Poiseuille profile
  ``1 - r^2/R^2`` of the inflow (the paper's inflow-profile paragraph in its
  simulation-setup section) on inlet cells of the x = 0 face, 0 elsewhere.
* the inlet amplitude is ``a0 * (1 + a1 * sin(2 pi t / period))`` with t the
  step index; only the three numbers travel with the case.

Geometry recipe of the aneurysm cases: cell centres at integer coordinates,
tube axis at (y_c, z_c) = (ny/2 - 1/2, nz/2 - 1/2), tube fluid where
(y - y_c)^2 + (z - z_c)^2 < R^2 (strict) for every x; sac = sphere of radius
R_s centred at (nx/2 - 1/2, y_c + D, z_c) with D = R + round(0.7 R_s), minus the
tube.  Sac porosity comes from a Gaussian random field: i.i.d. N(0, 1) noise from
``numpy.random.default_rng(seed)`` over the sphere's bounding box, a Gaussian
filter of standard deviation ``ell``, standardisation over the sac voxels to xi,
then phi = 0.65 + 0.30 * Phi(xi)^beta with Phi the standard normal CDF and
beta = 0.30/0.13 - 1, so that E[phi] = 0.78 on the range (0.65, 0.95).
"""

from __future__ import annotations

import dataclasses
import math
from typing import Dict, Optional, Tuple

import numpy as np
from scipy import ndimage, special

# Lattice-unit Carreau-Yasuda parameters shared by every configuration.
CY_DEFAULT = dict(nu0=0.1, nu_inf=0.01, lam=50.0, n=0.36, a=2.0)
BETA_PHI = 0.30 / 0.13 - 1.0


@dataclasses.dataclass
class Case:
    name: str
    nx: int
    ny: int
    nz: int
    periodic: Tuple[bool, bool, bool]
    solid: np.ndarray
    phi: np.ndarray
    sac: np.ndarray
    inlet: bool = False
    outlet: int = 0  # outflow on x = nx - 1: 0 none, 1 constant density, 2 extrapolation
    inlet_shape: Optional[np.ndarray] = None
    wave: Tuple[float, float, float] = (0.0, 0.0, 1.0)
    # optional: pre-run ramp length and a sampled waveform (one period, FP64)
    # that replaces the sine of ``wave`` (whose period still applies)
    ramp_steps: int = 0
    wave_table: Optional[np.ndarray] = None
    rho_out: float = 1.0
    rheology: Dict[str, float] = dataclasses.field(default_factory=lambda: dict(CY_DEFAULT))
    # Darcy/Forchheimer drag parameters: nu_d (kinematic viscosity in the
    # porous medium), kc (Kozeny-Carman constant), d (grain size), forchheimer
    # (0 = off, 1 = Ergun constant), g (body force per unit mass).
    porous: Dict[str, object] = dataclasses.field(
        default_factory=lambda: dict(nu_d=0.1, kc=180.0, d=2.0, forchheimer=0, g=(0.0, 0.0, 0.0)))
    steps: int = 0
    extra: Dict[str, object] = dataclasses.field(default_factory=dict)
    lattice: int = 19  # velocity set: 19 (D3Q19) or 27 (D3Q27, the paper's)

    @property
    def n_box(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def fluid(self) -> np.ndarray:
        return self.solid == 0

    @property
    def n_fluid(self) -> int:
        return int(np.count_nonzero(self.solid == 0))

    def fluid_index(self) -> np.ndarray:
        """Flat box indices of the fluid cells in ascending (z, y, x) order."""
        return np.flatnonzero(self.solid.reshape(-1) == 0)

    def with_(self, **kw) -> "Case":
        return dataclasses.replace(self, **kw)


def _zeros(nz, ny, nx, dtype):
    return np.zeros((nz, ny, nx), dtype=dtype)


def channel_case(n: int = 32, g: float = 1e-6, rheology=None, steps: int = 2000,
                 ny: Optional[int] = None, nx: Optional[int] = None, nz: Optional[int] = None,
                 phi: float = 1.0, nu_d: float = 0.1, kc: float = 180.0, d: float = 2.0,
                 forchheimer: int = 0) -> Case:
    """Plane channel: solid node layers at y = 0 and y = ny - 1, periodic x and z,
    body force g along x, uniform porosity ``phi`` (1 by default).

    With ny = 32 the fluid occupies y = 1 .. 30 and the halfway bounce-back walls
    sit at y = 0.5 and y = 30.5 (channel width 30).
    """
    nx = n if nx is None else nx
    ny = n if ny is None else ny
    nz = n if nz is None else nz
    solid = _zeros(nz, ny, nx, np.uint8)
    solid[:, 0, :] = 1
    solid[:, ny - 1, :] = 1
    ph = np.where(solid == 0, np.float32(phi), np.float32(0.0)).astype(np.float32)
    return Case(name=f"channel{nx}x{ny}x{nz}", nx=nx, ny=ny, nz=nz, periodic=(True, False, True),
                solid=solid, phi=ph, sac=np.zeros_like(solid, dtype=bool),
                rheology=dict(CY_DEFAULT if rheology is None else rheology),
                porous=dict(nu_d=nu_d, kc=kc, d=d, forchheimer=forchheimer, g=(g, 0.0, 0.0)),
                steps=steps)


def _grf_phi(shape, ell: float, rng: np.random.Generator, region: np.ndarray) -> np.ndarray:
    noise = rng.standard_normal(shape)
    field = ndimage.gaussian_filter(noise, sigma=ell, mode="reflect", truncate=4.0)
    vals = field[region]
    xi = (field - vals.mean()) / vals.std()
    u = special.ndtr(xi)
    return (0.65 + 0.30 * np.power(u, BETA_PHI)).astype(np.float32)


def aneurysm_case(nx: int, ny: int, nz: int, R: float, Rs: float, ell: float, seed: int,
                  steps: int = 20000, name: str = "aneurysm", wave=(0.05, 0.5, 4000.0),
                  kc: float = 180.0, d: float = 2.0, rheology=None) -> Case:
    """Straight tube along x with a spherical sac off its side (module docstring
    gives the recipe); GRF porosity in the sac; velocity inlet at x = 0, constant
    density outlet at x = nx - 1, walls elsewhere."""
    yc = ny / 2.0 - 0.5
    zc = nz / 2.0 - 0.5
    D = R + round(0.7 * Rs)
    cx, cy, cz = nx / 2.0 - 0.5, yc + D, zc
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    tube = (y - yc) ** 2 + (z - zc) ** 2 < R * R
    sphere = (x - cx) ** 2 + (y - cy) ** 2 + (z - cz) ** 2 < Rs * Rs
    fluid = tube | sphere
    sac = sphere & ~tube
    solid = (~fluid).astype(np.uint8)

    phi = np.where(fluid, np.float32(1.0), np.float32(0.0)).astype(np.float32)
    # GRF over the sphere's bounding box (clipped to the domain).
    lo = [max(0, int(math.floor(c - Rs))) for c in (cz, cy, cx)]
    hi = [min(nn, int(math.ceil(c + Rs)) + 1) for c, nn in zip((cz, cy, cx), (nz, ny, nx))]
    sl = tuple(slice(a, b) for a, b in zip(lo, hi))
    rng = np.random.default_rng(seed)
    sub = _grf_phi(tuple(b - a for a, b in zip(lo, hi)), ell, rng, sac[sl])
    phi_sub = phi[sl]
    phi_sub[sac[sl]] = sub[sac[sl]]
    phi[sl] = phi_sub

    r2 = (y[0, :, 0][None, :] - yc) ** 2 + (np.arange(nz)[:, None] - zc) ** 2
    shape = np.where(r2 < R * R, 1.0 - r2 / (R * R), 0.0).astype(np.float32)
    shape = np.where(solid[:, :, 0] == 0, shape, 0.0).astype(np.float32)
    return Case(name=name, nx=nx, ny=ny, nz=nz, periodic=(False, False, False), solid=solid,
                phi=phi, sac=sac, inlet=True, outlet=True, inlet_shape=shape, wave=tuple(wave),
                rho_out=1.0, rheology=dict(CY_DEFAULT if rheology is None else rheology),
                porous=dict(nu_d=0.1, kc=kc, d=d, forchheimer=0, g=(0.0, 0.0, 0.0)), steps=steps,
                extra=dict(R=R, Rs=Rs, D=D, ell=ell, seed=seed))


def coarsen2(case: Case, name: Optional[str] = None) -> Case:
    """2x-coarsened copy of an aneurysm case: same recipe at half the radii, with
    the sac porosity taken as the 2x2x2 block mean of the fine porosity."""
    e = case.extra
    nx, ny, nz = case.nx // 2, case.ny // 2, case.nz // 2
    c = aneurysm_case(nx, ny, nz, R=e["R"] / 2.0, Rs=e["Rs"] / 2.0, ell=e["ell"] / 2.0, seed=e["seed"],
                      steps=case.steps, name=name or case.name + "_coarse", wave=case.wave,
                      kc=case.porous["kc"], d=case.porous["d"], rheology=case.rheology)
    fine = case.phi.astype(np.float64)
    fine_fluid = (case.solid == 0).astype(np.float64)
    blk_sum = fine.reshape(nz, 2, ny, 2, nx, 2).sum(axis=(1, 3, 5))
    blk_cnt = fine_fluid.reshape(nz, 2, ny, 2, nx, 2).sum(axis=(1, 3, 5))
    mean = np.where(blk_cnt > 0, blk_sum / np.maximum(blk_cnt, 1), 1.0)
    phi = c.phi.copy()
    phi[c.sac] = np.clip(mean[c.sac], 0.05, 1.0).astype(np.float32)
    return c.with_(phi=phi)


def _coil_mask(case: Case, packing: float, wire_d: float, loop_r: Tuple[float, float], seed: int) -> np.ndarray:
    """Voxelised coil: a seeded random walk of helical loops inside the sac.

    Each loop picks a random axis through the current point, a radius drawn from
    ``loop_r`` and sweeps one helical turn with a pitch of one wire diameter;
    centreline samples (spacing 0.5 voxel) that would put the wire outside the
    sphere are skipped.  Voxels within wire_d/2 of a sample become coil.  The
    walk then moves on to a point of that loop at an angle drawn from
    [pi/2, 3pi/2] from its start (up to one loop diameter away), so successive
    loops spread through the sac instead of piling up at one spot.  Loops are
    added until the coil covers ``packing`` of the sac voxels.
    """
    e = case.extra
    rng = np.random.default_rng(seed)
    nx, ny, nz = case.nx, case.ny, case.nz
    yc, zc = ny / 2.0 - 0.5, nz / 2.0 - 0.5
    centre = np.array([nx / 2.0 - 0.5, yc + e["D"], zc])
    Rs = float(e["Rs"])
    rw = wire_d / 2.0
    coil = np.zeros((nz, ny, nx), dtype=bool)
    n_sac = int(np.count_nonzero(case.sac))
    target = packing * n_sac
    pos = centre.copy()
    offs = np.arange(-int(math.ceil(rw)), int(math.ceil(rw)) + 1)
    oz, oy, ox = np.meshgrid(offs, offs, offs, indexing="ij")
    ball = (ox ** 2 + oy ** 2 + oz ** 2) <= rw * rw + 1e-9
    bx, by, bz = ox[ball], oy[ball], oz[ball]
    count = 0
    loops = 0
    while count < target and loops < 100000:
        loops += 1
        axis = rng.standard_normal(3)
        axis /= np.linalg.norm(axis)
        tmp = np.array([1.0, 0.0, 0.0]) if abs(axis[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
        e1 = np.cross(axis, tmp)
        e1 /= np.linalg.norm(e1)
        e2 = np.cross(axis, e1)
        r = rng.uniform(*loop_r)
        # the loop passes through the current point: its centre sits r away along e1
        lc = pos - r * e1
        nsamp = max(8, int(2 * math.pi * r / 0.5))
        th_next = rng.uniform(0.5 * math.pi, 1.5 * math.pi)
        last = pos
        for k in range(nsamp + 1):
            th = 2 * math.pi * k / nsamp
            p = lc + r * (math.cos(th) * e1 + math.sin(th) * e2) + axis * wire_d * th / (2 * math.pi)
            if np.linalg.norm(p - centre) > Rs - rw - 0.5:
                continue
            if th <= th_next:
                last = p
            ix = np.rint(p[0] + bx).astype(int)
            iy = np.rint(p[1] + by).astype(int)
            iz = np.rint(p[2] + bz).astype(int)
            ok = (ix >= 0) & (ix < nx) & (iy >= 0) & (iy < ny) & (iz >= 0) & (iz < nz)
            coil[iz[ok], iy[ok], ix[ok]] = True
        pos = last
        if loops % 8 == 0:
            count = int(np.count_nonzero(coil & case.sac))
    coil &= case.sac
    return coil


def coil_cases(nx=384, ny=256, nz=256, R=24.0, Rs=40.0, packing=0.22, wire_d=3.0,
               loop_r=(6.0, 12.0), seed=3, window=8, steps=20000):
    """Fully resolved coil (coil voxels solid, porosity 1) and its volume-averaged
    twin (vessel mask only, porosity 1 - box-filter of the coil indicator over a
    window of ``window`` voxels with offsets -window/2 .. window/2 - 1)."""
    base = aneurysm_case(nx, ny, nz, R, Rs, ell=4.0, seed=seed, steps=steps, name="coil_base")
    coil = _coil_mask(base, packing, wire_d, loop_r, seed)
    solid_res = (base.solid.astype(bool) | coil).astype(np.uint8)
    phi_res = np.where(solid_res == 0, np.float32(1.0), np.float32(0.0)).astype(np.float32)
    resolved = base.with_(name="coil_resolved", solid=solid_res, phi=phi_res,
                          sac=base.sac & ~coil)
    frac = ndimage.uniform_filter(coil.astype(np.float64), size=window, mode="constant", origin=0)
    phi_avg = np.where(base.solid == 0, 1.0 - frac, 0.0)
    # floor 0.2: the porosity-jump collision term diverges (FP64 oracle and GPU
    # alike) where the porosity jumps sharply from 1 to 0.1 or below with these
    # drag parameters, and about 1 % of the width-8 windows are almost filled
    # by wire
    phi_avg = np.where(base.solid == 0, np.clip(phi_avg, 0.2, 1.0), 0.0).astype(np.float32)
    # inflow and outflow cells keep porosity 1
    phi_avg[:, :, 0] = np.where(base.solid[:, :, 0] == 0, 1.0, 0.0)
    phi_avg[:, :, -1] = np.where(base.solid[:, :, -1] == 0, 1.0, 0.0)
    averaged = base.with_(name="coil_averaged", phi=phi_avg)
    packing_got = float(np.count_nonzero(coil)) / max(1, int(np.count_nonzero(base.sac)))
    resolved.extra = dict(base.extra, packing=packing_got)
    averaged.extra = dict(base.extra, packing=packing_got)
    return resolved, averaged


def periodic_box_case(nx=512, ny=320, nz=320, ell=10.0, seed=5, g=1e-6, steps=2000) -> Case:
    """All-fluid box, periodic in every axis, body force along x, GRF porosity in
    every cell (the HBM-scale throughput case)."""
    rng = np.random.default_rng(seed)
    region = np.ones((nz, ny, nx), dtype=bool)
    phi = _grf_phi((nz, ny, nx), ell, rng, region)
    return Case(name=f"periodic{nx}x{ny}x{nz}", nx=nx, ny=ny, nz=nz, periodic=(True, True, True),
                solid=np.zeros((nz, ny, nx), np.uint8), phi=phi,
                sac=np.zeros((nz, ny, nx), bool),
                porous=dict(nu_d=0.1, kc=180.0, d=2.0, forchheimer=0, g=(g, 0.0, 0.0)), steps=steps)


def tiny_case(kind: str = "open", seed: int = 0, nx: int = 9, ny: int = 7, nz: int = 6) -> Case:
    """Small lattices with every cell type, for brute-force and parity checks.

    ``open``: non-periodic box, random solid voxels (about 15 %), velocity inlet
    on x = 0 and density outlet on x = nx - 1 (porosity 1 there), random porosity
    in [0.6, 1] elsewhere, fluid cells also touching the y/z faces (treated as
    walls).  ``periodic``: periodic x and z, solid layers at y = 0 and ny - 1 plus
    random solid voxels, random porosity, body force.  ``periodic3``: periodic
    in all three axes, random solid voxels, random porosity, body force.
    ``periodic_aniso``: ``periodic`` with Forchheimer drag and an anisotropic
    permeability shape (seeded SPD matrix, 6 fixed-point iterations).
    ``open_wave``: ``open`` with a 6-step pre-run ramp and a sampled 9-point
    inflow waveform of period 13 steps.  ``open_extrap``: ``open`` with the
    extrapolation outflow and one outflow cell whose -x neighbour is solid.
    ``bulk``: long rows (260 x 6 x 5, periodic in y and z, open in x) whose
    middles are wall-free, with uniform porosity 0.8 (1 near the open faces),
    a random-porosity patch and two solid voxels, so that whole waves of
    interior cells occur with uniform and with varying porosity.
    ``degenerate``: a 2 x 1 x 3 box periodic in all axes (both x neighbours
    are one cell, y neighbours are the cell's own row), random porosity.
    """
    if kind == "bulk":
        nx, ny, nz = 260, 6, 5
        rng = np.random.default_rng(1000 + seed)
        solid = np.zeros((nz, ny, nx), np.uint8)
        solid[2, 3, 230] = 1
        solid[4, 0, 20] = 1
        phi = np.full((nz, ny, nx), 0.8, np.float32)
        phi[:, :, :3] = 1.0
        phi[:, :, nx - 3:] = 1.0
        patch = rng.uniform(0.6, 1.0, (nz, ny, 30)).astype(np.float32)
        rows = (np.add.outer(np.arange(nz), np.arange(ny)) % 3 == 0)
        phi[:, :, 150:180] = np.where(rows[:, :, None], patch, phi[:, :, 150:180])
        shape = rng.uniform(0.2, 1.0, (nz, ny)).astype(np.float32)
        case = Case(name=f"tiny_bulk{seed}", nx=nx, ny=ny, nz=nz, periodic=(False, True, True),
                    solid=solid, phi=phi, sac=rng.random((nz, ny, nx)) < 0.5, inlet=True, outlet=True,
                    inlet_shape=shape, wave=(0.03, 0.5, 40.0), rho_out=1.0,
                    porous=dict(nu_d=0.1, kc=180.0, d=2.0, forchheimer=0, g=(0.0, 0.0, 0.0)))
        case.phi = np.where(case.solid == 0, case.phi, 0.0).astype(np.float32)
        case.sac = case.sac & (case.solid == 0)
        return case
    if kind == "degenerate":
        nx, ny, nz = 2, 1, 3
        rng = np.random.default_rng(1000 + seed)
        return Case(name=f"tiny_degenerate{seed}", nx=nx, ny=ny, nz=nz, periodic=(True, True, True),
                    solid=np.zeros((nz, ny, nx), np.uint8),
                    phi=rng.uniform(0.6, 1.0, (nz, ny, nx)).astype(np.float32),
                    sac=np.ones((nz, ny, nx), bool),
                    porous=dict(nu_d=0.1, kc=180.0, d=2.0, forchheimer=0, g=(1e-5, 2e-5, -1e-5)))
    rng = np.random.default_rng(1000 + seed)
    solid = (rng.random((nz, ny, nx)) < 0.15).astype(np.uint8)
    phi = rng.uniform(0.6, 1.0, (nz, ny, nx)).astype(np.float32)
    sac = rng.random((nz, ny, nx)) < 0.5
    if kind == "open":
        solid[:, :, 0] = 0
        solid[:, :, nx - 1] = 0
        solid[0, :, 0] = 1  # a few solid voxels on the open faces too
        solid[:, 0, nx - 1] = 1
        phi[:, :, 0] = 1.0
        phi[:, :, nx - 1] = 1.0
        shape = rng.uniform(0.2, 1.0, (nz, ny)).astype(np.float32)
        shape = np.where(solid[:, :, 0] == 0, shape, 0.0).astype(np.float32)
        case = Case(name=f"tiny_open{seed}", nx=nx, ny=ny, nz=nz, periodic=(False, False, False),
                    solid=solid, phi=phi, sac=sac, inlet=True, outlet=True, inlet_shape=shape,
                    wave=(0.03, 0.5, 40.0), rho_out=1.0,
                    porous=dict(nu_d=0.1, kc=180.0, d=2.0, forchheimer=0, g=(0.0, 0.0, 0.0)))
    elif kind == "open_wave":
        case = tiny_case("open", seed=seed, nx=nx, ny=ny, nz=nz)
        case.name = f"tiny_open_wave{seed}"
        case.ramp_steps = 6
        case.wave = (0.0, 0.0, 13.0)
        case.wave_table = sampled_waveform(9, peak=0.05, base=0.015)
        return case
    elif kind == "open_extrap":
        case = tiny_case("open", seed=seed, nx=nx, ny=ny, nz=nz)
        case.name = f"tiny_open_extrap{seed}"
        case.outlet = 2
        case.solid[nz // 2, ny // 2, nx - 2] = 1
        case.solid[nz // 2, ny // 2, nx - 1] = 0
        case.phi = np.where(case.solid == 0, case.phi, 0.0).astype(np.float32)
        case.phi[nz // 2, ny // 2, nx - 1] = 1.0
        case.sac = case.sac & (case.solid == 0)
        return case
    elif kind == "periodic":
        solid[:, 0, :] = 1
        solid[:, ny - 1, :] = 1
        case = Case(name=f"tiny_periodic{seed}", nx=nx, ny=ny, nz=nz, periodic=(True, False, True),
                    solid=solid, phi=phi, sac=sac,
                    porous=dict(nu_d=0.1, kc=180.0, d=2.0, forchheimer=0, g=(2e-5, -1e-5, 5e-6)))
    elif kind == "periodic_aniso":
        case = tiny_case("periodic", seed=seed, nx=nx, ny=ny, nz=nz)
        case.name = f"tiny_periodic_aniso{seed}"
        a = rng.standard_normal((3, 3))
        m = a @ a.T + 0.5 * np.eye(3)
        case.porous = dict(case.porous, forchheimer=1, aniso_iters=6,
                           aniso=(m[0, 0], m[1, 1], m[2, 2], m[0, 1], m[0, 2], m[1, 2]))
        return case
    elif kind == "periodic3":
        case = Case(name=f"tiny_periodic3_{seed}", nx=nx, ny=ny, nz=nz, periodic=(True, True, True),
                    solid=solid, phi=phi, sac=sac,
                    porous=dict(nu_d=0.1, kc=180.0, d=2.0, forchheimer=0, g=(1e-5, 2e-5, -1e-5)))
    else:
        raise ValueError(kind)
    case.phi = np.where(case.solid == 0, case.phi, 0.0).astype(np.float32)
    case.sac = case.sac & (case.solid == 0)
    return case


def tiny_random(seed: int) -> Case:
    """A random small lattice for broad parity checks: each extent in 1..10
    (x at least 2 with open faces), random periodic axes, an inflow and a
    constant-density or extrapolation outflow when x is not periodic, 0-30 %
    solid voxels, uniform or random porosity (1 on the open faces), random
    body force and Carreau-Yasuda lambda.  At least one fluid cell."""
    rng = np.random.default_rng(5000 + seed)
    per = tuple(bool(b) for b in rng.random(3) < 0.5)
    open_x = not per[0] and rng.random() < 0.7
    nx = int(rng.integers(2 if open_x else 1, 11))
    ny, nz = (int(v) for v in rng.integers(1, 11, 2))
    solid = (rng.random((nz, ny, nx)) < rng.uniform(0.0, 0.3)).astype(np.uint8)
    if open_x:
        solid[:, :, 0] = rng.random((nz, ny)) < 0.2
        solid[:, :, nx - 1] = rng.random((nz, ny)) < 0.2
    if solid.all():
        solid[nz // 2, ny // 2, nx // 2] = 0
    if rng.random() < 0.3:
        phi = np.full((nz, ny, nx), rng.uniform(0.6, 1.0), np.float32)
    else:
        phi = rng.uniform(0.6, 1.0, (nz, ny, nx)).astype(np.float32)
    g = tuple(float(v) for v in rng.uniform(-2e-5, 2e-5, 3))
    case = Case(name=f"tiny_random{seed}", nx=nx, ny=ny, nz=nz, periodic=per, solid=solid, phi=phi,
                sac=rng.random((nz, ny, nx)) < 0.5,
                rheology=dict(CY_DEFAULT, lam=float(rng.uniform(10.0, 200.0))),
                porous=dict(nu_d=0.1, kc=180.0, d=2.0, forchheimer=0, g=g))
    if open_x:
        case.phi[:, :, 0] = 1.0
        case.phi[:, :, nx - 1] = 1.0
        case.inlet = True
        case.outlet = int(rng.integers(1, 3))
        case.inlet_shape = np.where(solid[:, :, 0] == 0, rng.uniform(0.2, 1.0, (nz, ny)), 0.0).astype(np.float32)
        case.wave = (0.03, 0.5, 40.0)
    case.phi = np.where(case.solid == 0, case.phi, 0.0).astype(np.float32)
    case.sac = case.sac & (case.solid == 0)
    return case


def slab_of(case: Case, parts: int = 8, g: float = 1e-6) -> Case:
    """One GPU's share of an x-decomposition into ``parts`` slabs of equal
    fluid-cell counts, at its real shape: the narrowest even number of x-slices
    centred on the middle of ``case`` (for the aneurysm, through the sac centre,
    the thinnest slab of such a cut) that holds at least 1/parts of its fluid
    cells; periodic in x so that each cut face reads the other (standing in for
    the halo a neighbour would send), driven by a body force along x instead of
    the inlet."""
    per_x = (case.solid == 0).sum(axis=(0, 1))
    target = per_x.sum() / parts
    width = 2
    while width < case.nx and per_x[case.nx // 2 - width // 2: case.nx // 2 + width // 2].sum() < target:
        width += 2
    x0 = case.nx // 2 - width // 2
    sl = (slice(None), slice(None), slice(x0, x0 + width))
    porous = dict(case.porous)
    porous["g"] = (g, 0.0, 0.0)
    return Case(name=f"{case.name}_slab{width}", nx=width, ny=case.ny, nz=case.nz, periodic=(True, False, False),
                solid=np.ascontiguousarray(case.solid[sl]), phi=np.ascontiguousarray(case.phi[sl]),
                sac=np.ascontiguousarray(case.sac[sl]), rheology=dict(case.rheology), porous=porous,
                steps=case.steps, extra=dict(case.extra, slab_x0=x0), lattice=case.lattice)


def as_d3q27(case: Case) -> Case:
    """The same case on the D3Q27 velocity set."""
    case.lattice = 27
    case.name = case.name + "_q27"
    return case


def aniso_shape(seed: int = 9, ratio: float = 3.0) -> tuple:
    """A seeded permeability shape M (xx yy zz xy xz yz): a random rotation of
    diag(sqrt(ratio), 1, 1/sqrt(ratio)), i.e. permeability 'ratio' times larger
    along one direction than along another, as a coil's wire direction might
    impose.  An input, not part of the method."""
    rng = np.random.default_rng(1000 + seed)
    q, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    m = q @ np.diag([np.sqrt(ratio), 1.0, 1.0 / np.sqrt(ratio)]) @ q.T
    return (m[0, 0], m[1, 1], m[2, 2], m[0, 1], m[0, 2], m[1, 2])


def with_anisotropic_drag(case: Case, iters: int = 6, seed: int = 9) -> Case:
    """The case with Forchheimer drag and the anisotropic shape of aniso_shape."""
    case.porous = dict(case.porous, forchheimer=1, aniso=aniso_shape(seed), aniso_iters=iters)
    case.name = case.name + "_aniso"
    return case


def sampled_waveform(n: int = 128, peak: float = 0.05, base: float = 0.015) -> np.ndarray:
    """One period of a systole-like inflow waveform, n samples: a base level
    plus a raised-cosine systolic pulse in the first third of the period and a
    small secondary (dicrotic) bump.  Stands in for the paper's 1D-0D network
    waveform, which is not available."""
    s = np.arange(n, dtype=np.float64) / n
    pulse = np.where(s < 1.0 / 3.0, 0.5 * (1.0 - np.cos(6.0 * np.pi * s)), 0.0)
    bump = 0.15 * np.exp(-((s - 0.45) / 0.05) ** 2)
    return base + (peak - base) * (pulse + bump) / (1.0 + 0.15)


def fd_voxels(case: Case, count: int = 16, seed: int = 16) -> np.ndarray:
    """Flat box indices of ``count`` sac voxels drawn by default_rng(seed)."""
    cand = np.flatnonzero(case.sac.reshape(-1))
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(cand, size=min(count, cand.size), replace=False))


CONFIGS = {
    "c0": dict(kind="channel"),
    "c1": dict(kind="aneurysm", nx=192, ny=128, nz=128, R=12, Rs=20, ell=4, seed=1, steps=20000),
    "c2": dict(kind="aneurysm", nx=512, ny=320, nz=320, R=32, Rs=56, ell=10, seed=2, steps=20000),
    "c2c": dict(kind="coarse", of="c2"),
    "c3": dict(kind="coil"),
    "c4": dict(kind="aneurysm", nx=128, ny=96, nz=96, R=8, Rs=14, ell=4, seed=4, steps=4000),
    "hbm": dict(kind="periodic"),
}


def make_config(key: str):
    """Build one of the named workloads: c0 (32^3 channel), c1 (192x128x128
    aneurysm), c2 (512x320x320 aneurysm), c2c (c2 coarsened 2x), c3 (coil pair:
    returns (resolved, averaged)), c4 (128x96x96 aneurysm for gradients), hbm
    (512x320x320 periodic all-fluid box)."""
    cfg = CONFIGS[key]
    kind = cfg["kind"]
    if kind == "channel":
        return channel_case(32)
    if kind == "aneurysm":
        return aneurysm_case(cfg["nx"], cfg["ny"], cfg["nz"], cfg["R"], cfg["Rs"], cfg["ell"], cfg["seed"],
                             steps=cfg["steps"], name=key)
    if kind == "coarse":
        return coarsen2(make_config(cfg["of"]), name=key)
    if kind == "coil":
        return coil_cases()
    if kind == "periodic":
        return periodic_box_case()
    raise KeyError(key)
