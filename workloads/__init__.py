"""Seeded synthetic inputs shared by the oracle, the HIP path, the tests and the bench.

This module holds no arithmetic of the simulation method: it only draws numbers
(SplitMix64, a published counter-based generator by Steele, Lea and Flood, 2014)
and lays out particle beds, target height maps and per-instance parameters with
the geometry ratios of the paper's digging workload (flat bed in a box, surface
observed as a 40x40 height map, Sec. III-A "States and observations").

Everything here returns plain numpy arrays and dicts; both sides of every parity
test receive exactly the same arrays.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import List, Optional

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, count: int, offset: int = 0) -> np.ndarray:
    """Outputs ``offset .. offset+count-1`` of the SplitMix64 stream for ``seed``.

    SplitMix64's state after i draws is seed + i*golden, so output i is a pure
    function of (seed, i): the stream is evaluated vectorised.
    """
    with np.errstate(over="ignore"):
        i = np.arange(offset + 1, offset + count + 1, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + i * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, count: int, offset: int = 0) -> np.ndarray:
    """Uniform doubles in [0, 1) with 53 random bits each."""
    z = splitmix64(seed, count, offset)
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


class Stream:
    """Sequential draws from one SplitMix64 stream."""

    def __init__(self, seed: int):
        self.seed = seed
        self.pos = 0

    def uniform(self, count: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
        u = uniform01(self.seed, count, self.pos)
        self.pos += count
        return lo + (hi - lo) * u


# --------------------------------------------------------------------------
# Workload descriptions
# --------------------------------------------------------------------------

@dataclass
class Material:
    E: float = 3.5e5          # Young's modulus [Pa]
    nu: float = 0.3           # Poisson's ratio
    phi_deg: float = 30.0     # friction angle [deg]
    rho: float = 1600.0       # density [kg/m^3]
    cohesion: float = 0.0     # [Pa]


@dataclass
class Skill:
    """Skill parameters in physical units (Sec. III-B, phases 1-4)."""
    depth: float = 0.05       # insertion distance d2 [m]
    angle_deg: float = 30.0   # rotation phi1 [deg]
    push: float = 0.15        # push distance d3 [m]
    displace: float = 0.0     # phase-1 displacement d1 along x [m] (theta_displace = 0)
    push_angle_deg: float = 180.0   # push angle phi3 [deg] (theta_push_angle = 0)


@dataclass
class Workload:
    name: str
    dim: int
    n_grid: int
    dt: float
    steps: int
    precision: str                      # "f32" or "f64"
    ppc: int                            # particles per cell
    bed_lo: tuple                       # first bed cell per axis (build frame, y up)
    bed_hi: tuple                       # one past the last bed cell per axis
    seed: int
    material: Material = field(default_factory=Material)
    skill: Optional[Skill] = None       # None: no shovel
    bound: int = 3
    gravity: float = -9.8
    n_sub: int = 10                     # sub-steps per action
    skill_unrounded: bool = False       # phases 1 and 4 divide by T^float (Sec. III-B)
    particle_contact: bool = False      # particle-level collision of Algorithm 1
    w_emd: float = 0.0                  # weight of the EMD term (Eq. emd) in the loss
    checkpoint_every: int = 0
    target_seed: Optional[int] = None
    # Shovel and contact (the paper gives an SDF with Coulomb friction; sizes
    # are the 0.1 x 0.005 x 0.08 m blade, stored as half extents along the
    # blade's width, normal and pointing directions).
    shovel_half: tuple = (0.05, 0.0025, 0.04)
    mu_b: float = 0.5
    # Skill speeds and the fixed lift distance of phase 4.
    v_l: float = 3.0
    v_w: float = 10.0 * math.pi
    d_lift: float = 0.01
    # Loss: height-map window and the scoop-region mass term.
    hm_res: int = 40
    region_depth: float = 0.03
    m_ref: float = 1600.0 * 0.1 * 0.08 * 0.03
    m_target: float = 0.5 * 1600.0 * 0.1 * 0.08 * 0.03
    w_mass: float = 1.0
    w_hm: float = 1.0
    region_sign: int = -1

    @property
    def dx(self) -> float:
        return 1.0 / self.n_grid

    @property
    def n_particles(self) -> int:
        n = self.ppc
        for a in range(self.dim):
            n *= self.bed_hi[a] - self.bed_lo[a]
        return n

    @property
    def bed_top(self) -> float:
        return self.bed_hi[1] * self.dx

    @property
    def skin(self) -> float:
        """Contact skin: one cell, so that a blade thinner than dx is still seen."""
        return self.dx

    @property
    def hm_offset(self) -> float:
        """Height-map stencil offset: the particle spacing dx / ppc^(1/d)."""
        return self.dx / round(self.ppc ** (1.0 / self.dim))

    @property
    def hm_origin(self) -> tuple:
        return HM_ORIGIN if self.dim == 3 else (0.0, 0.0)

    @property
    def hm_size(self) -> float:
        return HM_SIZE if self.dim == 3 else 1.0

    @property
    def params(self) -> np.ndarray:
        """(E, nu, phi_deg, rho, depth, angle_deg, push, displace, push_angle_deg):
        the differentiable inputs."""
        m, s = self.material, self.skill or Skill()
        return np.array([m.E, m.nu, m.phi_deg, m.rho, s.depth, s.angle_deg, s.push, s.displace,
                         s.push_angle_deg], dtype=np.float64)

    @property
    def tip0(self) -> tuple:
        """Initial shovel tip: centre of the bed top (Sec. III-A, initial state),
        moved 0.3 dx along x off the node lattice.  On the lattice, the nodes on the
        insertion line would sit exactly on the mid-plane of a blade thinner than
        a cell, where the side a node is pushed to is decided by rounding."""
        c = [(self.bed_lo[a] + self.bed_hi[a]) * 0.5 * self.dx for a in range(self.dim)]
        c[0] += 0.3 * self.dx
        c[1] = self.bed_top
        return tuple(c)


def column_2d() -> Workload:
    """2D sand column collapse, FP64, 64^2 grid, 0.3 x 0.5 block at 4 ppc."""
    return Workload(name="column2d", dim=2, n_grid=64, dt=1e-4, steps=200, precision="f64",
                    ppc=4, bed_lo=(3, 3), bed_hi=(22, 35), seed=1)


def dig_3d(steps: int = 500, ppc: int = 8, n_grid: int = 64) -> Workload:
    """3D sand bed dig with the kinematic box shovel, FP32, 64^3 grid."""
    s = n_grid // 64
    return Workload(name="dig3d", dim=3, n_grid=n_grid, dt=2e-4, steps=steps, precision="f32",
                    ppc=ppc, bed_lo=(13 * s, 3 * s, 13 * s), bed_hi=(51 * s, 22 * s, 51 * s),
                    seed=2, skill=Skill(), target_seed=3)


def dig_3d_backward() -> Workload:
    """The 3D dig with 1000 steps, loss and gradient, checkpoint every 50 steps."""
    w = dig_3d(steps=1000)
    w.name = "dig3d_bwd"
    w.checkpoint_every = 50
    return w


def dig_3d_large() -> Workload:
    """128^3 grid, bed 77x38x77 cells at 8 ppc, cohesive soil, 2000 steps."""
    return Workload(name="dig3d_large", dim=3, n_grid=128, dt=1e-4, steps=2000, precision="f32",
                    ppc=8, bed_lo=(26, 6, 26), bed_hi=(103, 44, 103), seed=5,
                    material=Material(cohesion=500.0), skill=Skill(), checkpoint_every=100,
                    target_seed=3)


def tiny(dim: int, n_grid: int = 16, ppc: Optional[int] = None, steps: int = 20,
         shovel: bool = False, seed: int = 7) -> Workload:
    """Small cases for brute-force checks: a few cells of particles in a 16^d grid."""
    if dim == 2:
        lo, hi = (5, 3), (9, 7)
        ppc = ppc or 1
    else:
        lo, hi = (6, 3, 6), (10, 5, 8)
        ppc = ppc or 8
    w = Workload(name=f"tiny{dim}d", dim=dim, n_grid=n_grid, dt=2e-4 if dim == 3 else 1e-4,
                 steps=steps, precision="f64", ppc=ppc, bed_lo=lo, bed_hi=hi, seed=seed)
    if shovel:
        w.skill = Skill(depth=0.05, angle_deg=30.0, push=0.15)
        w.target_seed = seed + 100
    return w


# --------------------------------------------------------------------------
# Particle beds
# --------------------------------------------------------------------------

def bed_positions(w: Workload) -> np.ndarray:
    """Stratified jitter: every bed cell is split into ppc^(1/d) sub-cells per axis
    with one uniform point in each.  Returns float64 [N, dim], rounded to float32
    first when the workload runs in FP32 so both sides start from identical values.

    Particle order: cells lexicographic in (x, y[, z]) with the last axis fastest,
    then sub-cells in the same order.
    """
    d = w.dim
    k = round(w.ppc ** (1.0 / d))
    if k ** d != w.ppc:
        raise ValueError("ppc must be a perfect power of the dimension")
    ranges = [np.arange(w.bed_lo[a], w.bed_hi[a]) for a in range(d)]
    cells = np.stack(np.meshgrid(*ranges, indexing="ij"), axis=-1).reshape(-1, d)
    subs = np.stack(np.meshgrid(*([np.arange(k)] * d), indexing="ij"), axis=-1).reshape(-1, d)
    n = cells.shape[0] * subs.shape[0]
    u = uniform01(w.seed, n * d).reshape(cells.shape[0], subs.shape[0], d)
    pos = (cells[:, None, :] + (subs[None, :, :] + u) / k) / w.n_grid
    pos = pos.reshape(n, d)
    if w.precision == "f32":
        pos = pos.astype(np.float32).astype(np.float64)
    return np.ascontiguousarray(pos)


# --------------------------------------------------------------------------
# Loss targets: 40x40 height map over the bed footprint, minus a Gaussian dent
# --------------------------------------------------------------------------

HM_RES = 40
HM_ORIGIN = (0.2, 0.2)      # (x, z) corner of the height-map window
HM_SIZE = 0.6               # window edge [m]


def target_heightmap(w: Workload, seed: Optional[int] = None) -> np.ndarray:
    """Target surface: flat bed top inside the bed footprint (0 outside), minus a
    seeded Gaussian dent (centre within +-0.1 of the bed centre, depth U[0.02, 0.05],
    width U[0.03, 0.06]).  float64 [40, 40], indexed [ix, iz].  In 2D the target
    is a 40-pixel profile over x in [0, 1] with the same construction."""
    s = Stream(w.target_seed if seed is None else (seed if seed else 1))
    if w.dim == 2:
        cx = float(s.uniform(1, -0.1, 0.1)[0])
        depth = float(s.uniform(1, 0.02, 0.05)[0])
        sig = float(s.uniform(1, 0.03, 0.06)[0])
        pix = w.hm_size / w.hm_res
        px = w.hm_origin[0] + (np.arange(w.hm_res) + 0.5) * pix
        b0, b1 = w.bed_lo[0] * w.dx, w.bed_hi[0] * w.dx
        h = w.bed_top - depth * np.exp(-(px - (0.5 * (b0 + b1) + cx)) ** 2 / (2 * sig * sig))
        return np.where((px >= b0) & (px < b1), h, 0.0)
    cx, cz = s.uniform(2, -0.1, 0.1)
    depth = float(s.uniform(1, 0.02, 0.05)[0])
    sig = float(s.uniform(1, 0.03, 0.06)[0])
    dx = w.dx
    bx0, bx1 = w.bed_lo[0] * dx, w.bed_hi[0] * dx
    bz0, bz1 = w.bed_lo[2] * dx, w.bed_hi[2] * dx
    centre_x = 0.5 * (bx0 + bx1) + cx
    centre_z = 0.5 * (bz0 + bz1) + cz
    pix = HM_SIZE / HM_RES
    px = HM_ORIGIN[0] + (np.arange(HM_RES) + 0.5) * pix
    pz = HM_ORIGIN[1] + (np.arange(HM_RES) + 0.5) * pix
    X, Z = np.meshgrid(px, pz, indexing="ij")
    inside = (X >= bx0) & (X < bx1) & (Z >= bz0) & (Z < bz1)
    r2 = (X - centre_x) ** 2 + (Z - centre_z) ** 2
    h = w.bed_top - depth * np.exp(-r2 / (2.0 * sig * sig))
    return np.where(inside, h, 0.0)


# --------------------------------------------------------------------------
# Batched system-identification instances
# --------------------------------------------------------------------------

@dataclass
class Instance:
    workload: Workload
    material: Material


def target_points(w: Workload, seed: Optional[int] = None) -> np.ndarray:
    """Target surface point cloud for the EMD loss (Eq. emd): one point per
    pixel of the target height map, at the pixel centre and the target height
    (build frame, y up).  float64 [hm_res^2, 3], pixel order [ix, iz]."""
    H = target_heightmap(w, seed)
    res = w.hm_res
    pix = w.hm_size / res
    c = (np.arange(res) + 0.5) * pix
    X, Z = np.meshgrid(w.hm_origin[0] + c, w.hm_origin[1] + c, indexing="ij")
    return np.ascontiguousarray(np.stack([X.ravel(), H.reshape(-1), Z.ravel()], axis=1))


def sysid_batch(n_inst: int = 64, seed: int = 4, n_lo: int = 20000, n_hi: int = 200000,
                steps: int = 500) -> List[Workload]:
    """64 independent 64^3 instances with particle counts drawn uniformly in
    [n_lo, n_hi]: the bed keeps 19 cells of height at 8 ppc and gets a square
    footprint of s = round(sqrt(N / 152)) cells, centred, so N = 152 s^2.
    E is log-uniform in [1e4, 1e6] Pa, nu uniform in [0.2, 0.4], friction angle
    uniform in [20, 45] deg, density 1600.  dt is 2e-4 capped by a CFL guard
    0.3 dx / c_p with c_p = sqrt((lambda + 2 mu) / rho)."""
    s = Stream(seed)
    out = []
    n_target = s.uniform(n_inst, n_lo, n_hi)
    logE = s.uniform(n_inst, 4.0, 6.0)
    nus = s.uniform(n_inst, 0.2, 0.4)
    phis = s.uniform(n_inst, 20.0, 45.0)
    for i in range(n_inst):
        side = int(round(math.sqrt(n_target[i] / (19 * 8))))
        side = max(2, min(side, 52))
        lo = (64 - side) // 2
        mat = Material(E=float(10.0 ** logE[i]), nu=float(nus[i]), phi_deg=float(phis[i]), rho=1600.0)
        w = dig_3d(steps=steps)
        w = replace(w, name=f"sysid{i}", bed_lo=(lo, 3, lo), bed_hi=(lo + side, 22, lo + side),
                    seed=seed * 1000 + i + 1, material=mat, checkpoint_every=50,
                    target_seed=seed * 1000 + 500 + i)
        w.dt = cfl_dt(w)
        out.append(w)
    return out


def cfl_dt(w: Workload, dt_max: float = 2e-4, cfl: float = 0.3) -> float:
    """Time step cap from the P-wave speed sqrt(M / rho), M = E (1 - nu) /
    ((1 + nu)(1 - 2 nu)) the P-wave modulus: a stability guard on the inputs."""
    m = w.material
    cp = math.sqrt(m.E * (1.0 - m.nu) / ((1.0 + m.nu) * (1.0 - 2.0 * m.nu) * m.rho))
    return min(dt_max, cfl * w.dx / cp)
