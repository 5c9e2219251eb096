"""Seeded synthetic inputs: particle beds, hex boxes and tetrahedral meshes.

This module only draws inputs.  It holds none of the coarse-graining
arithmetic (no binning, no deposition, no operator, no solve), so the GPU
path and the CPU oracle can both be fed from it without sharing any of the
method.

The paper's own tests use 1000 quasi-random spheres whose positions are not
published (Section 4); every workload here is a seeded stand-in with the
shapes and value distributions stated in each function.  Positions are
float32 [N, 3] (x, y, z interleaved), per-particle values are float32 [F, N].
Sphere volumes are computed in float64 as pi d^3 / 6 and stored as float32.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

SEED_BASE = 14090100


@dataclasses.dataclass(frozen=True)
class HexBox:
    """Axis-aligned box [lo, hi] split into nx*ny*nz equal hexahedra."""
    lo: tuple
    hi: tuple
    shape: tuple  # (nx, ny, nz), x fastest in memory

    @property
    def n_cells(self) -> int:
        nx, ny, nz = self.shape
        return nx * ny * nz


@dataclasses.dataclass
class Particles:
    pos: np.ndarray      # float32 [N, 3]
    values: np.ndarray   # float32 [F, N]
    diam: np.ndarray | None = None  # float64 [N] (for reference only)


@dataclasses.dataclass
class Workload:
    name: str
    box: HexBox | None
    particles: Particles
    bandwidth: float
    n_steps: int
    rtol: float


def sphere_volume(d: np.ndarray) -> np.ndarray:
    """Volume of a sphere of diameter d, in float64."""
    return math.pi * np.asarray(d, dtype=np.float64) ** 3 / 6.0


def _lognormal_diam(rng, n, median=0.003, sigma=0.3):
    return np.exp(rng.normal(math.log(median), sigma, size=n))


def tiny(seed: int = SEED_BASE + 1) -> Workload:
    """Unit cube, 24^3 hexes, 20,000 uniform spheres of diameter 0.01.

    Bandwidth b = 0.05, 4 backward-Euler pseudo-steps.
    """
    rng = np.random.default_rng(seed)
    n = 20_000
    pos = rng.random((n, 3)).astype(np.float32)
    d = np.full(n, 0.01)
    vals = sphere_volume(d).astype(np.float32)[None, :]
    box = HexBox((0.0, 0.0, 0.0), (1.0, 1.0, 1.0), (24, 24, 24))
    return Workload("tiny-24^3-20k", box, Particles(pos, vals, d), 0.05, 4, 1e-7)


def _clumps(rng, n, n_clumps, sigma, lo, hi):
    """n points in n_clumps isotropic Gaussian clumps; out-of-box draws redrawn."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    centres = lo + (hi - lo) * rng.random((n_clumps, 3))
    which = rng.integers(0, n_clumps, size=n)
    out = centres[which] + sigma * rng.normal(size=(n, 3))
    bad = np.nonzero(((out < lo) | (out > hi)).any(axis=1))[0]
    while bad.size:
        out[bad] = centres[which[bad]] + sigma * rng.normal(size=(bad.size, 3))
        sub = ((out[bad] < lo) | (out[bad] > hi)).any(axis=1)
        bad = bad[sub]
    return out


def dense_bed(n_particles: int = 20_000_000, shape=(256, 256, 512), n_fields: int = 1,
              seed: int = SEED_BASE + 2, depth: float = 2.0) -> Workload:
    """Dense particle bed in a 1 x 1 x depth box (depth 2: h = 1/256 at the
    full shape; depth 1 with 256^3 cells and half the particles is the same
    bed in a cube, at the same per-volume density).

    Lognormal diameters (median 0.003, sigma 0.3).  70 % of the spheres are
    uniform in the bottom quarter [0,1]^2 x [0,depth/4]; 30 % sit in 50
    Gaussian clumps (sigma 0.05) with uniform centres.  Field 0 is the sphere
    volume; fields 1..3 (when n_fields = 4) are drag components drawn N(0, 1).
    Bandwidth b = 4 cell widths of the x spacing, 4 pseudo-steps, rtol 1e-6.
    A smaller shape keeps the box and the per-volume particle density when
    n_particles is scaled by the cell-count ratio.
    """
    rng = np.random.default_rng(seed)
    lo, hi = (0.0, 0.0, 0.0), (1.0, 1.0, float(depth))
    n_bed = int(round(0.7 * n_particles))
    n_clump = n_particles - n_bed
    bed = rng.random((n_bed, 3)) * np.array([1.0, 1.0, depth / 4.0])
    cl = _clumps(rng, n_clump, 50, 0.05, lo, hi)
    pos = np.concatenate([bed, cl]).astype(np.float32)
    del bed, cl
    d = _lognormal_diam(rng, n_particles)
    vals = np.empty((n_fields, n_particles), dtype=np.float32)
    vals[0] = sphere_volume(d)
    for f in range(1, n_fields):
        vals[f] = rng.normal(size=n_particles)
    box = HexBox(lo, hi, tuple(shape))
    b = 4.0 * (hi[0] - lo[0]) / shape[0]
    return Workload(f"dense-bed-{shape[0]}x{shape[1]}x{shape[2]}-{n_particles}p-F{n_fields}",
                    box, Particles(pos, vals, d), b, 4, 1e-6)


def uniform_bed(box: HexBox, n_particles: int, n_fields: int, seed: int,
                diam: float | None = None) -> Particles:
    """Uniform positions in the box; volume (+ N(0,1) drag) values."""
    rng = np.random.default_rng(seed)
    lo = np.asarray(box.lo)
    hi = np.asarray(box.hi)
    pos = (lo + (hi - lo) * rng.random((n_particles, 3))).astype(np.float32)
    d = np.full(n_particles, diam) if diam is not None else _lognormal_diam(rng, n_particles)
    vals = np.empty((n_fields, n_particles), dtype=np.float32)
    vals[0] = sphere_volume(d)
    for f in range(1, n_fields):
        vals[f] = rng.normal(size=n_particles)
    return Particles(pos, vals, d)


def batched_snapshot(j: int, shape=(128, 128, 128), n_range=(500_000, 4_000_000),
                     seed: int = SEED_BASE + 4) -> Particles:
    """Snapshot j of the batched workload: unit cube, N_j ~ U{n_range},
    uniform positions, lognormal diameters, 4 fields (volume + 3 N(0,1) drag)."""
    rng = np.random.default_rng(seed * 1000 + j)
    n = int(rng.integers(n_range[0], n_range[1] + 1))
    box = HexBox((0.0, 0.0, 0.0), (1.0, 1.0, 1.0), tuple(shape))
    return uniform_bed(box, n, 4, int(rng.integers(1 << 62)))


# ---------------------------------------------------------------------------
# Tetrahedral meshes: each hex of a lattice split into the 6 Kuhn tetrahedra
# that share its main diagonal, so that neighbouring hexes meet conformingly.
# ---------------------------------------------------------------------------

# The six monotone lattice paths from corner (0,0,0) to (1,1,1).
_KUHN_PERMS = ((0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0))


def kuhn_tet_mesh(n: int = 100, jitter: float = 0.2, seed: int = SEED_BASE + 3,
                  lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0)):
    """Vertices float64 [(n+1)^3, 3] and tets int32 [6 n^3, 4] of a unit-cube
    Kuhn mesh.  Interior vertices move by U(-jitter h, +jitter h) per axis.

    Tet 6*hexid + k is the k-th Kuhn tet of hex hexid = i + n (j + n k),
    vertices ordered so that every tet has positive orientation when unjittered.
    """
    rng = np.random.default_rng(seed)
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    m = n + 1
    g = np.arange(m, dtype=np.float64)
    h = (hi - lo) / n
    zz, yy, xx = np.meshgrid(g, g, g, indexing="ij")
    xyz = np.stack([lo[0] + xx.ravel() * h[0], lo[1] + yy.ravel() * h[1],
                    lo[2] + zz.ravel() * h[2]], axis=1)
    if jitter > 0:
        ii = np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1)
        interior = ((ii > 0) & (ii < n)).all(axis=1)
        shift = rng.uniform(-jitter, jitter, size=(interior.sum(), 3)) * h
        xyz[interior] += shift
    # hex corner (0,0,0) vertex ids
    c = np.arange(n)
    kk, jj, ii = np.meshgrid(c, c, c, indexing="ij")
    base = (ii + m * (jj + m * kk)).ravel()
    step = np.array([1, m, m * m])
    tets = np.empty((n ** 3, 6, 4), dtype=np.int64)
    for t, perm in enumerate(_KUHN_PERMS):
        v0 = base
        v1 = v0 + step[perm[0]]
        v2 = v1 + step[perm[1]]
        v3 = v2 + step[perm[2]]
        # odd permutations have negative orientation: swap two vertices
        parity = sum(1 for a in range(3) for b in range(a + 1, 3) if perm[a] > perm[b]) & 1
        if parity:
            tets[:, t, :] = np.stack([v0, v2, v1, v3], axis=1)
        else:
            tets[:, t, :] = np.stack([v0, v1, v2, v3], axis=1)
    return xyz, tets.reshape(-1, 4).astype(np.int32)


def unstructured(n_hex: int = 100, n_particles: int = 5_000_000, seed: int = SEED_BASE + 3):
    """Unit cube, n_hex^3 hexes x 6 jittered Kuhn tets, uniform spheres d=0.004.

    Bandwidth b = 4 hex spacings, 4 pseudo-steps, CG rtol 1e-6.
    Returns (xyz, tets, Particles, bandwidth, n_steps, rtol).
    """
    xyz, tets = kuhn_tet_mesh(n_hex, 0.2, seed)
    rng = np.random.default_rng(seed + 7)
    pos = rng.random((n_particles, 3)).astype(np.float32)
    d = np.full(n_particles, 0.004)
    vals = sphere_volume(d).astype(np.float32)[None, :]
    return xyz, tets, Particles(pos, vals, d), 4.0 / n_hex, 4, 1e-6


# ---------------------------------------------------------------- advected beds
# Inputs of the learned initial-guess workload: one particle bed carried by a
# steady divergence-free flow, sampled every few time steps.  The flow is an
# input generator only (the coarse graining never sees velocities).

@dataclasses.dataclass(frozen=True)
class FourierFlow:
    """u(x) = sum_m a_m cos(k_m . x + phi_m) with a_m perpendicular to k_m,
    so div u = 0; sum_m |a_m| = 1 bounds max |u|."""
    k: np.ndarray    # float64 [M, 3]
    a: np.ndarray    # float64 [M, 3]
    phi: np.ndarray  # float64 [M]


def fourier_flow(seed: int = SEED_BASE + 5, n_modes: int = 16, max_wavenumber: int = 4) -> FourierFlow:
    """n_modes random modes with |k_m| = 2 pi j_m, j_m uniform in 1..max_wavenumber."""
    rng = np.random.default_rng(seed)
    dirs = rng.normal(size=(n_modes, 3))
    dirs /= np.linalg.norm(dirs, axis=1, keepdims=True)
    j = rng.integers(1, max_wavenumber + 1, size=n_modes)
    k = 2.0 * math.pi * j[:, None] * dirs
    a = rng.normal(size=(n_modes, 3))
    a -= (a * dirs).sum(axis=1, keepdims=True) * dirs
    a /= np.linalg.norm(a, axis=1).sum()
    return FourierFlow(k, a, rng.uniform(0.0, 2.0 * math.pi, size=n_modes))


def bed_in_unit_cube(n_particles: int, seed: int, median_diam: float = 0.003):
    """The dense bed's recipe scaled to the unit cube: 70 % uniform in
    [0,1]^2 x [0,0.25], 30 % in 50 Gaussian clumps (sigma 0.05); lognormal
    diameters.  Returns (pos float64 [N, 3], volumes float32 [1, N])."""
    rng = np.random.default_rng(seed)
    n_bed = int(round(0.7 * n_particles))
    bed = rng.random((n_bed, 3)) * np.array([1.0, 1.0, 0.25])
    cl = _clumps(rng, n_particles - n_bed, 50, 0.05, (0.0, 0.0, 0.0), (1.0, 1.0, 1.0))
    d = _lognormal_diam(rng, n_particles, median=median_diam)
    return np.concatenate([bed, cl]), sphere_volume(d).astype(np.float32)[None, :]


class AdvectedSnapshots:
    """Snapshots j = 0, 1, ... of a bed (bed_in_unit_cube) advected through
    the unit cube by fourier_flow, with forward-Euler sub-steps of length
    dt = 0.5 h / sum|a_m| (no particle moves more than half a cell of the
    grid of `n_cells_x` cells per sub-step), `stride` sub-steps between
    snapshots, and specular reflection at the walls.

    Runs in torch float64 on `device` (CPU or GPU); positions are handed out
    as float32 [N, 3] tensors on that device, volumes as float32 [1, N]."""

    def __init__(self, n_particles: int = 2_000_000, n_cells_x: int = 128, stride: int = 4,
                 seed: int = SEED_BASE + 5, device=None):
        import torch
        self.torch = torch
        self.device = torch.device(device) if device is not None else torch.device("cpu")
        pos, vol = bed_in_unit_cube(n_particles, seed)
        flow = fourier_flow(seed + 1)
        self.pos = torch.from_numpy(pos).to(self.device)
        self.values = torch.from_numpy(vol).to(self.device)
        self.k = torch.from_numpy(flow.k).to(self.device)
        self.a = torch.from_numpy(flow.a).to(self.device)
        self.phi = torch.from_numpy(flow.phi).to(self.device)
        self.dt = 0.5 / n_cells_x / float(np.linalg.norm(flow.a, axis=1).sum())
        self.stride = stride
        self.index = 0

    def velocity(self, x):
        return self.torch.cos(x @ self.k.T + self.phi) @ self.a

    def current(self):
        return self.pos.float().contiguous(), self.values

    def advance(self):
        """Moves to the next snapshot."""
        for _ in range(self.stride):
            self.pos = self.pos + self.dt * self.velocity(self.pos)
            self.pos = self.torch.where(self.pos < 0.0, -self.pos, self.pos)
            self.pos = self.torch.where(self.pos > 1.0, 2.0 - self.pos, self.pos)
        self.index += 1
