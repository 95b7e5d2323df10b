"""Seeded synthetic inputs shared by the GPU library's callers and by the tests.

This module holds no lattice Boltzmann arithmetic: it builds solid masks
(plane channels, square ducts, random sphere packs, periodic cylinder
arrays), seeded uniform random numbers, and the parameter sets of the
benchmark workloads.  Both the GPU path and the oracle consume what it
produces; neither side's arithmetic lives here.

Random numbers come from SplitMix64 (Steele, Lea & Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014), which is counter based: the
k-th output (k = 1, 2, ...) of seed s is mix(s + k * 0x9E3779B97F4A7C15).
"""
from __future__ import annotations

import math

import numpy as np

_GOLDEN = 0x9E3779B97F4A7C15
_M1 = 0xBF58476D1CE4E5B9
_M2 = 0x94D049BB133111EB
_MASK64 = (1 << 64) - 1


def _mix64(z: int) -> int:
    z = ((z ^ (z >> 30)) * _M1) & _MASK64
    z = ((z ^ (z >> 27)) * _M2) & _MASK64
    return z ^ (z >> 31)


class SplitMix64:
    """Sequential SplitMix64 stream."""

    def __init__(self, seed: int):
        self.state = seed & _MASK64

    def next_u64(self) -> int:
        self.state = (self.state + _GOLDEN) & _MASK64
        return _mix64(self.state)

    def uniform(self) -> float:
        """Double in [0, 1) from the top 53 bits."""
        return (self.next_u64() >> 11) * (1.0 / 9007199254740992.0)


def splitmix64_array(seed: int, count: int, offset: int = 0) -> np.ndarray:
    """Outputs offset+1 .. offset+count of SplitMix64(seed), vectorised."""
    k = np.arange(offset + 1, offset + count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & _MASK64) + k * np.uint64(_GOLDEN)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(_M1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(_M2)
        z = z ^ (z >> np.uint64(31))
    return z


def uniform_array(seed: int, count: int, lo: float = 0.0, hi: float = 1.0,
                  offset: int = 0) -> np.ndarray:
    """Seeded doubles uniform in [lo, hi)."""
    z = splitmix64_array(seed, count, offset)
    u = (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    return lo + (hi - lo) * u


# ---------------------------------------------------------------------------
# Geometry.  Masks are uint8 with 1 = solid, flattened with x fastest
# (index x + nx*(y + ny*z)).  Walls of ducts and channels are not voxels: they
# sit half a node beyond the first and last node of every non-periodic axis.
# ---------------------------------------------------------------------------

def open_mask(nx: int, ny: int, nz: int = 1) -> np.ndarray:
    return np.zeros(nx * ny * nz, dtype=np.uint8)


def sphere_pack(dims, radius: float = 8.0, porosity: float = 0.7, seed: int = 1,
                max_trials: int = 50_000_000):
    """Random sequential addition of non-overlapping spheres in a periodic box.

    Centres are drawn uniformly in [0, n_a) on each axis (x, y, z order) from
    SplitMix64(seed); a candidate is rejected when its minimum-image distance
    to an accepted centre is below 2*radius.  A voxel (integer coordinates) is
    solid when its minimum-image squared distance to a centre is <= radius^2.
    Spheres are added until the voxel porosity first drops to <= porosity.
    Returns (mask, centres[k, 3]).
    """
    nx, ny, nz = (int(v) for v in dims)
    n = np.array([nx, ny, nz], dtype=np.float64)
    if 2.0 * radius >= min(nx, ny, nz) / 2.0:
        raise ValueError("box too small for minimum-image voxelisation")
    N = nx * ny * nz
    solid = np.zeros((nz, ny, nx), dtype=bool)
    rng = SplitMix64(seed)
    cell = 2.0 * radius
    ncell = [max(1, int(math.floor(v / cell))) for v in (nx, ny, nz)]
    csz = [v / c for v, c in zip((nx, ny, nz), ncell)]
    cells: dict = {}
    centres = []
    count = 0
    r = int(math.ceil(radius))
    trials = 0
    while 1.0 - count / N > porosity:
        if trials >= max_trials:
            raise RuntimeError("sphere_pack: porosity target not reached")
        trials += 1
        c = np.array([rng.uniform() * nx, rng.uniform() * ny, rng.uniform() * nz])
        ci = [int(c[a] // csz[a]) % ncell[a] for a in range(3)]
        ok = True
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    key = ((ci[0] + dx) % ncell[0], (ci[1] + dy) % ncell[1], (ci[2] + dz) % ncell[2])
                    for o in cells.get(key, ()):
                        d = c - o
                        d -= n * np.round(d / n)
                        if float(d @ d) < (2.0 * radius) ** 2:
                            ok = False
                            break
                    if not ok:
                        break
                if not ok:
                    break
            if not ok:
                break
        if not ok:
            continue
        cells.setdefault(tuple(ci), []).append(c)
        centres.append(c)
        count += _stamp_sphere(solid, c, radius)
    return solid.reshape(-1).astype(np.uint8), np.array(centres)


def _stamp_sphere(solid: np.ndarray, c, radius: float) -> int:
    """Mark the voxels within radius of centre c (periodic, minimum image)
    solid in the (nz, ny, nx) array; return how many were fluid before."""
    nz, ny, nx = solid.shape
    r = int(math.ceil(radius))
    ix = np.arange(int(math.floor(c[0])) - r, int(math.floor(c[0])) + r + 2)
    iy = np.arange(int(math.floor(c[1])) - r, int(math.floor(c[1])) + r + 2)
    iz = np.arange(int(math.floor(c[2])) - r, int(math.floor(c[2])) + r + 2)
    d2 = ((iz[:, None, None] - c[2]) ** 2 + (iy[None, :, None] - c[1]) ** 2
          + (ix[None, None, :] - c[0]) ** 2)
    inside = d2 <= radius * radius
    sub = np.ix_(iz % nz, iy % ny, ix % nx)
    newly = int((inside & ~solid[sub]).sum())
    solid[sub] |= inside
    return newly


def overlapping_spheres(dims, radius: float = 8.0, porosity: float = 0.15, seed: int = 1,
                        max_spheres: int = 10_000_000):
    """Tight porous medium: spheres whose centres are uniform in the periodic
    box (x, y, z order from SplitMix64(seed)) and may overlap (the Boolean
    model), added until the voxel porosity first drops to <= porosity.  Any
    porosity is reachable (non-overlapping packings jam near 0.6 solid); the
    pore space of this model stays connected down to a few percent.
    Returns (mask, centres[k, 3])."""
    nx, ny, nz = (int(v) for v in dims)
    if 2.0 * radius >= min(nx, ny, nz) / 2.0:
        raise ValueError("box too small for minimum-image voxelisation")
    N = nx * ny * nz
    solid = np.zeros((nz, ny, nx), dtype=bool)
    rng = SplitMix64(seed)
    centres = []
    count = 0
    while 1.0 - count / N > porosity:
        if len(centres) >= max_spheres:
            raise RuntimeError("overlapping_spheres: porosity target not reached")
        c = np.array([rng.uniform() * nx, rng.uniform() * ny, rng.uniform() * nz])
        centres.append(c)
        count += _stamp_sphere(solid, c, radius)
    return solid.reshape(-1).astype(np.uint8), np.array(centres)


def cylinder_array_mask(L: int, diameter: float, shift=(0.0, 0.0)) -> np.ndarray:
    """One circular cylinder in a periodic L x L cell (2-D, x fastest): node
    (x, y) is solid when its distance to the cell centre is <= diameter/2."""
    x = np.arange(L)[None, :] + 0.5 - L / 2.0 - shift[0]
    y = np.arange(L)[:, None] + 0.5 - L / 2.0 - shift[1]
    return ((x * x + y * y) <= (diameter / 2.0) ** 2).astype(np.uint8).reshape(-1)


# ---------------------------------------------------------------------------
# Workload parameter sets (lattice units, rho0 = 1).
# ---------------------------------------------------------------------------

C_MAX_SQUARE = 1.178741652  # square-duct coefficient quoted in Sec. 4.3.1


def channel_case(op: str, H: int = 64, nx: int = 4, nu_p: float = 0.1, g: float = 1e-5,
                 Bi: float = 1.0, m: float = 1e4):
    """Plane Bingham channel: nx periodic x H nodes, walls across y,
    Bi = 4 sigma_y / (rho g H)."""
    return dict(lattice="D2Q9", dims=(nx, H, 1), periodic=(1, 0, 1), op=op, nu_p=nu_p,
                sigma_y=Bi * g * H / 4.0, m=m, g=(g, 0.0, 0.0))


def duct_case(op: str, side: int = 128, length: int = 4, nu_p: float = 0.1, g: float = 4e-6,
              Bi: float = 0.0, m: float = 1e4, lattice: str = "D3Q19"):
    """Square duct: side x side cross-section in (x, y), walls on the four
    side faces, `length` periodic nodes along z (the slowest axis), force
    along z; Bi = 4 sigma_y / (rho g side)."""
    return dict(lattice=lattice, dims=(side, side, length), periodic=(0, 0, 1), op=op,
                nu_p=nu_p, sigma_y=Bi * g * side / 4.0, m=m, g=(0.0, 0.0, g))


def porous_case(op: str, n: int = 256, Bi: float = 1.0, nu_p: float = 0.1, g: float = 5e-5,
                m: float = 1e4, radius: float = 8.0, lattice: str = "D3Q27"):
    """Periodic box of random spheres, force along x,
    Bi = 4 sigma_y / (rho g 2R)."""
    return dict(lattice=lattice, dims=(n, n, n), periodic=(1, 1, 1), op=op, nu_p=nu_p,
                sigma_y=Bi * g * 2.0 * radius / 4.0, m=m, g=(g, 0.0, 0.0))


def cylinder_case(op: str, L: int = 80, D: float = 32.0, nu_p: float = 0.08, g: float = 1.25e-6,
                  sigma_y: float = 0.0, m: float = 1e7):
    """Periodic array of circular cylinders (Sec. 4.5): one cylinder of
    diameter D centred in an L x L periodic D2Q9 cell, body force along x.
    Defaults: the creeping-flow cell (D = 0.4 L, nu_p = 0.08, g = 1.25e-6).
    PR's Papanastasiou parameter is not printed for these runs; m = 1e7
    makes m sigma_y / rho large against nu_p for every yield stress used."""
    return dict(lattice="D2Q9", dims=(L, L, 1), periodic=(1, 1, 1), op=op, nu_p=nu_p, sigma_y=sigma_y,
                m=m if op == "PR" else 0.0, g=(g, 0.0, 0.0), mask=cylinder_array_mask(L, D), D=D)


def batch_sweep(count: int = 256, seed: int = 3, smin: int = 32, smax: int = 160,
                length: int = 4, nu_p: float = 0.1, bi_max: float = 10.0):
    """Independent square ducts of uneven section.  For each k: side s_k
    uniform integer in [smin, smax], Bi_k uniform in [0, bi_max), operator
    uniform in {PR m=1e3, PR m=1e4, PR m=1e5, IR}; force chosen so that the
    Newtonian centre-line velocity would be 0.05."""
    rng = SplitMix64(seed)
    cases = []
    for _ in range(count):
        s = smin + int(rng.uniform() * (smax - smin + 1))
        bi = rng.uniform() * bi_max
        kind = int(rng.uniform() * 4)
        g = 0.05 * nu_p * 16.0 / (C_MAX_SQUARE * s * s)
        op, m = ("IR", 0.0) if kind == 3 else ("PR", (1e3, 1e4, 1e5)[kind])
        cases.append(dict(lattice="D3Q19", dims=(s, s, length), periodic=(0, 0, 1), op=op,
                          nu_p=nu_p, sigma_y=bi * g * s / 4.0, m=m, g=(0.0, 0.0, g)))
    return cases
