"""Seeded synthetic inputs shared by the HIP path's tests/bench and the oracle.

This module holds no arithmetic of the method itself: it only draws random
numbers and rasterises solid indicators H (1 = solid, 0 = pore, the indicator
of Section 3, eq. Heaviside).  Both the oracle and the GPU path receive the
same H bytes from here.

Generator: SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom
number generators", OOPSLA 2014), written from its published definition.
Doubles in [0,1) take the top 53 bits.

Rasterisation rule: a voxel (centre at (i+1/2)h) is solid iff its centre lies
inside a disc/sphere under the periodic minimum-image distance; a centre
exactly on the boundary counts as solid.
"""
from __future__ import annotations

import numpy as np

_MASK = (1 << 64) - 1


class SplitMix64:
    """SplitMix64 stream; seed 0 yields 0xe220a8397b1dcdaf first."""

    def __init__(self, seed: int):
        self.state = seed & _MASK

    def next_u64(self) -> int:
        self.state = (self.state + 0x9E3779B97F4A7C15) & _MASK
        z = self.state
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _MASK
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _MASK
        return z ^ (z >> 31)

    def uniform(self) -> float:
        return (self.next_u64() >> 11) * (1.0 / (1 << 53))


def _stamp_ball(H: np.ndarray, centre, radius: float) -> int:
    """Mark voxels whose centre is within `radius` (unit-cell units) of `centre`;
    returns how many voxels became solid.

    H has numpy axis order [z][y][x] (3D) or [y][x] (2D); `centre` is given
    in (x, y[, z]) order.
    """
    shape = H.shape
    nd = len(shape)
    idx_ranges = []
    for c in range(nd):
        ax = nd - 1 - c
        n = shape[ax]
        h = 1.0 / n
        lo = int(np.floor((centre[c] - radius) / h - 0.5)) - 1
        hi = int(np.ceil((centre[c] + radius) / h - 0.5)) + 1
        idx = np.arange(lo, hi + 1)
        if idx.size > n:
            idx = np.arange(n)
        pos = (idx + 0.5) * h
        dist = pos - centre[c]
        dist -= np.round(dist)  # periodic minimum image
        idx_ranges.append((ax, idx % n, dist))
    # build the squared distance on the small box, axis order of H
    by_ax = {ax: (ii, dd) for ax, ii, dd in idx_ranges}
    grids = np.meshgrid(*[by_ax[a][1] for a in range(nd)], indexing="ij")
    d2 = sum(g * g for g in grids)
    inside = d2 <= radius * radius + 1e-15
    sel = np.ix_(*[by_ax[a][0] for a in range(nd)])
    sub = H[sel]
    added = int(np.count_nonzero(inside & (sub == 0)))
    sub[inside] = 1
    H[sel] = sub
    return added


def centred_disc(n: int, radius: float = 0.2) -> np.ndarray:
    """2D cell with one disc of radius `radius` centred at (0.5, 0.5)."""
    H = np.zeros((n, n), dtype=np.uint8)
    _stamp_ball(H, (0.5, 0.5), radius)
    return H


def slab_cell(shape, width_rows: int, axis: int = 1) -> np.ndarray:
    """Solid slab occupying indices [0, width_rows) along component `axis`."""
    H = np.zeros(shape, dtype=np.uint8)
    nd = len(shape)
    ax = nd - 1 - axis
    sl = [slice(None)] * nd
    sl[ax] = slice(0, width_rows)
    H[tuple(sl)] = 1
    return H


def overlapping_spheres(n, radius_vox: float, porosity: float, seed: int,
                        max_spheres: int = 1_000_000) -> np.ndarray:
    """Boolean model of overlapping spheres (discs in 2D).

    `n` is an int (cubic/square cell side, 3D) or a shape tuple.  Centres are
    uniform in the unit cell (x, y, z drawn in that order from SplitMix64).
    Spheres are added one at a time until the pore fraction first drops to or
    below `porosity`.  `radius_vox` is in voxels of the first axis.
    """
    shape = (n, n, n) if isinstance(n, int) else tuple(n)
    nd = len(shape)
    H = np.zeros(shape, dtype=np.uint8)
    rng = SplitMix64(seed)
    r = radius_vox / shape[-1]
    total = H.size
    solid = 0
    for _ in range(max_spheres):
        centre = tuple(rng.uniform() for _ in range(nd))
        solid += _stamp_ball(H, centre, r)
        if 1.0 - solid / total <= porosity:
            break
    return H


def random_field(shape, seed: int, scale: float = 1.0) -> np.ndarray:
    """Seeded uniform field in [-scale, scale) (float64), for warm starts / probes."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return (rng.random(shape) * 2.0 - 1.0) * scale


def random_mask(shape, seed: int, solid_fraction: float) -> np.ndarray:
    """Seeded i.i.d. voxel mask (uint8) for tiny brute-force cells."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return (rng.random(shape) < solid_fraction).astype(np.uint8)
