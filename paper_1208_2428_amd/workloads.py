"""Seeded synthetic inputs for the FHP workloads.

Input generators only: nothing here computes any part of the FHP dynamics.
Both the GPU tests/benchmark and the oracle-side golden scripts draw their
inputs from these functions.

The paper measures on synthetic flows too (arXiv:1208.2428, Sec. 4: lattices
sized to fill the memory, walls top and bottom, periodic in x, forcing); the
named workloads below fix their sizes and parameters.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np


@dataclass(frozen=True)
class Workload:
    name: str
    width: int
    height: int
    steps: int
    seed: int
    fill: float
    force_rate: float = 0.0
    walls: bool = False
    mask_seed: int | None = None   # porous disks when set
    mask_frac: float = 0.05
    rmin: int = 8
    rmax: int = 32

    def mask(self) -> np.ndarray | None:
        if self.mask_seed is None:
            return None
        return porous_mask(self.width, self.height, self.mask_seed, self.rmin, self.rmax,
                           self.mask_frac)

    def params(self) -> dict:
        return dict(width=self.width, height=self.height, seed=self.seed, fill=self.fill,
                    force_rate=self.force_rate, walls=self.walls)


# 256 x 256 periodic box, channels Bernoulli(0.2), no walls or forcing, 1000 steps.
SMALL_TORUS = Workload("torus-256", 256, 256, 1000, seed=1, fill=0.2)
# 4096 x 4096 channel: walls on rows 0 and H-1, fill 0.25, forcing 1e-3, 10000 steps.
CHANNEL = Workload("channel-4096", 4096, 4096, 10000, seed=2, fill=0.25, force_rate=1e-3,
                   walls=True)
# 16384 x 16384 porous medium: disks r in [8, 32] covering >= 5% (mask seed 33),
# periodic box, fill 0.3, forcing 5e-4, 2000 steps.
POROUS = Workload("porous-16384", 16384, 16384, 2000, seed=3, fill=0.3, force_rate=5e-4,
                  mask_seed=33)

WORKLOADS = {w.name: w for w in (SMALL_TORUS, CHANNEL, POROUS)}


def porous_mask(W: int, H: int, seed: int, rmin: int = 8, rmax: int = 32,
                frac: float = 0.05) -> np.ndarray:
    """Non-overlapping solid disks on the W x H periodic triangular lattice.

    Disks are drawn one at a time: centre a uniformly random node, radius a
    uniformly random integer in [rmin, rmax].  A disk is kept if its centre is
    farther than r1 + r2 from every kept centre (periodic distance between the
    nodes' physical positions); drawing stops once the solid fraction reaches
    `frac`.  Node (x, y) sits at (x + (y mod 2)/2, y*sqrt(3)/2), so in units of
    half a lattice constant 4*d^2 = dx^2 + 3*dy^2 with integer dx, dy: the
    whole construction is exact integer arithmetic.  A node is solid when its
    distance to a centre is at most r.  Raises ValueError when 100,000 draws in
    a row are rejected (the fraction lies beyond what such a packing reaches).
    """
    rng = np.random.default_rng(seed)
    solid = np.zeros((H, W), dtype=np.uint8)
    target = math.ceil(frac * W * H)
    count = 0
    cxh = np.zeros(0, dtype=np.int64)   # centre x in half units: 2x + (y mod 2)
    cys = np.zeros(0, dtype=np.int64)
    crs = np.zeros(0, dtype=np.int64)
    rows = np.arange(-rmax, rmax + 1)
    rejected = 0
    while count < target:
        x, y, r = (int(v) for v in (rng.integers(0, W), rng.integers(0, H),
                                    rng.integers(rmin, rmax + 1)))
        xh = 2 * x + (y & 1)
        if cxh.size:
            dx = (xh - cxh + W) % (2 * W) - W
            dy = (y - cys + H // 2) % H - H // 2
            if np.any(dx * dx + 3 * dy * dy <= 4 * (r + crs) ** 2):
                rejected += 1
                if rejected == 100_000:
                    raise ValueError(f"solid fraction {frac} not reached: {count} of {target} "
                                     "nodes solid when the disks stopped fitting")
                continue
        rejected = 0
        cxh = np.append(cxh, xh)
        cys = np.append(cys, y)
        crs = np.append(crs, r)
        ys = (y + rows[np.abs(rows) <= r]) % H
        dy = ys - y
        dy = (dy + H // 2) % H - H // 2
        xs = np.arange(x - r - 1, x + r + 2)
        XH = 2 * xs[None, :] + (ys[:, None] & 1)
        DX = XH - xh
        inside = DX * DX + 3 * (dy[:, None] ** 2) <= 4 * r * r
        yy, xx = np.nonzero(inside)
        sy, sx = ys[yy], xs[xx] % W
        count += int(np.count_nonzero(solid[sy, sx] == 0))
        solid[sy, sx] = 1
    return solid


def random_states(rng: np.random.Generator, H: int, W: int, p: float = 0.3,
                  solid_frac: float = 0.0) -> np.ndarray:
    """Arbitrary byte-per-node states: each channel bit Bernoulli(p), bit 7
    Bernoulli(solid_frac) independently (so solid nodes may hold particles)."""
    s = np.zeros((H, W), dtype=np.uint8)
    for c in range(7):
        s |= (rng.random((H, W)) < p).astype(np.uint8) << c
    if solid_frac > 0:
        s |= (rng.random((H, W)) < solid_frac).astype(np.uint8) << 7
    return s


@dataclass(frozen=True)
class BatchMember:
    width: int
    height: int
    seed: int
    fill: float


def batch_members(n: int = 512, seed: int = 4, lmin: int = 128, lmax: int = 2048,
                  fill_lo: float = 0.1, fill_hi: float = 0.4) -> list[BatchMember]:
    """Independent periodic square lattices: side uniform over the multiples of
    64 in [lmin, lmax], fill uniform in [fill_lo, fill_hi], 63-bit seeds."""
    rng = np.random.default_rng(seed)
    sides = np.arange(lmin, lmax + 1, 64)
    out = []
    for _ in range(n):
        L = int(rng.choice(sides))
        out.append(BatchMember(L, L, int(rng.integers(0, 2**63)), float(rng.uniform(fill_lo, fill_hi))))
    return out


@dataclass(frozen=True)
class Request:
    arrival: float  # seconds since the start of the stream
    side: int
    steps: int
    seed: int
    fill: float = 0.25
    force_rate: float = 1e-3
    walls: bool = True


def request_stream(n: int = 2000, rate: float = 200.0, seed: int = 5, side_lo: int = 256,
                   side_hi: int = 8192, steps_lo: int = 100, steps_hi: int = 10000) -> list[Request]:
    """Poisson arrivals of channel-flow jobs: exponential gaps of mean 1/rate,
    square side uniform in [side_lo, side_hi] rounded to a multiple of 64,
    step count log-uniform in [steps_lo, steps_hi]."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for _ in range(n):
        t += float(rng.exponential(1.0 / rate))
        side = int(round(rng.uniform(side_lo, side_hi) / 64.0)) * 64
        side = max(64, side)
        steps = int(round(math.exp(rng.uniform(math.log(steps_lo), math.log(steps_hi)))))
        out.append(Request(t, side, steps, int(rng.integers(0, 2**63))))
    return out
