"""Test-side geometry of the FHP triangular lattice, written from the physical
picture (floating point), independently of the oracle's integer offset tables.

The triangular lattice is stored as a rectangular array with every second row
shifted by half a lattice constant (arXiv:1208.2428, Sec. 2, Fig. 3).  Odd rows
are shifted by +1/2 and velocity c_i points at angle (i - 2) * 60 degrees.
"""
import math

import numpy as np

SQ3_2 = math.sqrt(3.0) / 2.0


def velocity(i: int):
    """Unit vector c_i (i = 0..5)."""
    a = math.radians((i - 2) * 60.0)
    return math.cos(a), math.sin(a)


def position(x: int, y: int):
    return x + 0.5 * (y % 2), y * SQ3_2


def node_at(px: float, py: float, W: int, H: int):
    """The node whose position equals (px, py) modulo the W x H torus
    (period W in x, H*sqrt(3)/2 in y), or None."""
    Ly = H * SQ3_2
    y = round((py % Ly) / SQ3_2) % H
    if abs(((py - y * SQ3_2) / Ly) - round((py - y * SQ3_2) / Ly)) > 1e-9:
        return None
    fx = (px - 0.5 * (y % 2)) % W
    x = round(fx) % W
    if abs(fx - round(fx)) > 1e-9:
        return None
    return x, y


def moving_momentum(state: int):
    """Total momentum of the moving particles of a 7-bit state, float vector."""
    px = py = 0.0
    for i in range(6):
        if (state >> i) & 1:
            cx, cy = velocity(i)
            px += cx
            py += cy
    return px, py


def mass(state: int) -> int:
    return bin(state & 0x7F).count("1")


# ---- numpy SplitMix64, written sequentially-free from the published generator
GAMMA = np.uint64(0x9E3779B97F4A7C15)


def sm64_mix_np(z):
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def hash_np(key, n):
    """H(key, n) = SplitMix64 output n+1 from state key, vectorised in numpy."""
    key = np.asarray(key, dtype=np.uint64)
    n = np.asarray(n, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return sm64_mix_np(key + (n + np.uint64(1)) * GAMMA)
