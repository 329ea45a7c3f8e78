"""Pins of the oracle's collision table (CPU only).

The paper's rule figure is missing (arXiv:1208.2428, Sec. 2, Fig. 2); the text
fixes only that collisions conserve mass and momentum and that there is a rest
channel (Sec. 2, itemised list).  The FHP-II reading is pinned here against
float geometry, not against the oracle's own bit indices.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
from tests.geometry import mass, moving_momentum, velocity


def rotate_state(state: int, sixths: int) -> int:
    """Rotates every moving particle by sixths*60 degrees, found geometrically."""
    out = state & 0x40
    for i in range(6):
        if (state >> i) & 1:
            cx, cy = velocity(i)
            a = math.radians(60.0 * sixths)
            rx, ry = cx * math.cos(a) - cy * math.sin(a), cx * math.sin(a) + cy * math.cos(a)
            j = [k for k in range(6)
                 if abs(velocity(k)[0] - rx) < 1e-9 and abs(velocity(k)[1] - ry) < 1e-9]
            assert len(j) == 1
            out |= 1 << j[0]
    return out


def expected_fhp2(state: int, chi: int) -> int:
    """FHP-II from its geometric description (no index arithmetic)."""
    rest = (state >> 6) & 1
    moving = [i for i in range(6) if (state >> i) & 1]
    px, py = moving_momentum(state)
    zero_p = abs(px) < 1e-9 and abs(py) < 1e-9
    # R1: exactly two moving particles, head on; rest particle is a spectator.
    if len(moving) == 2 and zero_p:
        return rotate_state(state, +1 if chi else -1)
    # R2: three moving particles at 120 degrees, no rest particle.
    if len(moving) == 3 and zero_p and not rest:
        return rotate_state(state, 1)
    # R3: one moving + rest  <->  two moving particles whose sum is a unit lattice vector.
    if rest and len(moving) == 1:
        i = moving[0]
        cx, cy = velocity(i)
        pair = [k for k in range(6)
                if abs(velocity(k)[0] * cx + velocity(k)[1] * cy - 0.5) < 1e-9]
        assert len(pair) == 2
        return (1 << pair[0]) | (1 << pair[1])
    if not rest and len(moving) == 2 and abs(math.hypot(px, py) - 1.0) < 1e-9:
        j = [k for k in range(6)
             if abs(velocity(k)[0] - px) < 1e-9 and abs(velocity(k)[1] - py) < 1e-9]
        assert len(j) == 1
        return (1 << j[0]) | 0x40
    return state


@pytest.mark.parametrize("chi", [0, 1])
def test_table_matches_geometric_fhp2(chi):
    t = oracle.collision_table(chi)
    for s in range(128):
        assert t[s] == expected_fhp2(s, chi), (chi, s)


@pytest.mark.parametrize("chi", [0, 1])
def test_conserves_mass_and_momentum(chi):
    t = oracle.collision_table(chi)
    for s in range(128):
        o = int(t[s])
        assert mass(o) == mass(s)
        a, b = moving_momentum(s), moving_momentum(o)
        assert abs(a[0] - b[0]) < 1e-9 and abs(a[1] - b[1]) < 1e-9


@pytest.mark.parametrize("chi", [0, 1])
def test_permutation_and_twenty_changes(chi):
    t = oracle.collision_table(chi)
    assert sorted(t.tolist()) == list(range(128))
    assert int(np.sum(t != np.arange(128))) == 20


def test_inverse_is_other_chirality():
    t0, t1 = oracle.collision_table(0), oracle.collision_table(1)
    for s in range(128):
        assert t0[t1[s]] == s and t1[t0[s]] == s


def test_head_on_rotation_sense():
    # chi = 1 turns the E-W pair (channels 2, 5) by +60 deg to NE-SW (3, 0).
    t1 = oracle.collision_table(1)
    t0 = oracle.collision_table(0)
    assert t1[0b100100] == 0b001001
    assert t0[0b100100] == 0b010010


def test_changes_stay_in_mass_momentum_class():
    # Independent check: group the 128 states by (mass, momentum); every change
    # must stay inside its class.
    def cls(s):
        px, py = moving_momentum(s)
        return mass(s), round(px, 6), round(py, 6)
    for chi in (0, 1):
        t = oracle.collision_table(chi)
        for s in range(128):
            assert cls(s) == cls(int(t[s]))


def test_fixed_points_of_full_and_empty():
    for chi in (0, 1):
        t = oracle.collision_table(chi)
        assert t[0] == 0 and t[127] == 127
        for i, r in itertools.product(range(6), (0, 0x40)):
            if r:
                continue
            assert t[1 << i] == 1 << i  # a lone moving particle never scatters
