"""Pins of the oracle's time step (CPU only): streaming brute-forced from the
lattice geometry, closed forms, global invariants, inverse dynamics, forcing
statistics and symmetries.

Model: arXiv:1208.2428, Sec. 2 -- motion then scattering, boundary nodes
reflect through the collision table, reflecting walls top and bottom with
periodic x, and a horizontal force realised by swapping bits 2 and 5.
"""
import math

import numpy as np
import pytest

import oracle
from tests.geometry import hash_np, node_at, position, velocity

M64 = (1 << 64) - 1
PX = np.array([-1, 1, 2, 1, -1, -2, 0])
PY = np.array([-1, -1, 0, 1, 1, 0, 0])


def bits(state):
    return np.stack([(state >> c) & 1 for c in range(8)]).astype(np.int64)


def totals(state):
    b = bits(state)[:7].reshape(7, -1).sum(axis=1)
    return int(b.sum()), int((b * PX).sum()), int((b * PY).sum())


def random_state(rng, H, W, p=0.3, solid=None):
    s = np.zeros((H, W), dtype=np.uint8)
    for c in range(7):
        s |= (rng.random((H, W)) < p).astype(np.uint8) << c
    if solid is not None:
        s |= solid.astype(np.uint8) << 7
    return s


# --------------------------------------------------------------- streaming
@pytest.mark.parametrize("W,H", [(2, 2), (4, 2), (6, 2), (2, 4), (4, 4), (6, 4)])
def test_single_particle_moves_to_geometric_neighbour(W, H):
    for y in range(H):
        for x in range(W):
            for i in range(6):
                s = np.zeros((H, W), dtype=np.uint8)
                s[y, x] = 1 << i
                out, swaps = oracle.step(s, t=5, seed=11)
                assert swaps == 0
                px, py = position(x, y)
                cx, cy = velocity(i)
                dest = node_at(px + cx, py + cy, W, H)
                assert dest is not None
                dx, dy = dest
                expect = np.zeros_like(s)
                expect[dy, dx] = 1 << i
                np.testing.assert_array_equal(out, expect, err_msg=f"{W}x{H} ({x},{y}) c{i}")
            # the rest particle stays
            s = np.zeros((H, W), dtype=np.uint8)
            s[y, x] = 0x40
            out, _ = oracle.step(s, t=0, seed=1)
            np.testing.assert_array_equal(out, s)


def test_east_particle_returns_after_W_steps():
    W, H = 12, 4
    s = np.zeros((H, W), dtype=np.uint8)
    s[1, 3] = 1 << 2
    for k in range(1, W + 1):
        s, _ = oracle.step(s, t=k, seed=3)
        assert s[1, (3 + k) % W] == 1 << 2
    assert s[1, 3] == 1 << 2


def test_northeast_particle_advances_half_H_per_H_steps():
    W, H = 10, 6
    s = np.zeros((H, W), dtype=np.uint8)
    s[2, 4] = 1 << 3
    out, _ = oracle.run(s, 0, H, seed=9)
    expect = np.zeros_like(s)
    expect[2, (4 + H // 2) % W] = 1 << 3
    np.testing.assert_array_equal(out, expect)


@pytest.mark.parametrize("channel,row", [(0, 1), (1, 1), (3, 4), (4, 4)])
def test_wall_reverses_particle_in_two_steps(channel, row):
    # A particle next to a wall row enters it, bounces back (c_i -> c_{i+3})
    # and is back on its starting node two steps later, reversed.
    W, H = 8, 6
    s = oracle.init(W, H, seed=0, fill=0.0, walls=True)
    s[row, 5] |= 1 << channel
    out, _ = oracle.run(s, 0, 2, seed=4)
    expect = oracle.init(W, H, seed=0, fill=0.0, walls=True)
    expect[row, 5] |= 1 << ((channel + 3) % 6)
    np.testing.assert_array_equal(out, expect)


def test_empty_and_full_are_fixed_points():
    for v in (0, 127):
        s = np.full((8, 64), v, dtype=np.uint8)
        out, _ = oracle.run(s, 0, 5, seed=2)
        np.testing.assert_array_equal(out, s)


# -------------------------------------------------------------- invariants
def test_mass_and_momentum_conserved_on_torus():
    rng = np.random.default_rng(1)
    s = random_state(rng, 16, 128)
    m0 = totals(s)
    for t in range(30):
        s, _ = oracle.step(s, t, seed=21)
        assert totals(s) == m0


def test_forcing_adds_four_px_per_swap():
    rng = np.random.default_rng(2)
    s = random_state(rng, 32, 256, p=0.25)
    m, px, py = totals(s)
    total_swaps = 0
    for t in range(40):
        s, sw = oracle.step(s, t, seed=5, force_rate=1.0 / 128)
        total_swaps += sw
        m2, px2, py2 = totals(s)
        assert m2 == m and py2 == py and px2 == px + 4 * sw
        px = px2
    assert total_swaps > 0


def test_mass_conserved_with_walls_and_obstacles():
    rng = np.random.default_rng(3)
    W, H = 128, 20
    mask = rng.random((H, W)) < 0.1
    s = oracle.init(W, H, seed=7, fill=0.3, mask=mask.astype(np.uint8), walls=True)
    m0 = totals(s)[0]
    for t in range(30):
        s, _ = oracle.step(s, t, seed=7, force_rate=1e-3)
        assert totals(s)[0] == m0
        assert np.array_equal(s >> 7, (mask | np.isin(np.arange(H), [0, H - 1])[:, None]))


# ---------------------------------------------------------- inverse dynamics
def inverse_step(state, t, seed, rules=oracle.RULES_FHP2):
    """Undoes one forcing-free step: invert the per-node map (table permutation
    for fluid nodes with this node's chirality, bounce-back for solid ones),
    then push every particle back along -c_i."""
    H, W = state.shape
    key_chir = oracle.hash64(seed, oracle.TAG_CHIR)
    ys, xs = np.mgrid[0:H, 0:W]
    h = hash_np(np.uint64(key_chir),
                (np.uint64(t) << np.uint64(40)) + (ys.astype(np.uint64) << np.uint64(20))
                + (xs // 64).astype(np.uint64))
    chi = ((h >> (xs % 64).astype(np.uint64)) & np.uint64(1)).astype(np.int64)
    inv = [np.argsort(oracle.rule_table(rules, c)) for c in (0, 1)]
    solid = state >> 7
    low = state & 0x7F
    pre = np.where(chi == 1, inv[1][low], inv[0][low]).astype(np.uint8)
    # bounce-back is its own inverse
    bb = low & 0x40
    for i in range(6):
        bb |= ((low >> ((i + 3) % 6)) & 1) << i
    pre = np.where(solid == 1, bb, pre).astype(np.uint8)
    # un-stream: particle c_i at node r came from r - c_i; push it back there
    out = (pre & 0x40) | (solid << 7).astype(np.uint8)
    for y in range(H):
        for x in range(W):
            px, py = position(x, y)
            for i in range(6):
                if (pre[y, x] >> i) & 1:
                    cx, cy = velocity(i)
                    sx, sy = node_at(px - cx, py - cy, W, H)
                    out[sy, sx] |= 1 << i
    return out.astype(np.uint8)


@pytest.mark.parametrize("rules", [oracle.RULES_FHP2, oracle.RULES_FHP1, oracle.RULES_FHP3])
def test_inverse_dynamics_recovers_initial_state(rules):
    rng = np.random.default_rng(4)
    W, H = 64, 8
    solid = rng.random((H, W)) < 0.15
    s0 = random_state(rng, H, W, p=0.35, solid=solid)
    s = s0.copy()
    n = 6
    for t in range(n):
        s, _ = oracle.step(s, t, seed=13, rules=rules)
    for t in reversed(range(n)):
        s = inverse_step(s, t, 13, rules)
    np.testing.assert_array_equal(s, s0)


# ------------------------------------------------------------------ forcing
def test_forcing_coin_rate_and_one_per_word():
    # Every node holds only a W-mover: it streams, does not scatter, and is
    # flipped to E exactly when the node's coin is up.
    W, H = 1024, 256
    f = 1.0 / 256
    s = np.full((H, W), 0x20, dtype=np.uint8)
    out, swaps = oracle.step(s, t=3, seed=17, force_rate=f)
    flipped = out == 0x04
    assert int(flipped.sum()) == swaps
    assert np.all((out == 0x04) | (out == 0x20))
    per_word = flipped.reshape(H, W // 64, 64).sum(axis=2)
    assert per_word.max() <= 1
    p = math.floor(f * 2**38) / 2**38
    mean, sd = W * H * p, math.sqrt(W * H * p * (1 - p))
    assert abs(swaps - mean) < 5 * sd


def test_forcing_flips_west_to_east_at_coin_node():
    # Find a coin with the test's own SplitMix64 and check the paper's pattern
    # (..1..0..) -> (..0..1..) on bits 5 and 2 (Sec. 2, last paragraph).
    seed, t, y, W, H = 23, 7, 3, 128, 6
    f = 1.0 / 100
    key_force = oracle.hash64(seed, oracle.TAG_FORCE)
    thr = math.floor(f * 2**38)
    # search t until row y has a coin and no other row does (keeps the check exact)
    tt = t
    while True:
        row_coins = {}
        for ty in range(H):
            for w in range(W // 64):
                h = int(hash_np(np.uint64(key_force), np.uint64((tt << 40) + (ty << 20) + w)))
                if (h & 0xFFFFFFFF) < thr:
                    row_coins.setdefault(ty, []).append(64 * w + (h >> 58))
        if len(row_coins) == 1:
            break
        tt += 1
    (cy, xs), = row_coins.items()
    cx = xs[0]
    s = np.zeros((H, W), dtype=np.uint8)
    s[cy, (cx + 1) % W] = 0x20  # arrives at (cx, cy) moving W
    out, swaps = oracle.step(s, tt, seed, force_rate=f)
    assert swaps == 1
    assert out[cy, cx] == 0x04
    # an E-mover already there blocks the swap; a third (SW) particle keeps the
    # E-W pair from scattering head on
    s[cy, (cx - 1) % W] = 0x04
    px, py = position(cx, cy)
    vx, vy = velocity(0)
    sx, sy = node_at(px - vx, py - vy, W, H)
    s[sy, sx] |= 0x01
    out, swaps = oracle.step(s, tt, seed, force_rate=f)
    assert swaps == 0 and out[cy, cx] == 0x25


# --------------------------------------------------------------- symmetries
def test_walls_equal_explicit_mask():
    W, H = 128, 12
    mask = np.zeros((H, W), dtype=np.uint8)
    mask[0] = mask[-1] = 1
    a = oracle.init(W, H, seed=31, fill=0.3, walls=True)
    b = oracle.init(W, H, seed=31, fill=0.3, mask=mask)
    np.testing.assert_array_equal(a, b)


def test_translation_invariance_with_fixed_chirality():
    rng = np.random.default_rng(5)
    W, H = 64, 10
    s = random_state(rng, H, W, p=0.4, solid=rng.random((H, W)) < 0.1)
    for dx, dy in [(1, 0), (7, 0), (0, 2), (5, 4)]:
        a, _ = oracle.run(s, 0, 4, seed=1, chir_mode=oracle.CHIR_ZERO)
        shifted = np.roll(np.roll(s, dx, axis=1), dy, axis=0)
        b, _ = oracle.run(shifted, 0, 4, seed=1, chir_mode=oracle.CHIR_ZERO)
        np.testing.assert_array_equal(np.roll(np.roll(a, dx, axis=1), dy, axis=0), b)


def test_threads_do_not_change_result():
    rng = np.random.default_rng(6)
    s = random_state(rng, 40, 192, p=0.3, solid=rng.random((40, 192)) < 0.05)
    a, sa = oracle.run(s, 0, 5, seed=2, force_rate=1e-2, threads=1)
    b, sb = oracle.run(s, 0, 5, seed=2, force_rate=1e-2, threads=4)
    np.testing.assert_array_equal(a, b)
    assert sa == sb


def chirality_field(seed, t, H, W):
    key = oracle.hash64(seed, oracle.TAG_CHIR)
    ys, xs = np.mgrid[0:H, 0:W].astype(np.uint64)
    h = hash_np(np.uint64(key), (np.uint64(t) << np.uint64(40)) + (ys << np.uint64(20))
                + xs // np.uint64(64))
    return ((h >> (xs % np.uint64(64))) & np.uint64(1)).astype(np.uint8)


def test_chirality_field_read_out_by_head_on_pairs():
    # A uniform E+W state streams onto itself, so every fluid node sees the
    # head-on pair {2, 5} and turns it by +60 deg (chi=1 -> {0, 3}) or -60 deg
    # (chi=0 -> {1, 4}): the output is a picture of the chirality field.
    W, H, seed, t = 256, 12, 77, 5
    s = np.full((H, W), 0x24, dtype=np.uint8)
    out, _ = oracle.step(s, t, seed)
    chi = chirality_field(seed, t, H, W)
    np.testing.assert_array_equal(out, np.where(chi == 1, 0x09, 0x12).astype(np.uint8))
    for mode, v in ((oracle.CHIR_ZERO, 0x12), (oracle.CHIR_ONE, 0x09)):
        out, _ = oracle.step(s, t, seed, chir_mode=mode)
        assert np.all(out == v)


def test_forcing_coin_positions_match_definition():
    W, H, seed, t = 512, 64, 19, 11
    f = 1.0 / 100
    s = np.full((H, W), 0x20, dtype=np.uint8)
    out, _ = oracle.step(s, t, seed, force_rate=f)
    key = oracle.hash64(seed, oracle.TAG_FORCE)
    ys, xs = np.mgrid[0:H, 0:W].astype(np.uint64)
    h = hash_np(np.uint64(key), (np.uint64(t) << np.uint64(40)) + (ys << np.uint64(20))
                + xs // np.uint64(64))
    thr = np.uint64(math.floor(f * 2**38))
    coin = ((h & np.uint64(0xFFFFFFFF)) < thr) & ((h >> np.uint64(58)) == xs % np.uint64(64))
    np.testing.assert_array_equal(out == 0x04, coin)
