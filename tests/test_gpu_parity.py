"""GPU vs oracle parity of the k = 1 step, the initial state, the layout
conversions and the observables.  Tolerance: none -- the dynamics is integer
bit logic with exactly one correct result, so every comparison is bit-exact.
"""
import numpy as np
import pytest

import oracle
from paper_1208_2428_amd import CHIR_HASH, CHIR_ONE, CHIR_ZERO, FhpError, Sim
from paper_1208_2428_amd import workloads as WL

pytestmark = pytest.mark.gpu

THREADS = oracle.default_threads()


def say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("W,H,fill,walls,masked", [
    (64, 2, 0.5, False, False), (128, 6, 0.2, True, False), (192, 10, 0.3, False, True),
    (256, 64, 1.0, True, True), (512, 30, 0.0, False, False)])
def test_initial_state(W, H, fill, walls, masked):
    say("init", W, H, fill, walls, masked)
    mask = WL.porous_mask(W, H, seed=W + H, rmin=2, rmax=4, frac=0.1) if masked else None
    s = Sim(W, H, seed=1234 + W, fill=fill, walls=walls, solid=mask)
    ref = oracle.init(W, H, 1234 + W, fill, mask=mask, walls=walls)
    np.testing.assert_array_equal(s.get_state(), ref)


@pytest.mark.parametrize("W,H", [(64, 2), (64, 4), (128, 6), (192, 10), (320, 34)])
@pytest.mark.parametrize("case", ["torus", "walls+force", "mask+force", "solid-particles"])
def test_tiny_lattices_every_step(W, H, case):
    say("tiny", W, H, case)
    rng = np.random.default_rng(W * 1000 + H)
    walls = "walls" in case
    f = 1.0 / 100 if "force" in case else 0.0
    s = Sim(W, H, seed=99, force_rate=f, walls=walls)
    if case == "solid-particles":
        st = WL.random_states(rng, H, W, p=0.4, solid_frac=0.2)
    elif case == "mask+force":
        st = WL.random_states(rng, H, W, p=0.3)
        st |= ((rng.random((H, W)) < 0.15).astype(np.uint8) << 7)
    else:
        st = WL.random_states(rng, H, W, p=0.3)
    if walls:
        st[0] |= 0x80
        st[-1] |= 0x80
    s.set_state(st, t=7)
    ref = st.copy()
    np.testing.assert_array_equal(s.get_state(), ref)
    for k in range(25):
        s.step(1)
        ref, _ = oracle.step(ref, 7 + k, 99, force_rate=f)
        np.testing.assert_array_equal(s.get_state(), ref, err_msg=f"step {k}")
    assert s.t == 7 + 25


def test_small_torus_every_step():
    wl = WL.SMALL_TORUS
    say("small torus", wl)
    s = Sim(**wl.params())
    ref = oracle.init(wl.width, wl.height, wl.seed, wl.fill)
    np.testing.assert_array_equal(s.get_state(), ref)
    for k in range(wl.steps):
        s.step(1)
        ref, _ = oracle.step(ref, k, wl.seed, threads=THREADS)
        got = s.get_state()
        if not np.array_equal(got, ref):
            bad = np.argwhere(got != ref)
            pytest.fail(f"step {k + 1}: {len(bad)} nodes differ, first {bad[:5].tolist()}")
    assert s.t == wl.steps


@pytest.mark.parametrize("mode", [CHIR_ZERO, CHIR_ONE])
def test_fixed_chirality_modes(mode):
    rng = np.random.default_rng(mode)
    W, H = 256, 16
    st = WL.random_states(rng, H, W, p=0.35)
    s = Sim(W, H, seed=5, chirality=mode)
    s.set_state(st, 0)
    s.step(6)
    ref, _ = oracle.run(st, 0, 6, 5, chir_mode=mode)
    np.testing.assert_array_equal(s.get_state(), ref)


@pytest.mark.parametrize("kind", ["empty", "full", "all-solid", "max-force", "full+walls"])
def test_edge_cases(kind):
    W, H = 256, 12
    f = 0.0
    walls = kind == "full+walls"
    if kind == "empty":
        st = np.zeros((H, W), np.uint8)
    elif kind in ("full", "full+walls"):
        st = np.full((H, W), 0x7F, np.uint8)
        if walls:
            st[0] = st[-1] = 0x80
    elif kind == "all-solid":
        st = WL.random_states(np.random.default_rng(3), H, W, p=0.5) | 0x80
    else:
        st = WL.random_states(np.random.default_rng(4), H, W, p=0.3)
        f = np.nextafter(1.0 / 64, 0.0)
    s = Sim(W, H, seed=8, force_rate=f, walls=walls)
    s.set_state(st, 3)
    s.step(10)
    ref, _ = oracle.run(st, 3, 10, 8, force_rate=f)
    np.testing.assert_array_equal(s.get_state(), ref)


def test_observables_match_oracle():
    rng = np.random.default_rng(11)
    W, H = 384, 50
    st = WL.random_states(rng, H, W, p=0.4, solid_frac=0.1)
    s = Sim(W, H, seed=1, walls=True)
    s.set_state(st, 0)
    ref = s.get_state()  # walls rows are solid on both sides now
    st[0] |= 0x80
    st[-1] |= 0x80
    np.testing.assert_array_equal(ref, st)
    g, og = s.observe_global(), oracle.observe_global(st)
    assert g == og
    for b in (1, 2, 4, 16, 32, 64, 128, 192):
        np.testing.assert_array_equal(s.observe_blocks(b), oracle.observe_blocks(st, b), err_msg=str(b))
    assert s.digest() == oracle.digest(st)


@pytest.mark.parametrize("H", [2, 12])
def test_block_sums_of_rows_wider_than_the_stage(H):
    """Short, wide lattices: one row of 1- to 4-node blocks (12 bytes each)
    holds more bytes than the idle buffer that stages host copies, so the
    row goes over in pieces; 8-node blocks take whole rows."""
    rng = np.random.default_rng(12)
    W = 32768
    st = WL.random_states(rng, H, W, p=0.4, solid_frac=0.1)
    s = Sim(W, H, seed=1)
    s.set_state(st, 0)
    for b in (1, 2, 4, 8, 64):
        say(f"block sums W={W} H={H} b={b}")
        np.testing.assert_array_equal(s.observe_blocks(b), oracle.observe_blocks(st, b), err_msg=str(b))


def test_channel_workload_first_steps():
    wl = WL.CHANNEL
    say("channel", wl)
    s = Sim(**wl.params())
    ref = oracle.init(wl.width, wl.height, wl.seed, wl.fill, walls=True)
    assert s.digest() == oracle.digest(ref)
    for k in range(6):
        s.step(1)
        ref, _ = oracle.step(ref, k, wl.seed, wl.force_rate, threads=THREADS)
        assert s.digest() == oracle.digest(ref), k
    np.testing.assert_array_equal(s.get_state(), ref)
    assert s.observe_global() == oracle.observe_global(ref)


def test_time_limit_and_bad_arguments():
    s = Sim(64, 2)
    with pytest.raises(FhpError) as e:
        s.step(1 << 24)
    assert e.value.code == -4
    with pytest.raises(FhpError):
        s.set_state(np.zeros((2, 64), np.uint8), t=1 << 24)
    with pytest.raises(FhpError):
        s.observe_blocks(3)
    with pytest.raises(FhpError):
        s.depth = 99
