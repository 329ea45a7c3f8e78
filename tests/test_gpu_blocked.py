"""GPU vs oracle parity of the temporally blocked step (K steps per HBM pass),
over depths, band heights, ragged lattice sizes and boundary cases.
Bit-exact: one correct result exists."""
import numpy as np
import pytest

import oracle
from paper_1208_2428_amd import Sim
from paper_1208_2428_amd import workloads as WL

pytestmark = pytest.mark.gpu

THREADS = oracle.default_threads()


def say(*a):
    print(*a, flush=True)


def make_state(rng, W, H, case):
    st = WL.random_states(rng, H, W, p=0.3)
    if case in ("mask", "mask+force", "solid-particles"):
        st |= ((rng.random((H, W)) < 0.15).astype(np.uint8) << 7)
    if case == "solid-particles":
        st |= WL.random_states(rng, H, W, p=0.5) & 0x7F
    if "walls" in case:
        st[0] |= 0x80
        st[-1] |= 0x80
    return st


@pytest.mark.parametrize("W,H", [(64, 2), (64, 6), (192, 10), (320, 34), (1024, 70), (4096, 40)])
@pytest.mark.parametrize("K", [2, 3, 4, 5])
@pytest.mark.parametrize("case", ["walls+force", "mask+force", "solid-particles"])
def test_depths_every_pass(W, H, K, case):
    say("blocked", W, H, K, case)
    rng = np.random.default_rng(W + 7 * H + K)
    f = 1.0 / 80 if "force" in case else 0.0
    walls = "walls" in case
    st = make_state(rng, W, H, case)
    s = Sim(W, H, seed=31, force_rate=f, walls=walls, depth=K)
    s.set_state(st, t=5)
    ref = st.copy()
    t = 5
    for n in (K, K, 1, K + 1, 2 * K + 3):
        s.step(n)
        ref, _ = oracle.run(ref, t, n, 31, f, threads=THREADS)
        t += n
        np.testing.assert_array_equal(s.get_state(), ref, err_msg=f"after step to t={t}")
    assert s.t == t


@pytest.mark.parametrize("band", [1, 2, 3, 7, 16, 33, 1000])
@pytest.mark.parametrize("K", [2, 4])
def test_band_heights(band, K):
    W, H = 512, 66
    say("band", band, K)
    rng = np.random.default_rng(band * 10 + K)
    st = make_state(rng, W, H, "solid-particles")
    s = Sim(W, H, seed=2, force_rate=1e-2, depth=K, band=min(band, H))
    s.set_state(st, 0)
    s.step(3 * K)
    ref, _ = oracle.run(st, 0, 3 * K, 2, 1e-2, threads=THREADS)
    np.testing.assert_array_equal(s.get_state(), ref)


@pytest.mark.parametrize("K", [1, 2, 3, 4, 5])
def test_depth_does_not_change_workload_result(K):
    # The channel workload at reduced size, 48 steps: every depth gives the
    # oracle's state.
    wl = WL.CHANNEL
    W, H = 2048, 256
    s = Sim(W, H, seed=wl.seed, fill=wl.fill, force_rate=wl.force_rate, walls=True, depth=K)
    s.step(48)
    ref = oracle.init(W, H, wl.seed, wl.fill, walls=True)
    ref, _ = oracle.run(ref, 0, 48, wl.seed, wl.force_rate, threads=THREADS)
    np.testing.assert_array_equal(s.get_state(), ref)


def test_fixed_points_blocked():
    for v in (0x00, 0x7F):
        s = Sim(256, 20, seed=4, depth=5)
        s.set_state(np.full((20, 256), v, np.uint8), 0)
        s.step(9)
        assert np.all(s.get_state() == v)


def test_state_buffer_above_4gib():
    """A state buffer whose seven planes span more than 4 GiB is addressed with
    one buffer resource per plane instead of one per buffer.  Its blocked
    passes (depths 5 and 2) must equal single steps, which use plain 64-bit
    pointers, on the same 32768 x 149798 channel (7 x 613 MB per buffer)."""
    import torch
    W, H = 32768, 149798
    assert 7 * (H * W // 64) * 8 > 2 ** 32
    got = {}
    for K in (1, 5):
        say("wide buffer", W, H, "depth", K)
        s = Sim(W, H, seed=9, fill=0.3, force_rate=1e-3, walls=True, depth=K)
        m0 = s.observe_global()["mass"]
        s.step(5)
        s.step(7)  # at depth 5: passes of 5 and 2 steps
        g = s.observe_global()
        got[K] = (s.digest(), int(g["mass"]), int(g["px"]), int(g["py"]))
        assert got[K][1] == m0
        s.close()
        del s
        torch.cuda.empty_cache()
    assert got[5] == got[1]


@pytest.mark.parametrize("band", [2, 4, 6, 12, 40])
@pytest.mark.parametrize("K", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("rules", [0, 1, 2])
def test_one_wave_rows(band, K, rules):
    """Rows of 64 words run the one-wave pass (carries between lanes by DPP,
    the periodic wrap from lane 63 to lane 0): every pass equals the oracle,
    for every band height, depth and rule set, with walls, obstacles,
    particles on solid nodes and forcing."""
    W, H = 4096, 40
    say("one-wave", band, K, rules)
    rng = np.random.default_rng(1000 * band + 10 * K + rules)
    st = make_state(rng, W, H, "solid-particles")
    st[0] |= 0x80   # the wall rows, as the state bytes of a lattice with walls hold them
    st[-1] |= 0x80
    f = 1.0 / 70
    s = Sim(W, H, seed=77, force_rate=f, walls=True, depth=K, band=band, rules=rules)
    s.set_state(st, t=3)
    ref, t = st.copy(), 3
    for n in (K, 2 * K + 1, 3):
        s.step(n)
        ref, _ = oracle.run(ref, t, n, 77, f, threads=THREADS, rules=rules)
        t += n
        np.testing.assert_array_equal(s.get_state(), ref, err_msg=f"t={t}")
    assert s.digest() == oracle.digest(ref)
    s.close()


@pytest.mark.parametrize("W,H,band", [(2048, 1002, 6), (4096, 262, 4), (1024, 4098, 8), (512, 130, 2)])
@pytest.mark.parametrize("K", [3, 5])
def test_band_runs_per_xcd(W, H, band, K):
    """Short bands (at most 8 rows) on rows of at most 64 words go to the
    XCDs in contiguous runs instead of launch order.  Band counts that are not
    a multiple of 8 (167, 66, 513, 65 here) and a short last band must still
    cover every row exactly once: every pass equals the oracle."""
    say("xcd runs", W, H, band, K)
    rng = np.random.default_rng(W + H + band + K)
    st = make_state(rng, W, H, "walls+force")
    f = 1.0 / 90
    s = Sim(W, H, seed=13, force_rate=f, walls=True, depth=K, band=band)
    assert s.band == band
    s.set_state(st, t=1)
    ref, t = st.copy(), 1
    for n in (K, 2 * K + 1):
        s.step(n)
        ref, _ = oracle.run(ref, t, n, 13, f, threads=THREADS)
        t += n
        np.testing.assert_array_equal(s.get_state(), ref, err_msg=f"t={t}")
    s.close()


def test_default_depth_and_band():
    """The default band is the largest even height up to 32 rows that gives
    every SIMD two waves (else one); the default depth is 3 on lattices too
    small to give every SIMD two waves, 4 at bands of 8 rows or fewer, else 5."""
    import torch
    simds = 4 * torch.cuda.get_device_properties(0).multi_processor_count

    def expected(W, H):
        waves = -(-W // 4096)

        def largest(need):
            for T in range(32, 1, -2):
                if -(-H // T) * waves >= need:
                    return T
            return 0
        T = largest(2 * simds)
        one = T < 4
        if one:
            T = max(largest(simds), 2)
        return (3 if one else 4 if T <= 8 else 5), min(T, H)

    for W, H in [(4096, 4096), (2048, 2048), (8192, 8192), (8192, 4096), (16384, 16384),
                 (4096, 65536), (256, 256)]:
        s = Sim(W, H, seed=1)
        assert (s.depth, s.band) == expected(W, H), (W, H)
        s.depth = 2
        assert s.depth == 2
        s.depth = 0  # back to the default
        assert s.depth == expected(W, H)[0]
        s.close()


@pytest.mark.parametrize("W,band", [(64, 2), (1024, 4), (4096, 2), (4096, 6), (8192, 2)])
@pytest.mark.parametrize("K", [2, 5])
def test_preloaded_and_streamed_fill(W, band, K):
    """A launch of at most one wave per SIMD loads the rows of its pipeline
    fill at once; with more waves it streams them two rows ahead.  Lattices
    with exactly as many band waves as the device has SIMDs, and with one band
    more, take the two paths; both must equal the oracle after every pass."""
    import torch
    simds = 4 * torch.cuda.get_device_properties(0).multi_processor_count
    waves_per_band = -(-W // 4096)
    bands = simds // waves_per_band
    for nb in (bands, bands + 1):
        H = nb * band
        say("fill", W, H, band, K, "bands", nb)
        rng = np.random.default_rng(W + H + K)
        st = make_state(rng, W, H, "walls+force")
        f = 1.0 / 75
        s = Sim(W, H, seed=5, force_rate=f, walls=True, depth=K, band=band)
        s.set_state(st, t=2)
        ref, t = st.copy(), 2
        for n in (K, K + 1):
            s.step(n)
            ref, _ = oracle.run(ref, t, n, 5, f, threads=THREADS)
            t += n
            np.testing.assert_array_equal(s.get_state(), ref, err_msg=f"H={H} t={t}")
        s.close()


@pytest.mark.parametrize("W", [64, 128, 256, 512, 1024, 2048])
@pytest.mark.parametrize("K", [2, 3, 5])
@pytest.mark.parametrize("rules", [0, 2])
def test_repeated_row_one_wave(W, K, rules):
    """Rows of 1 to 32 words run the one-wave pass with the row repeated
    across the wave's 64 lanes (a whole-wave rotation then brings every lane
    its periodic neighbour; only the first copy stores): every pass equals the
    oracle, with walls, obstacles, particles on solid nodes and forcing."""
    H = 46
    say("repeated row", W, K, rules)
    rng = np.random.default_rng(W + 10 * K + rules)
    st = make_state(rng, W, H, "solid-particles")
    st[0] |= 0x80
    st[-1] |= 0x80
    f = 1.0 / 70
    s = Sim(W, H, seed=19, force_rate=f, walls=True, depth=K, band=6, rules=rules)
    s.set_state(st, t=4)
    ref, t = st.copy(), 4
    for n in (K, 2 * K + 1, 3):
        s.step(n)
        ref, _ = oracle.run(ref, t, n, 19, f, threads=THREADS, rules=rules)
        t += n
        np.testing.assert_array_equal(s.get_state(), ref, err_msg=f"t={t}")
    s.close()


@pytest.mark.parametrize("W", [32768, 32704, 4160, 128 * 64 + 64])
@pytest.mark.parametrize("K", [2, 5])
def test_widest_rows(W, K):
    """The widest rows the blocked pass takes (512 words: eight waves per band
    exchanging carries through LDS), one word short of it (the last lane of the
    workgroup idle), and widths just past a wave (65 and 129 words: most lanes
    of the last wave idle): every pass equals the oracle."""
    H = 14
    say("widest", W, K)
    rng = np.random.default_rng(W + K)
    st = make_state(rng, W, H, "mask+force")
    f = 1.0 / 70
    s = Sim(W, H, seed=23, force_rate=f, depth=K)
    s.set_state(st, t=7)
    ref, t = st.copy(), 7
    for n in (K, 2 * K + 1):
        s.step(n)
        ref, _ = oracle.run(ref, t, n, 23, f, threads=THREADS)
        t += n
        np.testing.assert_array_equal(s.get_state(), ref, err_msg=f"t={t}")
    s.close()
