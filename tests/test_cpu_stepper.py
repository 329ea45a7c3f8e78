"""The host bit-plane stepper (libfhpcpu.so, include/fhp_cpu.h) against the
CPU oracle, bit for bit (CPU only): initial states, every step on small and
ragged lattices with walls, obstacles, forcing and particles on solid nodes,
several thread counts, arbitrary start times, digests."""
import numpy as np
import pytest

import oracle
from paper_1208_2428_amd import cpu_sim as C
from paper_1208_2428_amd import workloads as WL


@pytest.fixture(scope="module", autouse=True)
def lib():
    C.build()
    return C.load()


@pytest.mark.parametrize("W,H,walls,f,frac", [
    (64, 2, False, 0.0, 0.0), (64, 4, True, 0.015, 0.0), (128, 6, False, 0.01, 0.1),
    (192, 64, True, 0.005, 0.08), (320, 34, False, 0.0, 0.05), (576, 10, True, 1e-3, 0.0),
    (1024, 40, False, 0.0155, 0.02)])
def test_every_step_matches_oracle(W, H, walls, f, frac):
    mask = WL.porous_mask(W, H, seed=W + H, rmin=1, rmax=3, frac=frac) if frac else None
    seed = 1000 + W + H
    s = C.CpuSim(W, H, seed=seed, fill=0.3, force_rate=f, walls=walls, solid=mask)
    ref = oracle.init(W, H, seed, 0.3, mask=mask, walls=walls)
    np.testing.assert_array_equal(s.get_state(), ref)
    for t in range(12):
        s.step(1, threads=1 + t % 3)
        ref, _ = oracle.step(ref, t, seed, f)
        np.testing.assert_array_equal(s.get_state(), ref, err_msg=f"step {t}")
    assert s.t == 12 and s.digest() == oracle.digest(ref)


@pytest.mark.parametrize("seed", range(6))
def test_random_states_and_start_times(seed):
    rng = np.random.default_rng(seed)
    W = 64 * int(rng.integers(1, 9))
    H = 2 * int(rng.integers(1, 20))
    walls = bool(rng.integers(0, 2))
    f = float(rng.choice([0.0, 1e-3, 0.012]))
    st = WL.random_states(rng, H, W, p=float(rng.uniform(0.05, 0.7)), solid_frac=0.1)
    if walls:
        st[0] |= 0x80
        st[-1] |= 0x80
    t0 = int(rng.integers(0, 1 << 20))
    s = C.CpuSim(W, H, seed=seed, walls=walls, force_rate=f)
    s.set_state(st, t=t0)
    np.testing.assert_array_equal(s.get_state(), st)
    n = int(rng.integers(1, 25))
    s.step(n, threads=int(rng.integers(1, 5)))
    ref, _ = oracle.run(st, t0, n, seed, f)
    np.testing.assert_array_equal(s.get_state(), ref)
    assert s.t == t0 + n


def test_thread_count_does_not_matter():
    mask = WL.porous_mask(512, 64, seed=3, rmin=2, rmax=5, frac=0.06)
    states = []
    for threads in (1, 2, 5):
        s = C.CpuSim(512, 64, seed=9, fill=0.25, force_rate=5e-3, walls=True, solid=mask)
        s.step(15, threads=threads)
        states.append(s.get_state())
    assert all(np.array_equal(states[0], x) for x in states[1:])


def test_torus_workload_digest_matches_oracle_golden():
    """The 256^2 torus workload, 1000 steps, against the stored oracle digest."""
    import os
    wl = WL.WORKLOADS["torus-256"]
    s = C.CpuSim(**wl.params())
    s.step(wl.steps)
    path = os.path.join(os.path.dirname(__file__), "golden", "digests_torus-256.txt")
    gold = {int(l.split()[0]): int(l.split()[1], 16) for l in open(path) if not l.startswith("#")}
    assert s.digest() == gold[wl.steps]


def test_bad_arguments():
    with pytest.raises(RuntimeError, match="multiple of 64"):
        C.CpuSim(100, 4)
    with pytest.raises(RuntimeError, match="H even"):
        C.CpuSim(64, 3)
    with pytest.raises(RuntimeError, match="force rate"):
        C.CpuSim(64, 4, force_rate=1 / 64)
    s = C.CpuSim(64, 4)
    with pytest.raises(RuntimeError, match="2\\^24"):
        s.set_state(np.zeros((4, 64), np.uint8), t=1 << 24)
    s.set_state(np.zeros((4, 64), np.uint8), t=(1 << 24) - 2)
    s.step(1)
    with pytest.raises(RuntimeError, match="2\\^24"):
        s.step(1)
