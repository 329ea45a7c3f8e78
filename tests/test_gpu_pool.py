"""Pools and the serving loop on the GPU: each job's result is the same alone
(standalone simulation, and the oracle) and in the mix, whatever else is
resident and whenever it was admitted; admission respects the HBM budget.
Tolerance 0: the hash keys on the job's own seed and time."""
import numpy as np
import pytest

import oracle
from paper_1208_2428_amd import Pool, Sim
from paper_1208_2428_amd import serve
from paper_1208_2428_amd import workloads as WL

pytestmark = pytest.mark.gpu

THREADS = oracle.default_threads()


def alone_state(p, steps):
    s = Sim(**p)
    s.step(steps)
    st = s.get_state()
    s.close()
    return st


def oracle_state(p, steps):
    st = oracle.init(p["width"], p["height"], p["seed"], p["fill"], walls=p.get("walls", False))
    st, _ = oracle.run(st, 0, steps, p["seed"], p.get("force_rate", 0.0), threads=THREADS)
    return st


@pytest.mark.parametrize("depth", [4, 5])
def test_jobs_same_alone_and_in_the_mix(depth):
    pool = Pool(Pool.arena_bytes_for(16, 4096, 64 << 20), max_slots=16, max_bands=4096,
                group_threads=128, depth=depth)
    jobs = [
        (dict(width=256, height=256, seed=11, fill=0.25, force_rate=1e-3, walls=True), 37),
        (dict(width=128, height=64, seed=12, fill=0.3), 9),
        (dict(width=512, height=128, seed=13, fill=0.2, force_rate=5e-3, walls=True), 50),
        (dict(width=64, height=8, seed=14, fill=0.5), 3),   # fewer steps than a pass
        (dict(width=320, height=96, seed=15, fill=0.35), 0),  # nothing to do
        (dict(width=1024, height=64, seed=16, fill=0.25, force_rate=1e-3, walls=True), 24),
    ]
    slots = {}
    got = {}
    # admit in two waves, ticking in between: later jobs join a running mix
    for k, (p, n) in enumerate(jobs):
        slot = pool.admit(n, **p)
        assert slot is not None
        slots[slot] = k
        if k == 2:
            pool.tick(2)
            for s in pool.done():
                got[slots[s]] = pool.member(s).get_state()
                pool.release(s)
    while len(got) < len(jobs):
        pool.tick(3)
        for s in pool.done():
            got[slots[s]] = pool.member(s).get_state()
            pool.release(s)
    pool.sync()
    for k, (p, n) in enumerate(jobs):
        np.testing.assert_array_equal(got[k], alone_state(p, n), err_msg=f"job {k} vs alone")
        if p["width"] * p["height"] * max(n, 1) < 3e6:
            np.testing.assert_array_equal(got[k], oracle_state(p, n), err_msg=f"job {k} vs oracle")
    assert pool.usage()["active"] == 0


def test_admission_respects_budget():
    lattice = 3 * serve.job_bytes(512)
    pool = Pool(Pool.arena_bytes_for(8, 1024, lattice), max_slots=8, max_bands=1024)
    p = dict(width=512, height=512, seed=1, fill=0.2)
    slots = [pool.admit(10, **p) for _ in range(3)]
    assert None not in slots
    assert pool.admit(10, **p) is None          # arena full
    u = pool.usage()
    assert u["active"] == 3 and u["bytes_used"] <= lattice
    pool.release(slots[1])
    s = pool.admit(10, **p)
    assert s is not None                         # room again
    small = pool.admit(5, width=64, height=16, seed=2, fill=0.3)
    assert small is None or pool.usage()["bytes_used"] <= lattice


def test_serving_loop_results_match_alone():
    reqs = WL.request_stream(n=24, rate=1e6, seed=7, side_lo=128, side_hi=640, steps_lo=5,
                             steps_hi=60)
    srv = serve.Server(lattice_bytes=256 << 20, max_slots=8, max_bands=8192, passes_per_tick=2,
                       group_threads=64)
    out = srv.run(reqs, realtime=False, keep_results=set(range(len(reqs))))
    assert out["completed"] == len(reqs)
    for i, r in enumerate(reqs):
        s = Sim(**serve.job_params(r))
        s.step(r.steps)
        np.testing.assert_array_equal(out["results"][i], s.observe_blocks(16), err_msg=str(i))
        s.close()
    srv.close()


def test_serving_loop_rejects_a_job_larger_than_the_arena():
    """A request that an empty pool cannot admit is an error, not a wait."""
    srv = serve.Server(lattice_bytes=2 * serve.job_bytes(256), max_slots=4, max_bands=1024,
                       group_threads=64)
    ok = WL.Request(0.0, 256, 10, 1)
    big = WL.Request(0.0, 1024, 10, 2)
    out = srv.run([ok], realtime=False)
    assert out["completed"] == 1
    with pytest.raises(RuntimeError, match="does not fit"):
        srv.run([ok, big], realtime=False)
    srv.close()


def test_asynchronous_collection_matches_result():
    pool = Pool(Pool.arena_bytes_for(4, 1024, 16 << 20), max_slots=4, max_bands=1024)
    p = dict(width=256, height=128, seed=21, fill=0.3, force_rate=1e-3, walls=True)
    slot = pool.admit(18, **p)
    while not (done := pool.done()):
        pool.tick(2)
    assert done == [slot]
    out = pool.collect(slot, 16)
    for _ in range(2_000_000):
        if pool.collected(slot):
            break
    else:
        pytest.fail("the result copy did not complete")
    np.testing.assert_array_equal(out, pool.result(slot, 16))
    ref = oracle_state(p, 18)
    np.testing.assert_array_equal(out, oracle.observe_blocks(ref, 16))
    pool.release(slot)
