"""The batched ensemble and the served stream at their stated sizes.

Ensemble: all 512 lattices (sides 128..2048, fill 0.1..0.4, own seeds, torus)
advanced 500 steps by one graph-replayed batch at the tiling the benchmark
runs; every member's digest must equal the oracle's (stored by
tests/golden/make_golden.py ensemble-512, which calls only the oracle).

Serving: the first requests of the benchmark's Poisson stream (channel flow,
sides 256..8192, 100..10^4 steps) served with continuous batching; a seeded
sample of 32 jobs must give the same 16 x 16 block sums as the job run alone,
and the cheap ones the oracle's block sums.  Tolerance 0 throughout.
"""
import os

import numpy as np
import pytest

import oracle
from paper_1208_2428_amd import Batch, Sim
from paper_1208_2428_amd import ensemble
from paper_1208_2428_amd import serve
from paper_1208_2428_amd import workloads as WL

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
THREADS = oracle.default_threads()


def say(*a):
    print(*a, flush=True)


def golden_ensemble():
    path = os.path.join(HERE, "golden", "digests_ensemble-512.txt")
    if not os.path.exists(path):
        pytest.skip("oracle digests of the ensemble not written yet "
                    "(python tests/golden/make_golden.py ensemble-512)")
    out = {}
    with open(path) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                f = line.split()
                out[int(f[0])] = (int(f[1]), int(f[2]), int(f[3]), int(f[4], 16))
    return out


@pytest.mark.parametrize("tiling", [
    dict(depth=5, band=32, group_threads=64, passes_per_launch=1),   # the benchmark's tiling
    dict(depth=4, band=16, group_threads=256, passes_per_launch=1),
])
def test_ensemble_full_size_matches_oracle(tiling):
    say("ensemble 512 x 500 steps", tiling)
    gold = golden_ensemble()
    params = ensemble.ensemble_params()
    assert len(gold) == len(params) == 512
    for i, p in enumerate(params):  # the stored file describes these very members
        assert gold[i][:3] == (p["width"], p["height"], p["seed"]), i
    b = Batch(params, **tiling)
    b.step(500)
    b.sync()
    bad = [i for i in range(len(params)) if b[i].digest() != gold[i][3]]
    assert not bad, f"{len(bad)} members differ from the oracle, first {bad[:8]}"
    assert all(b[i].t == 500 for i in (0, 255, 511))
    b.close()


def test_ensemble_runner_digests_equal_alone_runs():
    """The timed runner's digests (fresh batch, tuned-style tiling) equal
    standalone runs of the same members (a slice, to keep it short)."""
    params = ensemble.ensemble_params()[:48]
    tiling = dict(depth=5, band=32, group_threads=64, passes_per_launch=1)
    res = ensemble.run_batched(params, 60, tiling=tiling, repeats=1)
    one = ensemble.run_one_by_one(params, 60)
    assert res["digests"] == one["digests"]


def test_served_stream_sample_matches_alone_and_oracle():
    reqs = WL.request_stream(n=2000, rate=200.0, seed=5)[:400]
    rng = np.random.default_rng(11)
    sample = set(int(i) for i in rng.choice(len(reqs), size=32, replace=False))
    cheap = [i for i, r in enumerate(reqs) if r.side * r.side * r.steps <= 4e8][:6]
    keep = sample | set(cheap)
    say(f"serving {len(reqs)} requests, checking {len(keep)} ({len(cheap)} against the oracle)")
    srv = serve.Server(lattice_bytes=32 << 30, max_slots=512, passes_per_tick=1, depth=5)
    out = srv.run(reqs, realtime=False, keep_results=keep)
    srv.close()
    assert out["completed"] == len(reqs)
    for i in sorted(keep):
        r = reqs[i]
        s = Sim(**serve.job_params(r))
        s.step(r.steps)
        np.testing.assert_array_equal(out["results"][i], s.observe_blocks(16),
                                      err_msg=f"request {i} ({r.side}^2, {r.steps} steps) vs alone")
        s.close()
    assert cheap, "the stream prefix holds no job cheap enough for the oracle"
    for i in cheap:
        r = reqs[i]
        p = serve.job_params(r)
        st = oracle.init(r.side, r.side, r.seed, r.fill, walls=r.walls)
        st, _ = oracle.run(st, 0, r.steps, r.seed, r.force_rate, threads=THREADS)
        assert p["walls"]
        np.testing.assert_array_equal(out["results"][i], oracle.observe_blocks(st, 16),
                                      err_msg=f"request {i} ({r.side}^2, {r.steps} steps) vs oracle")
