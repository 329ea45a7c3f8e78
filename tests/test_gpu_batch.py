"""Batches on the GPU: every member of a batch must equal its own oracle run
(and hence its standalone GPU run), bit for bit, for every tiling, with and
without graph replay and with several passes per launch."""
import numpy as np
import pytest

import oracle
from paper_1208_2428_amd import Batch, Sim
from paper_1208_2428_amd import workloads as WL

pytestmark = pytest.mark.gpu

THREADS = oracle.default_threads()


def say(*a):
    print(*a, flush=True)


def mixed_params():
    mask = WL.porous_mask(192, 64, seed=9, rmin=3, rmax=6, frac=0.08)
    return [
        dict(width=64, height=8, seed=1, fill=0.3),
        dict(width=128, height=128, seed=2, fill=0.25, force_rate=1e-2, walls=True),
        dict(width=192, height=64, seed=3, fill=0.4, solid=mask),
        dict(width=128, height=34, seed=4, fill=0.2, chirality=1),
        dict(width=320, height=96, seed=5, fill=0.35, force_rate=5e-3),
        dict(width=64, height=64, seed=6, fill=0.1),
        dict(width=128, height=128, seed=7, fill=0.3),
        dict(width=1024, height=40, seed=8, fill=0.3, walls=True),
        dict(width=64, height=10, seed=9, fill=0.5, chirality=2),
    ]


def oracle_state(kw, steps):
    st = oracle.init(kw["width"], kw["height"], kw["seed"], kw["fill"], mask=kw.get("solid"),
                     walls=kw.get("walls", False))
    out, _ = oracle.run(st, 0, steps, kw["seed"], kw.get("force_rate", 0.0),
                        chir_mode=kw.get("chirality", 0), threads=THREADS)
    return out


@pytest.mark.parametrize("depth,ppl,threads,graph", [
    (1, 1, 0, True), (2, 1, 0, True), (3, 1, 128, False), (4, 1, 0, True),
    (2, 0, 0, True), (3, 0, 256, True), (4, 0, 64, False), (3, 2, 0, True),
    (5, 1, 0, True), (5, 0, 128, True), (5, 2, 64, False)])
def test_mixed_batch_matches_oracle(depth, ppl, threads, graph):
    say("batch", depth, ppl, threads, graph)
    params = mixed_params()
    b = Batch(params, depth=depth, passes_per_launch=ppl, group_threads=threads, graph=graph)
    steps = 0
    for n in (12, 5, 7):
        b.step(n)
        steps += n
        b.sync()
        for i, kw in enumerate(params):
            np.testing.assert_array_equal(b[i].get_state(), oracle_state(kw, steps),
                                          err_msg=f"member {i} after {steps} steps")
            assert b[i].t == steps


def test_graph_replays_with_eager_work_between():
    params = mixed_params()[:6]
    b = Batch(params, depth=3, passes_per_launch=0, graph=True)
    side = Sim(256, 16, seed=5, fill=0.3)
    steps = 0
    for k in range(4):
        b.step(9)  # same (K, passes) every call: the captured graph is replayed
        steps += 9
        side.step(3)  # unrelated eager work on another stream
        b.sync()
        for i, kw in enumerate(params):
            assert b[i].digest() == oracle.digest(oracle_state(kw, steps)), (k, i)
    ref, _ = oracle.run(oracle.init(256, 16, 5, 0.3), 0, 12, 5)
    np.testing.assert_array_equal(side.get_state(), ref)


def test_member_views_set_state_and_single_steps():
    params = mixed_params()[:5]
    b = Batch(params, depth=2)
    rng = np.random.default_rng(3)
    W, H = params[2]["width"], params[2]["height"]
    st = WL.random_states(rng, H, W, p=0.3, solid_frac=0.1)
    b[2].set_state(st, t=11)
    b[0].step(3)  # one member alone
    b.step(8)
    b.sync()
    ref2, _ = oracle.run(st, 11, 8, params[2]["seed"], params[2].get("force_rate", 0.0))
    np.testing.assert_array_equal(b[2].get_state(), ref2)
    assert b[2].t == 19 and b[0].t == 11
    np.testing.assert_array_equal(b[0].get_state(), oracle_state(params[0], 11))
    np.testing.assert_array_equal(b[1].get_state(), oracle_state(params[1], 8))


def test_ensemble_sample_matches_oracle():
    # A slice of the 512-lattice ensemble (sides 128..2048, fill 0.1..0.4).
    members = WL.batch_members(n=512, seed=4)[:24]
    params = [dict(width=m.width, height=m.height, seed=m.seed, fill=m.fill) for m in members]
    b = Batch(params, depth=4, passes_per_launch=0)
    b.step(10)
    b.sync()
    for i, kw in enumerate(params):
        assert b[i].digest() == oracle.digest(oracle_state(kw, 10)), i


@pytest.mark.parametrize("depth,band", [(2, 0), (5, 8)])
def test_batch_with_widest_member(depth, band):
    """A member of the widest rows a batch takes (512 words: the workgroup is
    raised to 512 threads, eight waves per band) beside narrow ones: every
    member equals its oracle run."""
    params = [
        dict(width=32768, height=8, seed=31, fill=0.3, force_rate=1e-2, walls=True),
        dict(width=4160, height=10, seed=32, fill=0.25),
        dict(width=128, height=12, seed=33, fill=0.4, force_rate=5e-3),
    ]
    say("widest member", depth, band)
    b = Batch(params, depth=depth, band=band)
    steps = 0
    for n in (depth, 2 * depth + 1):
        b.step(n)
        steps += n
        b.sync()
        for i, kw in enumerate(params):
            np.testing.assert_array_equal(b[i].get_state(), oracle_state(kw, steps),
                                          err_msg=f"member {i} after {steps} steps")
    b.close()
