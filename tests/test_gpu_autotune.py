"""The autotuners time every candidate tiling on the caller's lattices, which
advances them; whatever tiling wins, the lattices must hold the oracle's
state at the time they reached, and the on-disk cache (keyed by the
candidate list actually tried) must hand back the same choice."""
import numpy as np
import pytest

import oracle
from paper_1208_2428_amd import Batch, Sim, autotune

pytestmark = pytest.mark.gpu

THREADS = oracle.default_threads()


def test_tune_sim_keeps_state_exact(tmp_path, monkeypatch):
    monkeypatch.setenv("FHP_TUNE_CACHE", str(tmp_path / "tune.json"))
    W, H, seed, fill, f = 512, 96, 21, 0.3, 1e-2
    s = Sim(W, H, seed=seed, fill=fill, force_rate=f, walls=True)
    cands = [dict(depth=k, band=b) for k in (1, 3, 5) for b in (2, 6, 32)]
    res = autotune.tune_sim(s, candidates=cands, steps=12)
    assert res["tiling"] in cands and len(res["trials"]) == len(cands)
    assert s.depth == res["tiling"]["depth"] and s.band == res["tiling"]["band"]
    t = s.t
    assert t == 2 * 12 * len(cands)
    ref = oracle.init(W, H, seed, fill, walls=True)
    ref, _ = oracle.run(ref, 0, t, seed, f, threads=THREADS)
    np.testing.assert_array_equal(s.get_state(), ref)
    # the same candidate list is answered from the cache, without stepping
    again = autotune.tune_sim(s, candidates=cands, steps=12)
    assert again["tiling"] == res["tiling"] and s.t == t
    # another list is not
    other = [dict(depth=2, band=4)]
    assert autotune.tune_sim(s, candidates=other, steps=12)["tiling"] == other[0]
    assert s.t > t
    s.close()


def test_tune_batch_keeps_state_exact(tmp_path, monkeypatch):
    monkeypatch.setenv("FHP_TUNE_CACHE", str(tmp_path / "tune.json"))
    params = [dict(width=64 * k, height=48 + 16 * k, seed=40 + k, fill=0.25, force_rate=1e-2,
                   walls=bool(k % 2)) for k in (1, 2, 5)]
    b = Batch(params)
    cands = [dict(depth=k, band=bd, group_threads=nt, passes_per_launch=1)
             for k, bd, nt in ((2, 8, 64), (5, 16, 256), (3, 32, 64))]
    res = autotune.tune_batch(b, params, candidates=cands, steps=12)
    assert res["tiling"] in cands and len(res["trials"]) == len(cands)
    b.sync()
    for i, p in enumerate(params):
        t = b[i].t
        ref = oracle.init(p["width"], p["height"], p["seed"], p["fill"], walls=p["walls"])
        ref, _ = oracle.run(ref, 0, t, p["seed"], p["force_rate"], threads=THREADS)
        np.testing.assert_array_equal(b[i].get_state(), ref, err_msg=f"member {i} at t={t}")
    b.close()
