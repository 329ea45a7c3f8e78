"""The batched ensemble workload: 512 independent periodic lattices with
sides uniform over the multiples of 64 in [128, 2048], fill uniform in
[0.1, 0.4], own seeds, 500 steps, advanced by one batch (persistent kernel,
graph replay, tiling from the autotuner)."""
from __future__ import annotations

import torch

from . import autotune
from . import workloads as WL
from .batch import Batch
from .sim import Sim


def ensemble_params(n: int = 512, seed: int = 4) -> list[dict]:
    return [dict(width=m.width, height=m.height, seed=m.seed, fill=m.fill)
            for m in WL.batch_members(n=n, seed=seed)]


def run_batched(params: list[dict], steps: int, tiling: dict | None = None, log=None,
                repeats: int = 3) -> dict:
    """Times `steps` steps of the whole ensemble and returns every member's
    state digest after `steps` steps from its initial state.

    With no tiling given, tunes on a scratch batch first.  The timed batch
    first makes one untimed call of `steps` steps, which captures and
    instantiates its graph; each of the `repeats` timed calls then replays
    that graph (HIP events on the batch's stream; the median is reported).
    A second batch, advanced `steps` steps from the initial state with the
    same tiling, gives the digests."""
    if tiling is None:
        scratch = Batch(params)
        res = autotune.tune_batch(scratch, params)
        tiling = res["tiling"]
        scratch.close()
        del scratch
        if log:
            log(f"ensemble: tuned tiling {tiling}")
    b = Batch(params, **tiling)
    b.step(steps)  # captures the graph of this launch sequence
    b.sync()
    times = []
    for _ in range(max(1, repeats)):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(b.stream)
        b.step(steps)
        e1.record(b.stream)
        e1.synchronize()
        times.append(e0.elapsed_time(e1) / 1e3)
    b.sync()
    b.close()
    del b
    fresh = Batch(params, **tiling)
    fresh.step(steps)
    fresh.sync()
    digests = [fresh[i].digest() for i in range(len(params))]
    fresh.close()
    sec = sorted(times)[len(times) // 2]
    nodes = sum(p["width"] * p["height"] for p in params)
    return {"value": nodes * steps / sec, "unit": "node-updates/s", "seconds": sec,
            "seconds_all": times, "steps": steps, "lattices": len(params), "nodes": nodes,
            "tiling": tiling, "digests": digests}


def run_one_by_one(params: list[dict], steps: int, depth: int = 0) -> dict:
    """The same ensemble as standalone simulations, each stepped with its own
    launches, one after the other on one stream; also returns every member's
    digest after `steps` steps."""
    sims = [Sim(**p, depth=depth) for p in params]
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for s in sims:
        s.step(steps)
    e1.record(stream)
    e1.synchronize()
    sec = e0.elapsed_time(e1) / 1e3
    nodes = sum(p["width"] * p["height"] for p in params)
    digests = [s.digest() for s in sims]
    for s in sims:
        s.close()
    return {"value": nodes * steps / sec, "unit": "node-updates/s", "seconds": sec,
            "digests": digests}


def main(argv=None) -> int:
    """python -m paper_1208_2428_amd.ensemble [--steps N] [--depth K] [--band T]
    [--threads NT]: times the 512-lattice ensemble at a fixed tiling."""
    import argparse
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--depth", type=int, default=5)
    ap.add_argument("--band", type=int, default=32)
    ap.add_argument("--threads", type=int, default=64)
    a = ap.parse_args(argv)
    tiling = dict(depth=a.depth, band=a.band, group_threads=a.threads, passes_per_launch=1)
    r = run_batched(ensemble_params(), a.steps, tiling)
    print(f"ensemble: {r['lattices']} lattices, {r['nodes']} nodes, {a.steps} steps, tiling {tiling}: "
          f"{r['value']:.3e} node-updates/s ({r['seconds'] * 1e3:.1f} ms)", flush=True)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
