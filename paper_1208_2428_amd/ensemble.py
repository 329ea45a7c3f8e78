"""The batched ensemble workload: 512 independent periodic lattices with
sides uniform over the multiples of 64 in [128, 2048], fill uniform in
[0.1, 0.4], own seeds, 500 steps, advanced by one batch (persistent kernel,
graph replay, tiling from the autotuner)."""
from __future__ import annotations

import time

import torch

from . import autotune
from . import workloads as WL
from .batch import Batch
from .sim import Sim


def ensemble_params(n: int = 512, seed: int = 4) -> list[dict]:
    return [dict(width=m.width, height=m.height, seed=m.seed, fill=m.fill)
            for m in WL.batch_members(n=n, seed=seed)]


def run_batched(params: list[dict], steps: int, tiling: dict | None = None, log=None) -> dict:
    """Times `steps` steps of the whole ensemble from its initial state.
    With no tiling given, tunes on a scratch batch first."""
    if tiling is None:
        scratch = Batch(params)
        res = autotune.tune_batch(scratch, params)
        tiling = res["tiling"]
        scratch.close()
        del scratch
        if log:
            log(f"ensemble: tuned tiling {tiling}")
    b = Batch(params, **tiling)
    # capture the launch sequence once on a scratch run of the same length
    warm = Batch(params, **tiling)
    warm.step(steps)
    warm.sync()
    warm.close()
    del warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b.step(steps)
    b.sync()
    wall = time.perf_counter() - t0
    nodes = sum(p["width"] * p["height"] for p in params)
    out = {"value": nodes * steps / wall, "unit": "node-updates/s", "seconds": wall,
           "steps": steps, "lattices": len(params), "nodes": nodes, "tiling": tiling}
    b.close()
    return out


def run_one_by_one(params: list[dict], steps: int, depth: int = 0) -> dict:
    """The same ensemble as standalone simulations, each stepped with its own
    launches, one after the other on one stream."""
    sims = [Sim(**p, depth=depth) for p in params]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in sims:
        s.step(steps)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    nodes = sum(p["width"] * p["height"] for p in params)
    for s in sims:
        s.close()
    return {"value": nodes * steps / wall, "unit": "node-updates/s", "seconds": wall}


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
