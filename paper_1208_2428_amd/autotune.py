"""Autotuner for the blocked kernels: picks the temporal-block depth K, the
band height, the workgroup size and the passes per launch by timed trials on
the GPU, and caches the choice on disk.

Trials run on the caller's lattices (they advance them; callers that need the
initial state create a fresh batch afterwards).  Timing uses HIP events
recorded on the stream the kernels run on.  The cache is a JSON file
(``$FHP_TUNE_CACHE``, default ``~/.cache/paper_1208_2428_amd/tune.json``)
keyed by the GPU name, a signature of the workload (sizes, rule set, forcing,
obstacles, walls), a hash of the candidate list and a hash of the kernel
sources, so that a choice made for other kernels or candidates is never reused.
"""
from __future__ import annotations

import glob
import hashlib
import json
import os
from collections import Counter

import torch

from ._binding import FhpError

DEFAULT_BATCH_CANDIDATES = [
    dict(depth=k, band=b, group_threads=nt, passes_per_launch=ppl)
    for k in (1, 2, 3, 4, 5) for b in (8, 16, 32, 64) for nt in (64, 256) for ppl in (1, 0)
]
# 2- and 6-row bands: the best heights on lattices of 32- and 64-word rows
# too small to give every SIMD two waves (2048^2, 4096^2)
DEFAULT_SIM_CANDIDATES = [dict(depth=k, band=b) for k in (1, 2, 3, 4, 5) for b in (2, 4, 6, 8, 16, 32, 64)]


def cache_path() -> str:
    return os.environ.get("FHP_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "paper_1208_2428_amd",
                                       "tune.json"))


def _load_cache() -> dict:
    try:
        with open(cache_path()) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store_cache(key: str, value: dict) -> None:
    data = _load_cache()
    data[key] = value
    path = cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp%d" % os.getpid()
        with open(tmp, "w") as fh:
            json.dump(data, fh, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass  # a read-only home only loses the cache


def _gpu_name() -> str:
    return torch.cuda.get_device_name(torch.cuda.current_device())


_SOURCES_HASH = None


def sources_hash() -> str:
    """Hash of every kernel source file of the library."""
    global _SOURCES_HASH
    if _SOURCES_HASH is None:
        h = hashlib.sha1()
        csrc = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc")
        for path in sorted(glob.glob(os.path.join(csrc, "*.h")) + glob.glob(os.path.join(csrc, "*.hip"))):
            h.update(os.path.basename(path).encode())
            with open(path, "rb") as fh:
                h.update(fh.read())
        _SOURCES_HASH = h.hexdigest()[:12]
    return _SOURCES_HASH


def _candidates_hash(candidates) -> str:
    return hashlib.sha1(json.dumps(candidates, sort_keys=True).encode()).hexdigest()[:12]


def batch_signature(params: list[dict]) -> str:
    sizes = Counter((p["width"], p["height"]) for p in params)
    flags = (any(p.get("force_rate", 0) > 0 for p in params),
             any(p.get("solid") is not None for p in params),
             any(p.get("walls", False) for p in params),
             sorted({int(p.get("rules", 0)) for p in params}))
    text = json.dumps([sorted(sizes.items()), flags])
    return hashlib.sha1(text.encode()).hexdigest()[:16]


def time_steps(step_fn, stream, steps: int, warmup: int) -> float:
    """Seconds per step of `step_fn(steps)`, timed with events on `stream`
    after `warmup` untimed calls of the same size (so that graphs are
    captured and code is loaded before the timed call)."""
    for _ in range(max(1, warmup)):
        step_fn(steps)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    step_fn(steps)
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / 1e3 / steps


def tune_batch(batch, params: list[dict], candidates=None, steps: int = 24,
               use_cache: bool = True) -> dict:
    """Returns {"tiling": best candidate, "trials": [(candidate, s/step)]} and
    leaves `batch` set to the best tiling."""
    cands = candidates or DEFAULT_BATCH_CANDIDATES
    key = (f"batch:{_gpu_name()}:{batch_signature(params)}:"
           f"{_candidates_hash(cands)}:{sources_hash()}")
    if use_cache:
        hit = _load_cache().get(key)
        if hit:
            batch.set_tiling(**hit["tiling"])
            return hit
    trials = []
    for cand in cands:
        batch.set_tiling(**cand)
        per = cand["depth"] * 3
        n = max(per, (steps // per) * per)
        dt = time_steps(batch.step, batch.stream, n, 1)
        batch.sync()
        trials.append((cand, dt))
    best = min(trials, key=lambda x: x[1])
    result = {"tiling": best[0], "s_per_step": best[1], "trials": trials}
    batch.set_tiling(**best[0])
    if use_cache:
        _store_cache(key, {"tiling": best[0], "s_per_step": best[1]})
    return result


def tune_sim(sim, candidates=None, steps: int = 48, use_cache: bool = True) -> dict:
    """Tunes depth and band of a standalone simulation (advances it)."""
    sig = json.dumps([sim.width, sim.height, sim.rules, sim.force_rate > 0, sim.has_mask, sim.walls])
    cands = candidates or DEFAULT_SIM_CANDIDATES
    key = f"sim:{_gpu_name()}:{sig}:{_candidates_hash(cands)}:{sources_hash()}"
    if use_cache:
        hit = _load_cache().get(key)
        if hit:
            sim.depth = hit["tiling"]["depth"]
            sim.set_band(hit["tiling"]["band"])
            return hit
    stream = torch.cuda.current_stream()
    trials = []
    for cand in cands:
        try:  # a depth this lattice does not take (width above 32768) is skipped
            sim.depth = cand["depth"]
            sim.set_band(min(cand["band"], sim.height))
        except FhpError:
            continue
        n = max(12, (steps // 12) * 12)
        trials.append((cand, time_steps(sim.step, stream, n, 1)))
    best = min(trials, key=lambda x: x[1])
    sim.depth = best[0]["depth"]
    sim.set_band(min(best[0]["band"], sim.height))
    result = {"tiling": best[0], "s_per_step": best[1], "trials": trials}
    if use_cache:
        _store_cache(key, {"tiling": best[0], "s_per_step": best[1]})
    return result
