"""Serving loop: continuous batching of FHP simulation jobs on one GPU.

Requests arrive over time (seeded Poisson stream of channel-flow jobs: walls
on rows 0 and H-1, fill 0.25, forcing 1e-3, the paper's flow set-up of Sec. 2
and Sec. 4).  Arrived requests wait in a FIFO queue; the head is admitted into
the pool whenever a slot and arena memory (the HBM budget) are free; every
resident job advances with each tick (one batch-kernel launch per pass over
all resident jobs); a finished job's 16 x 16 block sums of density and
momentum are copied to the host and its memory is freed for the queue.
Latency is measured from a request's arrival to its result on the host, and
split into the wait in the queue (arrival to admission) and the time in the
pool (admission to result); both are reported by job size (node updates).
"""
from __future__ import annotations

import time
from collections import deque

import numpy as np
import torch

from . import workloads as WL
from .pool import Pool


def job_params(r: WL.Request) -> dict:
    return dict(width=r.side, height=r.side, seed=r.seed, fill=r.fill,
                force_rate=r.force_rate, walls=r.walls)


def job_bytes(side: int) -> int:
    """Arena bytes one job of this side takes (two 7-plane buffers + obstacle plane)."""
    words = (side * side // 64 + 31) // 32 * 32
    return 15 * words * 8


class Server:
    def __init__(self, lattice_bytes: int = 32 << 30, max_slots: int = 512,
                 max_bands: int = 1 << 17, passes_per_tick: int = 1, depth: int = 0,
                 group_threads: int = 256, block: int = 16):
        arena = Pool.arena_bytes_for(max_slots, max_bands, lattice_bytes)
        self.pool = Pool(arena, max_slots=max_slots, max_bands=max_bands, depth=depth,
                         group_threads=group_threads)
        self.passes = passes_per_tick
        self.block = block
        self.ticks_ahead = 2  # ticks the host may enqueue before waiting for the GPU

    def run(self, requests: list[WL.Request], realtime: bool = True, keep_results=None,
            log=None) -> dict:
        """Serves `requests` (sorted by arrival time).  realtime=False admits
        every request as soon as there is room, ignoring arrival times.
        keep_results: optional set of request indices whose block sums are
        returned in the result under "results"."""
        pool = self.pool
        start = time.perf_counter()
        pending = deque(enumerate(requests))
        queue: deque = deque()
        inflight: dict[int, tuple[int, WL.Request]] = {}
        collecting: dict[int, np.ndarray] = {}
        in_flight: deque = deque()
        lat, results = [], {}
        admitted_at: dict[int, float] = {}
        waits, services, works = [], [], []
        node_updates = 0
        ticks = max_queue = max_active = 0
        while pending or queue or inflight:
            now = time.perf_counter() - start
            while pending and (not realtime or pending[0][1].arrival <= now):
                queue.append(pending.popleft())
            max_queue = max(max_queue, len(queue))
            while queue:
                idx, r = queue[0]
                slot = pool.admit(r.steps, **job_params(r))
                if slot is None:
                    if not inflight:  # an empty pool has no room for it: it never will
                        raise RuntimeError(
                            f"request {idx} ({r.side} x {r.side}, {job_bytes(r.side)} bytes) "
                            "does not fit the pool even when it is empty")
                    break
                queue.popleft()
                inflight[slot] = (idx, r)
                admitted_at[slot] = time.perf_counter() - start
            max_active = max(max_active, len(inflight))
            if not inflight:
                if pending:
                    time.sleep(max(0.0, min(0.01, pending[0][1].arrival - now)))
                continue
            any_work = len(collecting) < len(inflight)  # some job still has steps to run
            if not any_work:
                time.sleep(0.0002)  # only result copies in flight
            if any_work:
                pool.tick(self.passes)
                ticks += 1
                ev = torch.cuda.Event()
                ev.record(pool.stream)
                in_flight.append(ev)
                while len(in_flight) > self.ticks_ahead:  # bounded run-ahead of the host
                    in_flight.popleft().synchronize()
            # finished jobs: enqueue their results (pinned, asynchronous) ...
            for slot in pool.done():
                collecting[slot] = pool.collect(slot, self.block)
            # ... and hand back the ones whose copy has completed
            for slot in [s for s in collecting if pool.collected(s)]:
                blocks = collecting.pop(slot)
                idx, r = inflight.pop(slot)
                t_done = time.perf_counter() - start
                t_arr = r.arrival if realtime else 0.0
                t_adm = admitted_at.pop(slot)
                lat.append(t_done - t_arr)
                waits.append(max(0.0, t_adm - t_arr))
                services.append(t_done - t_adm)
                works.append(r.side * r.side * r.steps)
                node_updates += r.side * r.side * r.steps
                if keep_results is not None and idx in keep_results:
                    results[idx] = blocks.copy()
                pool.release(slot)
            if log and ticks % 200 == 0:
                log(f"serve: t={time.perf_counter() - start:.1f}s done={len(lat)} "
                    f"resident={len(inflight)} queued={len(queue)}")
        pool.sync()
        wall = time.perf_counter() - start
        lat_ms = np.array(lat) * 1e3
        out = {"requests": len(requests), "completed": len(lat), "seconds": wall,
               "node_updates": node_updates, "value": node_updates / wall,
               "unit": "node-updates/s", "ticks": ticks, "max_queue": max_queue,
               "max_resident": max_active,
               "p50_ms": float(np.percentile(lat_ms, 50)) if len(lat) else None,
               "p99_ms": float(np.percentile(lat_ms, 99)) if len(lat) else None,
               "mean_ms": float(lat_ms.mean()) if len(lat) else None}
        if len(lat):
            out.update(latency_breakdown(np.array(waits), np.array(services), np.array(works)))
        if keep_results is not None:
            out["results"] = results
        return out

    def close(self) -> None:
        self.pool.close()


def latency_breakdown(waits: np.ndarray, services: np.ndarray, works: np.ndarray) -> dict:
    """Where the latency goes: p50/p99 of the queue wait and of the time in
    the pool, overall and for the jobs in each third of the work (node
    updates), and the correlation of latency with work (logarithms)."""
    def pct(a, q):
        return float(np.percentile(a * 1e3, q)) if len(a) else None
    lat = waits + services
    out = {"queue_p50_ms": pct(waits, 50), "queue_p99_ms": pct(waits, 99),
           "pool_p50_ms": pct(services, 50), "pool_p99_ms": pct(services, 99)}
    edges = np.quantile(works, [1 / 3, 2 / 3])
    thirds = []
    for name, sel in (("small", works <= edges[0]),
                      ("medium", (works > edges[0]) & (works <= edges[1])),
                      ("large", works > edges[1])):
        thirds.append({"jobs": name, "count": int(sel.sum()),
                       "work_max": float(works[sel].max()) if sel.any() else None,
                       "latency_p50_ms": pct(lat[sel], 50), "latency_p99_ms": pct(lat[sel], 99),
                       "queue_p50_ms": pct(waits[sel], 50), "pool_p50_ms": pct(services[sel], 50)})
    out["by_work"] = thirds
    if len(lat) > 2:
        out["log_latency_log_work_corr"] = float(np.corrcoef(np.log(works), np.log(lat))[0, 1])
    return out


def offered_load(requests: list[WL.Request]) -> float:
    """Node updates per second the stream asks for."""
    span = requests[-1].arrival - requests[0].arrival if len(requests) > 1 else 1.0
    return sum(r.side * r.side * r.steps for r in requests) / max(span, 1e-9)
