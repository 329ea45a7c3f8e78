"""Writes the oracle's reference digests for the full-size workloads.

Calls only the CPU oracle (``oracle/``) and the seeded input generators
(``paper_1208_2428_amd.workloads``).  Output: one text file per workload,
``digests_<name>.txt``, with lines ``t digest mass px py swaps`` where the
digest is the oracle's state digest after t steps and swaps counts the forcing
exchanges applied in steps [0, t).

Usage: python tests/golden/make_golden.py [--threads N] [name ...]
"""
from __future__ import annotations

import argparse
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
from paper_1208_2428_amd import workloads as WL  # noqa: E402


def record_times(steps: int) -> list[int]:
    ts = set(range(0, min(steps, 24) + 1))
    ts |= set(range(0, min(steps, 240) + 1, 12))
    ts |= set(range(0, steps + 1, 120))
    ts.add(steps)
    return sorted(ts)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=oracle.default_threads())
    ap.add_argument("names", nargs="*", default=["channel-4096", "porous-16384"])
    args = ap.parse_args()
    for name in args.names:
        wl = WL.WORKLOADS[name]
        mask = wl.mask()
        state = oracle.init(wl.width, wl.height, wl.seed, wl.fill, mask=mask, walls=wl.walls)
        times = record_times(wl.steps)
        path = os.path.join(HERE, f"digests_{name}.txt")
        tmp = path + ".part"
        t0 = time.time()
        swaps = 0
        with open(tmp, "w") as fh:
            fh.write(f"# oracle digests for workload {name}: {wl}\n")
            fh.write("# written by: python tests/golden/make_golden.py " + name + "\n")
            fh.write("# t digest mass px py swaps\n")
            t = 0
            for target in times:
                if target > t:
                    state, sw = oracle.run(state, t, target - t, wl.seed, wl.force_rate,
                                           threads=args.threads)
                    swaps += sw
                    t = target
                g = oracle.observe_global(state)
                fh.write(f"{t} {oracle.digest(state):016x} {g['mass']} {g['px']} {g['py']} {swaps}\n")
                fh.flush()
                print(f"{name} t={t} ({time.time() - t0:.0f}s)", flush=True)
        os.replace(tmp, path)


if __name__ == "__main__":
    main()
