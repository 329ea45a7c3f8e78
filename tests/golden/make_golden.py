"""Writes the oracle's reference digests for the full-size workloads.

Calls only the CPU oracle (``oracle/``) and the seeded input generators
(``paper_1208_2428_amd.workloads``).  Output: one text file per workload,
``digests_<name>.txt``, with lines ``t digest mass px py swaps`` where the
digest is the oracle's state digest after t steps and swaps counts the forcing
exchanges applied in steps [0, t).

For the batched ensemble (``ensemble-512``: 512 periodic lattices of uneven
sides, fills and seeds, 500 steps) it writes ``digests_ensemble-512.txt`` with
one line per member, ``i width height seed digest mass px py``, the digest
taken after the full 500 steps; members run concurrently, one thread each,
and the file is resumable from its ``.part``.

Usage: python tests/golden/make_golden.py [--threads N] [name ...]
"""
from __future__ import annotations

import argparse
import concurrent.futures
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


ENSEMBLE = "ensemble-512"
ENSEMBLE_STEPS = 500


def ensemble(threads: int) -> None:
    """Oracle digests of every ensemble member after ENSEMBLE_STEPS steps."""
    members = WL.batch_members(n=512, seed=4)
    path = os.path.join(HERE, f"digests_{ENSEMBLE}.txt")
    tmp = path + ".part"
    done = {}
    if os.path.exists(tmp):
        with open(tmp) as fh:
            for line in fh:
                if line.strip() and not line.startswith("#"):
                    done[int(line.split()[0])] = line
    todo = sorted((i for i in range(len(members)) if i not in done),
                  key=lambda i: -members[i].width * members[i].height)

    def one(i):
        m = members[i]
        st = oracle.init(m.width, m.height, m.seed, m.fill)
        st, _ = oracle.run(st, 0, ENSEMBLE_STEPS, m.seed, 0.0, threads=1)
        g = oracle.observe_global(st)
        return i, (f"{i} {m.width} {m.height} {m.seed} {oracle.digest(st):016x} "
                   f"{g['mass']} {g['px']} {g['py']}\n")

    t0 = time.time()
    with open(tmp, "a") as fh, concurrent.futures.ThreadPoolExecutor(threads) as ex:
        for n, fut in enumerate(concurrent.futures.as_completed([ex.submit(one, i) for i in todo])):
            i, line = fut.result()
            done[i] = line
            fh.write(line)
            fh.flush()
            print(f"{ENSEMBLE} member {i} ({n + 1}/{len(todo)}, {time.time() - t0:.0f}s)",
                  flush=True)
    with open(path + ".tmp", "w") as fh:
        fh.write(f"# oracle digests of the {len(members)}-member batched ensemble "
                 f"(batch_members(n=512, seed=4), torus, no forcing) after {ENSEMBLE_STEPS} steps\n")
        fh.write("# written by: python tests/golden/make_golden.py " + ENSEMBLE + "\n")
        fh.write("# i width height seed digest mass px py\n")
        for i in range(len(members)):
            fh.write(done[i])
    os.replace(path + ".tmp", path)
    os.remove(tmp)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--threads", type=int, default=oracle.default_threads())
    ap.add_argument("names", nargs="*", default=["channel-4096", "porous-16384"])
    args = ap.parse_args()
    for name in args.names:
        if name == ENSEMBLE:
            ensemble(args.threads)
            continue
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
