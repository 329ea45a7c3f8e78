"""Summarises rocprofv3 output for the profiles/ notes.

    python -m paper_1208_2428_amd.profsum trace <kernel_stats.csv>
    python -m paper_1208_2428_amd.profsum pmc <counter_collection.csv> [<kernel substring>]

`trace` prints the per-kernel call count and average duration; `pmc` prints
the average counter value (per dispatch) of every counter, per kernel.
Also used by bench.py to read the HBM traffic recorded under profiles/.
"""
from __future__ import annotations

import csv
import hashlib
import os
import re
import sys
from collections import defaultdict

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
# Sources of the blocked single-lattice kernel, and the extra compiler flags of
# the depth-5 pass: the traffic recorded under profiles/ applies only while
# they are unchanged.
KERNEL_SOURCES = ["csrc/fhp_stepk.h", "csrc/fhp_stepk.hip", "csrc/fhp_stepk_k5.hip",
                  "csrc/fhp_sweep.h", "csrc/fhp_device.h"]


def kernel_source_hash() -> str:
    from . import build
    h = hashlib.sha1()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(PKG, rel), "rb") as fh:
            h.update(fh.read())
    h.update(repr(build.FILE_FLAGS.get("fhp_stepk_k5.hip", [])).encode())
    return h.hexdigest()[:12]


def short(name: str) -> str:
    name = name.replace("fhp::(anonymous namespace)::", "").replace("void ", "")
    return re.sub(r"\(.*", "", name)


def trace_summary(path: str) -> list[tuple[str, int, float]]:
    rows = []
    with open(path) as fh:
        for r in csv.DictReader(fh):
            rows.append((short(r["Name"]), int(r["Calls"]), float(r["AverageNs"]) / 1e3))
    return rows


def pmc_summary(path: str, match: str | None = None) -> dict:
    acc = defaultdict(list)
    with open(path) as fh:
        for r in csv.DictReader(fh):
            k = short(r["Kernel_Name"])
            if match and match not in k:
                continue
            acc[(k, r["Counter_Name"])].append(float(r["Counter_Value"]))
    return {k: (len(v), sum(v) / len(v)) for k, v in acc.items()}


def recorded_value(profile_md: str, key: str) -> float | None:
    """A `key: number` line of a profiles/ note, or None."""
    try:
        text = open(profile_md).read()
    except OSError:
        return None
    m = re.search(re.escape(key) + r":\s*([0-9.eE+]+)", text)
    return float(m.group(1)) if m else None


def recorded_traffic(profile_md: str) -> tuple[float | None, str | None, int | None]:
    """(bytes per launch, kernel source hash, depth) recorded in a profiles/ note."""
    try:
        text = open(profile_md).read()
    except OSError:
        return None, None, None
    m = re.search(r"traffic_bytes_per_launch:\s*([0-9.eE+]+)", text)
    s = re.search(r"kernel_source_hash:\s*([0-9a-f]+)", text)
    d = re.search(r"traffic_depth:\s*([0-9]+)", text)
    return ((float(m.group(1)) if m else None), (s.group(1) if s else None),
            (int(d.group(1)) if d else None))


def main(argv):
    if len(argv) < 2 or argv[0] not in ("trace", "pmc", "hash"):
        print(__doc__)
        return 2 if argv[:1] != ["hash"] else 0
    if argv[0] == "trace":
        for name, calls, us in trace_summary(argv[1]):
            print(f"| {name} | {calls} | {us:.1f} |")
    elif argv[0] == "pmc":
        for (k, c), (n, v) in sorted(pmc_summary(argv[1], argv[2] if len(argv) > 2 else None).items()):
            print(f"| {k} | {c} | {n} | {v:.1f} |")
    return 0


if __name__ == "__main__":
    if sys.argv[1:2] == ["hash"]:
        print(kernel_source_hash())
        sys.exit(0)
    sys.exit(main(sys.argv[1:]))
