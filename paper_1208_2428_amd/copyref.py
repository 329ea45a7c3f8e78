"""Reference device copy of a known size, used to calibrate HBM byte counters.

Copies a 1 GiB device buffer into another `--reps` times with torch (one copy
kernel per repetition, 1 GiB read + 1 GiB written each).  Profiling it with
the same counters as the FHP kernels gives the factor between the counter
reading and the true number of bytes.
"""
import argparse

import torch


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--mib", type=int, default=1024)
    ap.add_argument("--reps", type=int, default=5)
    a = ap.parse_args()
    n = a.mib << 20
    src = torch.ones(n, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(a.reps):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(f"copied {a.mib} MiB x {a.reps}", flush=True)


if __name__ == "__main__":
    main()
