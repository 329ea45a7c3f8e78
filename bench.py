"""Benchmark: FHP node updates per second on one MI355X, against the HBM roofline.

Workload: the 16384 x 16384 porous medium (solid disks r = 8..32 covering 5%,
periodic box, fill 0.3, forcing 5e-4), stepped with the library's temporally
blocked kernel.  One benchmark step is one FHP time step of the whole lattice
(motion + collision + bounce-back + forcing, arXiv:1208.2428 Sec. 2); the
unit is the paper's lattice-site update (Sec. 4).

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E peak
PLANE_BITS = 14        # 7 planes read + 7 written per node and HBM pass


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def golden_digest(name: str, t: int):
    path = os.path.join(ROOT, "tests", "golden", f"digests_{name}.txt")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        for line in fh:
            if line.startswith("#"):
                continue
            parts = line.split()
            if int(parts[0]) == t:
                return int(parts[1], 16)
    return None


def recorded_traffic(name: str, depth: int):
    """HBM bytes per launch from the rocprofv3 counters recorded under
    profiles/ for this kernel, or None if they were taken on other kernel
    sources or another depth."""
    from paper_1208_2428_amd import profsum
    path = os.path.join(ROOT, "profiles", f"k_stepk_{name}.md")
    traffic, src, rec_depth = profsum.recorded_traffic(path)
    if traffic is None or depth != rec_depth or src != profsum.kernel_source_hash():
        return None
    return traffic


def cpu_baseline(wl, mask, seconds: float):
    """Times the CPU oracle on a bounded sample of the workload: a full-width
    band of 1024 rows of the same lattice (same mask rows, fill and forcing),
    stepped until `seconds` have elapsed, on all host cores (capped at 16)."""
    import oracle
    threads = oracle.default_threads()
    rows = min(1024, wl.height)
    band = mask[:rows] if mask is not None else None
    state = oracle.init(wl.width, rows, wl.seed, wl.fill, mask=band, walls=wl.walls)
    steps, t0 = 0, time.perf_counter()
    while True:
        state, _ = oracle.step(state, steps, wl.seed, wl.force_rate, threads=threads)
        steps += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    rate = wl.width * rows * steps / el
    return {"value": rate, "unit": "node-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{wl.width}x{rows} band (rows 0-{rows - 1}) of {wl.name}, "
                      f"{steps} steps in {el:.1f} s"}


VALU_WAVE_INSTR_PEAK = 256 * 4 * 2.4e9 / 4  # SIMDs x clock / 4 cycles per wave64 instruction


def recorded_valu(name: str, depth: int):
    """VALU instructions per launch (all waves) from the rocprofv3 SQ_INSTS_VALU
    pass recorded under profiles/, if it was taken on these kernel sources at
    this depth."""
    from paper_1208_2428_amd import profsum
    path = os.path.join(ROOT, "profiles", f"k_stepk_{name}.md")
    _, src, rec_depth = profsum.recorded_traffic(path)
    insts = profsum.recorded_value(path, "valu_insts_per_launch")
    if insts is None or depth != rec_depth or src != profsum.kernel_source_hash():
        return None
    return insts


def depth_sweep(wl, mask, steps: int):
    """Throughput and HBM roofline fraction of the single-lattice kernel at
    every depth (the fraction of 14/K bits per node-step falls with K by
    construction; the HBM-bound regime is K <= 2)."""
    from paper_1208_2428_amd import _binding as B
    out = []
    for k in range(1, B.MAX_DEPTH + 1):
        n = steps - steps % k
        v = plain_rate(wl, mask, k, n)
        frac = v * PLANE_BITS / k / 8 / 1e9 / HBM_PEAK_GBS
        out.append({"depth": k, "value": v, "frac": frac, "steps": n})
        log(f"bench: depth {k}: {v:.3e} node-updates/s, {frac:.3f} of the HBM roofline")
    return out


def plain_rate(wl, mask, depth: int, steps: int) -> float:
    """Node updates/s of the single-lattice kernel at depth `depth`, timed
    with HIP events on the stream the kernels run on (after one untimed run
    of the same length)."""
    import torch

    from paper_1208_2428_amd import Sim
    from paper_1208_2428_amd.autotune import time_steps
    sim = Sim(**wl.params(), solid=mask, depth=depth)
    per_step = time_steps(sim.step, torch.cuda.current_stream(), steps, 1)
    sim.close()
    return wl.width * wl.height / per_step


def batched_leg(args, wl, mask, depth, value):
    """512 uneven lattices in one batch vs the plain single-lattice kernel."""
    from paper_1208_2428_amd import ensemble
    params = ensemble.ensemble_params()
    log(f"bench: ensemble of {len(params)} lattices, {args.ensemble_steps} steps (tuning first)")
    res = ensemble.run_batched(params, args.ensemble_steps, log=log)
    k = res["tiling"]["depth"]
    plain = value if k == depth else plain_rate(wl, mask, k, 480)
    log(f"bench: ensemble {res['value']:.3e} node-updates/s at depth {k}; plain {plain:.3e}")
    one = ensemble.run_one_by_one(params, args.ensemble_steps)
    log(f"bench: ensemble one lattice at a time: {one['value']:.3e} node-updates/s")
    return {"value": res["value"], "unit": "node-updates/s", "lattices": res["lattices"],
            "nodes": res["nodes"], "steps": res["steps"], "tiling": res["tiling"],
            "plain_value_same_depth": plain, "ratio_vs_plain": res["value"] / plain,
            "ratio_vs_headline": res["value"] / value,
            "one_by_one_value": one["value"], "ratio_vs_one_by_one": res["value"] / one["value"]}


def rules_leg(args, wl, mask, plain):
    """The headline workload under the other rule sets (FHP-I, FHP-III), each
    at its default depth: throughput and per-launch HBM roofline fraction."""
    import torch

    from paper_1208_2428_amd import Sim
    from paper_1208_2428_amd import _binding as B
    stream = torch.cuda.current_stream()
    nodes = wl.width * wl.height
    out = {}
    for name, rules, max_depth in (("fhp1", B.RULES_FHP1, B.MAX_DEPTH), ("fhp3", B.RULES_FHP3, 3)):
        sim = Sim(**wl.params(), solid=mask, rules=rules)
        depth = min(sim.depth, max_depth)  # steps per launch
        sim.step(8 * depth)
        torch.cuda.synchronize()
        steps = args.rules_steps
        t0 = time.perf_counter()
        sim.step(steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        launches = 50
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
               for _ in range(launches)]
        for a, b in evs:
            a.record(stream)
            sim.step(depth)
            b.record(stream)
        torch.cuda.synchronize()
        launch_s = sum(a.elapsed_time(b) for a, b in evs) / launches / 1e3
        sim.close()
        achieved = PLANE_BITS * nodes / 8 / launch_s / 1e9
        value = nodes * steps / wall
        out[name] = {"value": value, "unit": "node-updates/s", "depth": depth, "steps": steps,
                     "ratio_vs_fhp2": value / plain, "kernel_us": launch_s * 1e6,
                     "roofline_frac": achieved / HBM_PEAK_GBS}
        log(f"bench: {name} {value:.3e} node-updates/s at depth {depth}")
    return out


def served_leg(args, wl, mask, value, depth):
    """Continuous batching of a Poisson stream of channel-flow jobs, at the
    deepest depth pools take; compared with the plain kernel at that depth."""
    from paper_1208_2428_amd import _binding as B
    from paper_1208_2428_amd import serve
    from paper_1208_2428_amd import workloads as WL
    sdepth = min(depth, B.BATCH_MAX_DEPTH)
    plain = value if sdepth == depth else plain_rate(wl, mask, sdepth, 480)
    depth = sdepth
    reqs = WL.request_stream(n=args.serve_requests, rate=200.0, seed=5)
    offered = serve.offered_load(reqs)
    log(f"bench: serving {len(reqs)} requests at 200/s (offered {offered:.3e} node-updates/s)")
    srv = serve.Server(lattice_bytes=32 << 30, max_slots=512, passes_per_tick=1, depth=depth)
    hot = srv.run(reqs, realtime=True, log=log)
    log(f"bench: served {hot['completed']} in {hot['seconds']:.1f} s: {hot['value']:.3e} "
        f"node-updates/s, p50 {hot['p50_ms']:.0f} ms, p99 {hot['p99_ms']:.0f} ms")
    # a second point at about 80% of the measured capacity
    rate80 = 200.0 * 0.8 * hot["value"] / offered
    n80 = max(100, len(reqs) // 4)
    reqs80 = WL.request_stream(n=n80, rate=rate80, seed=6)
    at80 = srv.run(reqs80, realtime=True, log=log)
    log(f"bench: at {rate80:.0f} req/s: p50 {at80['p50_ms']:.0f} ms, p99 {at80['p99_ms']:.0f} ms")
    srv.close()
    keys = ("requests", "completed", "seconds", "value", "p50_ms", "p99_ms", "mean_ms",
            "max_queue", "max_resident", "ticks")
    return {"value": hot["value"], "unit": "node-updates/s", "depth": depth,
            "plain_value_same_depth": plain, "ratio_vs_plain": hot["value"] / plain,
            "ratio_vs_headline": hot["value"] / value,
            "offered_load": offered, "rate_per_s": 200.0, "arena_bytes": 32 << 30,
            "overloaded": {k: hot[k] for k in keys},
            "at_80pct_capacity": dict({k: at80[k] for k in keys}, rate_per_s=rate80,
                                      offered_load=serve.offered_load(reqs80))}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--depth", type=int, default=0, help="temporal-block depth k (0 = default)")
    ap.add_argument("--band", type=int, default=0, help="rows per workgroup band (0 = default)")
    ap.add_argument("--workload", default="porous-16384")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-ensemble", action="store_true",
                    help="skip the 512-lattice batched ensemble comparison")
    ap.add_argument("--ensemble-steps", type=int, default=500)
    ap.add_argument("--no-serve", action="store_true", help="skip the serving-loop leg")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--no-rules", action="store_true",
                    help="skip the FHP-I / FHP-III rule-set leg")
    ap.add_argument("--rules-steps", type=int, default=400)
    ap.add_argument("--no-depth-sweep", action="store_true",
                    help="skip the throughput / roofline sweep over depths 1..5")
    ap.add_argument("--sweep-steps", type=int, default=240)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              f"(asked for --gpus {args.gpus})", file=sys.stderr)
        return 2

    import torch

    from paper_1208_2428_amd import Sim
    from paper_1208_2428_amd import workloads as WL

    wl = WL.WORKLOADS[args.workload]
    torch.cuda.set_device(0)
    stream = torch.cuda.current_stream()
    log(f"bench: {wl.name} {wl.width}x{wl.height}, building mask")
    mask = wl.mask()
    solid_frac = float(mask.mean()) if mask is not None else 0.0

    warm = Sim(**wl.params(), solid=mask, depth=args.depth, band=args.band)
    depth = warm.depth
    log(f"bench: warmup {args.warmup} steps at depth {depth}")
    warm.step(args.warmup)
    warm.sync()
    warm.close()
    del warm

    sim = Sim(**wl.params(), solid=mask, depth=depth, band=args.band)
    nodes = wl.width * wl.height
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    sim.step(args.steps)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev_s = e0.elapsed_time(e1) / 1e3
    log(f"bench: {args.steps} steps in {wall * 1e3:.2f} ms wall, {ev_s * 1e3:.2f} ms events")

    digest = sim.digest()
    ref = golden_digest(wl.name, args.steps)
    parity = None if ref is None else (digest == ref)
    log(f"bench: digest at t={args.steps}: {digest:016x}, oracle {'n/a' if ref is None else f'{ref:016x}'}")

    # Per-launch duration of the step kernel, with events on the kernel's stream.
    launches = max(1, min(200, args.steps // depth))
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(launches)]
    for a, b in evs:
        a.record(stream)
        sim.step(depth)
        b.record(stream)
    torch.cuda.synchronize()
    launch_s = sum(a.elapsed_time(b) for a, b in evs) / launches / 1e3
    bytes_per_launch = PLANE_BITS * nodes / 8  # 14/k bits per node-step, k steps per launch
    achieved = bytes_per_launch / launch_s / 1e9
    sim.close()
    traffic = recorded_traffic(wl.name, depth)
    valu = recorded_valu(wl.name, depth)

    value = nodes * args.steps / wall
    out = {
        "metric": "FHP node updates/sec at 16384^2 vs HBM roofline",
        "value": value,
        "unit": "node-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": wl.name, "width": wl.width, "height": wl.height,
                   "fill": wl.fill, "force_rate": wl.force_rate,
                   "solid_fraction": round(solid_frac, 5), "depth": depth, "band": args.band,
                   "parity_digest_vs_oracle": parity},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel_us": launch_s * 1e6, "bytes_per_launch": bytes_per_launch},
    }
    if valu is not None:
        # the same launch against the VALU issue limit (wave64 instructions;
        # integer multiplies issue at the bit-operation rate on this GPU)
        rate = valu / launch_s
        out["alu"] = {"bound": "alu", "achieved": rate, "peak": VALU_WAVE_INSTR_PEAK,
                      "unit": "wave64 VALU instructions/s", "frac": rate / VALU_WAVE_INSTR_PEAK,
                      "valu_insts_per_launch": valu}
    if not args.no_depth_sweep:
        out["depth_sweep"] = depth_sweep(wl, mask, args.sweep_steps)
    if not args.no_ensemble:
        out["batched"] = batched_leg(args, wl, mask, depth, value)
    if not args.no_serve:
        out["served"] = served_leg(args, wl, mask, value, depth)
    if not args.no_rules:
        out["rule_sets"] = rules_leg(args, wl, mask, value)
    if not args.no_cpu_baseline:
        log(f"bench: timing the CPU oracle for ~{args.cpu_seconds:.0f} s")
        out["cpu_baseline"] = cpu_baseline(wl, mask, args.cpu_seconds)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
