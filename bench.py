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


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_band_rate(wl, mask, rows: int, threads: int, seconds: float):
    import oracle
    band = mask[:rows] if mask is not None else None
    state = oracle.init(wl.width, rows, wl.seed, wl.fill, mask=band, walls=wl.walls)
    steps, t0 = 0, time.perf_counter()
    while True:
        state, _ = oracle.step(state, steps, wl.seed, wl.force_rate, threads=threads)
        steps += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    return wl.width * rows * steps / el, steps, el


def cpu_baseline(wl, mask, seconds: float):
    """Times the CPU oracle on bounded samples of the workload: a full-width
    band of 1024 rows of the same lattice (same mask rows, fill and forcing)
    on every core this process may use (the affinity set, capped by
    OMP_NUM_THREADS when that is set), and a band of 64 rows on one core,
    each stepped until its share of `seconds` has elapsed."""
    import oracle
    threads = oracle.default_threads()
    rows = min(1024, wl.height)
    rate, steps, el = _oracle_band_rate(wl, mask, rows, threads, seconds * 2 / 3)
    rows1 = min(64, wl.height)
    rate1, steps1, el1 = _oracle_band_rate(wl, mask, rows1, 1, seconds / 3)
    return {"value": rate, "unit": "node-updates/s", "cores": threads, "kind": "oracle",
            "sample": f"{wl.width}x{rows} band (rows 0-{rows - 1}) of {wl.name}, "
                      f"{steps} steps in {el:.1f} s on {threads} threads",
            "single_core": {"value": rate1, "cores": 1,
                            "sample": f"{wl.width}x{rows1} band (rows 0-{rows1 - 1}), "
                                      f"{steps1} steps in {el1:.1f} s"},
            "cpu_model": cpu_model(), "nproc": os.cpu_count(),
            "affinity_cpus": len(os.sched_getaffinity(0))}


def cpu_simd_baseline(wl, mask, seconds: float):
    """The host bit-plane stepper (SIMD along rows, OpenMP over rows; the
    counterpart of the paper's pSSE/pAVX codes) on the same bounded samples
    as the oracle baseline, all allotted cores and one core; its digest of
    the 256^2 torus workload is checked against the oracle's."""
    import oracle
    from paper_1208_2428_amd import cpu_sim
    from paper_1208_2428_amd import workloads as WL

    def rate(rows, threads, budget):
        band = mask[:rows] if mask is not None else None
        s = cpu_sim.CpuSim(wl.width, rows, seed=wl.seed, fill=wl.fill, force_rate=wl.force_rate,
                           walls=wl.walls, solid=band)
        s.step(2, threads)
        steps, t0 = 0, time.perf_counter()
        while time.perf_counter() - t0 < budget:
            s.step(10, threads)
            steps += 10
        el = time.perf_counter() - t0
        s.close()
        return wl.width * rows * steps / el, steps, el

    threads = oracle.default_threads()
    rows = min(1024, wl.height)
    v, steps, el = rate(rows, threads, seconds * 2 / 3)
    v1, steps1, el1 = rate(min(256, wl.height), 1, seconds / 3)
    tw = WL.WORKLOADS["torus-256"]
    t = cpu_sim.CpuSim(**tw.params())
    t.step(tw.steps, threads)
    ref = golden_digest(tw.name, tw.steps)
    parity = None if ref is None else t.digest() == ref
    t.close()
    log(f"bench: CPU bit-plane stepper ({cpu_sim.isa()}): {v:.3e} node-updates/s on {threads} "
        f"threads, {v1:.3e} on one")
    return {"value": v, "unit": "node-updates/s", "cores": threads, "kind": "bit-plane SIMD",
            "isa": cpu_sim.isa(), "sample": f"{wl.width}x{rows} band of {wl.name}, {steps} steps "
                                            f"in {el:.1f} s on {threads} threads",
            "single_core": {"value": v1, "cores": 1, "steps": steps1, "seconds": el1},
            "cpu_model": cpu_model(), "parity_torus-256_digest_vs_oracle": parity}


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


def depth_sweep(wl, mask, min_seconds: float, last: int | None = None):
    """Throughput and HBM roofline fraction of the single-lattice kernel at
    every depth, each timed with HIP events over at least `min_seconds` (the
    fraction of 14/K bits per node-step falls with K by construction); depth
    `last` is measured last."""
    from paper_1208_2428_amd import _binding as B
    ks = [k for k in range(1, B.MAX_DEPTH + 1) if k != last] + ([last] if last else [])
    out = []
    for k in ks:
        v, n = plain_rate(wl, mask, k, min_seconds)
        frac = v * PLANE_BITS / k / 8 / 1e9 / HBM_PEAK_GBS
        out.append({"depth": k, "value": v, "frac": frac, "steps": n})
        log(f"bench: depth {k}: {v:.3e} node-updates/s over {n} steps, "
            f"{frac:.3f} of the HBM roofline")
    return sorted(out, key=lambda d: d["depth"])


def plain_rate(wl, mask, depth: int, min_seconds: float = 0.1):
    """(node updates/s, steps timed) of the single-lattice kernel at depth
    `depth`: a short untimed run sizes the measurement, which is then timed
    with HIP events on the stream the kernels run on over at least
    `min_seconds`, after an untimed run of the same length."""
    import torch

    from paper_1208_2428_amd import Sim
    from paper_1208_2428_amd.autotune import time_steps
    sim = Sim(**wl.params(), solid=mask, depth=depth)
    probe = time_steps(sim.step, torch.cuda.current_stream(), 12 * depth, 1)
    n = max(depth, int(min_seconds / probe) + 1)
    n = (n + depth - 1) // depth * depth
    per_step = time_steps(sim.step, torch.cuda.current_stream(), n, 1)
    sim.close()
    return wl.width * wl.height / per_step, n


def golden_ensemble():
    """Oracle digests of the ensemble members after its 500 steps, by index
    (written by tests/golden/make_golden.py ensemble-512), or None."""
    path = os.path.join(ROOT, "tests", "golden", "digests_ensemble-512.txt")
    if not os.path.exists(path):
        return None
    out = {}
    with open(path) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                f = line.split()
                out[int(f[0])] = int(f[4], 16)
    return out


def batched_leg(args, plain_at):
    """512 uneven lattices in one batch vs the plain single-lattice kernel at
    the same depth; every member's digest against the same lattice stepped
    alone and against the oracle's."""
    from paper_1208_2428_amd import ensemble
    params = ensemble.ensemble_params()
    log(f"bench: ensemble of {len(params)} lattices, {args.ensemble_steps} steps (tuning first)")
    res = ensemble.run_batched(params, args.ensemble_steps, log=log)
    k = res["tiling"]["depth"]
    plain = plain_at(k)
    log(f"bench: ensemble {res['value']:.3e} node-updates/s at depth {k}; plain {plain:.3e}")
    one = ensemble.run_one_by_one(params, args.ensemble_steps)
    log(f"bench: ensemble one lattice at a time: {one['value']:.3e} node-updates/s")
    same = sum(a == b for a, b in zip(res["digests"], one["digests"]))
    gold = golden_ensemble() if args.ensemble_steps == 500 else None
    vs_oracle = None
    if gold is not None and len(gold) == len(params):
        vs_oracle = sum(res["digests"][i] == gold[i] for i in range(len(params)))
    log(f"bench: ensemble digests: {same}/{len(params)} equal to the lattices stepped alone, "
        f"{'n/a' if vs_oracle is None else vs_oracle}/{len(params)} equal to the oracle's")
    parity = same == len(params) and (vs_oracle is None or vs_oracle == len(params))
    return {"value": res["value"], "unit": "node-updates/s", "lattices": res["lattices"],
            "nodes": res["nodes"], "steps": res["steps"], "tiling": res["tiling"],
            "timing": "HIP events on the batch stream, graph replay, median of "
                      f"{len(res['seconds_all'])} runs of {res['steps']} steps",
            "plain_value_same_depth": plain, "ratio_vs_plain": res["value"] / plain,
            "one_by_one_value": one["value"], "ratio_vs_one_by_one": res["value"] / one["value"],
            "members_equal_alone": same, "members_equal_oracle": vs_oracle, "parity": parity}


def rules_leg(args, wl, mask, plain_at):
    """The headline workload under the other rule sets (FHP-I, FHP-III), each
    at its default depth: throughput (HIP events) and per-launch HBM roofline
    fraction, against FHP-II at the same depth."""
    import torch

    from paper_1208_2428_amd import Sim
    from paper_1208_2428_amd import _binding as B
    from paper_1208_2428_amd.autotune import time_steps
    stream = torch.cuda.current_stream()
    nodes = wl.width * wl.height
    out = {}
    for name, rules, max_depth in (("fhp1", B.RULES_FHP1, B.MAX_DEPTH), ("fhp3", B.RULES_FHP3, 3)):
        sim = Sim(**wl.params(), solid=mask, rules=rules)
        depth = min(sim.depth, max_depth)  # steps per launch
        sim.depth = depth
        steps = args.rules_steps - args.rules_steps % depth
        per_step = time_steps(sim.step, stream, steps, 1)
        launch_s = launch_seconds(sim, stream, depth, 200)
        sim.close()
        achieved = PLANE_BITS * nodes / 8 / launch_s / 1e9
        value = nodes / per_step
        fhp2 = plain_at(depth)
        out[name] = {"value": value, "unit": "node-updates/s", "depth": depth, "steps": steps,
                     "fhp2_same_depth": fhp2, "ratio_vs_fhp2": value / fhp2,
                     "kernel_us": launch_s * 1e6, "roofline_frac": achieved / HBM_PEAK_GBS}
        log(f"bench: {name} {value:.3e} node-updates/s at depth {depth} "
            f"(FHP-II {fhp2:.3e})")
    return out


def served_leg(args, plain_at, depth):
    """Continuous batching of a Poisson stream of channel-flow jobs, at the
    deepest depth pools take; compared with the plain kernel at that depth.
    A seeded sample of the served jobs is run again alone: its 16 x 16 block
    sums must equal what the server returned."""
    import numpy as np

    from paper_1208_2428_amd import _binding as B
    from paper_1208_2428_amd import Sim
    from paper_1208_2428_amd import serve
    from paper_1208_2428_amd import workloads as WL
    depth = min(depth, B.BATCH_MAX_DEPTH)
    plain = plain_at(depth)
    reqs = WL.request_stream(n=args.serve_requests, rate=200.0, seed=5)
    offered = serve.offered_load(reqs)
    sample = sorted(int(i) for i in np.random.default_rng(7).choice(
        len(reqs), size=min(args.serve_check, len(reqs)), replace=False))
    log(f"bench: serving {len(reqs)} requests at 200/s (offered {offered:.3e} node-updates/s)")
    srv = serve.Server(lattice_bytes=32 << 30, max_slots=512, passes_per_tick=1, depth=depth)
    hot = srv.run(reqs, realtime=True, keep_results=set(sample), log=log)
    log(f"bench: served {hot['completed']} in {hot['seconds']:.1f} s: {hot['value']:.3e} "
        f"node-updates/s, p50 {hot['p50_ms']:.0f} ms, p99 {hot['p99_ms']:.0f} ms")
    # a second point at about 80% of the measured capacity
    rate80 = 200.0 * 0.8 * hot["value"] / offered
    n80 = max(100, len(reqs) // 4)
    reqs80 = WL.request_stream(n=n80, rate=rate80, seed=6)
    at80 = srv.run(reqs80, realtime=True, log=log)
    log(f"bench: at {rate80:.0f} req/s: p50 {at80['p50_ms']:.0f} ms, p99 {at80['p99_ms']:.0f} ms")
    for name, r in (("overloaded", hot), ("at 80%", at80)):
        log(f"bench: {name}: queue p50/p99 {r['queue_p50_ms']:.0f}/{r['queue_p99_ms']:.0f} ms, "
            f"in pool {r['pool_p50_ms']:.0f}/{r['pool_p99_ms']:.0f} ms; latency p99 by work third "
            + ", ".join(f"{t['latency_p99_ms']:.0f}" for t in r["by_work"])
            + f" ms; corr(log latency, log work) {r.get('log_latency_log_work_corr', 0):.2f}")
    srv.close()
    same = 0
    for i in sample:
        r = reqs[i]
        sim = Sim(**serve.job_params(r))
        sim.step(r.steps)
        same += int(np.array_equal(sim.observe_blocks(16), hot["results"][i]))
        sim.close()
    log(f"bench: {same}/{len(sample)} sampled served jobs equal to the same job run alone")
    keys = ("requests", "completed", "seconds", "value", "p50_ms", "p99_ms", "mean_ms",
            "max_queue", "max_resident", "ticks", "queue_p50_ms", "queue_p99_ms", "pool_p50_ms",
            "pool_p99_ms", "by_work", "log_latency_log_work_corr")
    return {"value": hot["value"], "unit": "node-updates/s", "depth": depth,
            "plain_value_same_depth": plain, "ratio_vs_plain": hot["value"] / plain,
            "timing": "wall clock from the first arrival to the last result on the host",
            "offered_load": offered, "rate_per_s": 200.0, "arena_bytes": 32 << 30,
            "overloaded": {k: hot[k] for k in keys},
            "at_80pct_capacity": dict({k: at80[k] for k in keys}, rate_per_s=rate80,
                                      offered_load=serve.offered_load(reqs80)),
            "sampled_jobs": len(sample), "sampled_equal_alone": same,
            "parity": same == len(sample)}


def launch_seconds(sim, stream, depth: int, launches: int) -> float:
    """Average duration of one pass of `depth` steps (one kernel launch):
    `launches` passes back to back between two HIP events on the kernel's
    stream, divided by their number (so the few microseconds between
    consecutive launches count as kernel time: an upper bound)."""
    import torch
    sim.step(depth)  # untimed
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(stream)
    sim.step(depth * launches)
    b.record(stream)
    torch.cuda.synchronize()
    return a.elapsed_time(b) / launches / 1e3


def memory_ceiling(wl, depth: int, band: int, has_mask: bool) -> dict:
    """The pass's own memory accesses without its arithmetic: the streaming
    reference kernel with the step kernel's shape (full-width bands of `band`
    rows, `depth` halo rows on each side, seven planes + mask read, seven
    planes written), and plain 16-byte streaming of 1 GiB, both timed here
    with HIP events.  The caller adds the step kernel's figures against them
    (`frac_of_pass_copy`: the reference kernel's time for the same accesses
    over the step kernel's time)."""
    from paper_1208_2428_amd import calib
    wd = wl.width // 64
    ref = calib.pass_rate("copy", wd, wl.height, band, depth, has_mask, launches=50)
    flat = calib.flat_rate("copy", 1 << 30, launches=20)
    log(f"bench: pass-shaped copy {ref['gbs']:.0f} GB/s ({ref['us']:.1f} us for "
        f"{ref['bytes'] / 1e6:.1f} MB), flat copy {flat['gbs']:.0f} GB/s")
    return {"pass_copy_gbs": ref["gbs"], "pass_copy_us": ref["us"], "pass_bytes": ref["bytes"],
            "pass_shape": {"words_per_row": wd, "rows": wl.height, "band": band,
                           "halo_rows": depth, "mask": has_mask},
            "flat_copy_gbs": flat["gbs"]}


def flow_leg(wl, mask) -> dict:
    """Darcy permeability of the workload's obstacle geometry (paper Sec. 2:
    forcing as a body force driving the flow), k = nu q / g.  nu: a forced
    channel of 2048 x 130 nodes at the workload's density (plane Poiseuille
    flow, u'' = -g / nu), 25,000 steps to settle, then profiles every 200
    steps for 40,000.  q, g: the workload's lattice and mask at a force rate
    low enough for linear (Darcy) flow, 60,000 steps to settle (the flow's
    relaxation time k / nu is about 10^4 steps), then global sums every 500
    steps for 20,000.  Both runs are GPU runs of the library; flow.py only
    averages and fits the sums."""
    from paper_1208_2428_amd import Sim, flow
    t0 = time.perf_counter()
    ch = Sim(2048, 130, seed=11, fill=wl.fill, force_rate=5e-5, walls=True)
    v = flow.channel_viscosity(ch, steps=40000, every=200, start=25000)
    ch.close()
    f_por = 2e-5
    sim = Sim(wl.width, wl.height, seed=wl.seed, fill=wl.fill, force_rate=f_por,
              walls=wl.walls, solid=mask)
    d = flow.darcy_sums(sim, steps=20000, every=500, start=60000)
    sim.close()
    k = flow.permeability(d["q"], d["g"], v["nu"])
    porosity = 1.0 - (float(mask.mean()) if mask is not None else 0.0)
    log(f"bench: viscosity {v['nu']:.4f} (channel fit R^2 {v['r2']:.4f}), permeability "
        f"{k:.1f} lattice constants^2 (q {d['q']:.4f}, g {d['g']:.3e}); "
        f"{time.perf_counter() - t0:.1f} s")
    return {"permeability": k, "unit": "lattice constants^2", "porosity": porosity,
            "superficial_velocity": d["q"], "body_force": d["g"], "force_rate": f_por,
            "steps": 80000, "viscosity": v["nu"],
            "viscosity_channel": {"width": 2048, "height": 130, "force_rate": 5e-5,
                                  "body_force": v["g"], "fit_r2": v["r2"], "peak": v["peak"],
                                  "steps": 65000},
            "fill": wl.fill}


def small_config(name: str, min_seconds: float):
    """A smaller named workload run in full from its initial state (digest
    against the oracle's at its last step), then timed with HIP events over
    further runs of the same length until `min_seconds` have been covered."""
    import torch

    from paper_1208_2428_amd import Sim
    from paper_1208_2428_amd import workloads as WL
    wl = WL.WORKLOADS[name]
    stream = torch.cuda.current_stream()
    sim = Sim(**wl.params(), solid=wl.mask())
    sim.step(wl.steps)
    digest = sim.digest()
    ref = golden_digest(name, wl.steps)
    parity = None if ref is None else digest == ref
    runs = 0
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(stream)
    while True:
        sim.step(wl.steps)
        runs += 1
        if time.perf_counter() - t0 >= min_seconds:
            break
    e1.record(stream)
    e1.synchronize()
    sec = e0.elapsed_time(e1) / 1e3
    depth = sim.depth
    sim.close()
    value = wl.width * wl.height * wl.steps * runs / sec
    log(f"bench: {name}: {value:.3e} node-updates/s at depth {depth} "
        f"({runs} runs of {wl.steps} steps); digest at t={wl.steps} "
        f"{'matches' if parity else 'DIFFERS FROM' if parity is False else 'has no'} oracle")
    return {"value": value, "unit": "node-updates/s", "width": wl.width, "height": wl.height,
            "steps": wl.steps, "depth": depth, "timed_steps": wl.steps * runs,
            "fill": wl.fill, "force_rate": wl.force_rate, "walls": wl.walls,
            "parity_digest_vs_oracle": parity}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=40)
    ap.add_argument("--depth", type=int, default=0, help="temporal-block depth k (0 = default)")
    ap.add_argument("--band", type=int, default=0, help="rows per workgroup band (0 = default)")
    ap.add_argument("--workload", default="porous-16384")
    ap.add_argument("--launches", type=int, default=200,
                    help="launches timed one by one for the per-launch kernel time")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-cpu-simd", action="store_true",
                    help="skip the host bit-plane stepper baseline")
    ap.add_argument("--cpu-simd-seconds", type=float, default=6.0)
    ap.add_argument("--no-ensemble", action="store_true",
                    help="skip the 512-lattice batched ensemble comparison")
    ap.add_argument("--ensemble-steps", type=int, default=500)
    ap.add_argument("--no-serve", action="store_true", help="skip the serving-loop leg")
    ap.add_argument("--serve-requests", type=int, default=2000)
    ap.add_argument("--serve-check", type=int, default=32,
                    help="served jobs run again alone and compared")
    ap.add_argument("--no-rules", action="store_true",
                    help="skip the FHP-I / FHP-III rule-set leg")
    ap.add_argument("--rules-steps", type=int, default=3000)
    ap.add_argument("--no-depth-sweep", action="store_true",
                    help="skip the throughput / roofline sweep over depths 1..5")
    ap.add_argument("--sweep-seconds", type=float, default=0.1,
                    help="HIP-event time covered at each depth of the sweep")
    ap.add_argument("--no-ceiling", action="store_true",
                    help="skip the measured memory ceilings (streaming reference kernels)")
    ap.add_argument("--no-flow", action="store_true",
                    help="skip the permeability of the workload's geometry")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the 256^2 torus and 4096^2 channel workloads")
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

    # The device raises its clock over a few tens of milliseconds of sustained
    # load: right after an idle spell (even the few milliseconds of setting up
    # a lattice) the step kernel's launches take up to 10% longer (the SQ
    # counters show 2.04 GHz rising to 2.27 GHz over the first launches).  So
    # both lattices are set up first, the reference measurements follow, and
    # the warm-up and the timed steps come right after them, as in the middle
    # of a long run.
    warm = Sim(**wl.params(), solid=mask, depth=args.depth, band=args.band)
    depth, band = warm.depth, warm.band
    sim = Sim(**wl.params(), solid=mask, depth=depth, band=args.band)
    ceiling = None
    if not args.no_ceiling:
        ceiling = memory_ceiling(wl, depth, band, has_mask=mask is not None)
    plain = {}
    sweep = None
    if not args.no_depth_sweep:
        sweep = depth_sweep(wl, mask, args.sweep_seconds, last=depth)
        plain = {d["depth"]: d["value"] for d in sweep}

    # Per-launch duration of the step kernel (events on the kernel's stream),
    # on the warm-up lattice: the same kernel, lattice and mask as the timed
    # one, so the timed lattice still starts from t = 0.
    launch_s = launch_seconds(warm, stream, depth, args.launches)
    bytes_per_launch = PLANE_BITS * wl.width * wl.height / 8  # 14/k bits per node-step, k steps per launch
    achieved = bytes_per_launch / launch_s / 1e9
    log(f"bench: {args.launches} launches of depth {depth}: {launch_s * 1e6:.1f} us each, "
        f"{achieved / HBM_PEAK_GBS:.3f} of the HBM roofline")

    log(f"bench: warmup {args.warmup} steps at depth {depth}")
    warm.step(args.warmup)
    warm.sync()

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

    sim.close()
    warm.close()
    del sim, warm
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
                   "solid_fraction": round(solid_frac, 5), "depth": depth, "band": band,
                   "parity_digest_vs_oracle": parity},
        "events_value": nodes * args.steps / ev_s,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel_us": launch_s * 1e6, "launches_timed": args.launches,
                     "bytes_per_launch": bytes_per_launch},
    }
    if ceiling is not None:
        moved = ceiling["pass_bytes"]
        ceiling["kernel_gbs_of_pass_bytes"] = moved / launch_s / 1e9
        ceiling["frac_of_pass_copy"] = ceiling["pass_copy_us"] / (launch_s * 1e6)
        ceiling["algorithmic_frac_of_flat_copy"] = achieved / ceiling["flat_copy_gbs"]
        out["roofline"]["ceiling"] = ceiling
    if valu is not None:
        # the same launch against the VALU issue limit (wave64 instructions;
        # integer multiplies issue at the bit-operation rate on this GPU)
        rate = valu / launch_s
        out["alu"] = {"bound": "alu", "achieved": rate, "peak": VALU_WAVE_INSTR_PEAK,
                      "unit": "wave64 VALU instructions/s", "frac": rate / VALU_WAVE_INSTR_PEAK,
                      "valu_insts_per_launch": valu}
    if sweep is not None:
        out["depth_sweep"] = sweep

    def plain_at(k: int) -> float:
        """The plain kernel's rate at depth k, HIP events over >= 100 ms."""
        if k not in plain:
            plain[k] = plain_rate(wl, mask, k, max(0.1, args.sweep_seconds))[0]
        return plain[k]

    if not args.no_configs:
        out["configs"] = {n: small_config(n, 0.1) for n in ("torus-256", "channel-4096")}
    if not args.no_ensemble:
        out["batched"] = batched_leg(args, plain_at)
    if not args.no_serve:
        out["served"] = served_leg(args, plain_at, depth)
    if not args.no_rules:
        out["rule_sets"] = rules_leg(args, wl, mask, plain_at)
    if not args.no_flow:
        out["flow"] = flow_leg(wl, mask)
    if not args.no_cpu_baseline:
        log(f"bench: timing the CPU oracle for ~{args.cpu_seconds:.0f} s")
        out["cpu_baseline"] = cpu_baseline(wl, mask, args.cpu_seconds)
    if not args.no_cpu_simd:
        out["cpu_simd_baseline"] = cpu_simd_baseline(wl, mask, args.cpu_simd_seconds)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
