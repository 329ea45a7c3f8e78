"""Randomised GPU vs oracle parity: 480 seeded single-lattice configurations
drawn over widths, heights, depths, band heights, walls, obstacles (solid
nodes holding particles included), forcing rates, chirality modes, rule sets
and step sequences; 64 seeded batches with random tilings; 32 seeded job
streams through pools.  Every result is compared bit for bit with the oracle.
The draws are fixed by the seeds, so a failure names a reproducible case."""
import numpy as np
import pytest

import oracle
from paper_1208_2428_amd import Batch, Pool, Sim
from paper_1208_2428_amd import workloads as WL

pytestmark = pytest.mark.gpu

THREADS = oracle.default_threads()
RULE_DEPTH = {oracle.RULES_FHP2: 5, oracle.RULES_FHP1: 5, oracle.RULES_FHP3: 3}


def draw(case: int) -> dict:
    rng = np.random.default_rng(1000 + case)
    rules = [oracle.RULES_FHP2, oracle.RULES_FHP2, oracle.RULES_FHP1, oracle.RULES_FHP3][case % 4]
    H = int(2 * rng.integers(1, 60))
    return dict(
        W=int(64 * rng.integers(1, 20)), H=H, rules=rules,
        depth=int(rng.integers(1, RULE_DEPTH[rules] + 1)),
        band=int(rng.integers(0, H + 1)),  # 0: the library's default
        walls=bool(rng.random() < 0.4),
        solid=float(rng.choice([0.0, 0.0, 0.05, 0.3])),
        force=float(rng.choice([0.0, 1e-3, 1.0 / 80])),
        chir=int(rng.choice([oracle.CHIR_HASH, oracle.CHIR_HASH, 1, 2])),
        fill=float(rng.uniform(0.05, 0.6)),
        seed=int(rng.integers(0, 2 ** 40)),
        t0=int(rng.integers(0, 50)),
        steps=[int(n) for n in rng.integers(1, 14, size=3)],
    )


@pytest.mark.parametrize("case", range(480))
def test_random_configuration(case):
    c = draw(case)
    print("random case", case, c, flush=True)
    rng = np.random.default_rng(case)
    st = WL.random_states(rng, c["H"], c["W"], p=c["fill"], solid_frac=c["solid"])
    if c["walls"]:
        st[0] |= 0x80
        st[-1] |= 0x80
    s = Sim(c["W"], c["H"], seed=c["seed"], force_rate=c["force"], walls=c["walls"],
            chirality=c["chir"], rules=c["rules"], depth=c["depth"])
    if c["band"]:
        s.set_band(c["band"])
    s.set_state(st, t=c["t0"])
    ref, t = st.copy(), c["t0"]
    for n in c["steps"]:
        s.step(n)
        ref, _ = oracle.run(ref, t, n, c["seed"], c["force"], chir_mode=c["chir"],
                            threads=THREADS, rules=c["rules"])
        t += n
        np.testing.assert_array_equal(s.get_state(), ref, err_msg=f"case {case} at t={t}")
    assert s.t == t
    s.close()


def draw_batch(case: int) -> dict:
    rng = np.random.default_rng(5000 + case)
    rules = [oracle.RULES_FHP2, oracle.RULES_FHP1, oracle.RULES_FHP3][case % 3]
    members = []
    for _ in range(int(rng.integers(2, 7))):
        H = int(2 * rng.integers(4, 40))  # batch members hold at least 8 rows
        members.append(dict(
            width=int(64 * rng.integers(1, 12)), height=H, seed=int(rng.integers(0, 2 ** 40)),
            fill=float(rng.uniform(0.05, 0.6)), walls=bool(rng.random() < 0.4),
            force_rate=float(rng.choice([0.0, 1e-3, 1.0 / 80])),
            chirality=int(rng.choice([oracle.CHIR_HASH, oracle.CHIR_HASH, 1, 2])),
            rules=rules))
    return dict(
        members=members,
        depth=int(rng.integers(1, RULE_DEPTH[rules] + 1)),
        band=int(rng.choice([0, 8, 16, 32])),
        threads=int(rng.choice([0, 64, 128, 256])),
        ppl=int(rng.choice([0, 1, 2])),
        graph=bool(rng.random() < 0.5),
        steps=[int(n) for n in rng.integers(1, 12, size=3)],
    )


@pytest.mark.parametrize("case", range(64))
def test_random_batch(case):
    """Seeded batches of 2-6 uneven lattices of one rule set with random
    tiling (depth, band height, workgroup size, passes per launch, graph
    replay), every member compared with the oracle after every call."""
    c = draw_batch(case)
    print("random batch", case, {k: v for k, v in c.items() if k != "members"},
          [(m["width"], m["height"]) for m in c["members"]], flush=True)
    b = Batch(c["members"], depth=c["depth"], band=c["band"], group_threads=c["threads"],
              passes_per_launch=c["ppl"], graph=c["graph"])
    refs = [oracle.init(m["width"], m["height"], m["seed"], m["fill"], walls=m["walls"])
            for m in c["members"]]
    t = 0
    for n in c["steps"]:
        b.step(n)
        b.sync()
        for i, m in enumerate(c["members"]):
            refs[i], _ = oracle.run(refs[i], t, n, m["seed"], m["force_rate"],
                                    chir_mode=m["chirality"], threads=THREADS, rules=m["rules"])
            np.testing.assert_array_equal(b[i].get_state(), refs[i],
                                          err_msg=f"batch case {case} member {i} at t={t + n}")
        t += n
    b.close()


@pytest.mark.parametrize("case", range(32))
def test_random_pool(case):
    """Seeded job streams through a pool: jobs of random size, step count and
    physics (one rule set per pool) admitted between ticks of random length,
    each finished job's state compared with the oracle."""
    rng = np.random.default_rng(9000 + case)
    rules = [oracle.RULES_FHP2, oracle.RULES_FHP1, oracle.RULES_FHP3][case % 3]
    depth = int(rng.integers(1, RULE_DEPTH[rules] + 1))
    pool = Pool(Pool.arena_bytes_for(16, 4096, 32 << 20), max_slots=16, max_bands=4096,
                depth=depth, rules=rules, group_threads=int(rng.choice([0, 64, 256])))
    jobs = []
    for _ in range(int(rng.integers(4, 10))):
        jobs.append((dict(width=int(64 * rng.integers(1, 8)), height=int(2 * rng.integers(4, 48)),
                          seed=int(rng.integers(0, 2 ** 40)), fill=float(rng.uniform(0.05, 0.6)),
                          walls=bool(rng.random() < 0.5),
                          force_rate=float(rng.choice([0.0, 1e-3, 1.0 / 80])), rules=rules),
                     int(rng.integers(0, 30))))
    print("random pool", case, depth, [(p["width"], p["height"], n) for p, n in jobs], flush=True)
    slot_of, got, pending = {}, {}, list(range(len(jobs)))
    while pending or len(got) < len(jobs):
        for _ in range(int(rng.integers(0, 3))):  # admit a few, then tick a few passes
            if pending:
                k = pending.pop(0)
                s = pool.admit(jobs[k][1], **jobs[k][0])
                assert s is not None
                slot_of[s] = k
        pool.tick(int(rng.integers(1, 4)))
        for s in pool.done():
            got[slot_of[s]] = pool.member(s).get_state()
            pool.release(s)
    for k, (p, n) in enumerate(jobs):
        ref = oracle.init(p["width"], p["height"], p["seed"], p["fill"], walls=p["walls"])
        ref, _ = oracle.run(ref, 0, n, p["seed"], p["force_rate"], threads=THREADS, rules=rules)
        np.testing.assert_array_equal(got[k], ref, err_msg=f"pool case {case} job {k}")
