"""GPU vs oracle parity of the rule-set variants (FHP-I, collision-saturated
FHP-III) on single lattices: every depth, walls, obstacles (including solid
nodes holding particles), forcing, ragged sizes, the one-step kernel and the
blocked kernel.  Bit-exact: one correct result exists."""
import numpy as np
import pytest

import oracle
from paper_1208_2428_amd import Batch, Pool, Sim
from paper_1208_2428_amd import _binding as B
from paper_1208_2428_amd import workloads as WL

pytestmark = pytest.mark.gpu

THREADS = oracle.default_threads()
RULES = {"FHP-I": (B.RULES_FHP1, oracle.RULES_FHP1), "FHP-III": (B.RULES_FHP3, oracle.RULES_FHP3)}


def say(*a):
    print(*a, flush=True)


def make_state(rng, W, H, case):
    # dense fills reach the mass >= 4 states that FHP-III handles by duality
    st = WL.random_states(rng, H, W, p=0.5)
    if case in ("mask+force", "solid-particles"):
        st |= ((rng.random((H, W)) < 0.15).astype(np.uint8) << 7)
    if case == "solid-particles":
        st |= WL.random_states(rng, H, W, p=0.5) & 0x7F
    if "walls" in case:
        st[0] |= 0x80
        st[-1] |= 0x80
    return st


@pytest.mark.parametrize("name", list(RULES))
@pytest.mark.parametrize("W,H", [(64, 2), (192, 10), (320, 34), (1024, 70)])
@pytest.mark.parametrize("K", [1, 2, 3, 4, 5])
@pytest.mark.parametrize("case", ["torus", "walls+force", "mask+force", "solid-particles"])
def test_rules_match_oracle(name, W, H, K, case):
    say("rules", name, W, H, K, case)
    gpu_rules, oracle_rules = RULES[name]
    rng = np.random.default_rng(W + 7 * H + 13 * K)
    f = 1.0 / 80 if "force" in case else 0.0
    walls = "walls" in case
    st = make_state(rng, W, H, case)
    s = Sim(W, H, seed=47, force_rate=f, walls=walls, depth=K, rules=gpu_rules)
    s.set_state(st, t=3)
    ref = st.copy()
    t = 3
    for n in (K, 1, K + 1, 2 * K + 3):
        s.step(n)
        ref, _ = oracle.run(ref, t, n, 47, f, threads=THREADS, rules=oracle_rules)
        t += n
        np.testing.assert_array_equal(s.get_state(), ref, err_msg=f"{name} after t={t}")
    s.close()


@pytest.mark.parametrize("name", list(RULES))
def test_rules_from_initial_state_with_chirality_modes(name):
    gpu_rules, oracle_rules = RULES[name]
    W, H = 256, 64
    for chir in (B.CHIR_ZERO, B.CHIR_ONE):
        s = Sim(W, H, seed=5, fill=0.45, force_rate=2e-3, walls=True, chirality=chir,
                rules=gpu_rules)
        s.step(20)
        ref = oracle.init(W, H, 5, 0.45, walls=True)
        ref, _ = oracle.run(ref, 0, 20, 5, 2e-3, chir_mode=chir, threads=THREADS,
                            rules=oracle_rules)
        np.testing.assert_array_equal(s.get_state(), ref)
        s.close()


def test_rule_sets_differ_and_conserve():
    W, H = 512, 128
    out = {}
    for rules in (B.RULES_FHP2, B.RULES_FHP1, B.RULES_FHP3):
        s = Sim(W, H, seed=9, fill=0.4, rules=rules)
        m0 = s.observe_global()
        s.step(40)
        m = s.observe_global()
        assert (m["mass"], m["px"], m["py"]) == (m0["mass"], m0["px"], m0["py"])
        out[rules] = s.get_state()
        s.close()
    assert not np.array_equal(out[B.RULES_FHP2], out[B.RULES_FHP1])
    assert not np.array_equal(out[B.RULES_FHP2], out[B.RULES_FHP3])


def mixed(rules):
    mask = WL.porous_mask(192, 64, seed=9, rmin=3, rmax=6, frac=0.08)
    return [
        dict(width=64, height=8, seed=1, fill=0.45, rules=rules),
        dict(width=128, height=128, seed=2, fill=0.5, force_rate=1e-2, walls=True, rules=rules),
        dict(width=192, height=64, seed=3, fill=0.4, solid=mask, rules=rules),
        dict(width=320, height=96, seed=5, fill=0.6, force_rate=5e-3, rules=rules),
        dict(width=1024, height=40, seed=8, fill=0.5, walls=True, rules=rules),
        dict(width=64, height=10, seed=9, fill=0.5, chirality=2, rules=rules),
    ]


def oracle_member(kw, steps, oracle_rules):
    st = oracle.init(kw["width"], kw["height"], kw["seed"], kw["fill"], mask=kw.get("solid"),
                     walls=kw.get("walls", False))
    st, _ = oracle.run(st, 0, steps, kw["seed"], kw.get("force_rate", 0.0),
                       chir_mode=kw.get("chirality", 0), threads=THREADS, rules=oracle_rules)
    return st


@pytest.mark.parametrize("name", list(RULES))
@pytest.mark.parametrize("depth,ppl", [(5, 1), (3, 0), (2, 2)])
def test_batch_of_a_rule_set_matches_oracle(name, depth, ppl):
    say("batch rules", name, depth, ppl)
    gpu_rules, oracle_rules = RULES[name]
    params = mixed(gpu_rules)
    b = Batch(params, depth=depth, passes_per_launch=ppl)
    steps = 0
    for n in (12, 5, 7):
        b.step(n)
        steps += n
        b.sync()
        for i, kw in enumerate(params):
            np.testing.assert_array_equal(b[i].get_state(), oracle_member(kw, steps, oracle_rules),
                                          err_msg=f"{name} member {i} after {steps} steps")
    b.close()


@pytest.mark.parametrize("name", list(RULES))
def test_pool_of_a_rule_set(name):
    gpu_rules, oracle_rules = RULES[name]
    pool = Pool(Pool.arena_bytes_for(8, 4096, 32 << 20), max_slots=8, max_bands=4096,
                rules=gpu_rules)
    # jobs of another rule set are refused
    with pytest.raises(RuntimeError, match="rule set"):
        pool.admit(4, width=128, height=32, seed=1, fill=0.2)
    jobs = [(dict(width=256, height=64, seed=21, fill=0.5, force_rate=1e-3, walls=True,
                  rules=gpu_rules), 23),
            (dict(width=128, height=40, seed=22, fill=0.4, rules=gpu_rules), 9)]
    slots = {pool.admit(n, **p): k for k, (p, n) in enumerate(jobs)}
    # the rule set changes only while the pool is empty
    with pytest.raises(RuntimeError, match="empty"):
        pool.set_rules(B.RULES_FHP2)
    got = {}
    while len(got) < len(jobs):
        pool.tick(2)
        for s in pool.done():
            got[slots[s]] = pool.member(s).get_state()
            pool.release(s)
    for k, (p, n) in enumerate(jobs):
        np.testing.assert_array_equal(got[k], oracle_member(p, n, oracle_rules), err_msg=str(k))
    pool.close()
