"""Pins of the oracle's rule-set variants (FHP-I, FHP-II, collision-saturated
FHP-III) against what the lattice gas itself fixes, computed here from the
geometry and not from the oracle's tables: conservation of mass and momentum,
invertibility with T_chi^-1 = T_{1-chi}, the classes of states that share mass
and momentum (which FHP-III must saturate), symmetry under the lattice's
rotations and reflections, particle-hole duality, and the collision counts.

The paper's rule figure is missing (arXiv:1208.2428, Sec. 2); FHP-II is the
reading of its model and these are the two standard variants of the same gas
(Frisch, Hasslacher & Pomeau 1986; Frisch et al. 1987)."""
from collections import defaultdict

import numpy as np
import pytest

import oracle
from tests.geometry import mass, moving_momentum

RULES = {"FHP-I": oracle.RULES_FHP1, "FHP-II": oracle.RULES_FHP2, "FHP-III": oracle.RULES_FHP3}
CHANGED = {"FHP-I": 10, "FHP-II": 20, "FHP-III": 76}


def table(name, chi):
    return [int(v) for v in oracle.rule_table(RULES[name], chi)]


def momentum_key(s):
    px, py = moving_momentum(s)
    return round(px * 2), round(py * 2)  # exact multiples of 1/2 for this lattice


def classes():
    """States grouped by (mass, momentum), from the geometry."""
    c = defaultdict(list)
    for s in range(128):
        c[(mass(s),) + momentum_key(s)].append(s)
    return c


def rot(s):
    """Lattice rotation by +60 degrees: channel i -> i+1, rest unchanged."""
    out = s & 64
    for i in range(6):
        if (s >> i) & 1:
            out |= 1 << ((i + 1) % 6)
    return out


def mirror(s):
    """Reflection in the x axis: angle (i-2)*60 -> -(i-2)*60, i.e. i -> 4-i."""
    out = s & 64
    for i in range(6):
        if (s >> i) & 1:
            out |= 1 << ((4 - i) % 6)
    return out


def bits(*chs, rest=False):
    return sum(1 << (c % 6) for c in chs) | (64 if rest else 0)


@pytest.mark.parametrize("name", list(RULES))
@pytest.mark.parametrize("chi", [0, 1])
def test_conserves_mass_and_momentum(name, chi):
    T = table(name, chi)
    for s in range(128):
        assert mass(T[s]) == mass(s)
        assert momentum_key(T[s]) == momentum_key(s)


@pytest.mark.parametrize("name", list(RULES))
def test_permutation_inverse_and_count(name):
    T0, T1 = table(name, 0), table(name, 1)
    assert sorted(T0) == list(range(128)) and sorted(T1) == list(range(128))
    for s in range(128):
        assert T0[T1[s]] == s and T1[T0[s]] == s
    assert sum(T1[s] != s for s in range(128)) == CHANGED[name]
    assert sum(T0[s] != s for s in range(128)) == CHANGED[name]


@pytest.mark.parametrize("name", list(RULES))
@pytest.mark.parametrize("chi", [0, 1])
def test_rotation_and_reflection_symmetry(name, chi):
    T, Tm = table(name, chi), table(name, 1 - chi)
    for s in range(128):
        assert T[rot(s)] == rot(T[s])
        # a reflection reverses the sense of rotation, i.e. the chirality
        assert T[mirror(s)] == mirror(Tm[s])


def test_fhp3_is_collision_saturated():
    can_change = {s for v in classes().values() if len(v) >= 2 for s in v}
    assert len(can_change) == 76
    for chi in (0, 1):
        T = table("FHP-III", chi)
        assert {s for s in range(128) if T[s] != s} == can_change


def test_fhp3_particle_hole_duality():
    for chi in (0, 1):
        T = table("FHP-III", chi)
        for s in range(128):
            assert T[~s & 127] == ~T[s] & 127


def test_fhp3_extends_fhp2_below_mass_four():
    for chi in (0, 1):
        T2, T3 = table("FHP-II", chi), table("FHP-III", chi)
        for s in range(128):
            if T2[s] != s:
                assert mass(s) <= 3
                assert T3[s] == T2[s]


def test_fhp3_head_on_pair_with_spectator_turns_like_fhp2():
    # pair {0, 3} with a spectator at 5: chi = 1 turns the pair by +60
    # degrees, as FHP-II turns a lone pair; the spectator stays
    T1, T0 = table("FHP-III", 1), table("FHP-III", 0)
    assert T1[bits(0, 3, 5)] == bits(1, 4, 5)
    assert table("FHP-II", 1)[bits(0, 3)] == bits(1, 4)
    # the class's third member: the spectator's two neighbours plus a rest
    # particle; chi = 0 runs the cycle backwards
    assert T1[bits(1, 4, 5)] == bits(0, 4, rest=True)
    assert T0[bits(0, 3, 5)] == bits(0, 4, rest=True)


def test_fhp1_rest_is_a_spectator():
    for chi in (0, 1):
        T1, T2 = table("FHP-I", chi), table("FHP-II", chi)
        for s in range(128):
            assert (T1[s] ^ s) & 64 == 0
            # without the rest bit's role FHP-I keeps only FHP-II's head-on
            # pairs and triples
            if T1[s] != s and (s & 63) in (bits(0, 3), bits(1, 4), bits(2, 5)):
                assert T1[s] == T2[s]
        # the triple exchanges whatever the rest bit (FHP-II needs it empty)
        assert T1[bits(0, 2, 4, rest=True)] == bits(1, 3, 5, rest=True)
        assert T2[bits(0, 2, 4, rest=True)] == bits(0, 2, 4, rest=True)


@pytest.mark.parametrize("rules", [oracle.RULES_FHP1, oracle.RULES_FHP3])
def test_dynamics_conserve_on_torus(rules):
    W, H = 128, 16
    s = oracle.init(W, H, seed=5, fill=0.45)
    g0 = oracle.observe_global(s)
    for t in range(12):
        s, _ = oracle.step(s, t, seed=5, rules=rules)
    g = oracle.observe_global(s)
    assert (g["mass"], g["px"], g["py"]) == (g0["mass"], g0["px"], g0["py"])
    # the rule sets differ in what they change, not in what they conserve
    s2, _ = oracle.run(oracle.init(W, H, seed=5, fill=0.45), 0, 12, seed=5)
    assert not np.array_equal(s, s2)


def test_unknown_rule_set_rejected():
    with pytest.raises(ValueError):
        oracle.rule_table(3, 0)
    with pytest.raises(ValueError):
        oracle.step(np.zeros((2, 64), dtype=np.uint8), 0, 1, rules=7)
