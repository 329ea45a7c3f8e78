"""Full-size parity: the GPU run of each named workload against the oracle's
digests and global observables recorded by tests/golden/make_golden.py
(the oracle stepped the same seeded initial state on the CPU).  Digests are
compared at every recorded step (every step up to 24, then every 12th, then
every 120th); fhp_step finishes a call that is not a multiple of the depth
with a shorter pass."""
import os

import pytest

from paper_1208_2428_amd import Sim
from paper_1208_2428_amd import workloads as WL

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def records(name):
    path = os.path.join(GOLDEN, f"digests_{name}.txt")
    if not os.path.exists(path):
        pytest.skip(f"no oracle digests for {name} yet ({path})")
    out = []
    with open(path) as fh:
        for line in fh:
            if line.startswith("#"):
                continue
            t, d, m, px, py, sw = line.split()
            out.append((int(t), int(d, 16), int(m), int(px), int(py)))
    return out


@pytest.mark.parametrize("name", ["channel-4096", "porous-16384"])
@pytest.mark.parametrize("depth", [1, 3, 4, 5])
def test_workload_matches_oracle_digests(name, depth):
    recs = records(name)
    wl = WL.WORKLOADS[name]
    print("golden", name, depth, len(recs), flush=True)
    sim = Sim(**wl.params(), solid=wl.mask(), depth=depth)
    t = 0
    for tr, digest, mass, px, py in recs:
        sim.step(tr - t)
        t = tr
        assert sim.digest() == digest, f"{name} depth {depth}: digest differs at t={tr}"
        g = sim.observe_global()
        assert (g["mass"], g["px"], g["py"]) == (mass, px, py), f"t={tr}"
    assert sim.t == recs[-1][0]
