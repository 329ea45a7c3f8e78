"""Flow observables on the GPU: the row sums equal the oracle's, the
time-averaged channel profile equals the one computed from the oracle's
states, and a larger forced channel relaxes to the plane Poiseuille profile
(the channel set-up of arXiv:1208.2428, Sec. 2)."""
import numpy as np
import pytest

import oracle
from paper_1208_2428_amd import Sim, flow
from paper_1208_2428_amd import workloads as WL

pytestmark = pytest.mark.gpu

THREADS = oracle.default_threads()


@pytest.mark.parametrize("W,H", [(64, 2), (192, 10), (1024, 70), (4096, 6)])
def test_row_sums_match_oracle(W, H):
    rng = np.random.default_rng(W + H)
    st = WL.random_states(rng, H, W, p=0.4)
    st |= ((rng.random((H, W)) < 0.1).astype(np.uint8) << 7)
    s = Sim(W, H, seed=3, force_rate=1e-2)
    s.set_state(st, 0)
    s.step(7)
    ref, _ = oracle.run(st, 0, 7, 3, 1e-2, threads=THREADS)
    np.testing.assert_array_equal(s.observe_rows(), oracle.observe_rows(ref))
    s.close()


def test_channel_profile_matches_oracle_states():
    W, H, f, seed = 512, 34, 2e-3, 3
    s = Sim(W, H, seed=seed, fill=0.2, force_rate=f, walls=True)
    u = flow.channel_profile(s, steps=600, every=50, start=300)
    s.close()
    st = oracle.init(W, H, seed, 0.2, walls=True)
    st, _ = oracle.run(st, 0, 300, seed, f, threads=THREADS)
    acc = np.zeros(H)
    for k in range(12):
        st, _ = oracle.run(st, 300 + 50 * k, 50, seed, f, threads=THREADS)
        acc += flow.row_velocity(oracle.observe_rows(st))
    np.testing.assert_array_equal(u, acc / 12)


def test_forced_channel_relaxes_to_poiseuille():
    # 130 rows: the momentum diffusion time H^2 / nu is a few 10^4 steps
    W, H = 2048, 130
    s = Sim(W, H, seed=11, fill=0.2, force_rate=5e-4, walls=True)
    u = flow.channel_profile(s, steps=40000, every=200, start=60000)
    s.close()
    fit = flow.poiseuille_fit(u)
    print("poiseuille", fit, flush=True)
    assert fit["r2"] > 0.99
    assert abs(fit["vertex"] - (H - 1) / 2) < 2.0
    assert fit["symmetry"] > 0.98
    assert fit["peak"] > 0.05 and fit["curvature"] < 0
    assert abs(fit["slip"][0]) < 0.15 and abs(fit["slip"][1]) < 0.15


def test_darcy_flow_through_obstacles_is_linear_in_the_force():
    # a dense field of small disks (radius 4..8 on 20% of the nodes: pores of
    # some 20 nodes, which settle within a few thousand steps) driven gently:
    # in this Darcy regime the mean velocity is proportional to the force
    W = H = 1024
    mask = WL.porous_mask(W, H, seed=5, rmin=4, rmax=8, frac=0.2)
    means = []
    for f in (5e-5, 1e-4):
        s = Sim(W, H, seed=13, fill=0.3, force_rate=f, solid=mask)
        means.append(flow.mean_velocity(s, steps=10000, every=200, start=10000))
        s.close()
    print("darcy", means, flush=True)
    assert means[0] > 0 and means[1] > 0
    assert 1.7 < means[1] / means[0] < 2.3


def test_permeability_chain_matches_oracle_states():
    """Superficial velocity, body force and the channel viscosity computed
    from the GPU's observables equal the ones computed from the oracle's
    states, float for float (a small obstacle field and a small channel)."""
    W, H, f, seed = 256, 96, 3e-3, 17
    mask = WL.porous_mask(W, H, seed=8, rmin=3, rmax=6, frac=0.15)
    s = Sim(W, H, seed=seed, fill=0.3, force_rate=f, solid=mask)
    got = flow.darcy_sums(s, steps=300, every=50, start=100)
    s.close()
    st = oracle.init(W, H, seed, 0.3, mask=mask)
    st, _ = oracle.run(st, 0, 100, seed, f, threads=THREADS)
    qs, gs = [], []
    for k in range(6):
        st, _ = oracle.run(st, 100 + 50 * k, 50, seed, f, threads=THREADS)
        glob = oracle.observe_global(st)
        qs.append(flow.superficial_velocity(glob, W * H))
        gs.append(flow.body_force(glob, W * H, f))
    assert got["q"] == float(np.mean(qs)) and got["g"] == float(np.mean(gs))

    W, H = 512, 34
    s = Sim(W, H, seed=seed, fill=0.3, force_rate=f, walls=True)
    nu = flow.channel_viscosity(s, steps=400, every=50, start=200)
    s.close()
    st = oracle.init(W, H, seed, 0.3, walls=True)
    st, _ = oracle.run(st, 0, 200, seed, f, threads=THREADS)
    acc, gs = np.zeros(H), []
    for k in range(8):
        st, _ = oracle.run(st, 200 + 50 * k, 50, seed, f, threads=THREADS)
        acc += flow.row_velocity(oracle.observe_rows(st))
        gs.append(flow.body_force(oracle.observe_global(st), W * H, f))
    np.testing.assert_equal(nu["nu"], flow.viscosity(acc / 8, float(np.mean(gs))))


def test_permeability_scales_with_obstacle_size_squared():
    """Darcy permeability of random disks at one solid fraction (20%) with
    every length doubled: about four times larger (k ~ R^2 at fixed
    porosity), measured with the full chain (channel viscosity at the same
    density, body force, superficial velocity)."""
    W = H = 1024
    f = 1e-3
    ch = Sim(2048, 66, seed=3, fill=0.3, force_rate=f, walls=True)
    nu = flow.channel_viscosity(ch, steps=20000, every=200, start=20000)["nu"]
    ch.close()
    ks = []
    for seed, (rmin, rmax) in ((51, (4, 8)), (52, (8, 16))):
        mask = WL.porous_mask(W, H, seed=seed, rmin=rmin, rmax=rmax, frac=0.2)
        s = Sim(W, H, seed=seed, fill=0.3, force_rate=f, solid=mask)
        d = flow.darcy_sums(s, steps=6000, every=100, start=4000)
        s.close()
        ks.append(flow.permeability(d["q"], d["g"], nu))
    print("viscosity", nu, "permeabilities", ks, flush=True)
    assert 0.05 < nu < 2.0
    assert ks[0] > 0 and 3.0 < ks[1] / ks[0] < 5.5
