"""Physics pin of the oracle beyond conservation: a channel with walls driven
by the horizontal forcing (arXiv:1208.2428, Sec. 2: no-slip walls top and
bottom, periodic in x, forcing that turns W-movers into E-movers) develops
the plane Poiseuille profile of a viscous fluid: a parabola across the
channel, symmetric about its middle, close to zero at the walls, flowing in
+x, with a velocity that grows with the force.  A dropped bounce-back, a
wrong forcing direction, broken collisions (no viscosity) or a wrong row
shift each break one of these."""
import numpy as np

import oracle

THREADS = oracle.default_threads()


def profile(W, H, f, steps, start, every, seed=3):
    s = oracle.init(W, H, seed, 0.2, walls=True)
    s, _ = oracle.run(s, 0, start, seed, f, threads=THREADS)
    acc, n, t = np.zeros(H), 0, start
    while t < start + steps:
        s, _ = oracle.run(s, t, every, seed, f, threads=THREADS)
        t += every
        r = oracle.observe_rows(s)
        acc += r[:, 1] / (2.0 * np.maximum(r[:, 0], 1))
        n += 1
    return acc / n


def fit(u):
    y = np.arange(1, len(u) - 1, dtype=float)
    v = u[1:-1]
    c = np.polyfit(y, v, 2)
    r2 = 1 - ((v - np.polyval(c, y)) ** 2).sum() / ((v - v.mean()) ** 2).sum()
    vertex = -c[1] / (2 * c[0])
    return r2, vertex, np.polyval(c, vertex), v


def test_forced_channel_develops_poiseuille_profile():
    W, H = 512, 34
    u = profile(W, H, 2e-3, steps=3000, start=3000, every=25)
    r2, vertex, peak, v = fit(u)
    assert r2 > 0.98
    assert abs(vertex - (H - 1) / 2) < 1.0          # symmetric about the middle row
    assert np.corrcoef(v, v[::-1])[0, 1] > 0.97
    assert peak > 0.1                               # flows in +x
    assert abs(v[0]) < 0.2 * peak and abs(v[-1]) < 0.2 * peak   # little slip at the walls
    # half the force, about half the flow (linear response, within noise and
    # the lattice gas's velocity-dependent corrections)
    u2 = profile(W, H, 1e-3, steps=3000, start=3000, every=25)
    ratio = peak / fit(u2)[2]
    assert 1.4 < ratio < 2.6


def test_no_force_no_flow():
    u = profile(256, 34, 0.0, steps=1000, start=500, every=25)
    assert np.abs(u[1:-1]).max() < 0.05


# ---------------------------------------------------------------- permeability
# The measurement chain of flow.py (body force, superficial velocity,
# viscosity, Darcy permeability), applied to the oracle's states.

from paper_1208_2428_amd import flow  # noqa: E402
from paper_1208_2428_amd import workloads as WL  # noqa: E402


def test_body_force_matches_counted_swaps():
    """The mean-field force per unit mass of flow.body_force against the
    exact momentum the forcing added: each swap turns a W-mover (p_x = -1)
    into an E-mover (+1), and the oracle counts the swaps."""
    W = H = 256
    f, seed = 2e-3, 9
    st = oracle.init(W, H, seed, 0.3)
    t, swaps, gs = 0, 0, []
    for _ in range(10):
        gs.append(flow.body_force(oracle.observe_global(st), W * H, f))
        st, s = oracle.run(st, t, 20, seed, f, threads=THREADS)
        t += 20
        swaps += s
    mass = oracle.observe_global(st)["mass"]
    counted = 2.0 * swaps / t / mass
    # ~4,850 swaps: 1.4% statistical error
    assert abs(np.mean(gs) / counted - 1.0) < 0.06, (np.mean(gs), counted)


def oracle_darcy(mask, f, seed, start, steps, every):
    H, W = mask.shape
    st = oracle.init(W, H, seed, 0.3, mask=mask)
    st, _ = oracle.run(st, 0, start, seed, f, threads=THREADS)
    t, qs, gs = start, [], []
    while t < start + steps:
        st, _ = oracle.run(st, t, every, seed, f, threads=THREADS)
        t += every
        g = oracle.observe_global(st)
        qs.append(flow.superficial_velocity(g, W * H))
        gs.append(flow.body_force(g, W * H, f))
    return float(np.mean(qs)), float(np.mean(gs))


def test_permeability_scales_with_obstacle_size_squared():
    """Darcy flow through random disks at one solid fraction: doubling every
    length of the geometry multiplies the permeability by about four
    (k ~ R^2 at fixed porosity, as in the Kozeny-Carman relation); the
    viscosity and body force cancel in the ratio, so the check pins the
    superficial velocity and the flow's linear (Darcy) regime."""
    W = H = 256
    f, seed = 2e-3, 21
    small = WL.porous_mask(W, H, seed=41, rmin=3, rmax=5, frac=0.2)
    large = WL.porous_mask(W, H, seed=42, rmin=6, rmax=10, frac=0.2)
    q1, g1 = oracle_darcy(small, f, seed, 600, 2400, 40)
    q2, g2 = oracle_darcy(large, f, seed, 1200, 2400, 40)
    assert q1 > 0 and q2 > 0
    ratio = (q2 / g2) / (q1 / g1)
    print("permeability ratio", ratio, q1, q2, flush=True)
    assert 2.5 < ratio < 7.0
