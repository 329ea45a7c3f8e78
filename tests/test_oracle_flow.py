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
