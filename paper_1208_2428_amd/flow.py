"""Flow observables of forced lattice-gas flows (the set-ups of arXiv:1208.2428,
Sec. 2 and Sec. 4: a channel with walls, or an obstacle field, driven by the
horizontal forcing).

All sums come from the GPU (``fhp_observe`` with FHP_OBS_ROWS or
FHP_OBS_GLOBAL); this module only averages them over time and fits them.

Units: a particle moves one lattice constant per step, so the mean velocity
of a row is p_x / (2 rho) lattice constants per step (p_x is counted in
units of 1/2)."""
from __future__ import annotations

import numpy as np


def row_velocity(rows: np.ndarray) -> np.ndarray:
    """Mean x velocity of each row from FHP_OBS_ROWS sums (0 for empty rows)."""
    rho = rows[:, 0].astype(np.float64)
    return np.where(rho > 0, rows[:, 1] / (2.0 * np.maximum(rho, 1.0)), 0.0)


def channel_profile(sim, steps: int, every: int, start: int = 0) -> np.ndarray:
    """Advances `sim` by `start` steps, then by `steps` more, and returns the
    mean x velocity of every row averaged over the states every `every`
    steps of the second stretch."""
    if start:
        sim.step(start)
    acc = np.zeros(sim.height)
    n = 0
    for _ in range(max(1, steps // every)):
        sim.step(every)
        acc += row_velocity(sim.observe_rows())
        n += 1
    return acc / n


def poiseuille_fit(u: np.ndarray) -> dict:
    """Fits a parabola to the profile of the fluid rows 1 .. H-2 of a channel
    whose rows 0 and H-1 are walls.  Returns the fit quality (r2), the vertex
    row, the peak velocity, the velocity next to each wall relative to the
    peak (slip), and the curvature u'' (lattice constants per step per row^2)."""
    y = np.arange(1, len(u) - 1, dtype=np.float64)
    v = np.asarray(u[1:-1], dtype=np.float64)
    c = np.polyfit(y, v, 2)
    fit = np.polyval(c, y)
    ss = ((v - v.mean()) ** 2).sum()
    r2 = 1.0 - ((v - fit) ** 2).sum() / ss if ss > 0 else 0.0
    vertex = -c[1] / (2.0 * c[0]) if c[0] != 0 else float("nan")
    peak = float(np.polyval(c, vertex)) if np.isfinite(vertex) else float(v.max())
    return {"r2": float(r2), "vertex": float(vertex), "peak": peak,
            "slip": (float(v[0] / peak), float(v[-1] / peak)) if peak else (0.0, 0.0),
            "curvature": float(2.0 * c[0]),
            "symmetry": float(np.corrcoef(v, v[::-1])[0, 1])}


def mean_velocity(sim, steps: int, every: int, start: int = 0) -> float:
    """Mean x velocity of all particles, averaged over time (for Darcy's law in
    an obstacle field: at small forcing it grows linearly with the force)."""
    if start:
        sim.step(start)
    acc, n = 0.0, 0
    for _ in range(max(1, steps // every)):
        sim.step(every)
        g = sim.observe_global()
        acc += g["px"] / (2.0 * g["mass"]) if g["mass"] else 0.0
        n += 1
    return acc / n
