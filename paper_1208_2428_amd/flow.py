"""Flow observables of forced lattice-gas flows (the set-ups of arXiv:1208.2428,
Sec. 2 and Sec. 4: a channel with walls, or an obstacle field, driven by the
horizontal forcing).

All sums come from the GPU (``fhp_observe`` with FHP_OBS_ROWS or
FHP_OBS_GLOBAL); this module only averages them over time and fits them.

Units: a particle moves one lattice constant per step, so the mean velocity
of a row is p_x / (2 rho) lattice constants per step (p_x is counted in
units of 1/2).  Rows are sqrt(3)/2 lattice constants apart.

Permeability (Darcy's law for a body force): in steady flow through an
obstacle field the superficial velocity q (momentum per unit area over the
mass density of the fluid) is q = k g / nu, with g the force per unit mass
and nu the kinematic viscosity of the lattice gas at that density.  nu comes
from a forced channel at the same density (plane Poiseuille flow:
u'' = -g / nu across the channel), q and g from the obstacle field, and
k = nu q / g, in lattice constants squared."""
from __future__ import annotations

import math

import numpy as np

ROW_PITCH = math.sqrt(3.0) / 2.0  # distance between rows (lattice constants)


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


def coin_rate(force_rate: float) -> float:
    """Per-node forcing rate the dynamics applies: floor(f * 2^38) / 2^38."""
    return math.floor(force_rate * 2.0 ** 38) / 2.0 ** 38


def body_force(glob: dict, nodes: int, force_rate: float) -> float:
    """Force per unit mass g (lattice constants per step^2) that the forcing
    exerts, from global sums (FHP_OBS_GLOBAL) of a lattice of `nodes` nodes.

    Each step a fluid node with channel 5 (W) occupied and channel 2 (E)
    empty has the W-mover turned into an E-mover with probability p = the
    coin rate, adding 2 to its x momentum.  Taking the channel occupations of
    the fluid nodes as independent (their equilibrium distribution at rest
    factorises; at the small velocities used here the correction is second
    order), the force per fluid node is 2 p d_5 (1 - d_2) and the mass per
    fluid node is sum_c d_c, with d_c the channel occupations of the fluid
    nodes (the few particles standing on solid nodes in the bounce-back step
    are counted with them)."""
    fluid = nodes - int(glob["solid"])
    if fluid <= 0 or glob["mass"] <= 0:
        return 0.0
    d = np.asarray(glob["channels"], dtype=np.float64) / fluid
    return 2.0 * coin_rate(force_rate) * d[5] * (1.0 - d[2]) / d.sum()


def superficial_velocity(glob: dict, nodes: int) -> float:
    """x momentum per node over the mass per fluid node: the Darcy (superficial)
    velocity, lattice constants per step."""
    fluid = nodes - int(glob["solid"])
    if glob["mass"] <= 0:
        return 0.0
    return (glob["px"] / 2.0) / glob["mass"] * fluid / nodes


def viscosity(u: np.ndarray, g: float) -> float:
    """Kinematic viscosity from a channel profile (rows 0 and H-1 walls):
    nu = -g / u'' with u'' the fitted curvature per row^2 converted to
    physical rows (ROW_PITCH apart)."""
    curv = poiseuille_fit(u)["curvature"] / ROW_PITCH ** 2
    return -g / curv if curv < 0 else float("nan")


def darcy_sums(sim, steps: int, every: int, start: int = 0) -> dict:
    """Advances `sim` by `start` steps, then averages the superficial velocity
    q and the body force g over the states every `every` steps of `steps`
    more: {"q", "g", "samples"}."""
    if start:
        sim.step(start)
    nodes = sim.width * sim.height
    qs, gs = [], []
    for _ in range(max(1, steps // every)):
        sim.step(every)
        glob = sim.observe_global()
        qs.append(superficial_velocity(glob, nodes))
        gs.append(body_force(glob, nodes, sim.force_rate))
    return {"q": float(np.mean(qs)), "g": float(np.mean(gs)), "samples": len(qs)}


def channel_viscosity(sim, steps: int, every: int, start: int = 0) -> dict:
    """Viscosity of the lattice gas from a forced channel `sim` (walls):
    profile and body force averaged as in channel_profile and darcy_sums."""
    if start:
        sim.step(start)
    nodes = sim.width * sim.height
    acc = np.zeros(sim.height)
    gs = []
    n = max(1, steps // every)
    for _ in range(n):
        sim.step(every)
        acc += row_velocity(sim.observe_rows())
        gs.append(body_force(sim.observe_global(), nodes, sim.force_rate))
    u = acc / n
    g = float(np.mean(gs))
    fit = poiseuille_fit(u)
    return {"nu": viscosity(u, g), "g": g, "r2": fit["r2"], "peak": fit["peak"]}


def permeability(q: float, g: float, nu: float) -> float:
    """Darcy permeability k = nu q / g (lattice constants squared)."""
    return nu * q / g if g > 0 else float("nan")
