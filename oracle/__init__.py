"""CPU oracle for the FHP lattice-gas time step -- TEST INFRASTRUCTURE ONLY.

Thin ctypes wrapper over ``fhp_oracle.c`` (plain C, one node at a time, one
byte per node).  Only the test suite, the smoke check and the CPU-baseline leg
of the benchmark may import this package; the GPU library never does, and the
two share no code.

State arrays are ``numpy.uint8`` of shape ``(H, W)`` in the paper's byte
layout (Sec. 2, Fig. 1): bits 0-5 moving particles, bit 6 rest particle,
bit 7 solid node.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fhp_oracle.c")
_LIB_PATH = os.path.join(_HERE, "libfhporacle.so")

CHIR_HASH, CHIR_ZERO, CHIR_ONE = 0, 1, 2
TAG_INIT, TAG_CHIR, TAG_FORCE = 1, 2, 3
RULES_FHP2, RULES_FHP1, RULES_FHP3 = 0, 1, 2

_lib = None


def build(force: bool = True) -> str:
    """Compiles the oracle with gcc (plain -O2, OpenMP over rows only)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.run(
            ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall",
             "-o", tmp, _SRC, "-lm"],
            check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    u8p = ctypes.POINTER(ctypes.c_uint8)
    i64p = ctypes.POINTER(ctypes.c_int64)
    i32p = ctypes.POINTER(ctypes.c_int32)
    lib.fhpo_hash.restype = ctypes.c_uint64
    lib.fhpo_hash.argtypes = [ctypes.c_uint64, ctypes.c_uint64]
    lib.fhpo_collision_table.restype = None
    lib.fhpo_collision_table.argtypes = [ctypes.c_int, u8p]
    lib.fhpo_rule_table.restype = ctypes.c_int
    lib.fhpo_rule_table.argtypes = [ctypes.c_int, ctypes.c_int, u8p]
    lib.fhpo_init.restype = ctypes.c_int
    lib.fhpo_init.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64,
                              ctypes.c_double, u8p, ctypes.c_int, u8p]
    lib.fhpo_step.restype = ctypes.c_int64
    lib.fhpo_step.argtypes = [u8p, u8p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64,
                              ctypes.c_uint64, ctypes.c_double, ctypes.c_int, ctypes.c_int]
    lib.fhpo_run.restype = ctypes.c_int
    lib.fhpo_run.argtypes = [u8p, u8p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64,
                             ctypes.c_uint64, ctypes.c_uint64, ctypes.c_double, ctypes.c_int,
                             ctypes.c_int, i64p]
    lib.fhpo_step_rules.restype = ctypes.c_int64
    lib.fhpo_step_rules.argtypes = [u8p, u8p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64,
                                    ctypes.c_uint64, ctypes.c_double, ctypes.c_int, ctypes.c_int,
                                    ctypes.c_int]
    lib.fhpo_run_rules.restype = ctypes.c_int
    lib.fhpo_run_rules.argtypes = [u8p, u8p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64,
                                   ctypes.c_uint64, ctypes.c_uint64, ctypes.c_double, ctypes.c_int,
                                   ctypes.c_int, ctypes.c_int, i64p]
    lib.fhpo_observe_global.restype = None
    lib.fhpo_observe_global.argtypes = [u8p, ctypes.c_uint32, ctypes.c_uint32, i64p]
    lib.fhpo_observe_rows.restype = None
    lib.fhpo_observe_rows.argtypes = [u8p, ctypes.c_uint32, ctypes.c_uint32, i64p]
    lib.fhpo_observe_blocks.restype = ctypes.c_int
    lib.fhpo_observe_blocks.argtypes = [u8p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                        i32p]
    lib.fhpo_digest.restype = ctypes.c_uint64
    lib.fhpo_digest.argtypes = [u8p, ctypes.c_uint32, ctypes.c_uint32]
    _lib = lib
    return lib


def _u8(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


def _check_state(state: np.ndarray) -> None:
    if state.dtype != np.uint8 or state.ndim != 2 or not state.flags.c_contiguous:
        raise ValueError("state must be a C-contiguous uint8 array of shape (H, W)")


def default_threads() -> int:
    """Every CPU this process may run on (its affinity set), capped by
    OMP_NUM_THREADS when that is set (a host's share of CPUs per GPU)."""
    try:
        n = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        n = os.cpu_count() or 1
    omp = os.environ.get("OMP_NUM_THREADS", "")
    if omp.isdigit() and int(omp) > 0:
        n = min(n, int(omp))
    return max(1, n)


def hash64(key: int, n: int) -> int:
    """H(key, n) = SplitMix64 output n+1 from state key."""
    return int(_load().fhpo_hash(key & (2**64 - 1), n & (2**64 - 1)))


def collision_table(chi: int) -> np.ndarray:
    out = np.zeros(128, dtype=np.uint8)
    _load().fhpo_collision_table(int(chi), _u8(out))
    return out


def rule_table(rules: int, chi: int) -> np.ndarray:
    """Collision table of rule set RULES_FHP2 / RULES_FHP1 / RULES_FHP3."""
    out = np.zeros(128, dtype=np.uint8)
    if _load().fhpo_rule_table(int(rules), int(chi), _u8(out)) != 0:
        raise ValueError("fhpo_rule_table: bad arguments")
    return out


def init(W: int, H: int, seed: int, fill: float, mask: np.ndarray | None = None,
         walls: bool = False) -> np.ndarray:
    state = np.empty((H, W), dtype=np.uint8)
    mptr = None
    if mask is not None:
        mask = np.ascontiguousarray(mask, dtype=np.uint8)
        if mask.shape != (H, W):
            raise ValueError("mask must have shape (H, W)")
        mptr = _u8(mask)
    rc = _load().fhpo_init(W, H, seed, float(fill), mptr, int(bool(walls)), _u8(state))
    if rc != 0:
        raise ValueError("fhpo_init: bad arguments")
    return state


def step(state: np.ndarray, t: int, seed: int, force_rate: float = 0.0,
         chir_mode: int = CHIR_HASH, threads: int = 1, rules: int = RULES_FHP2):
    """One step t -> t+1.  Returns (new_state, forcing swaps applied)."""
    _check_state(state)
    H, W = state.shape
    out = np.empty_like(state)
    r = _load().fhpo_step_rules(_u8(state), _u8(out), W, H, t, seed, float(force_rate),
                                int(chir_mode), int(rules), int(threads))
    if r < 0:
        raise ValueError("fhpo_step: bad arguments")
    return out, int(r)


def run(state: np.ndarray, t0: int, n: int, seed: int, force_rate: float = 0.0,
        chir_mode: int = CHIR_HASH, threads: int = 1, rules: int = RULES_FHP2):
    """n steps from time t0.  Returns (new_state, total forcing swaps)."""
    _check_state(state)
    H, W = state.shape
    cur = state.copy()
    tmp = np.empty_like(cur)
    swaps = ctypes.c_int64(0)
    rc = _load().fhpo_run_rules(_u8(cur), _u8(tmp), W, H, t0, n, seed, float(force_rate),
                                int(chir_mode), int(rules), int(threads), ctypes.byref(swaps))
    if rc != 0:
        raise ValueError("fhpo_run: bad arguments")
    return cur, int(swaps.value)


def observe_global(state: np.ndarray) -> dict:
    _check_state(state)
    H, W = state.shape
    out = (ctypes.c_int64 * 11)()
    _load().fhpo_observe_global(_u8(state), W, H, out)
    v = list(out)
    return {"mass": v[0], "px": v[1], "py": v[2], "channels": v[3:10], "solid": v[10]}


def observe_rows(state: np.ndarray) -> np.ndarray:
    """int64 (H, 3): (rho, p_x, p_y) summed over each row."""
    _check_state(state)
    H, W = state.shape
    out = np.zeros((H, 3), dtype=np.int64)
    _load().fhpo_observe_rows(_u8(state), W, H, out.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
    return out


def observe_blocks(state: np.ndarray, b: int) -> np.ndarray:
    _check_state(state)
    H, W = state.shape
    out = np.zeros(((H + b - 1) // b, (W + b - 1) // b, 3), dtype=np.int32)
    rc = _load().fhpo_observe_blocks(_u8(state), W, H, b,
                                     out.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
    if rc != 0:
        raise ValueError("fhpo_observe_blocks: bad arguments")
    return out


def digest(state: np.ndarray) -> int:
    _check_state(state)
    H, W = state.shape
    return int(_load().fhpo_digest(_u8(state), W, H))
