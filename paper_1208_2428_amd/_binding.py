"""ctypes binding of ``libfhp.so`` (the C ABI in ``include/fhp.h``).

Argument marshalling only: every step of the dynamics runs in the library's
HIP kernels.  PyTorch provides the device workspace and the HIP stream.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

from . import build as _build

ABI_VERSION = 1
MAX_DEPTH = 5
BATCH_MAX_DEPTH = 5

OK, E_INVAL, E_NOMEM, E_DEVICE, E_STATE, E_BUSY = 0, -1, -2, -3, -4, -5
WALLS_NONE, WALLS_CHANNEL = 0, 1
CHIR_HASH, CHIR_ZERO, CHIR_ONE = 0, 1, 2
RULES_FHP2, RULES_FHP1, RULES_FHP3 = 0, 1, 2
OBS_GLOBAL, OBS_BLOCKS, OBS_DIGEST, OBS_ROWS = 0, 1, 2, 3

_ERRNAMES = {E_INVAL: "FHP_E_INVAL", E_NOMEM: "FHP_E_NOMEM", E_DEVICE: "FHP_E_DEVICE",
             E_STATE: "FHP_E_STATE", E_BUSY: "FHP_E_BUSY"}


class FhpError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_ERRNAMES.get(code, code)}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [
        ("abi_version", ctypes.c_uint32),
        ("width", ctypes.c_uint32),
        ("height", ctypes.c_uint32),
        ("walls", ctypes.c_uint32),
        ("chirality", ctypes.c_uint32),
        ("rules", ctypes.c_uint32),
        ("seed", ctypes.c_uint64),
        ("fill", ctypes.c_double),
        ("force_rate", ctypes.c_double),
        ("solid", ctypes.POINTER(ctypes.c_uint8)),
    ]


_lib = None

_SIGNATURES = {
    "fhp_last_error": (ctypes.c_char_p, []),
    "fhp_workspace_bytes": (ctypes.c_int, [ctypes.POINTER(Params), ctypes.POINTER(ctypes.c_size_t)]),
    "fhp_create": (ctypes.c_int, [ctypes.POINTER(Params), ctypes.c_void_p, ctypes.c_size_t,
                                  ctypes.c_void_p, ctypes.POINTER(ctypes.c_void_p)]),
    "fhp_set_depth": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32]),
    "fhp_get_depth": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint32)]),
    "fhp_set_band": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32]),
    "fhp_get_band": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint32)]),
    "fhp_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64]),
    "fhp_observe": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_uint32, ctypes.c_void_p,
                                   ctypes.c_size_t]),
    "fhp_get_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t]),
    "fhp_set_state": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                     ctypes.c_uint64]),
    "fhp_time": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64)]),
    "fhp_sync": (ctypes.c_int, [ctypes.c_void_p]),
    "fhp_destroy": (None, [ctypes.c_void_p]),
    "fhp_batch_workspace_bytes": (ctypes.c_int, [ctypes.POINTER(Params), ctypes.c_uint32,
                                                 ctypes.POINTER(ctypes.c_size_t)]),
    "fhp_batch_create": (ctypes.c_int, [ctypes.POINTER(Params), ctypes.c_uint32, ctypes.c_void_p,
                                        ctypes.c_size_t, ctypes.c_void_p,
                                        ctypes.POINTER(ctypes.c_void_p)]),
    "fhp_batch_set_tiling": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32,
                                            ctypes.c_uint32, ctypes.c_uint32]),
    "fhp_batch_set_graph": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    "fhp_batch_step": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint64]),
    "fhp_batch_member": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32,
                                        ctypes.POINTER(ctypes.c_void_p)]),
    "fhp_batch_sync": (ctypes.c_int, [ctypes.c_void_p]),
    "fhp_batch_destroy": (None, [ctypes.c_void_p]),
    "fhp_pool_workspace_bytes": (ctypes.c_int, [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_size_t,
                                                ctypes.POINTER(ctypes.c_size_t)]),
    "fhp_pool_create": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_size_t, ctypes.c_uint32,
                                       ctypes.c_uint32, ctypes.c_void_p,
                                       ctypes.POINTER(ctypes.c_void_p)]),
    "fhp_pool_set_rules": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32]),
    "fhp_pool_set_tiling": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32,
                                           ctypes.c_uint32]),
    "fhp_pool_admit": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(Params), ctypes.c_uint64,
                                      ctypes.POINTER(ctypes.c_uint32)]),
    "fhp_pool_tick": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32]),
    "fhp_pool_done": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint32),
                                     ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint32)]),
    "fhp_pool_result": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32,
                                       ctypes.c_void_p, ctypes.c_size_t]),
    "fhp_pool_collect": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint32,
                                        ctypes.c_void_p, ctypes.c_size_t]),
    "fhp_pool_collected": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32,
                                          ctypes.POINTER(ctypes.c_int)]),
    "fhp_pool_member": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32,
                                       ctypes.POINTER(ctypes.c_void_p)]),
    "fhp_pool_release": (ctypes.c_int, [ctypes.c_void_p, ctypes.c_uint32]),
    "fhp_pool_usage": (ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint32),
                                      ctypes.POINTER(ctypes.c_size_t),
                                      ctypes.POINTER(ctypes.c_size_t)]),
    "fhp_pool_sync": (ctypes.c_int, [ctypes.c_void_p]),
    "fhp_pool_destroy": (None, [ctypes.c_void_p]),
    "fhp_step_noalloc": (ctypes.c_int, [ctypes.POINTER(Params), ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint64,
                                        ctypes.c_uint32, ctypes.c_void_p]),
    "fhp_calib_pass": (ctypes.c_int, [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                      ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64,
                                      ctypes.c_uint32, ctypes.c_uint32, ctypes.c_void_p]),
    "fhp_calib_flat": (ctypes.c_int, [ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                      ctypes.c_uint32, ctypes.POINTER(ctypes.c_uint32),
                                      ctypes.c_void_p]),
}

CALIB_COPY, CALIB_READ, CALIB_WRITE = 0, 1, 2

NOALLOC_MAX_STATE_BYTES = 64 << 20


def lib_path() -> str:
    return _build.LIB_PATH


def load():
    """Loads the HIP library; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    path = lib_path()
    if not os.path.exists(path):
        raise RuntimeError(
            f"{path} is missing: build the HIP library first "
            "(python -c 'import __graft_entry__ as g; g.build()')")
    # torch ships its own HIP runtime under the same soname (libamdhip64.so.7)
    # as the system one the library links; whichever is loaded first serves
    # the whole process.  Loading torch first keeps the library on the runtime
    # that owns torch's device memory and streams.
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    for name, (res, args) in _SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(rc: int) -> None:
    if rc != OK:
        msg = load().fhp_last_error()
        raise FhpError(rc, msg.decode() if msg else "")


def make_params(width, height, seed=0, fill=0.0, force_rate=0.0, walls=False,
                chirality=CHIR_HASH, solid=None, rules=RULES_FHP2):
    """Returns (Params, keepalive) where keepalive holds the mask buffer."""
    p = Params()
    p.abi_version = ABI_VERSION
    p.width, p.height = int(width), int(height)
    p.walls = WALLS_CHANNEL if walls else WALLS_NONE
    p.chirality = int(chirality)
    p.rules = int(rules)
    p.seed = int(seed) & (2**64 - 1)
    p.fill = float(fill)
    p.force_rate = float(force_rate)
    keep = None
    if solid is not None:
        keep = np.ascontiguousarray(solid, dtype=np.uint8)
        if keep.shape != (height, width):
            raise ValueError(f"solid mask must have shape ({height}, {width})")
        p.solid = keep.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    return p, keep


def workspace_bytes(params: Params) -> int:
    n = ctypes.c_size_t(0)
    check(load().fhp_workspace_bytes(ctypes.byref(params), ctypes.byref(n)))
    return int(n.value)
