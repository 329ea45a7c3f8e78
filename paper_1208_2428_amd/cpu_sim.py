"""ctypes binding of the host bit-plane stepper ``libfhpcpu.so``
(``include/fhp_cpu.h``): the FHP time step on the CPU's cores and SIMD units,
the counterpart of the paper's vectorised, threaded CPU codes (arXiv:1208.2428,
Sec. 3.1, Table 1).  It is a separate engine for CPU comparisons, not a
fallback of the GPU library.  Argument marshalling only."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(PKG, "cpu", "fhp_cpu.c")
LIB_PATH = os.path.join(PKG, "libfhpcpu.so")
INCLUDE = os.path.join(os.path.dirname(PKG), "include")

_lib = None


def build() -> str:
    """Compiles the stepper with gcc (-O3, OpenMP; AVX-512 and AVX2 versions of
    the update loop are picked at run time from the CPU's features)."""
    tmp = LIB_PATH + ".tmp%d" % os.getpid()
    subprocess.run(["gcc", "-O3", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wno-psabi",
                    "-I", INCLUDE, "-o", tmp, SRC, "-lm"], check=True)
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built (python -c 'import __graft_entry__ as g; g.build()')")
    lib = ctypes.CDLL(LIB_PATH)
    vp, u8p = ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint8)
    sig = {
        "fhpcpu_last_error": (ctypes.c_char_p, []),
        "fhpcpu_create": (ctypes.c_int, [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64,
                                         ctypes.c_double, ctypes.c_double, ctypes.c_int, u8p,
                                         ctypes.POINTER(vp)]),
        "fhpcpu_step": (ctypes.c_int, [vp, ctypes.c_uint64, ctypes.c_int]),
        "fhpcpu_get_state": (ctypes.c_int, [vp, u8p, ctypes.c_size_t]),
        "fhpcpu_set_state": (ctypes.c_int, [vp, u8p, ctypes.c_size_t, ctypes.c_uint64]),
        "fhpcpu_time": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_uint64)]),
        "fhpcpu_digest": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_uint64)]),
        "fhpcpu_isa": (ctypes.c_char_p, []),
        "fhpcpu_destroy": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype, f.argtypes = res, args
    _lib = lib
    return lib


def _check(rc: int) -> None:
    if rc != 0:
        raise RuntimeError(f"fhpcpu error {rc}: {load().fhpcpu_last_error().decode()}")


def isa() -> str:
    return load().fhpcpu_isa().decode()


def _u8(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))


class CpuSim:
    """``CpuSim(W, H, seed=..., fill=..., force_rate=..., walls=..., solid=mask)``
    on the host; ``step(n, threads)`` advances it on `threads` cores."""

    def __init__(self, width: int, height: int, seed: int = 0, fill: float = 0.0,
                 force_rate: float = 0.0, walls: bool = False, solid: np.ndarray | None = None):
        lib = load()
        self.width, self.height = int(width), int(height)
        mask = None
        if solid is not None:
            mask = np.ascontiguousarray(solid, dtype=np.uint8)
            if mask.shape != (self.height, self.width):
                raise ValueError("solid must have shape (H, W)")
        h = ctypes.c_void_p()
        _check(lib.fhpcpu_create(self.width, self.height, seed & (2**64 - 1), float(fill),
                                 float(force_rate), int(bool(walls)),
                                 _u8(mask) if mask is not None else None, ctypes.byref(h)))
        self._h, self._lib = h, lib

    def step(self, n: int = 1, threads: int = 0) -> None:
        _check(self._lib.fhpcpu_step(self._h, int(n), int(threads)))

    @property
    def t(self) -> int:
        v = ctypes.c_uint64()
        _check(self._lib.fhpcpu_time(self._h, ctypes.byref(v)))
        return int(v.value)

    def get_state(self) -> np.ndarray:
        out = np.empty((self.height, self.width), dtype=np.uint8)
        _check(self._lib.fhpcpu_get_state(self._h, _u8(out), out.nbytes))
        return out

    def set_state(self, state: np.ndarray, t: int = 0) -> None:
        st = np.ascontiguousarray(state, dtype=np.uint8)
        if st.shape != (self.height, self.width):
            raise ValueError("state must have shape (H, W)")
        _check(self._lib.fhpcpu_set_state(self._h, _u8(st), st.nbytes, int(t)))

    def digest(self) -> int:
        v = ctypes.c_uint64()
        _check(self._lib.fhpcpu_digest(self._h, ctypes.byref(v)))
        return int(v.value)

    def close(self) -> None:
        if self._h is not None:
            self._lib.fhpcpu_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
