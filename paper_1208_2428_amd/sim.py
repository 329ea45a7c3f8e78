"""Python front end of one FHP simulation on a GPU.

The lattice lives in a caller-visible torch ``uint8`` workspace on the device;
all work runs in the HIP library on the given torch stream.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _binding as B


def _stream_handle(stream, device):
    if stream is None:
        stream = torch.cuda.current_stream(device)
    return ctypes.c_void_p(stream.cuda_stream)


class Sim:
    """One lattice: ``Sim(W, H, seed=..., fill=..., force_rate=..., walls=...,
    solid=mask)``.  See ``include/fhp.h`` for the model and the readings of
    the paper it fixes."""

    def __init__(self, width: int, height: int, seed: int = 0, fill: float = 0.0,
                 force_rate: float = 0.0, walls: bool = False, chirality: int = B.CHIR_HASH,
                 solid: np.ndarray | None = None, device=None, stream=None, depth: int = 0,
                 band: int = 0, rules: int = B.RULES_FHP2):
        lib = B.load()
        if not torch.cuda.is_available():
            raise RuntimeError("the FHP library needs a ROCm GPU (torch.cuda is unavailable)")
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None \
            else torch.device(device)
        self.width, self.height = int(width), int(height)
        self.rules, self.force_rate, self.walls = int(rules), float(force_rate), bool(walls)
        self.has_mask = solid is not None
        params, keep = B.make_params(width, height, seed, fill, force_rate, walls, chirality, solid,
                                     rules)
        nbytes = B.workspace_bytes(params)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self._stream = stream
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            B.check(lib.fhp_create(ctypes.byref(params), ctypes.c_void_p(self.workspace.data_ptr()),
                                   nbytes, _stream_handle(stream, self.device), ctypes.byref(h)))
        del keep
        self._h = h
        self._lib = lib
        if depth:
            self.depth = depth
        if band:
            self.set_band(band)

    # ---------------------------------------------------------------- control
    def _handle(self):
        if self._h is None:
            raise RuntimeError("simulation is closed")
        return self._h

    def step(self, n: int = 1) -> None:
        B.check(self._lib.fhp_step(self._handle(), int(n)))

    @property
    def depth(self) -> int:
        k = ctypes.c_uint32()
        B.check(self._lib.fhp_get_depth(self._handle(), ctypes.byref(k)))
        return int(k.value)

    @depth.setter
    def depth(self, k: int) -> None:
        B.check(self._lib.fhp_set_depth(self._handle(), int(k)))

    def set_band(self, rows: int) -> None:
        B.check(self._lib.fhp_set_band(self._handle(), int(rows)))

    @property
    def band(self) -> int:
        """Rows per band of the blocked kernel (the default resolved)."""
        v = ctypes.c_uint32(0)
        B.check(self._lib.fhp_get_band(self._handle(), ctypes.byref(v)))
        return int(v.value)

    @property
    def t(self) -> int:
        v = ctypes.c_uint64()
        B.check(self._lib.fhp_time(self._handle(), ctypes.byref(v)))
        return int(v.value)

    def sync(self) -> None:
        B.check(self._lib.fhp_sync(self._handle()))

    def close(self) -> None:
        if self._h is not None:
            self._lib.fhp_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ------------------------------------------------------------ observables
    def observe_global(self) -> dict:
        out = np.zeros(11, dtype=np.int64)
        B.check(self._lib.fhp_observe(self._handle(), B.OBS_GLOBAL, 0,
                                      out.ctypes.data_as(ctypes.c_void_p), out.nbytes))
        v = [int(x) for x in out]
        return {"mass": v[0], "px": v[1], "py": v[2], "channels": v[3:10], "solid": v[10]}

    def observe_rows(self) -> np.ndarray:
        """int64 (H, 3): (rho, p_x, p_y) summed over each row."""
        out = np.zeros((self.height, 3), dtype=np.int64)
        B.check(self._lib.fhp_observe(self._handle(), B.OBS_ROWS, 0,
                                      out.ctypes.data_as(ctypes.c_void_p), out.nbytes))
        return out

    def observe_blocks(self, b: int) -> np.ndarray:
        out = np.zeros(((self.height + b - 1) // b, (self.width + b - 1) // b, 3), dtype=np.int32)
        B.check(self._lib.fhp_observe(self._handle(), B.OBS_BLOCKS, int(b),
                                      out.ctypes.data_as(ctypes.c_void_p), out.nbytes))
        return out

    def digest(self) -> int:
        out = np.zeros(1, dtype=np.uint64)
        B.check(self._lib.fhp_observe(self._handle(), B.OBS_DIGEST, 0,
                                      out.ctypes.data_as(ctypes.c_void_p), out.nbytes))
        return int(out[0])

    def get_state(self) -> np.ndarray:
        out = np.empty((self.height, self.width), dtype=np.uint8)
        B.check(self._lib.fhp_get_state(self._handle(), out.ctypes.data_as(ctypes.c_void_p),
                                        out.nbytes))
        return out

    def set_state(self, state: np.ndarray, t: int = 0) -> None:
        state = np.ascontiguousarray(state, dtype=np.uint8)
        if state.shape != (self.height, self.width):
            raise ValueError(f"state must have shape ({self.height}, {self.width})")
        B.check(self._lib.fhp_set_state(self._handle(), state.ctypes.data_as(ctypes.c_void_p),
                                        state.nbytes, int(t)))
