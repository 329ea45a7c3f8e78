"""Python front end of pools: continuous batching of simulation jobs in an
HBM arena (``fhp_pool_*`` in include/fhp.h)."""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _binding as B
from .batch import _MemberView


class Pool:
    """``Pool(arena_bytes, max_slots, max_bands)``: the arena is a torch uint8
    tensor on the device; jobs are admitted with ``admit`` (None when the pool
    is full), advanced with ``tick`` and read with ``result``."""

    def __init__(self, arena_bytes: int, max_slots: int = 256, max_bands: int = 1 << 16,
                 device=None, stream=None, depth: int = 0, band: int = 0,
                 group_threads: int = 0, rules: int = B.RULES_FHP2):
        lib = B.load()
        if not torch.cuda.is_available():
            raise RuntimeError("the FHP library needs a ROCm GPU (torch.cuda is unavailable)")
        self._lib = lib
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None \
            else torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        self.arena = torch.empty(int(arena_bytes), dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        B.check(lib.fhp_pool_create(ctypes.c_void_p(self.arena.data_ptr()), int(arena_bytes),
                                    int(max_slots), int(max_bands),
                                    ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h)))
        self._h = h
        self.max_slots = max_slots
        self._shapes = {}
        self._pinned = {}
        if depth or band or group_threads:
            B.check(lib.fhp_pool_set_tiling(h, int(depth), int(band), int(group_threads)))
        if rules != B.RULES_FHP2:
            B.check(lib.fhp_pool_set_rules(h, int(rules)))

    @staticmethod
    def arena_bytes_for(max_slots: int, max_bands: int, lattice_bytes: int) -> int:
        n = ctypes.c_size_t()
        B.check(B.load().fhp_pool_workspace_bytes(int(max_slots), int(max_bands),
                                                  int(lattice_bytes), ctypes.byref(n)))
        return int(n.value)

    def admit(self, steps: int, **params):
        """Slot number, or None when there is no room (FHP_E_BUSY)."""
        p, keep = B.make_params(**params)
        slot = ctypes.c_uint32()
        rc = self._lib.fhp_pool_admit(self._h, ctypes.byref(p), int(steps), ctypes.byref(slot))
        del keep
        if rc == B.E_BUSY:
            return None
        B.check(rc)
        self._shapes[int(slot.value)] = (params["width"], params["height"])
        return int(slot.value)

    def set_rules(self, rules: int) -> None:
        """Rule set of every job (FHP-II until set); only while the pool is empty."""
        B.check(self._lib.fhp_pool_set_rules(self._h, int(rules)))

    def tick(self, passes: int = 1) -> None:
        B.check(self._lib.fhp_pool_tick(self._h, int(passes)))

    def done(self) -> list[int]:
        out = (ctypes.c_uint32 * self.max_slots)()
        n = ctypes.c_uint32()
        B.check(self._lib.fhp_pool_done(self._h, out, self.max_slots, ctypes.byref(n)))
        return list(out[: n.value])

    def result(self, slot: int, block: int = 16) -> np.ndarray:
        W, H = self._shapes[slot]
        out = np.zeros(((H + block - 1) // block, (W + block - 1) // block, 3), dtype=np.int32)
        B.check(self._lib.fhp_pool_result(self._h, int(slot), int(block),
                                          out.ctypes.data_as(ctypes.c_void_p), out.nbytes))
        return out

    def collect(self, slot: int, block: int = 16) -> np.ndarray:
        """Enqueues the job's block sums into a pinned host array and returns
        it; valid once ``collected(slot)`` is True."""
        W, H = self._shapes[slot]
        shape = ((H + block - 1) // block, (W + block - 1) // block, 3)
        buf = torch.empty(shape, dtype=torch.int32, pin_memory=True)
        out = buf.numpy()
        B.check(self._lib.fhp_pool_collect(self._h, int(slot), int(block),
                                           ctypes.c_void_p(buf.data_ptr()), out.nbytes))
        self._pinned[slot] = buf
        return out

    def collected(self, slot: int) -> bool:
        r = ctypes.c_int()
        B.check(self._lib.fhp_pool_collected(self._h, int(slot), ctypes.byref(r)))
        return bool(r.value)

    def member(self, slot: int):
        v = ctypes.c_void_p()
        B.check(self._lib.fhp_pool_member(self._h, int(slot), ctypes.byref(v)))
        W, H = self._shapes[slot]
        view = _MemberView.__new__(_MemberView)
        view._lib, view._h, view._batch, view.index = self._lib, v, self, slot
        view.width, view.height, view.device = W, H, self.device
        return view

    def release(self, slot: int) -> None:
        B.check(self._lib.fhp_pool_release(self._h, int(slot)))
        self._shapes.pop(slot, None)
        self._pinned.pop(slot, None)

    def usage(self) -> dict:
        a, u, f = ctypes.c_uint32(), ctypes.c_size_t(), ctypes.c_size_t()
        B.check(self._lib.fhp_pool_usage(self._h, ctypes.byref(a), ctypes.byref(u), ctypes.byref(f)))
        return {"active": int(a.value), "bytes_used": int(u.value), "bytes_free": int(f.value)}

    def sync(self) -> None:
        B.check(self._lib.fhp_pool_sync(self._h))

    def close(self) -> None:
        if self._h is not None:
            self._lib.fhp_pool_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
