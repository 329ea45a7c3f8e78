"""Python front end of batches: many lattices advanced by one persistent
kernel (``fhp_batch_*`` in include/fhp.h)."""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _binding as B
from .sim import Sim


class _MemberView(Sim):
    """A member of a batch: observables, state access and single stepping go
    through the same calls as a standalone simulation."""

    def __init__(self, batch: "Batch", index: int, handle, width: int, height: int):  # noqa: D401
        self._lib = batch._lib
        self._h = handle
        self._batch = batch
        self.index = index
        self.width, self.height = width, height
        self.device = batch.device

    def close(self) -> None:  # owned by the batch
        self._h = None

    def __del__(self):
        pass


class Batch:
    """``Batch(params)`` where params is a list of dicts with the keys of
    ``Sim`` (width, height, seed, fill, force_rate, walls, chirality, solid).

    The batch runs on its own torch stream (graph replay needs a stream other
    than the default one)."""

    def __init__(self, params: list[dict], device=None, stream=None, depth: int = 0,
                 band: int = 0, group_threads: int = 0, passes_per_launch: int = 1,
                 graph: bool = True):
        lib = B.load()
        if not torch.cuda.is_available():
            raise RuntimeError("the FHP library needs a ROCm GPU (torch.cuda is unavailable)")
        self._lib = lib
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None \
            else torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.Stream(device=self.device)
        n = len(params)
        arr = (B.Params * n)()
        keep = []
        for i, kw in enumerate(params):
            p, k = B.make_params(**kw)
            arr[i] = p
            keep.append(k)
        nbytes = ctypes.c_size_t()
        B.check(lib.fhp_batch_workspace_bytes(arr, n, ctypes.byref(nbytes)))
        self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=self.device)
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            B.check(lib.fhp_batch_create(arr, n, ctypes.c_void_p(self.workspace.data_ptr()),
                                         int(nbytes.value), ctypes.c_void_p(self.stream.cuda_stream),
                                         ctypes.byref(h)))
        del keep
        self._h = h
        self.n = n
        self.members = []
        for i in range(n):
            v = ctypes.c_void_p()
            B.check(lib.fhp_batch_member(h, i, ctypes.byref(v)))
            self.members.append(_MemberView(self, i, v, params[i]["width"], params[i]["height"]))
        self.set_tiling(depth, band, group_threads, passes_per_launch)
        self.set_graph(graph)

    def _handle(self):
        if self._h is None:
            raise RuntimeError("batch is closed")
        return self._h

    def set_tiling(self, depth: int = 0, band: int = 0, group_threads: int = 0,
                   passes_per_launch: int = 1) -> None:
        B.check(self._lib.fhp_batch_set_tiling(self._handle(), int(depth), int(band),
                                               int(group_threads), int(passes_per_launch)))

    def set_graph(self, enable: bool) -> None:
        B.check(self._lib.fhp_batch_set_graph(self._handle(), int(bool(enable))))

    def step(self, n: int) -> None:
        B.check(self._lib.fhp_batch_step(self._handle(), int(n)))

    def sync(self) -> None:
        B.check(self._lib.fhp_batch_sync(self._handle()))

    def __getitem__(self, i: int) -> Sim:
        return self.members[i]

    def __len__(self) -> int:
        return self.n

    def close(self) -> None:
        if self._h is not None:
            for m in self.members:
                m.close()
            self._lib.fhp_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
