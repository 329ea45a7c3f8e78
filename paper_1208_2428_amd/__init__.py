"""MI355X (gfx950) FHP lattice-gas library: Python front end.

``Sim`` drives one lattice through the C ABI of ``libfhp.so`` (include/fhp.h).
Importing this package does not load the GPU library; the first ``Sim`` does,
and fails loudly when it has not been built.
"""
from ._binding import (CHIR_HASH, CHIR_ONE, CHIR_ZERO, MAX_DEPTH, FhpError,  # noqa: F401
                       load)

__all__ = ["Sim", "Batch", "Pool", "FhpError", "CHIR_HASH", "CHIR_ZERO", "CHIR_ONE", "MAX_DEPTH", "load"]


def __getattr__(name):
    if name == "Sim":
        from .sim import Sim
        return Sim
    if name == "Batch":
        from .batch import Batch
        return Batch
    if name == "Pool":
        from .pool import Pool
        return Pool
    raise AttributeError(name)
