"""Memory ceilings measured on the device itself (``include/fhp_calib.h``).

``pass_rate`` times the streaming kernel that makes exactly the memory
accesses of one blocked pass (seven planes plus the obstacle plane read over
every band and its halo rows, seven planes written) with no arithmetic;
``flat_rate`` times plain 16-byte-per-thread streaming of a flat buffer.  Both
time every launch with HIP events on the stream the kernels run on.
"""
from __future__ import annotations

import ctypes

import torch

from . import _binding as B

MODES = {"copy": B.CALIB_COPY, "read": B.CALIB_READ, "write": B.CALIB_WRITE}


def pass_bytes(mode: str, wd: int, H: int, band: int, halo: int, mask: bool) -> int:
    """Bytes one pass-shaped launch moves: every band reads its rows and
    `halo` rows on each side (wrapping at the lattice edges) of 7 planes (+ the
    mask), and writes its own rows of 7 planes."""
    read_rows = sum(min(band, H - y0) + 2 * halo for y0 in range(0, H, band))
    planes_in = 7 + (1 if mask else 0)
    rd = 0 if mode == "write" else read_rows * wd * 8 * planes_in
    wr = 0 if mode == "read" else H * wd * 8 * 7
    return rd + wr


def _time(launch, stream, launches: int) -> float:
    launch()  # untimed
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(launches)]
    for a, b in evs:
        a.record(stream)
        launch()
        b.record(stream)
    torch.cuda.synchronize()
    return sum(a.elapsed_time(b) for a, b in evs) / launches / 1e3


def pass_rate(mode: str, wd: int, H: int, band: int, halo: int = 0, mask: bool = True,
              launches: int = 50, device=None) -> dict:
    """Bandwidth of the pass-shaped streaming kernel: {"bytes", "us", "gbs"}."""
    lib = B.load()
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else device
    ps = (H * wd + 31) // 32 * 32
    src = torch.zeros(7 * ps, dtype=torch.int64, device=dev)
    dst = torch.empty(7 * ps, dtype=torch.int64, device=dev)
    msk = torch.zeros(ps, dtype=torch.int64, device=dev) if mask else None
    stream = torch.cuda.current_stream(dev)
    sh = ctypes.c_void_p(stream.cuda_stream)
    args = (MODES[mode], ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()),
            ctypes.c_void_p(msk.data_ptr()) if mask else None, wd, H, ps, band, halo, sh)

    def launch():
        B.check(lib.fhp_calib_pass(*args))

    sec = _time(launch, stream, launches)
    nbytes = pass_bytes(mode, wd, H, band, halo, mask)
    return {"bytes": nbytes, "us": sec * 1e6, "gbs": nbytes / sec / 1e9}


def flat_rate(mode: str, nbytes: int = 1 << 30, launches: int = 20, device=None) -> dict:
    """Bandwidth of plain streaming over `nbytes` bytes (read and written
    bytes both count for a copy): {"bytes", "us", "gbs"}."""
    lib = B.load()
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else device
    src = torch.zeros(nbytes // 8, dtype=torch.int64, device=dev)
    dst = torch.empty(nbytes // 8, dtype=torch.int64, device=dev)
    stream = torch.cuda.current_stream(dev)
    used = ctypes.c_uint32(0)

    def launch():
        B.check(lib.fhp_calib_flat(MODES[mode], ctypes.c_void_p(src.data_ptr()),
                                   ctypes.c_void_p(dst.data_ptr()), nbytes, 0, ctypes.byref(used),
                                   ctypes.c_void_p(stream.cuda_stream)))

    sec = _time(launch, stream, launches)
    moved = nbytes * (2 if mode == "copy" else 1)
    return {"bytes": moved, "us": sec * 1e6, "gbs": moved / sec / 1e9}


def main(argv=None) -> int:
    """Runs the reference kernels once each (used for the rocprofv3 counter
    calibration): python -m paper_1208_2428_amd.calib [--wd 256 --height 16384
    --band 32 --halo 5] [--launches N]."""
    import argparse
    import json
    ap = argparse.ArgumentParser()
    ap.add_argument("--wd", type=int, default=256)
    ap.add_argument("--height", type=int, default=16384)
    ap.add_argument("--band", type=int, default=32)
    ap.add_argument("--halo", type=int, default=5)
    ap.add_argument("--launches", type=int, default=20)
    ap.add_argument("--flat-mib", type=int, default=1024)
    a = ap.parse_args(argv)
    out = {}
    for mode in ("copy", "read", "write"):
        out[f"pass_{mode}_halo0"] = pass_rate(mode, a.wd, a.height, a.band, 0, True, a.launches)
        out[f"pass_{mode}_halo{a.halo}"] = pass_rate(mode, a.wd, a.height, a.band, a.halo, True,
                                                     a.launches)
        out[f"flat_{mode}"] = flat_rate(mode, a.flat_mib << 20, a.launches)
    for k, v in out.items():
        print(f"{k}: {v['bytes']} bytes in {v['us']:.1f} us = {v['gbs']:.0f} GB/s", flush=True)
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
