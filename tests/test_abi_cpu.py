"""C-ABI checks that need no GPU: the library loads, exports every function
that include/fhp.h declares, and rejects bad parameters before touching the
device."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1208_2428_amd import _binding as B

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"\b(fhp_\w+)\s*\(", text):
            names.add(m.group(1))
    return names


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(B.lib_path()):
        from paper_1208_2428_amd import build
        build.build()
    return B.load()


def test_exports_every_declared_function(lib):
    names = declared_functions()
    assert {"fhp_create", "fhp_step", "fhp_observe"} <= names
    for n in sorted(names):
        assert hasattr(lib, n), n
    assert set(B._SIGNATURES) <= names


def test_struct_layout_matches_header():
    # abi_version .. reserved: 6 x u32, seed u64, fill/force f64, pointer
    assert ctypes.sizeof(B.Params) == 6 * 4 + 8 + 8 + 8 + 8
    assert B.Params.seed.offset == 24


@pytest.mark.parametrize("kw,code", [
    (dict(width=100), B.E_INVAL), (dict(width=0), B.E_INVAL), (dict(width=1 << 20), B.E_INVAL),
    (dict(height=3), B.E_INVAL), (dict(height=0), B.E_INVAL), (dict(fill=1.5), B.E_INVAL),
    (dict(fill=float("nan")), B.E_INVAL), (dict(force_rate=1.0 / 64), B.E_INVAL),
    (dict(force_rate=-1e-9), B.E_INVAL), (dict(chirality=7), B.E_INVAL)])
def test_bad_params_rejected(lib, kw, code):
    args = dict(width=128, height=4)
    args.update(kw)
    p, _ = B.make_params(**args)
    n = ctypes.c_size_t()
    assert lib.fhp_workspace_bytes(ctypes.byref(p), ctypes.byref(n)) == code
    assert lib.fhp_last_error()


def test_workspace_size_and_create_argument_checks(lib):
    p, _ = B.make_params(16384, 16384)
    n = B.workspace_bytes(p)
    planes = 16384 * 16384 // 8
    assert 15 * planes <= n < 15 * planes + 65536
    h = ctypes.c_void_p()
    # NULL and misaligned workspaces, and a workspace that is too small, fail
    # before any device call
    assert lib.fhp_create(ctypes.byref(p), None, n, None, ctypes.byref(h)) == B.E_INVAL
    assert lib.fhp_create(ctypes.byref(p), ctypes.c_void_p(8), n, None, ctypes.byref(h)) == B.E_INVAL
    assert lib.fhp_create(ctypes.byref(p), ctypes.c_void_p(4096), n - 1, None,
                          ctypes.byref(h)) == B.E_NOMEM
    p.abi_version = 99
    assert lib.fhp_workspace_bytes(ctypes.byref(p), ctypes.byref(ctypes.c_size_t())) == B.E_INVAL


def test_null_handle_calls_fail_cleanly(lib):
    assert lib.fhp_step(None, 1) == B.E_INVAL
    assert lib.fhp_sync(None) == B.E_INVAL
    assert lib.fhp_set_depth(None, 1) == B.E_INVAL
    lib.fhp_destroy(None)


def test_batch_and_pool_argument_checks(lib):
    n = ctypes.c_size_t()
    arr = (B.Params * 2)()
    arr[0], _ = B.make_params(128, 64)
    arr[1], _ = B.make_params(128, 4)          # below the batch's minimum height
    assert lib.fhp_batch_workspace_bytes(arr, 2, ctypes.byref(n)) == B.E_INVAL
    arr[1], _ = B.make_params(256, 32)
    assert lib.fhp_batch_workspace_bytes(arr, 2, ctypes.byref(n)) == B.OK
    planes = (128 * 64 + 256 * 32) // 8
    assert n.value >= 15 * planes
    assert lib.fhp_batch_workspace_bytes(arr, 0, ctypes.byref(n)) == B.E_INVAL
    # a member whose seven planes exceed 4 GiB (32768 x 149800: 7 x 613.6 MB):
    # batches address a member's planes through one 32-bit-offset resource
    arr[1], _ = B.make_params(32768, 149800)
    assert lib.fhp_batch_workspace_bytes(arr, 2, ctypes.byref(n)) == B.E_INVAL
    arr[1], _ = B.make_params(32768, 149700)  # 7 x 613.2 MB: fits
    assert lib.fhp_batch_workspace_bytes(arr, 2, ctypes.byref(n)) == B.OK
    h = ctypes.c_void_p()
    assert lib.fhp_batch_create(arr, 2, None, n.value, None, ctypes.byref(h)) == B.E_INVAL
    assert lib.fhp_pool_workspace_bytes(0, 16, 1 << 20, ctypes.byref(n)) == B.E_INVAL
    assert lib.fhp_pool_workspace_bytes(16, 1024, 1 << 20, ctypes.byref(n)) == B.OK
    assert n.value > 1 << 20
    assert lib.fhp_pool_create(None, n.value, 16, 1024, None, ctypes.byref(h)) == B.E_INVAL
    assert lib.fhp_pool_create(ctypes.c_void_p(256), 1024, 16, 1024, None,
                               ctypes.byref(h)) == B.E_NOMEM   # arena smaller than its tables
    assert lib.fhp_pool_tick(None, 1) == B.E_INVAL
    assert lib.fhp_batch_step(None, 1) == B.E_INVAL


def test_rule_set_checks(lib):
    n = ctypes.c_size_t()
    for rules in (B.RULES_FHP2, B.RULES_FHP1, B.RULES_FHP3):
        p, _ = B.make_params(128, 64, rules=rules)
        assert lib.fhp_workspace_bytes(ctypes.byref(p), ctypes.byref(n)) == B.OK
    p, _ = B.make_params(128, 64, rules=3)
    assert lib.fhp_workspace_bytes(ctypes.byref(p), ctypes.byref(n)) == B.E_INVAL
    # a batch runs one rule set: any one, not a mix (checked before the device)
    arr = (B.Params * 2)()
    arr[0], _ = B.make_params(128, 64, rules=B.RULES_FHP3)
    arr[1], _ = B.make_params(256, 32, rules=B.RULES_FHP3)
    assert lib.fhp_batch_workspace_bytes(arr, 2, ctypes.byref(n)) == B.OK
    arr[1], _ = B.make_params(256, 32, rules=B.RULES_FHP1)
    assert lib.fhp_batch_workspace_bytes(arr, 2, ctypes.byref(n)) == B.E_INVAL
    assert b"rule set" in lib.fhp_last_error()
    assert lib.fhp_pool_set_rules(None, B.RULES_FHP1) == B.E_INVAL


def test_step_noalloc_argument_checks(lib):
    """fhp_step_noalloc rejects what it cannot run before touching the device
    (the pointers below are never dereferenced)."""
    x, y = ctypes.c_void_p(1 << 20), ctypes.c_void_p(2 << 20)
    W, H = 8192, 9400  # 7 planes of 77M nodes: above the 64 MiB limit
    assert 7 * W * H // 8 > B.NOALLOC_MAX_STATE_BYTES
    p, _ = B.make_params(W, H)
    assert lib.fhp_step_noalloc(ctypes.byref(p), x, y, None, 0, 5, 0, None) == B.E_NOMEM
    assert b"at most" in lib.fhp_last_error()
    p, _ = B.make_params(128, 8)
    assert lib.fhp_step_noalloc(ctypes.byref(p), x, x, None, 0, 5, 0, None) == B.E_INVAL
    assert lib.fhp_step_noalloc(ctypes.byref(p), x, ctypes.c_void_p((1 << 20) + 8), None,
                                0, 5, 0, None) == B.E_INVAL  # overlapping
    assert lib.fhp_step_noalloc(ctypes.byref(p), ctypes.c_void_p((1 << 20) + 8), y, None,
                                0, 5, 0, None) == B.E_INVAL  # misaligned
    assert lib.fhp_step_noalloc(ctypes.byref(p), x, y, None, 0, 5, 6, None) == B.E_INVAL
    assert lib.fhp_step_noalloc(ctypes.byref(p), x, y, None, (1 << 24) - 2, 5, 0,
                                None) == B.E_STATE
    mask = np.zeros((8, 128), np.uint8)
    p, keep = B.make_params(128, 8, solid=mask)
    assert lib.fhp_step_noalloc(ctypes.byref(p), x, y, None, 0, 5, 0, None) == B.E_INVAL


def test_calibration_argument_checks(lib):
    """The streaming reference kernels reject what they cannot run before any
    launch (the pointers below are never dereferenced)."""
    x, y = ctypes.c_void_p(1 << 20), ctypes.c_void_p(2 << 20)
    ok = dict(wd=256, H=64, ps=256 * 64, band=32, halo=5)

    def cp(mode=B.CALIB_COPY, src=x, dst=y, **kw):
        a = {**ok, **kw}
        return lib.fhp_calib_pass(mode, src, dst, None, a["wd"], a["H"], a["ps"], a["band"],
                                  a["halo"], None)

    assert cp(mode=3) == B.E_INVAL
    assert cp(wd=0) == B.E_INVAL and cp(wd=513) == B.E_INVAL
    assert cp(H=0) == B.E_INVAL and cp(band=0) == B.E_INVAL
    assert cp(halo=9) == B.E_INVAL
    assert cp(ps=256 * 64 - 1) == B.E_INVAL
    assert cp(ps=1 << 27) == B.E_INVAL  # seven planes of 1 GiB
    assert cp(src=None) == B.E_INVAL and cp(dst=None) == B.E_INVAL
    n = ctypes.c_uint32(0)
    assert lib.fhp_calib_flat(B.CALIB_COPY, x, y, 24, 4, ctypes.byref(n), None) == B.E_INVAL
    assert lib.fhp_calib_flat(B.CALIB_COPY, x, y, 0, 4, ctypes.byref(n), None) == B.E_INVAL
    assert lib.fhp_calib_flat(B.CALIB_COPY, ctypes.c_void_p((1 << 20) + 8), y, 1 << 20, 4,
                              ctypes.byref(n), None) == B.E_INVAL
    assert lib.fhp_calib_flat(B.CALIB_READ, None, y, 1 << 20, 4, ctypes.byref(n), None) == B.E_INVAL
    assert lib.fhp_calib_flat(5, x, y, 1 << 20, 4, ctypes.byref(n), None) == B.E_INVAL
