"""Builds the gfx950 HIP library ``libfhp.so`` in-tree with hipcc."""
from __future__ import annotations

import concurrent.futures
import glob
import os
import subprocess

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
LIB_PATH = os.path.join(PKG, "libfhp.so")
ARCH = "gfx950"

HIPCC_FLAGS = [
    "-O3", "-std=c++17", "-fPIC",
    f"--offload-arch={ARCH}",
    # keep hipcc from forming packed fp32 instructions (none are used here)
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


# Per-source extra flags.  The depth-5 pass of wide lattices is scheduled for
# instruction-level parallelism (see fhp_stepk_k5.hip).
FILE_FLAGS = {
    "fhp_stepk_k5.hip": ["-mllvm", "-amdgpu-sched-strategy=max-ilp"],
}


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed:\n" + " ".join(cmd) + "\n" + r.stdout + r.stderr)


def build(verbose: bool = False) -> str:
    """Compiles every source to an object in parallel, then links the library."""
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    inc = ["-I", os.path.join(os.path.dirname(PKG), "include")]
    objdir = os.path.join(PKG, "_build")
    os.makedirs(objdir, exist_ok=True)
    tag = "%d" % os.getpid()
    objs, cmds = [], []
    for src in sources():
        obj = os.path.join(objdir, os.path.basename(src) + "." + tag + ".o")
        objs.append(obj)
        extra = FILE_FLAGS.get(os.path.basename(src), [])
        cmds.append([hipcc, *HIPCC_FLAGS, *extra, "-c", *inc, "-o", obj, src])
    jobs = max(1, min(len(cmds), os.cpu_count() or 1, 8))
    try:
        with concurrent.futures.ThreadPoolExecutor(jobs) as ex:
            for f in [ex.submit(_run, c, verbose) for c in cmds]:
                f.result()
        tmp = LIB_PATH + ".tmp" + tag
        _run([hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp, *objs], verbose)
        os.replace(tmp, LIB_PATH)
    finally:
        for o in objs:
            if os.path.exists(o):
                os.remove(o)
    return LIB_PATH


if __name__ == "__main__":
    print(build(verbose=True))
