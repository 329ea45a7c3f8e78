"""The GPU library's per-word update, built for the host with hipcc and
checked exhaustively against the oracle's collision table (CPU only)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    if not os.path.exists(hipcc) or not shutil.which("gcc"):
        pytest.skip("hipcc or gcc not available")
    d = tmp_path_factory.mktemp("logic")
    obj = str(d / "oracle.o")
    subprocess.run(["gcc", "-O2", "-c", os.path.join(ROOT, "oracle", "fhp_oracle.c"), "-o", obj],
                   check=True)
    exe = str(d / "update_check")
    subprocess.run([hipcc, "-x", "hip", "--offload-arch=gfx950", "-O2", "-std=c++17",
                    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                    os.path.join(HERE, "native", "update_check.cpp"), "-x", "none", obj,
                    "-o", exe, "-lm"], check=True, capture_output=True)
    return exe


def test_update_matches_oracle_table_exhaustively(checker):
    r = subprocess.run([checker], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "OK" in r.stdout


def test_batch_band_packing(tmp_path):
    """Packing of lattice bands into the batch kernel's work items (host code
    of the batch engine, built with g++): coverage, class purity, one member
    per wave, the kernel's lane-to-band mapping and the queue order."""
    if not shutil.which("g++"):
        pytest.skip("g++ not available")
    exe = str(tmp_path / "groups_check")
    subprocess.run(["g++", "-O2", "-std=c++17", "-I",
                    os.path.join(ROOT, "paper_1208_2428_amd", "csrc"),
                    os.path.join(HERE, "native", "groups_check.cpp"), "-o", exe], check=True)
    r = subprocess.run([exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("OK")
