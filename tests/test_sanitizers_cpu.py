"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the host-side C
and C++ (CPU only, gcc): the oracle driven through every entry point on small
and ragged lattices (tests/native/oracle_check.c), the GPU library's per-word
update built for the host and checked against the oracle's tables
(update_check.cpp), and the batch engine's band packing (groups_check.cpp).
Any sanitizer report aborts the program and fails the test."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
NATIVE = os.path.join(HERE, "native")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1")

pytestmark = pytest.mark.skipif(not (shutil.which("gcc") and shutil.which("g++")),
                                reason="gcc/g++ not available")


def run(exe):
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr
    return r.stdout


@pytest.fixture(scope="module")
def oracle_obj(tmp_path_factory):
    d = tmp_path_factory.mktemp("san")
    obj = str(d / "fhp_oracle.o")
    subprocess.run(["gcc", *SAN, "-std=c11", "-fopenmp", "-c",
                    os.path.join(ROOT, "oracle", "fhp_oracle.c"), "-o", obj], check=True)
    return obj


def test_oracle_entry_points_sanitized(oracle_obj, tmp_path):
    exe = str(tmp_path / "oracle_check")
    subprocess.run(["gcc", *SAN, "-std=c11", "-fopenmp", os.path.join(NATIVE, "oracle_check.c"),
                    oracle_obj, "-o", exe, "-lm"], check=True)
    out = run(exe)
    assert out.rstrip().endswith("OK")
    assert out.count("case ") == 45


def test_device_update_host_build_sanitized(oracle_obj, tmp_path):
    if not os.path.isdir("/opt/rocm/include"):
        pytest.skip("HIP headers not available")
    exe = str(tmp_path / "update_check")
    subprocess.run(["g++", *SAN, "-std=c++17", "-fopenmp", "-D__HIP_PLATFORM_AMD__",
                    "-I/opt/rocm/include", "-x", "c++", os.path.join(NATIVE, "update_check.cpp"),
                    "-x", "none", oracle_obj, "-o", exe, "-lm"], check=True)
    assert "OK" in run(exe)


def test_band_packing_sanitized(tmp_path):
    exe = str(tmp_path / "groups_check")
    subprocess.run(["g++", *SAN, "-std=c++17", "-I", os.path.join(ROOT, "paper_1208_2428_amd", "csrc"),
                    os.path.join(NATIVE, "groups_check.cpp"), "-o", exe], check=True)
    assert run(exe).startswith("OK")
