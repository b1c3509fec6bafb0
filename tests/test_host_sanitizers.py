"""The library's host-side C++ (mesh canonicalisation, start grid,
tree-cotree split, field and Gauss-law assembly, the particle checkpoint
file) and the C oracle built with
AddressSanitizer and UndefinedBehaviorSanitizer on the CPU (gcc/g++ only, no
GPU code) and driven through their paths by the programs in tests/sanitize/:
no sanitizer report, and every driver check holds."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2208_12795_amd", "csrc")
SAN = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=all", "-g", "-O1"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="2")


def _run(cmd, **kw):
    return subprocess.run(cmd, capture_output=True, text=True, timeout=600, **kw)


@pytest.fixture(scope="module")
def outdir(tmp_path_factory):
    if shutil.which("g++") is None or shutil.which("gcc") is None:
        pytest.skip("no gcc/g++")
    return tmp_path_factory.mktemp("sanitize")


def test_host_cpp_under_asan_ubsan(outdir):
    exe = str(outdir / "host_driver")
    b = _run(["g++", "-std=c++17", *SAN, "-I", CSRC, os.path.join(ROOT, "tests", "sanitize", "host_driver.cpp"),
              os.path.join(CSRC, "mesh_host.cpp"), os.path.join(CSRC, "field_host.cpp"),
              os.path.join(CSRC, "checkpoint_host.cpp"), "-o", exe])
    assert b.returncode == 0, b.stderr[-4000:]
    r = _run([exe, str(outdir)], env=ENV)
    assert r.returncode == 0 and "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr, \
        (r.stdout[-2000:], r.stderr[-4000:])
    assert "all checks passed" in r.stdout


def test_oracle_under_asan_ubsan(outdir):
    exe = str(outdir / "oracle_driver")
    b = _run(["gcc", "-std=c11", "-fopenmp", *SAN, os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"),
              os.path.join(ROOT, "oracle", "oracle.c"), "-lm", "-o", exe])
    assert b.returncode == 0, b.stderr[-4000:]
    r = _run([exe], env=ENV)
    assert r.returncode == 0 and "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr, \
        (r.stdout[-2000:], r.stderr[-4000:])
    assert "all calls succeeded" in r.stdout
