"""AddressSanitizer + UndefinedBehaviorSanitizer builds of the host code (no
GPU): the library's host unit (generators, CSR validation, hierarchy set-up,
K P, SELL-C images and their host walk) and, separately, the oracle, each
driven by a small program under tests/sanitize/ that also checks its results.
Any invalid access, leak or undefined operation aborts the driver."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2511_21268_amd", "csrc")
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-ffp-contract=off"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1", UBSAN_OPTIONS="print_stacktrace=1",
           OMP_NUM_THREADS="4")


def _need(tool):
    if shutil.which(tool) is None:
        pytest.skip(f"{tool} not found")


def _build(cmd, tmp_path):
    r = subprocess.run(cmd, cwd=tmp_path, capture_output=True, text=True)
    if r.returncode != 0 and "libasan" in (r.stderr + r.stdout):
        pytest.skip("sanitizer runtime not installed")
    assert r.returncode == 0, r.stderr[-4000:]


def _run(exe):
    r = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=600)
    assert r.returncode == 0, (r.stdout + r.stderr)[-6000:]
    return r.stdout


def test_host_code_under_sanitizers(tmp_path):
    _need("g++")
    exe = str(tmp_path / "host_check")
    _build(["g++", "-std=c++17", "-pthread"] + SAN + ["-I", CSRC, "-I", os.path.join(ROOT, "include"),
            os.path.join(CSRC, "host_setup.cpp"), os.path.join(ROOT, "tests", "sanitize", "host_check.cpp"),
            "-o", exe], tmp_path)
    assert "host checks ok" in _run(exe)


def test_oracle_under_sanitizers(tmp_path):
    _need("gcc")
    exe = str(tmp_path / "oracle_check")
    odir = os.path.join(ROOT, "oracle")
    srcs = [os.path.join(odir, f) for f in ("amg.c", "cube.c", "iga.c", "krylov.c", "mlp.c")]
    _build(["gcc", "-std=gnu11", "-fopenmp"] + SAN + ["-I", odir] + srcs +
           [os.path.join(ROOT, "tests", "sanitize", "oracle_check.c"), "-lm", "-o", exe], tmp_path)
    assert "oracle checks ok" in _run(exe)
