"""The library's host logic and the oracle built with AddressSanitizer and
UndefinedBehaviorSanitizer (CPU only, no GPU calls).

* ``sanitize/planner_check.cpp`` drives the planner (``plan.cpp``: tile geometry, exact
  accumulation windows, output types, work accounting) over 200,000 seeded argument
  combinations, valid and invalid, the exact inverse of the tile numbering (Sec. 4.2) over
  two million indices, and the tune cache's JSON-lines save / load, including malformed
  and overlong files.
* ``sanitize/oracle_check.c`` runs the oracle's C library on every sample format and the
  edge shapes (no samples, no channels selected, one station, one polarisation), compares
  each result with a second evaluation of Eq. 4 in another loop order, and checks that
  bad arguments are refused before anything is read.

A sanitizer report aborts the program (``-fno-sanitize-recover=all``), so a non-zero exit
status is the failure.
"""

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1107_4264_amd", "csrc")
SAN = ["-g", "-O1", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def _need(tool):
    if shutil.which(tool) is None:
        pytest.skip(f"{tool} not available")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300, **kw)
    assert r.returncode == 0, f"{' '.join(cmd[:3])}... exited {r.returncode}\n{r.stdout[-2000:]}\n{r.stderr[-4000:]}"
    return r.stdout


def test_planner_and_tune_cache_under_sanitizers(tmp_path):
    _need("g++")
    exe = str(tmp_path / "planner_check")
    rocm_inc = os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "include")
    _run(["g++", "-std=c++17", *SAN, "-D__HIP_PLATFORM_AMD__", "-I" + rocm_inc, "-I" + os.path.join(ROOT, "include"),
          "-I" + CSRC, os.path.join(CSRC, "plan.cpp"), os.path.join(CSRC, "tune.cpp"),
          os.path.join(HERE, "sanitize", "planner_check.cpp"), "-o", exe])
    out = _run([exe, str(tmp_path)], env=ENV)
    assert out.strip().endswith("ok")


def test_oracle_under_sanitizers(tmp_path):
    _need("gcc")
    exe = str(tmp_path / "oracle_check")
    _run(["gcc", "-std=c99", "-fopenmp", *SAN, os.path.join(ROOT, "oracle", "xcorr_oracle.c"),
          os.path.join(HERE, "sanitize", "oracle_check.c"), "-o", exe])
    out = _run([exe], env=dict(ENV, OMP_NUM_THREADS="4"))
    assert out.strip().endswith("ok")
