"""Host code under the address and undefined-behaviour sanitizers.

Two small native harnesses are built here with gcc/g++ and run:

* ``native/host_checks.cpp``: the sorting and merge networks of
  ``csrc/netgen.hpp`` on every 0-1 input, the serving arena (``csrc/arena.hpp``)
  against a page-bitmap model, and the argument checks of
  ``csrc/host_common.hpp`` at their limits;
* ``native/oracle_checks.c``: the oracle (``oracle/fnr_oracle.c``) on random tiny
  frames, large windows, padded pitches and adversarial introsort inputs,
  against a brute-force statement of the method written in the harness.

A sanitizer report or a failed check makes the harness exit non-zero."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NATIVE = os.path.join(ROOT, "tests", "native")
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def _build_and_run(cmd, exe):
    res = subprocess.run(cmd, capture_output=True, text=True)
    assert res.returncode == 0, res.stdout + res.stderr
    run = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=120)
    assert run.returncode == 0 and run.stdout.strip() == "ok", run.stdout + run.stderr
    assert "runtime error" not in run.stderr and "AddressSanitizer" not in run.stderr, run.stderr


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ is not installed")
def test_host_checks_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_checks")
    rocm = os.environ.get("ROCM_PATH", "/opt/rocm")
    _build_and_run(["g++", "-std=c++17", *SAN, "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(rocm, "include"),
                    "-o", exe, os.path.join(NATIVE, "host_checks.cpp"), "-L", os.path.join(rocm, "lib"),
                    "-lamdhip64", "-Wl,-rpath," + os.path.join(rocm, "lib")], exe)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc is not installed")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_checks")
    _build_and_run(["gcc", "-std=c11", *SAN, "-Wall", "-Werror", "-o", exe, os.path.join(NATIVE, "oracle_checks.c"),
                    os.path.join(ROOT, "oracle", "fnr_oracle.c")], exe)
