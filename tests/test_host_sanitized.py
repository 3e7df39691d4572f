"""CPU builds with AddressSanitizer and UndefinedBehaviorSanitizer.

* tests/host_check.cpp with paper_2511_08427_amd/csrc/pn_geometry.cpp: the
  library's host-only code (validation, per-view tables, matrix
  composition entry points) and the cached-memory rules of pn_cache.hpp
  under graph capture (pinned plans, retired buffers), with a counting
  fake allocator;
* tests/oracle_check.c with oracle/oracle.c: every routine of the FP64
  oracle's C part on small edge-case geometries.
Both are plain host programs: no device code is built with a sanitizer.
"""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = ["-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def _build_and_run(cmd, exe, marker):
    subprocess.run(cmd + ["-o", exe], check=True, cwd=ROOT)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert marker in r.stdout


def test_host_logic_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_check")
    _build_and_run(["g++", "-std=c++17", *SAN, "-Wall", "-I", "include", "tests/host_check.cpp",
                    "paper_2511_08427_amd/csrc/pn_geometry.cpp"], exe, "host_check OK")


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_check")
    _build_and_run(["gcc", "-std=c99", *SAN, "-Wall", "-Wno-unknown-pragmas", "tests/oracle_check.c",
                    "oracle/oracle.c", "-lm"], exe, "oracle_check OK")
