"""The oracle and the library's host-side argument checks, built with the
address and undefined-behaviour sanitizers and run on the CPU.

tests/sanitize/oracle_checks.c drives every entry point of oracle/oracle.c
(both shift rules, the quadratic start, fixed T, no exceptional shift,
invalid inputs, mixed degrees, density, local density, backward and the
exposed building blocks) on inputs with known results.
tests/sanitize/host_checks.cpp drives the C ABI's window and option checks
(csrc/validate.hpp) and the sorted-density workspace plan (csrc/sortplan.hpp)
over edge cases and every size class the entry points accept.  Both print
"... ok" and exit 0; any sanitizer report aborts them.
"""
from __future__ import annotations

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def _needs(compiler):
    if shutil.which(compiler) is None:
        pytest.skip(f"{compiler} not found")


def _run(exe):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    env.pop("LD_PRELOAD", None)
    p = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=120)
    return p.returncode, p.stdout + p.stderr


def test_oracle_under_sanitizers(tmp_path):
    _needs("gcc")
    exe = str(tmp_path / "oracle_checks")
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-Wall", "-ffp-contract=off", *SAN,
           os.path.join(ROOT, "oracle", "oracle.c"), os.path.join(HERE, "oracle_checks.c"),
           "-o", exe, "-lm"]
    subprocess.run(cmd, check=True, capture_output=True)
    rc, out = _run(exe)
    assert rc == 0 and "oracle checks ok" in out, out


def test_host_checks_under_sanitizers(tmp_path):
    _needs("g++")
    exe = str(tmp_path / "host_checks")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-Wall", "-Wextra", *SAN,
           "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "paper_2507_02164_amd", "csrc"),
           os.path.join(HERE, "host_checks.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True)
    rc, out = _run(exe)
    assert rc == 0 and "host checks ok" in out, out
