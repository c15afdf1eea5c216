"""Address and undefined-behaviour sanitizer builds (host code only, with
gcc / g++) of the oracle and of the library's host-side plan compiler
(schedule.cpp), each driven over random small codes by its own driver in
tests/sanitize/.  Any sanitizer report aborts the driver and fails the
test.  The rest of the library's host code calls the HIP runtime and runs
under the GPU tests."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
       "-g", "-O1"]
ENV = {**os.environ, "ASAN_OPTIONS": "detect_leaks=1:abort_on_error=1",
       "UBSAN_OPTIONS": "print_stacktrace=1:halt_on_error=1"}


def _build_and_run(tmp_path, compiler, sources, includes, extra=()):
    if shutil.which(compiler) is None:
        pytest.skip(f"{compiler} not available")
    exe = str(tmp_path / "driver")
    cmd = [compiler, *SAN, *[f"-I{i}" for i in includes], *sources, "-o", exe, *extra]
    b = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert b.returncode == 0, b.stderr[-2000:]
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=ENV)
    assert r.returncode == 0, (r.stdout[-1000:], r.stderr[-4000:])
    return r.stdout


def test_oracle_under_sanitizers(tmp_path):
    out = _build_and_run(tmp_path, "gcc",
                         [os.path.join(ROOT, "tests", "sanitize", "oracle_main.c"),
                          os.path.join(ROOT, "oracle", "polar_oracle.c")],
                         [os.path.join(ROOT, "oracle")],
                         ["-std=c99", "-D_POSIX_C_SOURCE=200809L", "-ffp-contract=off", "-lm",
                          "-lpthread"])
    assert "decoder calls" in out


def test_schedule_compiler_under_sanitizers(tmp_path):
    csrc = os.path.join(ROOT, "paper_1505_01466_amd", "csrc")
    out = _build_and_run(tmp_path, "g++",
                         [os.path.join(ROOT, "tests", "sanitize", "schedule_main.cpp"),
                          os.path.join(csrc, "schedule.cpp")],
                         [csrc], ["-std=c++17"])
    assert "schedules" in out
