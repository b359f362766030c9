"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU
only): the exact finish of libf2m (f2m_finish.cpp, through the CPU harness
that feeds it brute-force pair data) and the C oracle.  Each is built as a
standalone program with g++/gcc and run on random, tie-heavy, lattice and
b-matching instances in every workspace mode; the sanitizers abort on the
first invalid access, leak or undefined operation."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2011_08170_amd", "csrc")
NATIVE = os.path.join(HERE, "native")
SAN = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1:abort_on_error=0:verify_asan_link_order=0",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="4")


def run(cmd_build, exe, timeout):
    r = subprocess.run(cmd_build, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    p = subprocess.run([exe], capture_output=True, text=True, env=ENV, timeout=timeout)
    assert "ERROR: AddressSanitizer" not in p.stderr and "runtime error" not in p.stderr, p.stderr[-4000:]
    assert "LeakSanitizer" not in p.stderr, p.stderr[-4000:]
    assert p.returncode == 0, (p.returncode, p.stdout[-2000:], p.stderr[-4000:])
    return p.stdout


def test_finish_under_sanitizers(tmp_path):
    exe = str(tmp_path / "sanitize_finish")
    out = run(["g++", "-std=c++17", "-pthread"] + SAN + ["-I", CSRC, os.path.join(NATIVE, "sanitize_finish.cpp"),
                                                         os.path.join(NATIVE, "finish_harness.cpp"),
                                                         os.path.join(CSRC, "f2m_finish.cpp"), "-o", exe],
              exe, 600)
    assert "failures 0" in out


def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "sanitize_oracle")
    out = run(["gcc", "-std=c11", "-fopenmp"] + SAN + [os.path.join(NATIVE, "sanitize_oracle.c"),
                                                       os.path.join(ROOT, "oracle", "f2m_oracle.c"), "-lm", "-o", exe],
              exe, 600)
    assert "failures 0" in out
