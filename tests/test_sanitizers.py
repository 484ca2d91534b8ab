"""AddressSanitizer and UndefinedBehaviorSanitizer builds of the host code
that the parity tests trust: the C oracle and the CPU candidate filter.

tests/sanitize/check_host.cpp drives both over small random collections (all
four similarity functions, the merge trace, both filter modes, probe pieces
that do not fit their buffer, argument errors); the build aborts on the first
sanitizer report.  CPU only; no GPU code is built here.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
FLAGS = ["-g", "-O1", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]


def _build(tmp_path):
    if shutil.which("gcc") is None or shutil.which("g++") is None:
        pytest.skip("gcc/g++ not available")
    obj = tmp_path / "verify_ref.o"
    subprocess.run(["gcc", "-std=gnu99", "-fopenmp", *FLAGS, "-c", os.path.join(ROOT, "oracle", "verify_ref.c"),
                    "-o", str(obj)], check=True)
    exe = tmp_path / "check_host"
    subprocess.run(["g++", "-std=c++17", "-fopenmp", "-pthread", *FLAGS,
                    os.path.join(ROOT, "tests", "sanitize", "check_host.cpp"),
                    os.path.join(ROOT, "ssj_inputs", "csrc", "allpairs.cpp"), str(obj), "-o", str(exe)],
                   check=True)
    return exe


def test_oracle_and_filter_under_asan_ubsan(tmp_path):
    exe = _build(tmp_path)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="2")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "sanitized host checks passed" in r.stdout
