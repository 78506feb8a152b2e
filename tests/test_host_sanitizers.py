"""Host-side code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The library's host mathematics (csrc/host_math.cpp: Léja table, Alg. 1,
squared-basis coefficients, probe generator, error strings, the tridiagonal
eigen-solver of the Lanczos bound) is plain C++; it is built here with g++
and both sanitizers into a driver that exercises every entry point over
ordinary and edge-case arguments.  Values are checked by the other host
tests; this one fails on memory errors and undefined behaviour.  A second
driver calls the Léja table, Alg. 1 and the squared-basis coefficients from
several threads at once while the shared Léja table grows, under
ThreadSanitizer and under AddressSanitizer.
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2603_02207_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_host_code_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "host_sanitize")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           os.path.join(CSRC, "host_math.cpp"), os.path.join(ROOT, "tests", "host", "host_sanitize_main.cpp"),
           "-o", exe]
    build = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert build.returncode == 0, build.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    env.pop("LD_PRELOAD", None)
    run = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert run.returncode == 0, (run.stdout[-2000:], run.stderr[-3000:])
    assert "host checks passed" in run.stdout


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
@pytest.mark.parametrize("sanitizer", ["thread", "address,undefined"])
def test_host_code_from_several_threads(tmp_path, sanitizer):
    exe = str(tmp_path / "host_threads")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-pthread",
           f"-fsanitize={sanitizer}", "-fno-sanitize-recover=all",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC,
           os.path.join(CSRC, "host_math.cpp"), os.path.join(ROOT, "tests", "host", "host_threads_main.cpp"),
           "-o", exe]
    build = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert build.returncode == 0, build.stderr[-3000:]
    env = dict(os.environ, TSAN_OPTIONS="halt_on_error=1", ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    env.pop("LD_PRELOAD", None)
    run = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert run.returncode == 0, (run.stdout[-2000:], run.stderr[-3000:])
    assert "thread checks passed" in run.stdout
