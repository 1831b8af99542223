"""Host code under sanitizers, on the CPU: the oracle (naive vs KMP) with
AddressSanitizer + UndefinedBehaviorSanitizer, the server's result-arena ring
allocator with the same, the server's batch formation with a mock executor
under ThreadSanitizer, and the server's serving core (batching, admission by
result memory with deferral, eviction and refusal, completion) with a mock
executor under ThreadSanitizer and under AddressSanitizer. Each driver prints
"ok"."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1012_2547_amd", "csrc")
TESTS = os.path.join(ROOT, "tests")

pytestmark = pytest.mark.skipif(shutil.which("g++") is None or shutil.which("gcc") is None,
                                reason="gcc/g++ not available")

ASAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-g", "-O1"]


def run(exe):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1")
    out = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.strip().splitlines()[-1] == "ok"


def test_oracle_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_check")
    subprocess.check_call(["gcc", "-std=c11", *ASAN, "-o", exe, os.path.join(TESTS, "oracle_check.c"),
                           os.path.join(ROOT, "oracle", "sm_oracle.c")])
    run(exe)


def test_ring_asan_ubsan(tmp_path):
    exe = str(tmp_path / "ring_check")
    subprocess.check_call(["g++", "-std=c++17", *ASAN, "-I" + CSRC, "-o", exe,
                           os.path.join(TESTS, "ring_check.cpp")])
    run(exe)


def test_scheduler_mock_executor_tsan(tmp_path):
    exe = str(tmp_path / "sched_check")
    subprocess.check_call(["g++", "-std=c++17", "-fsanitize=thread", "-g", "-O1", "-pthread",
                           "-I" + CSRC, "-o", exe, os.path.join(TESTS, "sched_check.cpp")])
    out = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "WARNING: ThreadSanitizer" not in out.stderr, out.stderr
    assert out.stdout.strip().splitlines()[-1] == "ok"


def _serve_check(tmp_path, flags, name):
    exe = str(tmp_path / name)
    subprocess.check_call(["g++", "-std=c++17", *flags, "-pthread", "-I" + CSRC, "-o", exe,
                           os.path.join(TESTS, "serve_check.cpp")])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", UBSAN_OPTIONS="print_stacktrace=1")
    out = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "WARNING: ThreadSanitizer" not in out.stderr, out.stderr
    assert out.stdout.strip().splitlines()[-1] == "ok", out.stdout


def test_serving_core_mock_executor_tsan(tmp_path):
    _serve_check(tmp_path, ["-fsanitize=thread", "-g", "-O1"], "serve_check_tsan")


def test_serving_core_mock_executor_asan_ubsan(tmp_path):
    _serve_check(tmp_path, ASAN, "serve_check_asan")
