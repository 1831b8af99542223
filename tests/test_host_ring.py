"""Host logic of the server's pinned result arena: the ring allocator in
csrc/sm_ring.h, built with g++ and checked by a randomised driver."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1012_2547_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")
def test_ring_allocator(tmp_path):
    exe = str(tmp_path / "ring_check")
    subprocess.check_call(["g++", "-O1", "-std=c++17", "-Wall", "-I" + CSRC,
                           os.path.join(ROOT, "tests", "ring_check.cpp"), "-o", exe])
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.strip() == "ok"
