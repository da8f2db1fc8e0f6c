"""CPU-only tests of the serving loop's admission policy (the header
paper_2006_05226_amd/csrc/admission.h, no device code): tests/cpu/admission_test.cpp
drives it against a mock device allocator (budget accounting, FIFO with
backfill, the host-memory bound, an event-driven simulation over random
request mixes, and submitter/lane threads around one mutex).  Built with g++
under the address and undefined-behaviour sanitizers, and under the thread
sanitizer for the threaded part."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "cpu", "admission_test.cpp")
INC = os.path.join(ROOT, "paper_2006_05226_amd", "csrc")

pytestmark = pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not available")


def build_and_run(tmp_path, flags, args=()):
    exe = str(tmp_path / "admission_test")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", *flags, f"-I{INC}", SRC, "-o", exe,
                    "-pthread"], check=True, capture_output=True, text=True)
    r = subprocess.run([exe, *args], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "all checks passed" in r.stdout


def test_admission_asan_ubsan(tmp_path):
    build_and_run(tmp_path, ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined"])


def test_admission_threads_tsan(tmp_path):
    build_and_run(tmp_path, ["-fsanitize=thread"], ["threads"])
