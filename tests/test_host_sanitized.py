"""The library's host logic (plan validation, work schedule, default tile
choice, byte-range overlap, tile-cache keys and the tile-cache reader) built
for the CPU with g++ under AddressSanitizer and UndefinedBehaviorSanitizer,
and run over a sweep of shapes and over truncated and corrupted cache text
(tests/host_logic_check.cpp).  No GPU and no HIP runtime are involved: the
logic lives in bf_host.cpp, which has no HIP dependency."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1412_4907_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_host_logic_under_sanitizers(tmp_path):
    exe = str(tmp_path / "host_logic_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I", CSRC, "-I", os.path.join(ROOT, "include"),
           os.path.join(CSRC, "bf_host.cpp"), os.path.join(ROOT, "tests", "host_logic_check.cpp"),
           "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stdout + r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe, os.path.join(ROOT, "paper_1412_4907_amd", "tune_cache.json")],
                       capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0 and r.stdout.startswith("OK"), r.stdout + r.stderr
