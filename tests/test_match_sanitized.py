"""The library's host-side candidate consumers built with AddressSanitizer
and UndefinedBehaviorSanitizer (host code only, g++) and driven by
tests/match_driver.cpp on seeded random inputs: no memory or UB errors, and
the documented invariants of their outputs hold."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_consumers_under_sanitizers(tmp_path):
    exe = str(tmp_path / "match_driver")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-Wall", "-fsanitize=address,undefined",
           "-fno-omit-frame-pointer", "-fno-sanitize-recover=undefined",
           f"-I{os.path.join(ROOT, 'include')}",
           os.path.join(ROOT, "tests", "match_driver.cpp"),
           os.path.join(ROOT, "paper_2108_05602_amd", "csrc", "pulse_match.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr
    # verify_asan_link_order=0: the runtime need not be the first library
    # the process loads
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0 and r.stdout.strip() == "ok", r.stdout + r.stderr
