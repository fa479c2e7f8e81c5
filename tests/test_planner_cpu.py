"""CPU test of the host planner of a search, under address and undefined-behaviour
sanitizers.

tests/planner_check.cpp plans thousands of random searches (databases laid out as
sw_db_load lays them out, empty to 40,000-residue queries, every knob setting, 1 to 256
compute units) with the library's own planner source and checks that every (query,
sequence) pair is covered exactly once, that split pairs chain only backwards through
their boundary rows, and that every offset fits its buffer.  Host code only: no GPU.
"""
from __future__ import annotations

import os
import subprocess

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_planner_covers_every_pair_once_with_sanitizers(tmp_path):
    exe = tmp_path / "planner_check"
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
           "-I", os.path.join(ROOT, "include"),
           os.path.join(ROOT, "tests", "planner_check.cpp"),
           os.path.join(ROOT, "paper_1702_07195_amd", "csrc", "planner.cpp"), "-o", str(exe)]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("planner ok"), r.stdout
