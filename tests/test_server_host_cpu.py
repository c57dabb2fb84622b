"""Host bookkeeping of the serving loop, without a GPU: the device arena's
first-fit allocator and the per-ticket live ranges, built from their header
with g++ and checked against brute force on seeded random operation mixes."""

import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "csrc", "serve_ranges_check.cpp")
INC = os.path.join(os.path.dirname(HERE), "paper_1411_2484_amd", "csrc")


def test_arena_and_live_ranges(tmp_path):
    exe = str(tmp_path / "serve_ranges_check")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                    "-I", INC, "-o", exe, SRC], check=True)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip() == "ok"
