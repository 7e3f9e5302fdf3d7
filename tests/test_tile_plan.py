"""Host logic of the batched Euler step: tile plans and the per-slot
descriptor the kernel decodes (no GPU).  The C++ check compiles the
library's own tile header with the host compiler, under the address and
undefined-behaviour sanitizers, and compares every slot against brute force."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2602_21911_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_tile_plans_match_brute_force(tmp_path):
    exe = str(tmp_path / "tile_plan_check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I", CSRC, os.path.join(ROOT, "tests", "tile_plan_check.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    res = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert res.returncode == 0, res.stdout + res.stderr
    assert res.stdout.startswith("ok "), res.stdout
    assert int(res.stdout.split()[1]) > 1_000_000
