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


# Mistakes planted in a copy of the tile header (host code, on the CPU): the
# brute-force check above must reject every one.  (Marking from slot 1 instead
# of 2 is not among them: slot 1 is the first owned cell, whose domain is the
# tile's first domain, so that change alters nothing.)
TILE_MUTANTS = [
    ("periodic left halo one past the domain's last cell",
     "(periodic ? off[z + 1] - 1 : -1)", "(periodic ? off[z + 1] : -1)"),
    ("right halo allowed one cell past the domain",
     "last + 1 < off[w + 1] ? last + 1 :", "last + 1 <= off[w + 1] ? last + 1 :"),
    ("a domain starting at the last owned slot left unmarked",
     "if (e >= 2 && e <= count && start + e - 1 == off[s + 1]) {",
     "if (e >= 2 && e < count && start + e - 1 == off[s + 1]) {"),
    ("word base domain taken one slot late",
     "if ((e & 63) == 0) d.base[e >> 6] = s;", "if ((e & 63) == 1) d.base[e >> 6] = s;"),
    ("tiles of block - 1 owned cells",
     "const int T = block - 2;", "const int T = block - 1;"),
    ("split pieces without the remainder",
     "const int cnt = base + (k < extra ? 1 : 0);", "const int cnt = base;"),
    ("segment tiles always full length",
     "t.push_back({st, std::min(T, off[s + 1] - st), s, s});", "t.push_back({st, T, s, s});"),
]


def _tile_mutant_caught(args):
    k, (name, old, new), work = args
    src = open(os.path.join(CSRC, "grprec_tiles.h")).read()
    assert src.count(old) == 1, f"{name}: expression not found once in grprec_tiles.h"
    d = os.path.join(work, f"m{k}")
    os.makedirs(d)
    with open(os.path.join(d, "grprec_tiles.h"), "w") as fh:
        fh.write(src.replace(old, new))
    exe = os.path.join(d, "check")
    cmd = ["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I", d, os.path.join(ROOT, "tests", "tile_plan_check.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    try:
        res = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    except subprocess.TimeoutExpired:
        return name, False
    return name, res.returncode != 0 or not res.stdout.startswith("ok ")


@pytest.mark.skipif(shutil.which("g++") is None, reason="no host C++ compiler")
def test_planted_tile_mistakes_are_rejected(tmp_path):
    import concurrent.futures as cf
    jobs = max(1, min(8, len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else 4))
    with cf.ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(_tile_mutant_caught, [(k, m, str(tmp_path)) for k, m in enumerate(TILE_MUTANTS)]))
    missed = [name for name, caught in results if not caught]
    assert not missed, missed
