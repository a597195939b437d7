"""Host-side C++ of the library built with g++ under AddressSanitizer and
UndefinedBehaviorSanitizer and run on the CPU (no GPU, no HIP runtime).

* quadtree.h: the adaptive quadtree and the FMM interaction lists, checked
  pair by pair against the definitions of the lists (tests/host/quadtree_check.cpp).
* arena.h: the serving arena's first-fit node ranges and memory-budget admission
  (tests/host/arena_check.cpp).
"""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1810_04131_amd", "csrc")
FLAGS = ["-std=c++17", "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
         "-fno-omit-frame-pointer", "-I", CSRC]


def _build_and_run(src, tmp_path):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not found")
    exe = str(tmp_path / "check")
    r = subprocess.run([gxx, *FLAGS, os.path.join(ROOT, "tests", "host", src), "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().splitlines()[-1].startswith("ok")


def test_quadtree_lists_under_sanitizers(tmp_path):
    _build_and_run("quadtree_check.cpp", tmp_path)


def test_serving_arena_under_sanitizers(tmp_path):
    _build_and_run("arena_check.cpp", tmp_path)
