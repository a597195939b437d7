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


def _refine_configs():
    import math

    import numpy as np

    import workloads

    def pair(gap):
        c = 1.0 + gap / 2
        return workloads.Particles(np.array([[-c, 0.0], [c, 0.0]]), np.array([0.0, math.pi]),
                                   np.array([[1.0, 0.5], [1.0, 0.5]]), 1.0)

    # a side-by-side pair at an angle and a tight cluster of four
    skew = workloads.Particles(np.array([[0.0, 0.0], [0.3, 1.02]]), np.array([0.1, 0.05]),
                               np.array([[1.0, 0.5], [1.2, 0.5]]), 1.0)
    four = workloads.Particles(np.array([[0.0, 0.0], [2.04, 0.0], [0.0, 1.03], [2.2, 1.1]]),
                               np.array([0.0, 0.0, 0.0, 0.3]), np.array([[1.0, 0.5]] * 4), 1.0)
    return [(pair(0.02), 16, 3), (pair(0.005), 16, 4), (skew, 12, 3), (four, 16, 2)]


def test_refinement_matches_the_oracle_under_sanitizers(tmp_path):
    """The library's host refinement (refine.h) takes the same split decisions as the
    oracle's (oracle/geometry.py refine_panels) on near-contact configurations."""
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not found")
    import oracle
    from oracle.geometry import Params
    exe = str(tmp_path / "refine")
    r = subprocess.run([gxx, *FLAGS, os.path.join(ROOT, "tests", "host", "refine_check.cpp"), "-o",
                        exe], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0")
    for parts, P, levels in _refine_configs():
        lines = [f"{parts.n} {P} {levels} 2.0 2"]
        for c, a, ax in zip(parts.center, parts.angle, parts.axes):
            lines.append(" ".join(f"{float(v):.17g}" for v in (c[0], c[1], a, ax[0], ax[1])))
        r = subprocess.run([exe], input="\n".join(lines) + "\n", capture_output=True, text=True,
                           env=env, timeout=120)
        assert r.returncode == 0, r.stderr
        got = [[int(v) for v in ln.split()] for ln in r.stdout.strip().splitlines()]
        want = oracle.geometry.refine_panels(parts, Params(panels=P, refine_levels=levels,
                                                           refine_ratio=2.0, qbx_window=2))
        assert len(got) == len(want)
        for g, w in zip(got, want):
            assert g[0] == len(w)
            assert [tuple(g[1 + 3 * a:4 + 3 * a]) for a in range(g[0])] == [tuple(d) for d in w]
        assert any(len(w) > P for w in want)     # each case refines something
