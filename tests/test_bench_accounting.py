"""Host logic of bench.py's roofline accounting (CPU only): the pair-class mix
that weights the per-class flop and instruction counts."""
import os
import sys

import numpy as np

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402


def _two_clusters(gap):
    """Two 256-node lines of nodes, `gap` apart along x (each line 1 unit long)."""
    t = np.linspace(0.0, 1.0, 256)
    x = np.concatenate([t, t + 1.0 + gap])
    y = np.zeros_like(x)
    return x, y


def test_class_mix_sums_to_one_and_panels_only_move_close_pairs():
    rng = np.random.default_rng(0)
    x, y = rng.uniform(0, 20, 4096), rng.uniform(0, 20, 4096)
    tile = bench.far_class_mix(x, y, 1.0)
    pan = bench.far_class_mix(x, y, 1.0, panels=True)
    assert abs(sum(tile.values()) - 1.0) < 1e-12 and abs(sum(pan.values()) - 1.0) < 1e-12
    # the panel split refines only the tiles with close pairs
    assert pan["z8"] >= tile["z8"] and pan["z4"] >= tile["z4"] and pan["z2"] >= tile["z2"]
    assert pan["general"] <= tile["general"]
    moved = tile["general"] - pan["general"]
    gained = sum(pan[c] - tile[c] for c in ("z8", "z4", "z2"))
    assert abs(moved - gained) < 1e-12


def test_class_mix_of_separated_clusters():
    # gap 9 between the lines: the cross pairs (half of all pairs) are z >= 8 at
    # kappa = 1, the pairs within a line are close
    x, y = _two_clusters(9.0)
    mix = bench.far_class_mix(x, y, 1.0)
    assert abs(mix["z8"] - 0.5) < 1e-12
    assert abs(mix["general"] - 0.5) < 1e-12
    # kappa = 0.5 halves every gap: the cross pairs drop to the z >= 4 class
    mix = bench.far_class_mix(x, y, 0.5)
    assert abs(mix["z4"] - 0.5) < 1e-12


def test_weighted_counts():
    mix = {"z8": 0.5, "z4": 0.25, "z2": 0.125, "general": 0.125}
    assert bench.flops_per_pair(mix, bench.F32_CLASS) == 0.5 * 23 + 0.25 * 25 + 0.125 * 29 + 0.125 * 31
    assert bench.flops_per_pair(mix, bench.F32_VALU) == 0.5 * 16 + 0.25 * 17 + 0.125 * 19 + 0.125 * 43
    assert bench.VALU_ISSUE == 256 * 4 * 16 * 2.4e9
