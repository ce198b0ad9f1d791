"""Host logic of bench.py that runs without a GPU: the training-set selection of the learned
proposal (two-cluster split of the cold samples)."""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_dominant_mode_splits_two_separated_modes():
    rng = np.random.default_rng(0)
    a = 0.01 * rng.standard_normal((8000, 14))
    b = 0.01 * rng.standard_normal((2000, 14))
    b[:, 5] += 0.15
    b[:, 6] += 0.4
    kept, frac = bench.dominant_mode(np.vstack([a, b]))
    assert frac == 0.8 and kept.shape == (8000, 14)
    assert np.abs(kept[:, 5]).max() < 0.075           # every kept sample from the larger mode


def test_dominant_mode_keeps_unimodal_samples():
    rng = np.random.default_rng(1)
    g = rng.standard_normal((10000, 14))
    kept, frac = bench.dominant_mode(g)
    assert frac == 1.0 and kept.shape == g.shape
    c = rng.standard_normal((10000, 14))
    c[:, 1] = 0.99 * c[:, 0] + 0.01 * c[:, 1]          # a narrow correlated ridge is one mode
    kept, frac = bench.dominant_mode(c)
    assert frac == 1.0


def test_dominant_mode_ignores_a_tiny_cluster():
    rng = np.random.default_rng(2)
    a = 0.01 * rng.standard_normal((9950, 6))
    b = 0.01 * rng.standard_normal((50, 6)) + 1.0      # 0.5 %: below the 2 % floor
    kept, frac = bench.dominant_mode(np.vstack([a, b]))
    assert frac == 1.0


def test_flow_gemm_flops_counts_every_weight_three_times():
    # one multiply-add per weight of W1[H][|A|], W2[H][H], W3[2|B|][H] in each pass
    for d, layers, hidden in ((10, 8, 256), (14, 8, 256), (5, 3, 16)):
        a, b = d // 2, d - d // 2
        weights = layers * (hidden * a + hidden * hidden + 2 * b * hidden)
        assert bench.flow_gemm_flops(d, layers, hidden) == 3 * 2 * weights


def test_split_modes_marks_the_larger_cluster():
    """The mask of the larger of two separated clusters (each flow of a mixture proposal trains on
    one side of it), None for one Gaussian."""
    rng = np.random.default_rng(4)
    a = rng.normal(size=(3000, 5))
    b = rng.normal(size=(1200, 5)) + np.array([0.0, 14.0, 0.0, 0.0, 0.0])
    s = np.vstack([a, b])
    keep = bench.split_modes(s)
    assert keep is not None and keep.sum() == 3000 and keep[:3000].all() and not keep[3000:].any()
    assert bench.split_modes(a) is None
