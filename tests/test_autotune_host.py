"""Host-side logic of the launch-shape autotuner (no GPU needed)."""

import ctypes

from paper_0905_2441_amd import _lib as L
from paper_0905_2441_amd import autotune


def test_candidates_respect_limits():
    # N above the split cap: at most 16 slices (one workgroup per tile)
    assert autotune.candidates(1000, 131072) == [1, 2, 3, 4, 8, 12, 16]
    # small N, long data: every candidate up to 128 slices
    assert autotune.candidates(10000, 8192) == list(autotune.CANDIDATES)
    # short data: at least MIN_PER_SLICE observations per slice
    assert autotune.candidates(20, 100) == [1, 2]
    assert autotune.candidates(1, 100) == [1]
    # the MFMA form takes at most 16
    assert max(autotune.candidates(65536, 16384, "bf16x3")) == 16


def test_buckets_are_power_of_two_ranges():
    assert autotune.bucket(1) == (1, 1)
    assert autotune.bucket(1000) == (512, 1023)
    assert autotune.bucket(1024) == (1024, 2047)
    assert autotune.bucket(131072) == (131072, 262143)


def test_launch_rule_layout_matches_header():
    # int32 k, d, prec, slices; int64 n_lo, n_hi, N_lo, N_hi
    assert ctypes.sizeof(L.SmcLaunchRule) == 4 * 4 + 4 * 8
    assert L.SmcLaunchRule.n_lo.offset == 16
