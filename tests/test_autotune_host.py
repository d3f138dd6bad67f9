"""Host logic of the launch-plan autotuner: the ef-class split that mirrors
the device's classification, and the rule that keeps the default plan
unless another is clearly faster.  No device work."""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
from paper_2402_11354_amd import autotune  # noqa: E402


def test_ef_classes_follow_the_power_of_two_bins():
    # class c holds effective list sizes max(ef, k) in (32 << (c-1), 32 << c]
    k = np.array([10, 10, 100, 1, 10, 1])
    ef = np.array([16, 64, 128, 256, 33, 32])
    np.testing.assert_array_equal(autotune.ef_classes(k, ef), [0, 1, 2, 3, 1, 0])


def test_ef_classes_take_k_when_it_exceeds_ef():
    # a query asking for more results than its ef searches with a list of k
    np.testing.assert_array_equal(autotune.ef_classes(np.array([100, 10]), np.array([32, 256])),
                                  [2, 3])


def test_ef_classes_single_and_capped():
    assert (autotune.ef_classes(np.array([1, 10]), np.array([8, 32])) == 0).all()
    # at most 8 classes: every size above 32 << 6 = 2048 lands in the last one
    cls = autotune.ef_classes(np.array([1, 1, 1]), np.array([2048, 2049, 4096]))
    np.testing.assert_array_equal(cls, [6, 7, 7])


def test_pick_keeps_the_default_unless_clearly_faster():
    keep = 1.0 - autotune.KEEP_DEFAULT
    assert autotune._pick({0: 1.0, 1024: keep + 0.005}) == 0
    assert autotune._pick({0: 1.0, 1024: keep - 0.005, 2048: 0.99}) == 1024
    assert autotune._pick({0: 1.0}) == 0
