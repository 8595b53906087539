"""Pins of the oracle's loop-closure classification (Section III-C): strong
above the new-keyframe quality threshold, weak above 75 % of it (both strict,
as the text says "higher than"), none for failed registrations; the keyframe
switched to is the strong closure with the highest inlier ratio."""
import numpy as np

import oracle as O


def test_thresholds_are_strict():
    thr = 0.5  # 3/4 of it, 0.375, is exact in binary
    r = [0.51, 0.5, 0.38, 0.375, 0.3751, 0.0, 1.0]
    st = [0] * len(r)
    cls, best = O.loop_closure_classes(r, st, thr)
    assert cls.tolist() == [2, 1, 1, 0, 1, 0, 2]
    assert best == 6


def test_failed_registrations_close_nothing():
    cls, best = O.loop_closure_classes([0.9, 0.9, 0.9, 0.9, 0.9], [0, 1, 2, 3, 4], 0.5)
    assert cls.tolist() == [2, 2, 0, 0, 2]
    assert best == 0


def test_best_is_first_of_equals_and_none_without_strong():
    cls, best = O.loop_closure_classes([0.7, 0.8, 0.8, 0.3], [0, 0, 0, 0], 0.5)
    assert best == 1
    cls, best = O.loop_closure_classes([0.45, 0.3], [0, 0], 0.5)
    assert cls.tolist() == [1, 0] and best == -1
