"""The error norms of the parity tests (CPU): a receiver whose terms are all
zero (A_i = 0 or P_i = 0) is gated, not skipped."""
import math

import numpy as np

from tests._metrics import cond_max, l2_rel, phi_cond_max


def test_cond_max_scales_each_receiver_by_its_own_magnitude_sum():
    ref = np.array([[1.0, 0.0, 0.0], [0.0, 2.0, 0.0]])
    got = ref + np.array([[0.0, 3e-6, 4e-6], [1e-6, 0.0, 0.0]])
    amag = np.array([10.0, 0.5])
    assert cond_max(got, ref, amag) == max(5e-6 / 10.0, 1e-6 / 0.5)


def test_zero_magnitude_sum_demands_an_exact_zero():
    ref = np.zeros((2, 3))
    amag = np.array([0.0, 1.0])
    assert cond_max(ref, ref, amag) == 0.0
    bad = ref.copy()
    bad[0, 2] = 1e-300
    assert math.isinf(cond_max(bad, ref, amag))
    assert math.isinf(phi_cond_max(np.array([1e-30, 0.0]), np.zeros(2), np.array([0.0, 1.0])))
    assert phi_cond_max(np.array([0.0, 1.0 + 1e-7]), np.array([0.0, 1.0]), np.array([0.0, 2.0])) <= 5.1e-8


def test_l2_and_empty_inputs():
    assert l2_rel(np.array([3.0, 4.0]), np.array([0.0, 0.0])) == 5.0
    assert cond_max(np.zeros((0, 3)), np.zeros((0, 3)), np.zeros(0)) == 0.0
