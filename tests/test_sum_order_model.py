"""CPU checks of the summation-order model used by the GPU parity tests of
desc_reduce_sum_f32: it stays within the error bound of its own order
against the exact sum (the oracle), is exact where every partial sum is
representable, and reduces to plain sequential addition for one lane."""
import numpy as np

import oracle
import workloads
from sum_order_model import CHUNK, chain_bound, fixed_order_sum, grid


def _bound(x):
    return chain_bound(x.size) * 2.0 ** -53 * float(np.abs(x.astype(np.float64)).sum())


def test_model_within_bound_of_exact_sum():
    for n in (1, 17, 4095, 4096, 4097, 3 * 4096 + 5, 2048 * 4096 + 3 * 4096 + 11):
        x = workloads.wide_f32(n, 40 + n % 13)
        exact = oracle.sum_f32(x)
        assert abs(fixed_order_sum(x) - exact) <= _bound(x), n


def test_model_exact_on_small_integers():
    # integers below 2^24 sum exactly in FP64 whatever the order
    x = workloads.int_uniform(5 * CHUNK + 123, 41).astype(np.float32)
    assert fixed_order_sum(x) == oracle.sum_f32(x) == float(x.astype(np.int64).sum())


def test_model_one_lane_is_sequential():
    # n <= 4: lane 0 of block 0 holds everything, added from 0.0 in order
    x = np.array([1.0, 2.0 ** -60, -1.0, 2.0 ** -60], np.float32)
    s = 0.0
    for v in x.astype(np.float64):
        s += v
    assert fixed_order_sum(x) == s
    assert grid(0) == 1 and fixed_order_sum(np.zeros(0, np.float32)) == 0.0


def test_model_order_shows_in_rounding():
    # the model is not the exact sum: a cancellation the order loses
    x = np.zeros(CHUNK, np.float32)
    x[0], x[1], x[4] = 2.0 ** 60, 1.0, -(2.0 ** 60)   # lanes 0, 0 and 1
    assert oracle.sum_f32(x) == 1.0
    assert fixed_order_sum(x) == 0.0
