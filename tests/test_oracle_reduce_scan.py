"""Pins of the oracle's reduce and scan against closed forms, brute force and
library routines (none of which re-types the oracle's own loop).

Sum reduction and inclusive scan are the "block-wide parallel reduction" and
"scan" benchmarks of the paper's evaluation (Sec. 5).
"""
import itertools

import numpy as np
import pytest

import oracle
import workloads


# ------------------------------------------------------------------ reduce
@pytest.mark.parametrize("n,a,d", [(1, 5, 0), (1000, -500, 1), (4097, 1024, -1),
                                   (1 << 16, -1024, 0), (123457, 3, 0)])
def test_reduce_arithmetic_closed_form(n, a, d):
    x = workloads.arithmetic_i32(n, a, d)
    assert oracle.reduce_i32(x) == n * a + d * n * (n - 1) // 2


def test_reduce_periodic_closed_form():
    # x_i = (i mod 2049) - 1024: each full period sums to 0, the tail is an
    # arithmetic run starting at -1024.
    n = 3 * 2049 + 700
    x = ((np.arange(n) % 2049) - 1024).astype(np.int32)
    t = n % 2049
    assert oracle.reduce_i32(x) == t * -1024 + t * (t - 1) // 2


def test_reduce_bruteforce_tiny():
    vals = (-2, -1, 0, 1, 2)
    for length in range(0, 5):
        for xs in itertools.product(vals, repeat=length):
            assert oracle.reduce_i32(np.array(xs, dtype=np.int32)) == sum(xs)


def test_reduce_no_int32_overflow():
    # 2^20 copies of INT32_MAX / INT32_MIN: the exact total needs 51 bits.
    n = 1 << 20
    assert oracle.reduce_i32(np.full(n, 2**31 - 1, np.int32)) == n * (2**31 - 1)
    assert oracle.reduce_i32(np.full(n, -2**31, np.int32)) == n * -2**31


def test_reduce_matches_numpy_and_is_additive():
    x = workloads.int_uniform(1 << 22, seed=1)
    total = oracle.reduce_i32(x)
    assert total == int(x.sum(dtype=np.int64))
    cut = 1234567
    assert total == oracle.reduce_i32(x[:cut]) + oracle.reduce_i32(x[cut:])


def test_reduce_empty():
    assert oracle.reduce_i32(np.zeros(0, np.int32)) == 0


# ------------------------------------------------------------------ scan
def _wrap32(v: int) -> int:
    v &= 0xFFFFFFFF
    return v - (1 << 32) if v >= (1 << 31) else v


@pytest.mark.parametrize("n,a,d", [(1, -7, 0), (1000, -500, 1), (5000, 1024, -1), (70000, 3, 2)])
def test_scan_arithmetic_closed_form(n, a, d):
    x = workloads.arithmetic_i32(n, a, d)
    y = oracle.scan_i32(x)
    i = np.arange(n, dtype=object)
    expect = [(_wrap32(int(k + 1) * a + d * int(k) * int(k + 1) // 2)) for k in i]
    assert y.tolist() == expect


def test_scan_bruteforce_tiny():
    vals = (-2, 0, 1, 2)
    for length in range(0, 5):
        for xs in itertools.product(vals, repeat=length):
            y = oracle.scan_i32(np.array(xs, dtype=np.int32))
            assert y.tolist() == [sum(xs[: k + 1]) for k in range(length)]


def test_scan_invariants_random():
    x = workloads.int_uniform(1 << 20, seed=2)
    y, wrapped, m = oracle.scan_i32(x, return_info=True)
    assert not wrapped and m < 2**31
    # last element == reduction (mod 2^32; no wrap here)
    assert int(y[-1]) == oracle.reduce_i32(x)
    # differences recover the input
    d = np.diff(y.astype(np.int64))
    assert np.array_equal(d, x[1:].astype(np.int64)) and y[0] == x[0]
    # library cumsum
    assert np.array_equal(y, np.cumsum(x, dtype=np.int64).astype(np.int32))


def test_scan_wraps_modulo_2_32():
    n = 4
    x = np.full(n, 2**31 - 1, np.int32)
    y, wrapped, m = oracle.scan_i32(x, return_info=True)
    assert wrapped and m == n * (2**31 - 1)
    assert y.tolist() == [_wrap32(k * (2**31 - 1)) for k in range(1, n + 1)]
    # wrap arithmetic still recovers the input from differences
    d = (y.astype(np.int64)[1:] - y.astype(np.int64)[:-1]) & 0xFFFFFFFF
    assert np.array_equal(d.astype(np.uint32).view(np.int32), x[1:])


def test_scan_last_equals_reduce_mod_2_32_under_wrap():
    x = np.full(3000, 2**30 + 12345, np.int32)
    y = oracle.scan_i32(x)
    assert int(y[-1]) == _wrap32(oracle.reduce_i32(x))


def test_scan_empty():
    assert oracle.scan_i32(np.zeros(0, np.int32)).size == 0


def test_scan_workload_never_wraps():
    # The 2^28 workload keeps every prefix far inside int32, so the wrapped
    # and exact scans coincide.  Checked on a 2^24 prefix of the same stream
    # here (the full size is covered by the GPU parity test).
    x = workloads.int_uniform(1 << 24, seed=2)
    _, wrapped, m = oracle.scan_i32(x, return_info=True)
    assert not wrapped and m < 2**28


# ----------------------------------------------------------------- exclusive scan
@pytest.mark.parametrize("n,a,d", [(1, -7, 0), (1000, -500, 1), (5000, 1024, -1), (70000, 3, 2)])
def test_scan_exclusive_arithmetic_closed_form(n, a, d):
    # x_k = a + d k: the sum of the k terms before position k is k a + d k (k - 1) / 2
    x = workloads.arithmetic_i32(n, a, d)
    y = oracle.scan_exclusive_i32(x)
    expect = [_wrap32(int(k) * a + d * int(k) * (int(k) - 1) // 2) for k in range(n)]
    assert y.tolist() == expect


def test_scan_exclusive_bruteforce_tiny():
    vals = (-2, 0, 1, 2)
    for length in range(0, 5):
        for xs in itertools.product(vals, repeat=length):
            y = oracle.scan_exclusive_i32(np.array(xs, dtype=np.int32))
            assert y.tolist() == [sum(xs[:k]) for k in range(length)]


def test_scan_exclusive_invariants_random():
    x = workloads.int_uniform(1 << 20, seed=2)
    y = oracle.scan_exclusive_i32(x)
    assert y[0] == 0
    # the last exclusive prefix plus the last element is the total
    assert int(y[-1]) + int(x[-1]) == oracle.reduce_i32(x)
    # differences recover the input
    assert np.array_equal(np.diff(y.astype(np.int64)), x[:-1].astype(np.int64))


def test_scan_exclusive_wraps_modulo_2_32():
    x = np.full(5, 2**31 - 1, np.int32)
    y = oracle.scan_exclusive_i32(x)
    assert y.tolist() == [_wrap32(k * (2**31 - 1)) for k in range(5)]


# ------------------------------------------------------------------ min / max
def test_minmax_bruteforce_tiny():
    vals = (-3, -1, 0, 2, 5)
    for length in range(1, 5):
        for xs in itertools.product(vals, repeat=length):
            assert oracle.minmax_i32(np.array(xs, dtype=np.int32)) == (min(xs), max(xs))


def test_minmax_matches_numpy_and_extremes():
    x = workloads.int_uniform(100003, 21, -(1 << 31), (1 << 31) - 1)
    assert oracle.minmax_i32(x) == (int(x.min()), int(x.max()))
    y = np.zeros(4099, np.int32)
    y[4098] = -(1 << 31)
    y[0] = (1 << 31) - 1
    assert oracle.minmax_i32(y) == (-(1 << 31), (1 << 31) - 1)
    # a sorted run: the ends are the answer
    z = np.arange(-777, 5000, dtype=np.int32)
    assert oracle.minmax_i32(z) == (-777, 4999)
    assert oracle.minmax_i32(z[::-1]) == (-777, 4999)


def test_minmax_empty_gives_identities():
    assert oracle.minmax_i32(np.zeros(0, np.int32)) == ((1 << 31) - 1, -(1 << 31))


# ------------------------------------------------------------------ float sum
def _fraction_sum(x):
    from fractions import Fraction
    return float(sum((Fraction(float(v)) for v in x), Fraction(0)))   # rounds once


def test_sum_f32_matches_exact_rationals():
    # Python's float(Fraction) rounds the exact rational correctly; the
    # inputs span the whole float32 range, denormals and zeros included.
    g = np.random.default_rng(31)
    for trial in range(40):
        n = int(g.integers(1, 200))
        exp = g.integers(-149, 127, size=n)
        sig = 1.0 + g.random(n)
        x = (np.where(g.random(n) < 0.5, -1.0, 1.0) * np.ldexp(sig, exp))
        x = np.clip(x, -3.4e38, 3.4e38).astype(np.float32)
        x[g.random(n) < 0.1] = 0.0
        assert oracle.sum_f32(x) == _fraction_sum(x), trial


def test_sum_f32_matches_fsum():
    import math
    for seed, (lo, hi) in [(32, (-40, 40)), (33, (-126, 100)), (34, (-2, 2))]:
        x = workloads.wide_f32(200001, seed, lo, hi)
        assert oracle.sum_f32(x) == math.fsum(x.astype(np.float64))


def test_sum_f32_closed_forms():
    # integers 1..n are exact in float32 up to 2^24; their sum is n(n+1)/2
    n = 1 << 20
    assert oracle.sum_f32(np.arange(1, n + 1, dtype=np.float32)) == n * (n + 1) / 2
    # catastrophic cancellation keeps the small term exactly
    assert oracle.sum_f32(np.array([2.0 ** 100, 1.0, -(2.0 ** 100)], np.float32)) == 1.0
    assert oracle.sum_f32(np.array([2.0 ** 100, 2.0 ** -100, -(2.0 ** 100)], np.float32)) \
        == 2.0 ** -100
    # 2^k copies of the smallest denormal, and of the largest float
    tiny = np.full(1 << 12, np.float32(2.0 ** -149))
    assert oracle.sum_f32(tiny) == 2.0 ** -137
    big = np.full(1 << 20, np.finfo(np.float32).max)
    assert oracle.sum_f32(big) == float(np.finfo(np.float32).max) * 2.0 ** 20
    assert oracle.sum_f32(-big) == -float(np.finfo(np.float32).max) * 2.0 ** 20


def test_sum_f32_rounds_once_to_nearest_even():
    t = 2.0 ** 53
    cases = [([t, 1.0], t),                    # halfway, even below
             ([t, 1.0, 2.0], t + 4.0),         # 2^53 + 3: halfway, even above
             ([t, 1.0, 2.0 ** -20], t + 2.0),  # just above halfway
             ([t, 1.0, -(2.0 ** -20)], t),     # just below halfway
             ([t, t, 1.0], 2 * t)]             # 2^54 + 1: below halfway of step 4
    for xs, want in cases:
        x = np.array(xs, np.float32)
        assert oracle.sum_f32(x) == want, xs
        assert oracle.sum_f32(-x) == -want, xs


def test_sum_f32_is_order_free_and_empty_is_zero():
    x = workloads.wide_f32(50000, 35)
    p = np.random.default_rng(36).permutation(x.size)
    assert oracle.sum_f32(x[p]) == oracle.sum_f32(x)
    assert oracle.sum_f32(x[::-1]) == oracle.sum_f32(x)
    assert oracle.sum_f32(np.zeros(0, np.float32)) == 0.0
    assert oracle.sum_f32(np.array([-0.0, -0.0], np.float32)) == 0.0


def test_sum_f32_non_finite_follow_ieee():
    inf, nan = np.float32(np.inf), np.float32(np.nan)
    assert oracle.sum_f32(np.array([1.0, inf, -5.0], np.float32)) == np.inf
    assert oracle.sum_f32(np.array([1.0, -inf], np.float32)) == -np.inf
    assert np.isnan(oracle.sum_f32(np.array([inf, 2.0, -inf], np.float32)))
    assert np.isnan(oracle.sum_f32(np.array([1.0, nan, inf], np.float32)))


# ------------------------------------------------------------------ float scan
def test_scan_f32_matches_exact_rationals():
    from fractions import Fraction
    g = np.random.default_rng(37)
    for trial in range(25):
        n = int(g.integers(1, 120))
        x = (np.where(g.random(n) < 0.5, -1.0, 1.0) *
             np.ldexp(1.0 + g.random(n), g.integers(-149, 127, size=n)))
        x = np.clip(x, -3.4e38, 3.4e38).astype(np.float32)
        acc, want = Fraction(0), []
        for v in x:
            acc += Fraction(float(v))
            want.append(float(acc))        # rounds once
        assert oracle.scan_f32(x).tolist() == want, trial


def test_scan_f32_closed_forms_and_cancellation():
    n = 1 << 16
    k = np.arange(1, n + 1, dtype=np.float64)
    assert np.array_equal(oracle.scan_f32(k.astype(np.float32)), k * (k + 1) / 2)
    x = np.array([2.0 ** 100, 1.0, -(2.0 ** 100), 1.0, 2.0 ** -149], np.float32)
    # 2^100 + 1 is not a double: it rounds to 2^100; the exact sum keeps the 1
    # 2 + 2^-149 needs 150 significant bits: it rounds to 2
    assert oracle.scan_f32(x).tolist() == [2.0 ** 100, 2.0 ** 100, 1.0, 2.0, 2.0]


def test_scan_f32_positions_last_and_fsum():
    import math
    x = workloads.wide_f32(100_003, 38)
    full = oracle.scan_f32(x)
    idx = np.sort(np.random.default_rng(39).choice(x.size, 500, replace=False))
    idx = np.concatenate([[0, 0], idx, [x.size - 1]]).astype(np.int64)
    assert np.array_equal(oracle.scan_f32(x, idx), full[idx])
    assert full[-1] == oracle.sum_f32(x)
    for i in idx[::25]:
        assert full[i] == math.fsum(x[: i + 1].astype(np.float64))
    with pytest.raises(ValueError):
        oracle.scan_f32(x, np.array([5, 4], np.int64))
    with pytest.raises(ValueError):
        oracle.scan_f32(x, np.array([x.size], np.int64))
    assert oracle.scan_f32(np.zeros(0, np.float32)).size == 0
