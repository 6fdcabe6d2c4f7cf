"""The all-core CPU baseline loops (oracle/cpu_parallel.c) give the oracle's
results: the benchmark reports their throughput beside the single-thread
oracle, so they must compute the same thing."""
import numpy as np
import pytest

import oracle
import workloads


@pytest.mark.parametrize("n", [0, 1, 7, 1000, (1 << 20) + 3])
def test_omp_reduce_and_scan_equal_the_oracle(n):
    x = workloads.int_uniform(n, seed=70)
    assert oracle.omp_reduce_i32(x) == oracle.reduce_i32(x)
    assert np.array_equal(oracle.omp_scan_i32(x), oracle.scan_i32(x))


def test_omp_scan_wraps_like_the_oracle():
    x = np.full(100003, 2**31 - 5, np.int32)
    assert np.array_equal(oracle.omp_scan_i32(x), oracle.scan_i32(x))


@pytest.mark.parametrize("rows,cols", [(1, 1), (3, 200), (64, 64), (130, 67), (1000, 513)])
def test_omp_transpose_equals_the_oracle(rows, cols):
    m = workloads.self_describing_u32(rows, cols)
    assert np.array_equal(oracle.omp_transpose_u32(m), oracle.transpose_u32(m).view(np.uint32))
