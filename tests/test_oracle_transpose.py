"""Pins of the oracle transpose (Sec. 1 Listings 1-2, Sec. 5 "matrix
transposition"): involution, self-describing inputs, bit preservation and a
library routine."""
import numpy as np
import pytest

import oracle
import workloads


@pytest.mark.parametrize("rows,cols", [(1, 1), (1, 37), (37, 1), (64, 64), (65, 129), (300, 7)])
def test_self_describing(rows, cols):
    m = workloads.self_describing_u32(rows, cols)
    t = oracle.transpose_u32(m)
    assert t.shape == (cols, rows)
    r = np.arange(rows)[None, :]
    c = np.arange(cols)[:, None]
    assert np.array_equal(t, (r * cols + c).astype(np.uint32))


def test_involution_and_numpy():
    m = workloads.matrix_f32(333, 517, seed=3)
    t = oracle.transpose_u32(m)
    assert np.array_equal(t, m.T)
    assert np.array_equal(oracle.transpose_u32(t).view(np.uint32), m.view(np.uint32))


def test_bits_preserved():
    pats = np.array([0x7FC00001, 0xFFBADBAD, 0x80000000, 0x00000001, 0x7F800000, 0x3F800000],
                    dtype=np.uint32)
    m = np.tile(pats, (5, 3))  # 5 x 18
    t = oracle.transpose_u32(m.view(np.float32)).view(np.uint32)
    assert np.array_equal(t, m.T)
    assert sorted(t.ravel().tolist()) == sorted(m.ravel().tolist())


def test_empty():
    assert oracle.transpose_u32(np.zeros((0, 5), np.float32)).shape == (5, 0)
