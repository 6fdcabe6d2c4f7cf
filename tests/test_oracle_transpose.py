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


# ----------------------------------------------------------------- 1-, 2-, 8-byte elements
DTYPES = [np.uint8, np.uint16, np.uint32, np.uint64]


@pytest.mark.parametrize("dtype", DTYPES)
@pytest.mark.parametrize("rows,cols", [(1, 1), (1, 37), (37, 1), (65, 129), (300, 7)])
def test_bytes_self_describing(dtype, rows, cols):
    # element (r, c) holds its own index r * cols + c modulo the element range
    bits = 8 * np.dtype(dtype).itemsize
    idx = np.arange(rows * cols, dtype=np.uint64).reshape(rows, cols)
    m = (idx % (1 << bits) if bits < 64 else idx).astype(dtype)
    t = oracle.transpose_bytes(m)
    r = np.arange(rows, dtype=np.uint64)[None, :]
    c = np.arange(cols, dtype=np.uint64)[:, None]
    want = r * cols + c
    assert np.array_equal(t, (want % (1 << bits) if bits < 64 else want).astype(dtype))


@pytest.mark.parametrize("dtype", DTYPES)
def test_bytes_involution_and_numpy(dtype):
    m = workloads.rng(50).integers(0, np.iinfo(dtype).max, size=(123, 77), dtype=dtype,
                                   endpoint=True)
    t = oracle.transpose_bytes(m)
    assert np.array_equal(t, m.T)
    assert np.array_equal(oracle.transpose_bytes(t), m)


def test_bytes_f64_bits_preserved():
    # the paper's own example transposes doubles: NaN payloads, -0.0,
    # subnormals and infinities move unchanged
    pats = np.array([0x7FF8000000000001, 0xFFF0DEADBEEF0001, 0x8000000000000000,
                     0x0000000000000001, 0x7FF0000000000000, 0x3FF0000000000000],
                    dtype=np.uint64)
    m = np.tile(pats, (4, 3))  # 4 x 18
    t = oracle.transpose_bytes(m.view(np.float64)).view(np.uint64)
    assert np.array_equal(t, m.T)


def test_bytes_matches_32_bit_form():
    m = workloads.matrix_f32(65, 33, seed=51)
    assert np.array_equal(oracle.transpose_bytes(m), oracle.transpose_u32(m))


# ----------------------------------------------------------------- reversal (the reverse view)
@pytest.mark.parametrize("n", [0, 1, 2, 3, 4, 5, 1000, 4097])
def test_reverse_self_describing_and_involution(n):
    x = np.arange(n, dtype=np.uint32)
    y = oracle.reverse_u32(x)
    assert np.array_equal(y, np.arange(n - 1, -1, -1, dtype=np.uint32) if n else y)
    assert np.array_equal(oracle.reverse_u32(y), x)


def test_reverse_matches_numpy_and_keeps_bits():
    x = workloads.matrix_f32(1, 12345, seed=52).ravel()
    x[:4] = np.array([0x7FC00001, 0x80000000, 0x00000001, 0xFF800000], np.uint32).view(np.float32)
    y = oracle.reverse_u32(x)
    assert np.array_equal(y.view(np.uint32), x[::-1].view(np.uint32))
