"""Seeded synthetic inputs for the hot-path workloads.

This module only draws random numbers and lays them out; it holds none of
the arithmetic of the operations themselves.  Both the CPU oracle (through
the tests) and the GPU library (through the tests and the benchmark) are fed
from here, so that they always see identical inputs.

Generator: numpy ``Generator(PCG64(seed))``.

* integers: ``integers(-1024, 1025, dtype=int32)``, i.e. uniform over the
  closed range [-1024, 1024] (2049 values);
* normal FP32: ``standard_normal(dtype=float64).astype(float32)`` (the cast
  rounds to nearest even);
* segment lengths: ``floor(2 ** (u * log2(2**20 + 1)))`` with ``u`` uniform in
  [0, 1), which is log-uniform over [1, 2**20]; the offsets array is the
  exclusive running total of the lengths (``offsets[0] = 0``,
  ``offsets[S] = T``);
* wide-range FP32: sign from ``random() < 0.5``, significand ``1 + random()``,
  exponent ``integers(emin, emax + 1)`` (default [-40, 40]), cast to float32;
* grouped GEMM shapes: ``64 * integers(1, 17, size=(G, 3))`` -> (M, N, K)
  each uniform over {64, 128, ..., 1024}.

Seeds of the named workloads are collected in ``SEEDS``.
"""
from __future__ import annotations

import math

import numpy as np

SEEDS = {
    "reduce": 1,            # 2**22 int32
    "scan": 2,              # 2**28 int32
    "transpose": 3,         # 8192 x 8192 f32
    "gemm4096_a": 4, "gemm4096_b": 5, "gemm4096_samples": 6,
    "gemm8192_a": 7, "gemm8192_b": 8, "gemm8192_samples": 9,
    "seg_lengths": 10, "seg_values": 11,
    "grouped_shapes": 12, "grouped_values": 13, "grouped_samples": 14,
    "reduce_f32": 15,       # 2**28 float32, wide exponent range
}

SIZES = {
    "reduce_n": 1 << 22,
    "scan_n": 1 << 28,
    "transpose_rows": 8192, "transpose_cols": 8192,
    "gemm_sizes": (4096, 8192),
    "gemm_samples": 4096,
    "seg_count": 4096, "seg_max_len": 1 << 20,
    "grouped_count": 512, "grouped_samples_per_problem": 64,
}


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def int_uniform(n: int, seed: int, lo: int = -1024, hi: int = 1024) -> np.ndarray:
    """``n`` int32 values uniform over the closed range [lo, hi]."""
    return rng(seed).integers(lo, hi + 1, size=n, dtype=np.int32)


def normal_f32(shape, seed: int) -> np.ndarray:
    """N(0, 1) drawn in float64 and rounded to float32."""
    return rng(seed).standard_normal(size=shape, dtype=np.float64).astype(np.float32)


def wide_f32(n: int, seed: int, emin: int = -40, emax: int = 40) -> np.ndarray:
    """``n`` float32 values with a random sign, a significand uniform in
    [1, 2) and an exponent uniform over [emin, emax] (a wide dynamic range,
    so that the order of a floating-point sum shows in its rounding)."""
    g = rng(seed)
    sig = 1.0 + g.random(n)
    exp = g.integers(emin, emax + 1, size=n)
    sign = np.where(g.random(n) < 0.5, -1.0, 1.0)
    return (sign * np.ldexp(sig, exp)).astype(np.float32)


def matrix_f32(rows: int, cols: int, seed: int) -> np.ndarray:
    return normal_f32((rows, cols), seed)


def segment_lengths(num_segments: int, seed: int, max_len: int = 1 << 20) -> np.ndarray:
    """Log-uniform lengths in [1, max_len] (int64)."""
    u = rng(seed).random(num_segments)
    lengths = np.floor(2.0 ** (u * math.log2(max_len + 1))).astype(np.int64)
    return np.clip(lengths, 1, max_len)


def offsets_from_lengths(lengths) -> np.ndarray:
    """Exclusive running total of the lengths, with the total appended."""
    lengths = np.asarray(lengths, dtype=np.int64)
    out = np.zeros(len(lengths) + 1, dtype=np.int64)
    np.cumsum(lengths, out=out[1:])
    return out


def segmented_input(num_segments: int = 4096, len_seed: int = 10, val_seed: int = 11,
                    max_len: int = 1 << 20):
    """(values int32[T], offsets int64[S+1]) of the segmented workload."""
    offsets = offsets_from_lengths(segment_lengths(num_segments, len_seed, max_len))
    values = int_uniform(int(offsets[-1]), val_seed)
    return values, offsets


def grouped_shapes(count: int = 512, seed: int = 12, step: int = 64, max_mult: int = 16):
    """(count, 3) int64 array of (M, N, K)."""
    return step * rng(seed).integers(1, max_mult + 1, size=(count, 3)).astype(np.int64)


def grouped_operands(shapes, seed: int = 13):
    """List of (A[M,K], B[K,N]) float32 pairs drawn in problem order."""
    g = rng(seed)
    out = []
    for m, n, k in np.asarray(shapes):
        a = g.standard_normal(size=(int(m), int(k)), dtype=np.float64).astype(np.float32)
        b = g.standard_normal(size=(int(k), int(n)), dtype=np.float64).astype(np.float32)
        out.append((a, b))
    return out


def sample_pairs(rows: int, cols: int, count: int, seed: int):
    """``count`` distinct (i, j) positions of a rows x cols matrix (int64 arrays)."""
    count = min(count, rows * cols)
    flat = rng(seed).choice(rows * cols, size=count, replace=False)
    return (flat // cols).astype(np.int64), (flat % cols).astype(np.int64)


def arithmetic_i32(n: int, a: int, d: int) -> np.ndarray:
    """x_i = a + d*i as int32 (caller keeps it in range)."""
    return (a + d * np.arange(n, dtype=np.int64)).astype(np.int32)


def self_describing_u32(rows: int, cols: int) -> np.ndarray:
    """Matrix whose element (r, c) holds the bit pattern r*cols + c."""
    return np.arange(rows * cols, dtype=np.uint64).astype(np.uint32).reshape(rows, cols)
