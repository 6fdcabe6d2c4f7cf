"""CPU oracle for the data-parallel hot path -- TEST INFRASTRUCTURE ONLY.

A thin numpy front end over ``oracle.c`` (plain C, built with gcc, loaded with
ctypes).  Only the tests, the smoke check and the benchmark's CPU-baseline leg
may import this package; the GPU library never does, and the two share no
code.  See the header of ``oracle.c`` for what each function computes and
which passage of the paper it follows.

Parity status of every function is pinned by ``tests/test_oracle_*.py``
against closed forms, brute force, invariants and library routines.  The
error of the sampled FP8 GEMM against the exact product (as opposed to its
own quantised operands) is reported, not gated: parity unpinned for that
comparison only.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
CFLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared"]


_OMP_SRC = os.path.join(_HERE, "cpu_parallel.c")
_OMP_LIB = os.path.join(_HERE, "liboracle_omp.so")


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (a plain host build), and
    the all-core baseline loops of cpu_parallel.c into liboracle_omp.so."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", *CFLAGS, _SRC, "-o", tmp, "-lm"], check=True)
        os.replace(tmp, _LIB)
    if force or not os.path.exists(_OMP_LIB) or \
            os.path.getmtime(_OMP_LIB) < os.path.getmtime(_OMP_SRC):
        tmp = _OMP_LIB + ".tmp%d" % os.getpid()
        subprocess.run(["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", _OMP_SRC,
                        "-o", tmp], check=True)
        os.replace(tmp, _OMP_LIB)
    return _LIB


_omp = None


def omp_lib() -> ctypes.CDLL:
    """The all-core OpenMP loops (measurement baseline, not the oracle)."""
    global _omp
    if _omp is None:
        if not os.path.exists(_OMP_LIB) or os.path.getmtime(_OMP_LIB) < os.path.getmtime(_OMP_SRC):
            build(force=True)
        L = ctypes.CDLL(_OMP_LIB)
        P, I64 = ctypes.c_void_p, ctypes.c_int64
        L.omp_threads.restype = ctypes.c_int
        L.omp_reduce_i32.argtypes = [P, I64]
        L.omp_reduce_i32.restype = I64
        L.omp_scan_i32.argtypes = [P, P, I64]
        L.omp_transpose_u32.argtypes = [P, P, I64, I64]
        _omp = L
    return _omp


def omp_threads() -> int:
    return omp_lib().omp_threads()


def omp_reduce_i32(x) -> int:
    x = _c(x, np.int32)
    return int(omp_lib().omp_reduce_i32(_p(x), x.size))


def omp_scan_i32(x):
    x = _c(x, np.int32)
    y = np.empty_like(x)
    omp_lib().omp_scan_i32(_p(x), _p(y), x.size)
    return y


def omp_transpose_u32(m):
    m = np.ascontiguousarray(m).view(np.uint32)
    rows, cols = m.shape
    out = np.empty((cols, rows), np.uint32)
    omp_lib().omp_transpose_u32(_p(m), _p(out), rows, cols)
    return out


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        L = ctypes.CDLL(_LIB)
        P, I64, F = ctypes.c_void_p, ctypes.c_int64, ctypes.c_float
        L.oracle_reduce_i32.argtypes = [P, I64]
        L.oracle_reduce_i32.restype = I64
        L.oracle_scan_i32.argtypes = [P, P, I64, P]
        L.oracle_scan_i32.restype = ctypes.c_int
        L.oracle_scan_exclusive_i32.argtypes = [P, P, I64]
        L.oracle_transpose_u32.argtypes = [P, P, I64, I64]
        L.oracle_transpose_bytes.argtypes = [P, P, I64, I64, I64]
        L.oracle_reverse_u32.argtypes = [P, P, I64]
        L.oracle_gemm_ref_sampled.argtypes = [P, I64, P, I64, I64, P, P, I64, P, P]
        L.oracle_bf16_rne.argtypes = [F]
        L.oracle_bf16_rne.restype = ctypes.c_uint16
        L.oracle_bf16_to_f32.argtypes = [ctypes.c_uint16]
        L.oracle_bf16_to_f32.restype = F
        L.oracle_split_bf16.argtypes = [P, P, P, I64]
        L.oracle_gemm_bf16x3_sampled.argtypes = [P, I64, P, I64, I64, P, P, I64, P, P]
        L.oracle_e4m3_encode.argtypes = [F]
        L.oracle_e4m3_encode.restype = ctypes.c_uint8
        L.oracle_e4m3_encode_n.argtypes = [P, P, I64]
        L.oracle_e4m3_decode.argtypes = [ctypes.c_uint8]
        L.oracle_e4m3_decode.restype = ctypes.c_double
        L.oracle_quant_rows_e4m3.argtypes = [P, I64, I64, I64, P, I64, P, P]
        L.oracle_quant_cols_e4m3.argtypes = [P, I64, I64, I64, P, I64, P, P]
        L.oracle_gemm_fp8_sampled.argtypes = [P, I64, P, I64, P, P, I64, P, P, I64, P, P]
        L.oracle_reduce_segmented_i32.argtypes = [P, P, I64, P]
        L.oracle_scan_segmented_i32.argtypes = [P, P, P, I64]
        L.oracle_minmax_i32.argtypes = [P, I64, P]
        L.oracle_sum_f32.argtypes = [P, I64]
        L.oracle_sum_f32.restype = ctypes.c_double
        L.oracle_scan_f32_at.argtypes = [P, I64, P, I64, P]
        L.oracle_scan_f32_at.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


# ----------------------------------------------------------------- reduce / scan
def reduce_i32(x) -> int:
    x = _c(x, np.int32)
    return int(lib().oracle_reduce_i32(_p(x), x.size))


def minmax_i32(x):
    """(min, max) of int32 values; (INT32_MAX, INT32_MIN) for an empty array."""
    x = _c(x, np.int32)
    out = np.empty(2, np.int32)
    lib().oracle_minmax_i32(_p(x), x.size, _p(out))
    return int(out[0]), int(out[1])


def sum_f32(x) -> float:
    """The exact sum of FP32 values rounded once to the nearest double (IEEE
    rules for non-finite inputs; a zero total is +0)."""
    x = _c(x, np.float32)
    return float(lib().oracle_sum_f32(_p(x), x.size))


def scan_f32(x, idx=None) -> np.ndarray:
    """Exact inclusive prefix sums of FP32 values, each rounded once to the
    nearest double, at the ascending positions ``idx`` (all when None)."""
    x = _c(x, np.float32)
    idx = np.arange(x.size, dtype=np.int64) if idx is None else _c(idx, np.int64)
    out = np.empty(idx.size, np.float64)
    if lib().oracle_scan_f32_at(_p(x), x.size, _p(idx), idx.size, _p(out)) != 0:
        raise ValueError("positions must be ascending and below n")
    return out


def scan_i32(x, return_info: bool = False):
    x = _c(x, np.int32)
    y = np.empty_like(x)
    m = ctypes.c_int64(0)
    wrapped = lib().oracle_scan_i32(_p(x), _p(y), x.size, ctypes.byref(m))
    if return_info:
        return y, bool(wrapped), int(m.value)
    return y


def scan_exclusive_i32(x):
    """y[0] = 0, y[i] = (x[0] + ... + x[i-1]) mod 2^32 as int32."""
    x = _c(x, np.int32)
    y = np.empty_like(x)
    lib().oracle_scan_exclusive_i32(_p(x), _p(y), x.size)
    return y


# ----------------------------------------------------------------- transpose
def transpose_u32(m) -> np.ndarray:
    """Transpose of a 2-D array of 32-bit words (any 4-byte dtype; bits kept)."""
    m = np.ascontiguousarray(m)
    assert m.ndim == 2 and m.dtype.itemsize == 4
    rows, cols = m.shape
    out = np.empty((cols, rows), dtype=m.dtype)
    lib().oracle_transpose_u32(_p(m), _p(out), rows, cols)
    return out


def transpose_bytes(m) -> np.ndarray:
    """Transpose of a 2-D array of 1-, 2-, 4- or 8-byte elements (bits kept)."""
    m = np.ascontiguousarray(m)
    assert m.ndim == 2 and m.dtype.itemsize in (1, 2, 4, 8)
    rows, cols = m.shape
    out = np.empty((cols, rows), dtype=m.dtype)
    lib().oracle_transpose_bytes(_p(m), _p(out), rows, cols, m.dtype.itemsize)
    return out


def reverse_u32(x) -> np.ndarray:
    """out[i] = x[n - 1 - i] for a 1-D array of 32-bit elements (bits kept)."""
    x = np.ascontiguousarray(x)
    assert x.ndim == 1 and x.dtype.itemsize == 4
    out = np.empty_like(x)
    lib().oracle_reverse_u32(_p(x), _p(out), x.size)
    return out


# ----------------------------------------------------------------- GEMM
def gemm_ref_sampled(A, B, ii, jj):
    """(R, D) in float64 for the sampled entries of A @ B."""
    A = _c(A, np.float32); B = _c(B, np.float32)
    ii = _c(ii, np.int64); jj = _c(jj, np.int64)
    K = A.shape[1]
    assert B.shape[0] == K
    R = np.empty(ii.size, np.float64); D = np.empty(ii.size, np.float64)
    lib().oracle_gemm_ref_sampled(_p(A), A.shape[1], _p(B), B.shape[1], K,
                                  _p(ii), _p(jj), ii.size, _p(R), _p(D))
    return R, D


def bf16_rne(x):
    """bfloat16 bit patterns (uint16) of float32 values."""
    return split_bf16(x)[0]


def bf16_to_f32(h):
    h = _c(h, np.uint16)
    return (h.astype(np.uint32) << 16).view(np.float32)


def split_bf16(x):
    """(hi, lo) bfloat16 bit patterns of the two-term split of float32 x."""
    x = _c(x, np.float32)
    shape = x.shape
    x = x.ravel()
    hi = np.empty(x.size, np.uint16); lo = np.empty(x.size, np.uint16)
    lib().oracle_split_bf16(_p(x), _p(hi), _p(lo), x.size)
    return hi.reshape(shape), lo.reshape(shape)


def gemm_bf16x3_sampled(A, B, ii, jj):
    A = _c(A, np.float32); B = _c(B, np.float32)
    ii = _c(ii, np.int64); jj = _c(jj, np.int64)
    R = np.empty(ii.size, np.float64); D = np.empty(ii.size, np.float64)
    lib().oracle_gemm_bf16x3_sampled(_p(A), A.shape[1], _p(B), B.shape[1], A.shape[1],
                                     _p(ii), _p(jj), ii.size, _p(R), _p(D))
    return R, D


def e4m3_encode(x):
    x = _c(x, np.float32)
    q = np.empty(x.shape, np.uint8)
    lib().oracle_e4m3_encode_n(_p(x), _p(q), x.size)
    return q


def e4m3_decode(q):
    q = _c(q, np.uint8).ravel()
    return np.array([lib().oracle_e4m3_decode(int(v)) for v in q], dtype=np.float64)


def quant_rows_e4m3(A):
    """(q uint8[M,K], alpha f32[M], scale f32[M]) -- per-row absmax scaling."""
    A = _c(A, np.float32)
    M, K = A.shape
    q = np.empty((M, K), np.uint8); al = np.empty(M, np.float32); sc = np.empty(M, np.float32)
    lib().oracle_quant_rows_e4m3(_p(A), M, K, K, _p(q), K, _p(al), _p(sc))
    return q, al, sc


def quant_cols_e4m3(B):
    """(q uint8[K,N], beta f32[N], scale f32[N]) -- per-column absmax scaling."""
    B = _c(B, np.float32)
    K, N = B.shape
    q = np.empty((K, N), np.uint8); be = np.empty(N, np.float32); sc = np.empty(N, np.float32)
    lib().oracle_quant_cols_e4m3(_p(B), K, N, N, _p(q), N, _p(be), _p(sc))
    return q, be, sc


def gemm_fp8_sampled(qa, qb, sa, sb, ii, jj):
    qa = _c(qa, np.uint8); qb = _c(qb, np.uint8)
    sa = _c(sa, np.float32); sb = _c(sb, np.float32)
    ii = _c(ii, np.int64); jj = _c(jj, np.int64)
    K = qa.shape[1]
    R = np.empty(ii.size, np.float64); D = np.empty(ii.size, np.float64)
    lib().oracle_gemm_fp8_sampled(_p(qa), qa.shape[1], _p(qb), qb.shape[1], _p(sa), _p(sb), K,
                                  _p(ii), _p(jj), ii.size, _p(R), _p(D))
    return R, D


# ----------------------------------------------------------------- segmented
def reduce_segmented_i32(x, offsets):
    x = _c(x, np.int32); off = _c(offsets, np.int64)
    S = off.size - 1
    out = np.empty(S, np.int64)
    lib().oracle_reduce_segmented_i32(_p(x), _p(off), S, _p(out))
    return out


def scan_segmented_i32(x, offsets, fill: int = 0):
    """Segmented inclusive scan; positions outside every segment keep ``fill``."""
    x = _c(x, np.int32); off = _c(offsets, np.int64)
    y = np.full_like(x, fill)
    lib().oracle_scan_segmented_i32(_p(x), _p(y), _p(off), off.size - 1)
    return y
