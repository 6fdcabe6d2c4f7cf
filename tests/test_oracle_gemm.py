"""Pins of the GEMM references (Sec. 5 "matrix multiplication") and of the
precision forms: split-BF16 operands and OCP e4m3 row/column quantisation.

Pins used: exact integer products (numpy int64 matmul), the identity matrix,
a correctly rounded sum (math.fsum of exact products), torch's bfloat16 and
float8_e4m3fn conversions (library round-to-nearest-even), values fixed by
the format definitions, and algebraic properties of the split.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import workloads


def _int_matrix(rows, cols, seed, lo=-4, hi=4):
    return workloads.rng(seed).integers(lo, hi + 1, size=(rows, cols)).astype(np.float32)


# ------------------------------------------------------------------ FP64 reference
def test_ref_exact_on_integers_nonsquare():
    M, N, K = 37, 53, 301
    A = _int_matrix(M, K, 1); B = _int_matrix(K, N, 2)
    ii, jj = np.meshgrid(np.arange(M), np.arange(N), indexing="ij")
    R, D = oracle.gemm_ref_sampled(A, B, ii.ravel(), jj.ravel())
    exact = A.astype(np.int64) @ B.astype(np.int64)
    assert np.array_equal(R, exact.ravel().astype(np.float64))
    absx = np.abs(A).astype(np.int64) @ np.abs(B).astype(np.int64)
    assert np.array_equal(D, absx.ravel().astype(np.float64))


def test_ref_identity():
    A = workloads.matrix_f32(24, 40, seed=4)
    I = np.eye(40, dtype=np.float32)
    ii, jj = np.meshgrid(np.arange(24), np.arange(40), indexing="ij")
    R, D = oracle.gemm_ref_sampled(A, I, ii.ravel(), jj.ravel())
    assert np.array_equal(R, A.ravel().astype(np.float64))
    assert np.array_equal(D, np.abs(A).ravel().astype(np.float64))


def test_ref_within_fp64_bound_of_correctly_rounded_sum():
    M, N, K = 8, 9, 4096
    A = workloads.matrix_f32(M, K, seed=4); B = workloads.matrix_f32(K, N, seed=5)
    ii, jj = workloads.sample_pairs(M, N, 30, seed=6)
    R, D = oracle.gemm_ref_sampled(A, B, ii, jj)
    for s in range(ii.size):
        exact = math.fsum(float(A[ii[s], k]) * float(B[k, jj[s]]) for k in range(K))
        assert abs(R[s] - exact) <= K * 2.0**-53 * D[s]
        assert D[s] >= abs(exact)


# ------------------------------------------------------------------ bfloat16
BF16_CASES = [
    (0x3F800000, 0x3F80),  # 1.0
    (0x3F808000, 0x3F80),  # tie, even stays
    (0x3F818000, 0x3F82),  # tie, odd rounds up
    (0x3F808001, 0x3F81),  # above the tie
    (0x3F807FFF, 0x3F80),  # below the tie
    (0x7F7FFFFF, 0x7F80),  # largest float rounds to +inf
    (0xFF800000, 0xFF80),  # -inf
    (0x80000000, 0x8000),  # -0
    (0x00008000, 0x0000),  # subnormal tie to even (zero)
    (0x00018000, 0x0002),  # subnormal tie, odd rounds up
    (0x007FFFFF, 0x0080),  # largest subnormal rounds into the normals
]


@pytest.mark.parametrize("bits,expect", BF16_CASES)
def test_bf16_fixed_values(bits, expect):
    x = np.array([bits], np.uint32).view(np.float32)
    assert int(oracle.bf16_rne(x)[0]) == expect


def test_bf16_nan_stays_quiet_nan():
    x = np.array([0x7F800001, 0xFFA00000, 0x7FC00000], np.uint32).view(np.float32)
    h = oracle.bf16_rne(x)
    assert all(((v & 0x7F80) == 0x7F80) and (v & 0x7F) != 0 and (v & 0x40) for v in h.tolist())


def test_bf16_matches_torch_on_random_patterns():
    pats = workloads.rng(21).integers(0, 2**32, size=1 << 22, dtype=np.uint64).astype(np.uint32)
    x = pats.view(np.float32)
    finite = np.isfinite(x) | np.isinf(x)
    x = x[finite]
    ours = oracle.bf16_rne(x)
    ref = torch.from_numpy(x.copy()).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    assert np.array_equal(ours, ref)


def test_split_properties():
    a = workloads.normal_f32(1 << 20, seed=22)
    h, l = oracle.split_bf16(a)
    hf = oracle.bf16_to_f32(h).astype(np.float64)
    lf = oracle.bf16_to_f32(l).astype(np.float64)
    # torch reproduces both halves with its own RNE conversion
    th = torch.from_numpy(a).to(torch.bfloat16)
    rest = torch.from_numpy(a) - th.to(torch.float32)
    assert np.array_equal(h, th.view(torch.int16).numpy().view(np.uint16))
    assert np.array_equal(l, rest.to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16))
    a64 = a.astype(np.float64)
    # |a - h| <= 2^-9 |a|, and the two-term error is <= 2^-17 |a| (+ subnormal slack)
    assert np.all(np.abs(a64 - hf) <= 2.0**-8 * np.abs(a64))
    assert np.all(np.abs(a64 - hf - lf) <= 2.0**-16 * np.abs(a64) + 1e-44)
    # values with at most 16 significant bits split exactly
    b = (workloads.rng(23).integers(-2**15, 2**15, size=4096)).astype(np.float32)
    bh, bl = oracle.split_bf16(b)
    assert np.array_equal(oracle.bf16_to_f32(bh) + oracle.bf16_to_f32(bl), b)


def test_bf16x3_reference_exact_for_integer_operands():
    # small integers are exact in bf16: lo = 0 and R3 is the exact product
    M, N, K = 16, 12, 257
    A = _int_matrix(M, K, 7); B = _int_matrix(K, N, 8)
    ii, jj = np.meshgrid(np.arange(M), np.arange(N), indexing="ij")
    R3, D3 = oracle.gemm_bf16x3_sampled(A, B, ii.ravel(), jj.ravel())
    exact = (A.astype(np.int64) @ B.astype(np.int64)).ravel()
    assert np.array_equal(R3, exact.astype(np.float64))


def test_bf16x3_reference_close_to_true_product():
    M, N, K = 6, 7, 2048
    A = workloads.matrix_f32(M, K, 9); B = workloads.matrix_f32(K, N, 10)
    ii, jj = workloads.sample_pairs(M, N, 42, seed=11)
    R, D = oracle.gemm_ref_sampled(A, B, ii, jj)
    R3, D3 = oracle.gemm_bf16x3_sampled(A, B, ii, jj)
    # dropped al*bl term and the residual of the split: <= ~3 * 2^-16 per |a||b|
    assert np.all(np.abs(R3 - R) <= 3 * 2.0**-16 * D)
    assert np.max(np.abs(R3 - R) / D) < 1e-5


def test_bf16x3_short_sums_reach_past_1e5():
    # K = 1: each entry is one product, so the split's error does not average
    # out; the 3-product scheme exceeds 1e-5 on some entries and stays inside
    # its a-priori bound 3 * 2^-16 on all (why the GPU tests use that bound
    # for K < 64)
    M, N, K = 64, 64, 1
    A = workloads.matrix_f32(M, K, 24); B = workloads.matrix_f32(K, N, 25)
    ii, jj = np.meshgrid(np.arange(M), np.arange(N), indexing="ij")
    R, D = oracle.gemm_ref_sampled(A, B, ii.ravel(), jj.ravel())
    R3, _ = oracle.gemm_bf16x3_sampled(A, B, ii.ravel(), jj.ravel())
    e = np.abs(R3 - R) / D
    assert e.max() > 1e-5
    assert e.max() <= 3 * 2.0**-16


# ------------------------------------------------------------------ e4m3
def _e4m3_value_from_definition(code: int) -> float:
    s = -1.0 if code & 0x80 else 1.0
    e, m = (code >> 3) & 0xF, code & 7
    if e == 15 and m == 7:
        return math.nan
    if e == 0:
        return s * m * 2.0**-9
    return s * (1 + m / 8.0) * 2.0 ** (e - 7)


def test_e4m3_decode_all_codes():
    codes = np.arange(256, dtype=np.uint8)
    ours = oracle.e4m3_decode(codes)
    lib = torch.from_numpy(codes.copy()).view(torch.float8_e4m3fn).to(torch.float64).numpy()
    for c in range(256):
        want = _e4m3_value_from_definition(c)
        if math.isnan(want):
            assert math.isnan(ours[c]) and math.isnan(lib[c])
        else:
            assert ours[c] == want == lib[c]
    assert ours[0x7E] == 448.0 and ours[0x08] == 2.0**-6 and ours[0x01] == 2.0**-9
    assert ours[0x38] == 1.0


def test_e4m3_encode_matches_torch_in_range():
    g = workloads.rng(31)
    x = np.concatenate([
        g.uniform(-463.9, 463.9, 200000),
        g.standard_normal(200000) * 2.0**g.integers(-14, 4, 200000),
        np.array([0.0, -0.0, 2.0**-10, 3 * 2.0**-10, 2.0**-6, 2.0**-6 * 0.999, 463.99, 240.0]),
    ]).astype(np.float32)
    ours = oracle.e4m3_encode(x)
    lib = torch.from_numpy(x).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    assert np.array_equal(ours, lib)


def test_e4m3_roundtrip_and_saturation():
    codes = np.array([c for c in range(256) if (c & 0x7F) != 0x7F], np.uint8)
    vals = oracle.e4m3_decode(codes).astype(np.float32)
    assert np.array_equal(oracle.e4m3_encode(vals), codes)
    sat = np.array([448.0, 449.0, 464.0, 470.0, 1e30, np.inf, -500.0, -np.inf], np.float32)
    assert oracle.e4m3_encode(sat).tolist() == [0x7E] * 6 + [0xFE] * 2
    assert oracle.e4m3_encode(np.array([np.nan], np.float32))[0] & 0x7F == 0x7F


def test_quant_rows_cols():
    A = workloads.matrix_f32(33, 70, seed=12)
    A[5] = 0.0
    q, al, sc = oracle.quant_rows_e4m3(A)
    assert np.array_equal(al, np.abs(A).max(axis=1))
    assert al[5] == 0.0 and sc[5] == 0.0 and not q[5].any()
    # every row contains a code of magnitude 448 (its absmax element)
    for i in range(33):
        if i != 5:
            assert (q[i] & 0x7F).max() == 0x7E
    # columns of B are rows of B^T
    B = workloads.matrix_f32(70, 21, seed=13)
    qc, be, scc = oracle.quant_cols_e4m3(B)
    qr, ber, scr = oracle.quant_rows_e4m3(np.ascontiguousarray(B.T))
    assert np.array_equal(qc, qr.T) and np.array_equal(be, ber) and np.array_equal(scc, scr)


def test_fp8_reference_exact_when_codes_are_exact():
    # Rows whose values are already e4m3 numbers with absmax 448 quantise
    # losslessly (scale 1); the reference is then the exact product.
    g = workloads.rng(14)
    grid = oracle.e4m3_decode(np.arange(0, 0x7F, dtype=np.uint8))  # non-negative finite values
    M, N, K = 5, 6, 64
    A = (g.choice(grid, (M, K)) * g.choice([-1, 1], (M, K))).astype(np.float32)
    B = (g.choice(grid, (K, N)) * g.choice([-1, 1], (K, N))).astype(np.float32)
    A[:, 0] = 448.0; B[0, :] = 448.0
    qa, _, sa = oracle.quant_rows_e4m3(A)
    qb, _, sb = oracle.quant_cols_e4m3(B)
    assert np.all(sa == 1.0) and np.all(sb == 1.0)
    ii, jj = np.meshgrid(np.arange(M), np.arange(N), indexing="ij")
    Rq, Dq = oracle.gemm_fp8_sampled(qa, qb, sa, sb, ii.ravel(), jj.ravel())
    for s, (i, j) in enumerate(zip(ii.ravel(), jj.ravel())):
        exact = math.fsum(float(A[i, k]) * float(B[k, j]) for k in range(K))
        assert Rq[s] == exact
