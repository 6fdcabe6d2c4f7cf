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


# ------------------------------------------------------------------ FP8 pins at general scales
def _e4m3_codes_by_library(t):
    """OCP e4m3 codes of float32 values |t| < 464 (torch's round-to-nearest-even)."""
    return torch.from_numpy(np.ascontiguousarray(t, np.float32)).to(
        torch.float8_e4m3fn).view(torch.uint8).numpy()


def _quant_rows_float32_steps(A, inv_step="f32", mul_step="f32"):
    """Row quantisation written with numpy float32 arithmetic, one operation
    per rounding: alpha = max|a|, inv = 448 / alpha (float32 division),
    t = a * inv (float32 product), codes by the library encoder, scale =
    alpha / 448.  inv_step / mul_step select deliberately wrong variants."""
    alpha = np.abs(A).max(axis=1).astype(np.float32)
    nz = alpha > 0
    if inv_step == "f32":
        inv = np.where(nz, np.float32(448.0) / np.where(nz, alpha, 1), np.float32(1.0))
        inv = inv.astype(np.float32)
    else:  # inverse kept in FP64
        inv = np.where(nz, 448.0 / np.where(nz, alpha, 1).astype(np.float64), 1.0)
    if mul_step == "f32":
        t = (A * inv[:, None]).astype(np.float32)
    elif mul_step == "div":   # a / (alpha / 448) instead of a * (448 / alpha)
        s = (alpha / np.float32(448.0)).astype(np.float32)
        t = np.where(nz[:, None], A / np.where(nz, s, 1)[:, None], A).astype(np.float32)
    else:                     # product in FP64 encoded without the float32 rounding
        t = A.astype(np.float64) * inv[:, None].astype(np.float64)
        return _e4m3_encode_f64(t), alpha, (alpha / np.float32(448.0)).astype(np.float32)
    return _e4m3_codes_by_library(t), alpha, (alpha / np.float32(448.0)).astype(np.float32)


def _e4m3_encode_f64(t):
    """Nearest e4m3 value of doubles |t| <= 448, ties to the even code."""
    codes = np.arange(0, 0x7F, dtype=np.int64)
    vals = np.array([_e4m3_value_from_definition(int(c)) for c in codes])
    a = np.abs(t).ravel()
    hi = np.clip(np.searchsorted(vals, a), 1, vals.size - 1)
    lo = hi - 1
    dlo, dhi = a - vals[lo], vals[hi] - a
    pick = np.where(dlo < dhi, lo, np.where(dhi < dlo, hi, np.where(codes[lo] % 2 == 0, lo, hi)))
    q = codes[pick] | np.where(np.signbit(t.ravel()), 0x80, 0)
    return q.astype(np.uint8).reshape(t.shape)


def test_quant_rows_equal_float32_steps_and_separate_wrong_steps():
    # Rows of very different magnitudes; the codes, absmax and scales must be
    # those of the float32 steps bit for bit, and the same data must separate
    # the plausible wrong steps (inverse in FP64, product in FP64, division
    # by the scale), so that each of them fails this pin.
    # Besides random values, each row holds values whose scaled image lies
    # within a few float32 steps of an e4m3 rounding point (the midpoint of two
    # neighbouring codes), where one rounding more or less changes the code.
    g = workloads.rng(41)
    M, K = 512, 1024
    A = (g.standard_normal((M, K)) * 2.0 ** g.integers(-20, 20, (M, 1))).astype(np.float32)
    grid = np.unique(oracle.e4m3_decode(np.arange(0, 0x7F, dtype=np.uint8)))
    mids = (grid[:-1] + grid[1:]) / 2.0
    for i in range(M):
        alpha = np.float32(np.abs(A[i]).max())
        m = g.choice(mids, 128)
        a = (m * (float(alpha) / 448.0)).astype(np.float32)
        near = np.concatenate([a, np.nextafter(a, np.float32(np.inf)),
                               np.nextafter(a, np.float32(0))])
        near = np.minimum(near, alpha)                    # alpha stays the absmax
        A[i, 1:1 + near.size] = near * g.choice([-1, 1], near.size).astype(np.float32)
    A[7] = 0.0
    q, al, sc = oracle.quant_rows_e4m3(A)
    want_q, want_al, want_sc = _quant_rows_float32_steps(A)
    assert np.array_equal(q, want_q)
    assert np.array_equal(al, want_al) and np.array_equal(sc, want_sc)
    for inv_step, mul_step in (("f64", "f32"), ("f32", "f64"), ("f32", "div")):
        wrong_q = _quant_rows_float32_steps(A, inv_step, mul_step)[0]
        assert not np.array_equal(q, wrong_q), (inv_step, mul_step)
    # columns: the same steps on B^T
    B = np.ascontiguousarray(A[:300, :200].T)
    qc, be, scc = oracle.quant_cols_e4m3(B)
    wq, wal, wsc = _quant_rows_float32_steps(np.ascontiguousarray(B.T))
    assert np.array_equal(qc, wq.T) and np.array_equal(be, wal) and np.array_equal(scc, wsc)


def test_quant_rows_within_half_spacing():
    # deq(q) * 448 / alpha approximates a to within half an e4m3 spacing at the
    # scaled value, plus the two float32 roundings of the scaling (2^-23
    # relative); spacing 2^(floor(log2|u|) - 3) for |u| >= 2^-6, else 2^-9.
    g = workloads.rng(42)
    A = (g.standard_normal((64, 700)) * 2.0 ** g.integers(-30, 30, (64, 1))).astype(np.float32)
    q, al, _ = oracle.quant_rows_e4m3(A)
    u = A.astype(np.float64) * (448.0 / al.astype(np.float64))[:, None]
    dq = np.array([_e4m3_value_from_definition(int(c)) for c in q.ravel()]).reshape(q.shape)
    au = np.abs(u)
    spacing = np.where(au >= 2.0**-6, 2.0 ** (np.floor(np.log2(np.maximum(au, 2.0**-6))) - 3),
                       2.0**-9)
    assert np.all(np.abs(dq - u) <= 0.5 * spacing + 2.0**-23 * au * 1.0000001)
    assert np.all(np.abs(dq) <= 448.0)


def test_fp8_reference_power_of_two_scales():
    # Scaling A by 2^a and B by 2^b leaves every code unchanged and multiplies
    # the scales by exactly 2^a and 2^b (448/alpha and alpha/448 move by exact
    # powers of two), so Rq and Dq move by exactly 2^(a+b): a reference that
    # drops a scale, or uses one twice, fails for a != b.
    A = workloads.matrix_f32(40, 192, seed=43)
    B = workloads.matrix_f32(192, 30, seed=44)
    ii, jj = workloads.sample_pairs(40, 30, 300, seed=45)
    qa, ala, sa = oracle.quant_rows_e4m3(A)
    qb, alb, sb = oracle.quant_cols_e4m3(B)
    Rq, Dq = oracle.gemm_fp8_sampled(qa, qb, sa, sb, ii, jj)
    for a, b in ((5, -3), (-11, 7), (0, 9)):
        qa2, ala2, sa2 = oracle.quant_rows_e4m3((A * np.float32(2.0**a)).astype(np.float32))
        qb2, alb2, sb2 = oracle.quant_cols_e4m3((B * np.float32(2.0**b)).astype(np.float32))
        assert np.array_equal(qa2, qa) and np.array_equal(qb2, qb)
        assert np.array_equal(sa2, sa * np.float32(2.0**a)) and np.array_equal(sb2, sb * np.float32(2.0**b))
        Rq2, Dq2 = oracle.gemm_fp8_sampled(qa2, qb2, sa2, sb2, ii, jj)
        assert np.array_equal(Rq2, Rq * 2.0 ** (a + b)) and np.array_equal(Dq2, Dq * 2.0 ** (a + b))


def test_fp8_reference_is_the_exact_scaled_sum_rounded_once():
    # With general (non power-of-two) scales the reference equals the exact
    # rational s_a s_b sum_k deq(qa) deq(qb), rounded once to a double: every
    # product of two e4m3 values is a multiple of 2^-18 below 2^18, so the FP64
    # sum of up to 2^12 of them is exact, s_a s_b (two floats) is exact in FP64,
    # and only the final product rounds.  Decoding here follows the format
    # definition, not the oracle's decoder.
    from fractions import Fraction
    g = workloads.rng(46)
    M, N, K = 12, 9, 320
    A = (g.standard_normal((M, K)) * g.uniform(0.01, 30.0, (M, 1))).astype(np.float32)
    B = (g.standard_normal((K, N)) * g.uniform(0.01, 30.0, (1, N))).astype(np.float32)
    qa, _, sa = oracle.quant_rows_e4m3(A)
    qb, _, sb = oracle.quant_cols_e4m3(B)
    assert len(set(sa.tolist())) == M and not np.any(np.log2(sa) == np.round(np.log2(sa)))
    ii, jj = np.meshgrid(np.arange(M), np.arange(N), indexing="ij")
    ii, jj = ii.ravel(), jj.ravel()
    Rq, Dq = oracle.gemm_fp8_sampled(qa, qb, sa, sb, ii, jj)
    val = {c: Fraction(_e4m3_value_from_definition(c)) for c in range(256) if (c & 0x7F) != 0x7F}
    for s, (i, j) in enumerate(zip(ii, jj)):
        terms = [val[int(qa[i, k])] * val[int(qb[k, j])] for k in range(K)]
        sc = Fraction(float(sa[i])) * Fraction(float(sb[j]))
        assert Rq[s] == float(sc * sum(terms))
        assert Dq[s] == float(abs(sc) * sum(abs(t) for t in terms))
