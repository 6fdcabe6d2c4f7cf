"""Parity of the HIP GEMM paths with the FP64 oracle, through the C ABI.

Error measure (a reading of the stated 1e-5 bound, since an elementwise
relative error is unbounded where an entry is near zero): the componentwise
error e_ij = |C_ij - R_ij| / D_ij with R the FP64 product and
D_ij = sum_k |a_ik| |b_kj|, the normalisation of the standard dot-product
error bound.  Exactly representable cases (small integers, identity) must be
bit-exact."""
import numpy as np
import pytest
import torch

import oracle
import paper_2305_03448_amd as desc
import workloads
from gpu_util import bf16x3_bound, case, dev, needs_gpu, to_dev

pytestmark = [pytest.mark.gpu, needs_gpu]

TOL = {"f32": 1e-5, "bf16x3": 1e-5}
MODES_EXACT = ["f32", "bf16x3"]      # modes exact on small-integer operands
FP8_ACC_TOL = 3e-5                   # fp8 vs the FP64 sum of its own codes (see below)


def _int_matrix(rows, cols, seed, lo=-4, hi=4):
    return workloads.rng(seed).integers(lo, hi + 1, size=(rows, cols)).astype(np.float32)


def _run(A, B, mode, lda_pad=0, ldc_pad=0):
    M, K = A.shape
    N = B.shape[1]
    if lda_pad:
        Ab = to_dev(np.pad(A, ((0, 0), (0, lda_pad))))[:, :K]
    else:
        Ab = to_dev(A)
    Bt = to_dev(B)
    Cbuf = torch.full((M, N + ldc_pad), float("nan"), dtype=torch.float32, device=dev())
    C = Cbuf[:, :N]
    desc.desc_gemm(Ab, Bt, C, mode=mode)
    torch.cuda.synchronize()
    if ldc_pad:
        assert torch.isnan(Cbuf[:, N:]).all(), "wrote outside C"
    return C.cpu().numpy()


def _check_sampled(A, B, C, tol, samples=2048, seed=6):
    M, N = C.shape
    ii, jj = workloads.sample_pairs(M, N, samples, seed)
    R, D = oracle.gemm_ref_sampled(A, B, ii, jj)
    err = np.abs(C[ii, jj].astype(np.float64) - R) / np.maximum(D, 1e-300)
    assert err.max() <= tol, f"componentwise error {err.max():.3e} > {tol}"
    return err.max()


SHAPES = [(1, 1, 1), (5, 7, 3), (32, 32, 2), (64, 64, 16), (100, 37, 129), (128, 128, 128),
          (129, 257, 65), (255, 300, 500), (512, 256, 1024), (33, 1000, 17)]


@pytest.mark.parametrize("M,N,K", SHAPES)
@pytest.mark.parametrize("mode", MODES_EXACT)
def test_gemm_integer_exact(M, N, K, mode):
    case(f"gemm {mode} integer {M}x{N}x{K}")
    A = _int_matrix(M, K, 1); B = _int_matrix(K, N, 2)
    C = _run(A, B, mode)
    exact = (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float32)
    assert np.array_equal(C, exact)


@pytest.mark.parametrize("mode", ["f32", "bf16x3"])
def test_gemm_identity_and_k0(mode):
    case(f"gemm {mode} identity")
    A = workloads.matrix_f32(70, 96, seed=4)
    C = _run(A, np.eye(96, dtype=np.float32), mode)
    if mode == "f32":
        assert np.array_equal(C, A)
    else:
        # C = lo*1 + hi*0 + hi*1 accumulated in FP32: exactly lo + hi
        hi, lo = oracle.split_bf16(A)
        want = oracle.bf16_to_f32(lo) + oracle.bf16_to_f32(hi)
        assert np.array_equal(C, want)
    case(f"gemm {mode} K=0")
    Ct = torch.full((3, 4), 7.0, device=dev())
    desc.desc_gemm(torch.empty((3, 0), device=dev()), torch.empty((0, 4), device=dev()), Ct,
                   mode=mode)
    assert (Ct == 0).all()


@pytest.mark.parametrize("mode", ["f32", "bf16x3"])
@pytest.mark.parametrize("M,N,K", [(96, 160, 300), (257, 129, 1000), (1024, 1024, 1024)])
def test_gemm_normal_within_bound(M, N, K, mode):
    case(f"gemm {mode} N(0,1) {M}x{N}x{K}")
    A = workloads.matrix_f32(M, K, seed=4); B = workloads.matrix_f32(K, N, seed=5)
    C = _run(A, B, mode)
    _check_sampled(A, B, C, TOL[mode])


@pytest.mark.parametrize("K", [1, 3, 16, 40])
def test_gemm_bf16x3_short_k_within_a_priori_bound(K):
    # short sums: the two-plane representation error dominates (see bf16x3_bound)
    case(f"gemm bf16x3 N(0,1) 130x70x{K}")
    A = workloads.matrix_f32(130, K, seed=20); B = workloads.matrix_f32(K, 70, seed=21)
    C = _run(A, B, "bf16x3")
    e = _check_sampled(A, B, C, bf16x3_bound(K), samples=130 * 70)
    print(f"[result] gemm bf16x3 K={K} max componentwise error {e:.3e} "
          f"(bound {bf16x3_bound(K):.3e})", flush=True)


@pytest.mark.parametrize("cfg", ["m128n128k32_fused", "m256n256k32_w8d1_fused"])
def test_gemm_bf16x3_fused_shapes(cfg):
    # operands split while staged: ragged edges, K not a multiple of the
    # stage, an unaligned row stride (single loads), K = 0 (pre-pass form)
    op = "gemm_bf16x3"
    names = [desc.desc_config_name(op, c) for c in range(desc.desc_config_count(op))]
    idx = names.index(cfg)
    try:
        for M, N, K, pad in [(77, 53, 45, 3), (300, 260, 100, 0), (1, 1, 1, 0),
                             (257, 129, 1000, 1), (64, 300, 0, 0), (513, 70, 96, 0)]:
            case(f"gemm bf16x3 {cfg} {M}x{N}x{K} lda pad {pad}")
            for cls in range(4):
                desc.desc_config_set(op, cls, idx)
            A = workloads.matrix_f32(M, K, seed=40); B = workloads.matrix_f32(K, N, seed=41)
            C = _run(A, B, "bf16x3", lda_pad=pad, ldc_pad=2)
            if K == 0:
                assert (C == 0).all()
                continue
            tol = TOL["bf16x3"] if K >= 64 else bf16x3_bound(K)
            _check_sampled(A, B, C, tol, samples=min(M * N, 4096))
    finally:
        for cls in range(4):
            desc.desc_config_set(op, cls, -1)


@pytest.mark.parametrize("mode", ["f32", "bf16x3"])
def test_gemm_strided_rows(mode):
    case(f"gemm {mode} strided lda/ldc")
    A = workloads.matrix_f32(77, 45, seed=8); B = workloads.matrix_f32(45, 53, seed=9)
    C = _run(A, B, mode, lda_pad=3, ldc_pad=5)
    _check_sampled(A, B, C, TOL[mode], samples=77 * 53)


@pytest.mark.parametrize("M,N,K,pad", [(300, 200, 136, 0), (77, 53, 45, 3), (260, 516, 68, 0)])
def test_gemm_f32_every_config(M, N, K, pad):
    # aligned groups of four with ragged tiles, then single loads (odd K, N,
    # unaligned rows)
    A = _int_matrix(M, K, 11); B = _int_matrix(K, N, 12)
    exact = (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float32)
    cls = desc.desc_size_class("gemm_f32", M * N * K)
    try:
        for cfg in range(desc.desc_config_count("gemm_f32")):
            case(f"gemm f32 config {desc.desc_config_name('gemm_f32', cfg)} {M}x{N}x{K}")
            desc.desc_config_set("gemm_f32", cls, cfg)
            assert np.array_equal(_run(A, B, "f32", lda_pad=pad, ldc_pad=pad), exact)
    finally:
        desc.desc_config_set("gemm_f32", cls, -1)


@pytest.mark.parametrize("mode", ["f32", "bf16x3"])
def test_gemm_workload_4096(mode):
    case(f"gemm {mode} 4096^3 (seeds 4/5, 4096 samples seed 6)")
    A = workloads.matrix_f32(4096, 4096, seed=4); B = workloads.matrix_f32(4096, 4096, seed=5)
    C = _run(A, B, mode)
    e = _check_sampled(A, B, C, TOL[mode], samples=4096, seed=6)
    print(f"[result] gemm {mode} 4096 max componentwise error {e:.3e}", flush=True)


@pytest.fixture(scope="module")
def workload_8192():
    """The 8192^3 precision workload: A (seed 7), B (seed 8), 4096 sampled
    entries (seed 9) and their FP64 references."""
    A = workloads.matrix_f32(8192, 8192, seed=7); B = workloads.matrix_f32(8192, 8192, seed=8)
    ii, jj = workloads.sample_pairs(8192, 8192, 4096, seed=9)
    R, D = oracle.gemm_ref_sampled(A, B, ii, jj)
    return A, B, ii, jj, R, D


@pytest.mark.parametrize("mode", ["f32", "bf16x3"])
def test_gemm_workload_8192(workload_8192, mode):
    A, B, ii, jj, R, D = workload_8192
    case(f"gemm {mode} 8192^3 (seeds 7/8, 4096 samples seed 9)")
    C = _run(A, B, mode)
    e = _check_against(C[ii, jj], R, D, TOL[mode], f"{mode} 8192")
    print(f"[result] gemm {mode} 8192 max componentwise error {e:.3e}", flush=True)


# A-priori bound of the FP8 product against the exact one, componentwise.
# With inv = fl32(448 / alpha) and s = fl32(alpha / 448), a normal code is
# within half an e4m3 spacing of the scaled value, relative 2^-4, and a
# subnormal one within 2^-10 in scaled units, 2^-10 alpha / 448 in the
# input's; the FP32 steps add a few 2^-24.  So each operand carries
# |e_a| <= (2^-4 + 2^-20) |a| + t_a, t_a = 2^-10 alpha (1 + 2^-20) / 448, and
# a product |(a + e_a)(b + e_b) - a b| <= (2^-3 + 2^-7) |a b| +
# (1 + 2^-3)(|a| t_b + |b| t_a) + t_a t_b, with |a| <= alpha, |b| <= beta.
# Summed over k, plus the accumulation tolerance on the quantised sum
# (whose absolute sum is at most (1 + 2^-3) D).  Loose, but a wrong scale or
# layout exceeds it; the observed error is reported beside it.
def _fp8_apriori(A, B, ii, jj, D):
    al = np.abs(A).max(axis=1).astype(np.float64)[ii]
    be = np.abs(B).max(axis=0).astype(np.float64)[jj]
    K = A.shape[1]
    ta, tb = 2.0 ** -10 * al * (1 + 2.0 ** -20) / 448, 2.0 ** -10 * be * (1 + 2.0 ** -20) / 448
    per_k = (1 + 2.0 ** -3) * (al * tb + be * ta) + ta * tb
    return (2.0 ** -3 + 2.0 ** -7 + (1 + 2.0 ** -3) * FP8_ACC_TOL) * D + K * per_k


def _fp8_workload(A, B, ii, jj, R, D, size):
    C = _run(A, B, "fp8")
    qa, _, sa = oracle.quant_rows_e4m3(A)
    qb, _, sb = oracle.quant_cols_e4m3(B)
    Rq, Dq = oracle.gemm_fp8_sampled(qa, qb, sa, sb, ii, jj)
    e_q = _check_against(C[ii, jj], Rq, Dq, FP8_ACC_TOL, f"fp8 {size} vs Rq")
    dev_abs = np.abs(C[ii, jj].astype(np.float64) - R)
    assert (dev_abs <= _fp8_apriori(A, B, ii, jj, D)).all(), "fp8 beyond its a-priori bound"
    e = dev_abs / D
    print(f"[result] fp8 {size}: vs its own codes {e_q:.3e}; vs the exact product max "
          f"{e.max():.3e} median {np.median(e):.3e}", flush=True)


def test_fp8_workload_4096():
    case("gemm fp8 4096^3 (seeds 4/5, 4096 samples seed 6)")
    A = workloads.matrix_f32(4096, 4096, seed=4); B = workloads.matrix_f32(4096, 4096, seed=5)
    ii, jj = workloads.sample_pairs(4096, 4096, 4096, seed=6)
    R, D = oracle.gemm_ref_sampled(A, B, ii, jj)
    _fp8_workload(A, B, ii, jj, R, D, "4096^3")


def test_fp8_workload_8192(workload_8192):
    A, B, ii, jj, R, D = workload_8192
    case("gemm fp8 8192^3 (seeds 7/8, 4096 samples seed 9)")
    _fp8_workload(A, B, ii, jj, R, D, "8192^3")


# ------------------------------------------------------------------ operand preparation
def _patterns(rows, cols, seed):
    g = workloads.rng(seed)
    a = g.standard_normal((rows, cols)).astype(np.float32) * 2.0 ** g.integers(-30, 30, (rows, cols))
    flat = a.reshape(-1)
    special = np.array([0.0, -0.0, np.inf, -np.inf, np.nan, 1e-40, -3e-39, 3.4e38, 1.0 + 2**-8,
                        1.0 + 2**-9 + 2**-16], np.float32)
    n = min(flat.size, special.size)
    flat[:n] = special[:n]
    return a.astype(np.float32)


@pytest.mark.parametrize("M,K", [(1, 1), (7, 33), (130, 257), (512, 1024)])
def test_split_bf16_rows_cols_bit_exact(M, K):
    case(f"split bf16 rows/cols {M}x{K}")
    A = _patterns(M, K, 3)
    hi, lo = oracle.split_bf16(A)
    h = torch.empty((M, K), dtype=torch.int16, device=dev())
    l = torch.empty_like(h)
    desc.desc_split_bf16_rows(to_dev(A), h, l)
    assert np.array_equal(h.cpu().numpy().view(np.uint16), hi)
    assert np.array_equal(l.cpu().numpy().view(np.uint16), lo)
    # columns of B = A^T
    B = np.ascontiguousarray(A.T)
    ht = torch.empty((M, K), dtype=torch.int16, device=dev())
    lt = torch.empty_like(ht)
    desc.desc_split_bf16_cols(to_dev(B), ht, lt)
    assert np.array_equal(ht.cpu().numpy().view(np.uint16), hi)
    assert np.array_equal(lt.cpu().numpy().view(np.uint16), lo)


@pytest.mark.parametrize("M,K", [(1, 1), (5, 70), (129, 300), (600, 2048)])
def test_quant_e4m3_rows_cols_bit_exact(M, K):
    case(f"quant e4m3 rows/cols {M}x{K}")
    A = workloads.matrix_f32(M, K, seed=12) * np.float32(3.0)
    A[M // 2] = 0.0                        # an all-zero row
    if K > 3:
        A[0, 1] = 1e-30; A[0, 2] = -7e-5     # deep subnormal and small codes
    q, al, sa = oracle.quant_rows_e4m3(A)
    qd = torch.empty((M, K), dtype=torch.uint8, device=dev())
    sd = torch.empty(M, dtype=torch.float32, device=dev())
    desc.desc_quant_e4m3_rows(to_dev(A), qd, sd)
    assert np.array_equal(qd.cpu().numpy(), q)
    assert np.array_equal(sd.cpu().numpy(), sa)
    # columns: B = A^T, codes come back transposed (N x K)
    B = np.ascontiguousarray(A.T)
    qc, be, sb = oracle.quant_cols_e4m3(B)
    qt = torch.empty((M, K), dtype=torch.uint8, device=dev())
    st = torch.empty(M, dtype=torch.float32, device=dev())
    desc.desc_quant_e4m3_cols(to_dev(B), qt, st)
    assert np.array_equal(qt.cpu().numpy(), qc.T)
    assert np.array_equal(st.cpu().numpy(), sb)


def _e4m3_rounding_points():
    """Every e4m3 code value, every midpoint between neighbouring codes (the
    ties) and the floats one ulp either side of each, over the whole range
    including subnormals, with both signs; then random bit patterns of
    magnitude <= 448.  Each row also holds 448, so its scale is 1 and the
    encoder sees these values unscaled."""
    pts = []
    for e in range(-9, 9):                     # code spacing 2^(e-3) in [2^e, 2^(e+1))
        step = 2.0 ** (max(e, -6) - 3)
        lo = 0.0 if e == -9 else 2.0 ** e
        v = np.arange(lo, min(2.0 ** (e + 1), 448.0) + step, step / 2)
        pts.append(v)
    p = np.unique(np.concatenate(pts)).astype(np.float32)
    p = p[p <= 448.0]
    up = np.nextafter(p, np.float32(np.inf))
    dn = np.nextafter(p, np.float32(0))
    p = np.unique(np.concatenate([p, up[up <= 448.0], dn]))
    p = np.concatenate([p, -p])
    g = workloads.rng(77)
    bits = g.integers(0, 0x43e00001, 1 << 20, dtype=np.uint32) | \
        (g.integers(0, 2, 1 << 20, dtype=np.uint32) << 31)
    return np.concatenate([p, bits.view(np.float32)])


def test_quant_e4m3_every_rounding_point():
    # the quantisers encode with the hardware conversion where it agrees with
    # the format definition (finite magnitudes up to 448): checked here on
    # all ties and code boundaries against the oracle's encoder
    vals = _e4m3_rounding_points()
    K = 4096
    rows = (vals.size + K - 2) // (K - 1)
    A = np.zeros((rows, K), np.float32)
    A[:, 0] = 448.0
    flat = np.zeros(rows * (K - 1), np.float32)
    flat[:vals.size] = vals
    A[:, 1:] = flat.reshape(rows, K - 1)
    case(f"quant e4m3 rounding points {vals.size} values")
    q, _, sa = oracle.quant_rows_e4m3(A)
    assert np.all(sa == 1.0)
    qd = torch.empty((rows, K), dtype=torch.uint8, device=dev())
    sd = torch.empty(rows, dtype=torch.float32, device=dev())
    desc.desc_quant_e4m3_rows(to_dev(A), qd, sd)
    assert np.array_equal(qd.cpu().numpy(), q)
    B = np.ascontiguousarray(A.T)
    qc, _, _ = oracle.quant_cols_e4m3(B)
    qt = torch.empty((rows, K), dtype=torch.uint8, device=dev())
    st = torch.empty(rows, dtype=torch.float32, device=dev())
    desc.desc_quant_e4m3_cols(to_dev(B), qt, st)
    assert np.array_equal(qt.cpu().numpy(), qc.T)


# ------------------------------------------------------------------ precision modes
def _check_against(C, R, D, tol, what):
    err = np.abs(C.astype(np.float64) - R) / np.maximum(D, 1e-300)
    assert err.max() <= tol, f"{what}: componentwise error {err.max():.3e} > {tol}"
    return err.max()


@pytest.mark.parametrize("M,N,K", [(64, 64, 64), (130, 250, 700), (1024, 768, 2048)])
def test_bf16x3_against_its_own_operands(M, N, K):
    case(f"gemm bf16x3 vs R3 {M}x{N}x{K}")
    A = workloads.matrix_f32(M, K, seed=21); B = workloads.matrix_f32(K, N, seed=22)
    C = _run(A, B, "bf16x3")
    ii, jj = workloads.sample_pairs(M, N, 1500, seed=23)
    R3, D3 = oracle.gemm_bf16x3_sampled(A, B, ii, jj)
    # only FP32 accumulation error remains against the three-product reference
    _check_against(C[ii, jj], R3, D3, 2e-6, "bf16x3 vs R3")


def test_fp8_exact_on_e4m3_integers():
    case("gemm fp8 exact integer codes")
    g = workloads.rng(31)
    M, N, K = 96, 80, 256
    A = g.integers(-8, 9, (M, K)).astype(np.float32)
    B = g.integers(-8, 9, (K, N)).astype(np.float32)
    # unit scales (every row of A and column of B has absmax 448), placed so
    # that the 448s always meet a zero: every product is a small integer, and
    # the sum is exact whatever the width of the instruction's internal adder
    A[:, 0] = 448.0; B[0, :] = 0.0
    A[:, 1] = 0.0; B[1, :] = 448.0
    C = _run(A, B, "fp8")
    exact = (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float32)
    assert np.array_equal(C, exact)


@pytest.mark.parametrize("M,N,K", [(100, 37, 129), (512, 512, 1024)])
def test_fp8_against_its_own_codes(M, N, K):
    case(f"gemm fp8 vs Rq {M}x{N}x{K}")
    A = workloads.matrix_f32(M, K, seed=24); B = workloads.matrix_f32(K, N, seed=25)
    C = _run(A, B, "fp8")
    qa, _, sa = oracle.quant_rows_e4m3(A)
    qb, _, sb = oracle.quant_cols_e4m3(B)
    ii, jj = workloads.sample_pairs(M, N, 1500, seed=26)
    Rq, Dq = oracle.gemm_fp8_sampled(qa, qb, sa, sb, ii, jj)
    # The fp8 matrix-core instruction sums its 64 products with an adder
    # narrower than FP32 (measured: 448^2 + 2^2 comes back as 448^2), so the
    # bound against the FP64 sum of the same codes is the accumulation
    # tolerance FP8_ACC_TOL, not FP32 rounding.  It stays two orders below the
    # quantisation error (~3e-3), so a wrong code, scale or layout still fails.
    _check_against(C[ii, jj], Rq, Dq, FP8_ACC_TOL, "fp8 vs Rq")
    R, D = oracle.gemm_ref_sampled(A, B, ii, jj)
    e = np.abs(C[ii, jj] - R) / D
    print(f"[result] fp8 {M}x{N}x{K} vs exact product: max {e.max():.3e} mean {e.mean():.3e}")


@pytest.mark.parametrize("op,mode", [("gemm_bf16x3", "bf16x3"), ("gemm_fp8", "fp8")])
def test_lowp_every_config(op, mode):
    M, N, K = 300, 520, 384
    if mode == "bf16x3":
        A = _int_matrix(M, K, 13); B = _int_matrix(K, N, 14)
    else:
        g = workloads.rng(15)
        A = g.integers(-8, 9, (M, K)).astype(np.float32)
        B = g.integers(-8, 9, (K, N)).astype(np.float32)
        A[:, 0] = 448.0; B[0, :] = 0.0
        A[:, 1] = 0.0; B[1, :] = 448.0
    exact = (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float32)
    cls = desc.desc_size_class(op, M * N * K)
    try:
        for cfg in range(desc.desc_config_count(op)):
            case(f"{op} config {desc.desc_config_name(op, cfg)}")
            desc.desc_config_set(op, cls, cfg)
            assert np.array_equal(_run(A, B, mode), exact), desc.desc_config_name(op, cfg)
    finally:
        desc.desc_config_set(op, cls, -1)
