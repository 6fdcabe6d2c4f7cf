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

import fp8_mfma_model as fp8_model
import oracle
import paper_2305_03448_amd as desc
import workloads
from gpu_util import bf16x3_bound, case, dev, needs_gpu, to_dev

pytestmark = [pytest.mark.gpu, needs_gpu]

TOL = {"f32": 1e-5, "bf16x3": 1e-5}
MODES_EXACT = ["f32", "bf16x3"]      # modes exact on small-integer operands
# FP8 against the FP64 sum of its own codes: the library must follow the
# model of the fp8 matrix instruction (tests/fp8_mfma_model.py): bit for bit
# where a single sub-group sum is nonzero, elsewhere within
# the model's derived limit for the order of the FP32 additions
# (fp8_mfma_model.combine_bound); the model's own deviation from that sum is
# bounded per entry from its definition (fp8_mfma_model.entry_bounds; for
# normal operands at most 2^-10 + 9 G 2^-24 of the absolute sum, G the number
# of 64-product groups).


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


@pytest.mark.parametrize("M,N,K,pad", [(300, 200, 136, 0), (77, 53, 45, 3), (260, 516, 68, 0),
                                       (300, 200, 128, 0), (520, 392, 96, 4)])
def test_gemm_f32_every_config(M, N, K, pad):
    # aligned groups of four with ragged tiles, then single loads (odd K, N,
    # unaligned rows); with K a multiple of 16 the tiles wholly inside C take
    # the buffer-range loads and the others the guarded ones, in one call
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
# Summed over k: the quantisation part; the instruction's own deviation from
# the quantised sum (the model's per-entry bound) is added by the caller.
# Loose, but a wrong scale or layout exceeds it; the observed error is
# reported beside it.
def _fp8_apriori(A, B, ii, jj, D):
    al = np.abs(A).max(axis=1).astype(np.float64)[ii]
    be = np.abs(B).max(axis=0).astype(np.float64)[jj]
    K = A.shape[1]
    ta, tb = 2.0 ** -10 * al * (1 + 2.0 ** -20) / 448, 2.0 ** -10 * be * (1 + 2.0 ** -20) / 448
    per_k = (1 + 2.0 ** -3) * (al * tb + be * ta) + ta * tb
    return (2.0 ** -3 + 2.0 ** -7) * D + K * per_k


_E4M3 = None


def _e4m3_values(q):
    global _E4M3
    if _E4M3 is None:
        _E4M3 = np.array([float(np.asarray(oracle.e4m3_decode(c)).ravel()[0]) for c in range(256)])
    return _E4M3[q]


def _fp8_model_check(C_s, qa, qb, sa, sb, ii, jj, what):
    """The sampled FP8 entries follow the instruction model (bit for bit where
    it is exact, within combine_bound elsewhere), and lie within the model's
    per-entry bound of the exact scaled sum Rq.  Returns the largest deviation
    from Rq relative to the absolute sum, and the per-entry bound of that
    deviation."""
    va, vb = _e4m3_values(qa), _e4m3_values(qb)
    a, b = va[ii, :], vb[:, jj].T
    model = fp8_model.gemm_fp8_sampled(va, vb, sa, sb, ii, jj)
    got = np.ascontiguousarray(C_s, np.float32)
    scale = sa.astype(np.float64)[ii] * sb.astype(np.float64)[jj]
    single = fp8_model.single_term(a, b)
    diff = np.nonzero(single & (got.view(np.uint32) != model.view(np.uint32)))[0]
    assert diff.size == 0, (f"{what}: {diff.size} entries differ from the instruction model "
                            f"where it is exact, first {got[diff[0]]!r} vs {model[diff[0]]!r}")
    lim = scale * fp8_model.combine_bound(a, b) * (1 + 2.0 ** -20) + \
        np.abs(model.astype(np.float64)) * 2.0 ** -22
    dev_m = np.abs(got.astype(np.float64) - model.astype(np.float64))
    bad = np.nonzero(dev_m > lim)[0]
    assert bad.size == 0, (f"{what}: {bad.size} entries beyond the instruction model's limit, "
                           f"first {got[bad[0]]!r} vs {model[bad[0]]!r} (limit {lim[bad[0]]:.3e})")
    Rq, Dq = oracle.gemm_fp8_sampled(qa, qb, sa, sb, ii, jj)
    tol = scale * fp8_model.entry_bounds(a, b) + lim + np.abs(Rq) * 2.0 ** -22 + 1e-300
    dev_q = np.abs(got.astype(np.float64) - Rq)
    assert (dev_q <= tol).all(), f"{what}: beyond the model's bound of Rq"
    print(f"[result] {what}: {np.mean(dev_m == 0):.4f} of entries equal the model bit for bit "
          f"({int(single.sum())} exact by construction); largest deviation "
          f"{(dev_m / np.maximum(lim, 1e-300)).max():.3f} of the limit", flush=True)
    return (dev_q / np.maximum(Dq, 1e-300)).max(), tol


def _fp8_workload(A, B, ii, jj, R, D, size):
    C = _run(A, B, "fp8")
    qa, _, sa = oracle.quant_rows_e4m3(A)
    qb, _, sb = oracle.quant_cols_e4m3(B)
    e_q, tol_q = _fp8_model_check(C[ii, jj], qa, qb, sa, sb, ii, jj, f"fp8 {size}")
    dev_abs = np.abs(C[ii, jj].astype(np.float64) - R)
    assert (dev_abs <= _fp8_apriori(A, B, ii, jj, D) + tol_q).all(), "fp8 beyond its a-priori bound"
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


# (8200, 4100): the column encode of a 4100 x 8200 B has more than 8192 tiles of
# 64 x 64, so it runs in 128-k tiles, with a ragged last k tile and column block
@pytest.mark.parametrize("M,K", [(1, 1), (5, 70), (129, 300), (600, 2048), (8200, 4100)])
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


@pytest.mark.parametrize("M,N,K", [(100, 37, 129), (512, 512, 1024), (64, 64, 4096)])
def test_fp8_against_its_own_codes(M, N, K):
    case(f"gemm fp8 vs the instruction model and Rq {M}x{N}x{K}")
    A = workloads.matrix_f32(M, K, seed=24); B = workloads.matrix_f32(K, N, seed=25)
    C = _run(A, B, "fp8")
    qa, _, sa = oracle.quant_rows_e4m3(A)
    qb, _, sb = oracle.quant_cols_e4m3(B)
    ii, jj = workloads.sample_pairs(M, N, 1500, seed=26)
    e_q, _ = _fp8_model_check(C[ii, jj], qa, qb, sa, sb, ii, jj, "fp8 vs model")
    R, D = oracle.gemm_ref_sampled(A, B, ii, jj)
    e = np.abs(C[ii, jj] - R) / D
    print(f"[result] fp8 {M}x{N}x{K}: vs Rq max {e_q:.3e}; vs the exact product: max "
          f"{e.max():.3e} mean {e.mean():.3e}")


def test_fp8_instruction_model_on_crafted_groups():
    """The measurement behind the model, as a test on the product path: with
    unit scales (each row of A and column of B holds 448 against a zero
    partner) the diagonal C[i][i] is the instruction's sum of the products
    placed in row i / column i, for big products of every exponent sum next
    to small ones one quantum above and below the cut, of either sign, in one
    sub-group, in the next sub-group of the same group (not cut by the big
    one), or in the next group (FP32 rounding between groups, ties
    included).  One cut per whole group of 64 fails these cases."""
    cases = []
    for a, b in ((448.0, 448.0), (256.0, 256.0), (448.0, 256.0), (320.0, 320.0), (16.0, 16.0),
                 (24.0, 16.0), (1.0, 1.0), (1.5, 1.5), (0.25, 0.5), (2.0 ** -6, 1.0)):
        s = int(fp8_model.e4m3_exponent(np.array([a]))[0] + fp8_model.e4m3_exponent(np.array([b]))[0])
        for e in range(s - 16, s + 2):
            x, y = 2.0 ** (e // 2), 2.0 ** (e - e // 2)
            if not (2.0 ** -9 <= x <= 256 and 2.0 ** -9 <= y <= 256):
                continue
            for sign in (1.0, -1.0):
                cases.append([(2, a, b), (3, sign * x, y)])
                cases.append([(2, -a, b), (3, sign * x, y)])
                if x >= 2.0 ** -5:
                    cases.append([(2, a, b), (3, sign * 1.75 * x, y)])
            cases.append([(2, a, b), (3, x, y), (4, x, y)])            # cut one by one
            cases.append([(2, a, b), (5, -a, b), (3, x, y)])           # big ones cancel
            cases.append([(2, a, b), (64, x, y)])                      # next group: FP32 add
            cases.append([(2, a, b), (9, sign * x, y)])                # next sub-group: not cut
            cases.append([(2, a, b), (13, -a, b), (15, x, y)])         # cancel in another one
    for t_a, t_b in ((1.75, 2.0 ** -6), (-1.75, 2.0 ** -6), (1.0, 2.0 ** -7), (1.25, 2.0 ** -6)):
        cases.append([(0, 448.0, 448.0), (64, t_a, t_b)])
    n, K = len(cases), 128
    A = np.zeros((n, K), np.float32); B = np.zeros((K, n), np.float32)
    for i, terms in enumerate(cases):
        A[i, 120] = 448.0; B[121, i] = 448.0
        for k, x, y in terms:
            A[i, k] = x; B[k, i] = y
    assert (np.abs(A).max(1) == 448).all() and (np.abs(B).max(0) == 448).all()
    case(f"gemm fp8 crafted instruction groups ({n} cases)")
    C = _run(A, B, "fp8")
    qa, _, sa = oracle.quant_rows_e4m3(A)
    qb, _, sb = oracle.quant_cols_e4m3(B)
    assert (sa == 1).all() and (sb == 1).all()
    ii = np.arange(n)
    assert np.array_equal(_e4m3_values(qa), A) and np.array_equal(_e4m3_values(qb), B)
    _fp8_model_check(C[ii, ii], qa, qb, sa, sb, ii, ii, "crafted groups")
    va, vb = _e4m3_values(qa), _e4m3_values(qb)
    flat = fp8_model.gemm_fp8_sampled(va, vb, sa, sb, ii, ii, sub=64).astype(np.float64)
    lim = fp8_model.combine_bound(va, vb.T) * (1 + 2.0 ** -20) + np.abs(flat) * 2.0 ** -22
    assert (np.abs(C[ii, ii] - flat) > lim).sum() > 0, "the crafted cases do not test the sub-groups"
    exact = np.array([sum(x * y for _, x, y in t) for t in cases])
    lost = int((C[ii, ii] != exact).sum())
    print(f"[result] fp8 instruction: {lost} of {n} crafted sums differ from the exact sum, "
          f"all as the model predicts")
    assert lost > 0


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
