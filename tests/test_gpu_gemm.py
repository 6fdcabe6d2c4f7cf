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
from gpu_util import case, dev, needs_gpu, to_dev

pytestmark = [pytest.mark.gpu, needs_gpu]

TOL = {"f32": 1e-5, "bf16x3": 1e-5}


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
@pytest.mark.parametrize("mode", ["f32"])
def test_gemm_integer_exact(M, N, K, mode):
    case(f"gemm {mode} integer {M}x{N}x{K}")
    A = _int_matrix(M, K, 1); B = _int_matrix(K, N, 2)
    C = _run(A, B, mode)
    exact = (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float32)
    assert np.array_equal(C, exact)


@pytest.mark.parametrize("mode", ["f32"])
def test_gemm_identity_and_k0(mode):
    case(f"gemm {mode} identity")
    A = workloads.matrix_f32(70, 96, seed=4)
    C = _run(A, np.eye(96, dtype=np.float32), mode)
    assert np.array_equal(C, A)
    case(f"gemm {mode} K=0")
    Ct = torch.full((3, 4), 7.0, device=dev())
    desc.desc_gemm(torch.empty((3, 0), device=dev()), torch.empty((0, 4), device=dev()), Ct,
                   mode=mode)
    assert (Ct == 0).all()


@pytest.mark.parametrize("mode", ["f32"])
@pytest.mark.parametrize("M,N,K", [(96, 160, 300), (257, 129, 1000), (1024, 1024, 1024)])
def test_gemm_normal_within_bound(M, N, K, mode):
    case(f"gemm {mode} N(0,1) {M}x{N}x{K}")
    A = workloads.matrix_f32(M, K, seed=4); B = workloads.matrix_f32(K, N, seed=5)
    C = _run(A, B, mode)
    _check_sampled(A, B, C, TOL[mode])


@pytest.mark.parametrize("mode", ["f32"])
def test_gemm_strided_rows(mode):
    case(f"gemm {mode} strided lda/ldc")
    A = workloads.matrix_f32(77, 45, seed=8); B = workloads.matrix_f32(45, 53, seed=9)
    C = _run(A, B, mode, lda_pad=3, ldc_pad=5)
    _check_sampled(A, B, C, TOL[mode], samples=77 * 53)


def test_gemm_f32_every_config():
    M, N, K = 300, 200, 136
    A = _int_matrix(M, K, 11); B = _int_matrix(K, N, 12)
    exact = (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float32)
    cls = desc.desc_size_class("gemm_f32", M * N * K)
    try:
        for cfg in range(desc.desc_config_count("gemm_f32")):
            case(f"gemm f32 config {desc.desc_config_name('gemm_f32', cfg)}")
            desc.desc_config_set("gemm_f32", cls, cfg)
            assert np.array_equal(_run(A, B, "f32"), exact)
    finally:
        desc.desc_config_set("gemm_f32", cls, -1)


@pytest.mark.parametrize("mode", ["f32"])
def test_gemm_workload_4096(mode):
    case(f"gemm {mode} 4096^3 (seeds 4/5, 4096 samples seed 6)")
    A = workloads.matrix_f32(4096, 4096, seed=4); B = workloads.matrix_f32(4096, 4096, seed=5)
    C = _run(A, B, mode)
    e = _check_sampled(A, B, C, TOL[mode], samples=4096, seed=6)
    print(f"[result] gemm {mode} 4096 max componentwise error {e:.3e}", flush=True)
