"""Parity of the uniform batched forms with the oracle through the C ABI:
row-by-row reduce and scan of a batch x len int32 matrix (the segmented
oracle with offsets s * len, bit for bit), and the strided batched GEMM in
the FP32 and split-BF16 modes (every entry of every batch within the
componentwise bound, padded strides included)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2305_03448_amd as desc
import workloads
from gpu_util import bf16x3_bound, case, dev, needs_gpu, to_dev

pytestmark = [pytest.mark.gpu, needs_gpu]

SHAPES = [(1, 1), (3, 5), (1, 70000), (1000, 4097), (4096, 1000), (64, 65536 + 3), (7, 0)]


def _offsets(B, L):
    return np.arange(B + 1, dtype=np.int64) * L


@pytest.mark.parametrize("B,L", SHAPES)
def test_reduce_batched(B, L):
    case(f"reduce_batched B={B} L={L}")
    x = workloads.int_uniform(B * L, seed=500 + B % 31).reshape(B, L)
    out = torch.full((B,), -7, dtype=torch.int64, device=dev())
    desc.desc_reduce_batched_i32(to_dev(x), out)
    want = oracle.reduce_segmented_i32(x.ravel(), _offsets(B, L))
    assert np.array_equal(out.cpu().numpy(), want)


@pytest.mark.parametrize("B,L", SHAPES)
def test_scan_batched(B, L):
    case(f"scan_batched B={B} L={L}")
    x = workloads.int_uniform(B * L, seed=600 + B % 37).reshape(B, L)
    out = torch.full((B, L), -7, dtype=torch.int32, device=dev())
    desc.desc_scan_batched_i32(to_dev(x), out)
    want = oracle.scan_segmented_i32(x.ravel(), _offsets(B, L)).reshape(B, L)
    assert np.array_equal(out.cpu().numpy(), want)


def test_batched_unaligned_and_workspace_reuse():
    # one workspace for both operations, sized for the larger
    ws = torch.zeros(max(desc.desc_scan_batched_i32_workspace(300, 4099),
                         desc.desc_reduce_batched_i32_workspace(300, 4099)), dtype=torch.uint8,
                     device=dev())
    for rep, (B, L, off) in enumerate([(300, 4099, 1), (5, 3, 3), (299, 4097, 2), (300, 4099, 0)]):
        case(f"batched reuse rep {rep} B={B} L={L} offset={off}")
        x = workloads.int_uniform(B * L, seed=700 + rep).reshape(B, L)
        xt = to_dev(x, off)
        y = torch.empty((B, L), dtype=torch.int32, device=dev())
        desc.desc_scan_batched_i32(xt, y, ws=ws)
        assert np.array_equal(y.cpu().numpy(),
                              oracle.scan_segmented_i32(x.ravel(), _offsets(B, L)).reshape(B, L))
        r = torch.empty(B, dtype=torch.int64, device=dev())
        desc.desc_reduce_batched_i32(xt, r, ws=ws)
        assert np.array_equal(r.cpu().numpy(), oracle.reduce_segmented_i32(x.ravel(),
                                                                           _offsets(B, L)))


def _gemm_case(G, M, N, K, pad, seed, mode):
    g = workloads.rng(seed)
    A = g.standard_normal((G, M, K)).astype(np.float32)
    B = g.standard_normal((G, K, N)).astype(np.float32)
    # padded rows and batches: lda = K + pad, batch stride = M * lda + 5 * pad
    def padded(X):
        Gx, R, Cc = X.shape
        buf = torch.zeros(Gx * (R * (Cc + pad) + 5 * pad) + 8, dtype=torch.float32, device=dev())
        v = buf.as_strided((Gx, R, Cc), (R * (Cc + pad) + 5 * pad, Cc + pad, 1))
        v.copy_(torch.from_numpy(X))
        return v
    At, Bt = padded(A), padded(B)
    Ct = padded(np.full((G, M, N), np.nan, np.float32))
    desc.desc_gemm_strided_batched(At, Bt, Ct, mode=mode)
    C = Ct.cpu().numpy()
    worst = 0.0
    for b in range(G):
        ii, jj = np.meshgrid(np.arange(M), np.arange(N), indexing="ij")
        R, D = oracle.gemm_ref_sampled(A[b], B[b], ii.ravel(), jj.ravel())
        worst = max(worst, float((np.abs(C[b].ravel() - R) / np.maximum(D, 1e-300)).max()))
    return worst


@pytest.mark.parametrize("mode", ["f32", "bf16x3"])
@pytest.mark.parametrize("G,M,N,K,pad", [(1, 64, 64, 64, 0), (8, 200, 136, 260, 3),
                                         (33, 96, 64, 128, 0), (4, 130, 257, 1, 1),
                                         (3, 17, 9, 700, 5)])
def test_gemm_strided_batched(mode, G, M, N, K, pad):
    case(f"gemm_strided_batched {mode} G={G} {M}x{N}x{K} pad={pad}")
    worst = _gemm_case(G, M, N, K, pad, seed=800 + G, mode=mode)
    tol = 1e-5 if (mode == "f32" or K >= 64) else bf16x3_bound(K)
    print(f"[result] strided batched {mode} worst {worst:.3e}")
    assert worst <= tol


@pytest.mark.parametrize("mode", ["f32", "bf16x3"])
def test_gemm_strided_batched_k0_writes_zeros(mode):
    case(f"gemm_strided_batched K=0 {mode}")
    A = torch.empty((3, 5, 0), dtype=torch.float32, device=dev())
    B = torch.empty((3, 0, 7), dtype=torch.float32, device=dev())
    C = torch.full((3, 5, 7), float("nan"), dtype=torch.float32, device=dev())
    desc.desc_gemm_strided_batched(A, B, C, mode=mode)
    assert torch.count_nonzero(C).item() == 0


def test_batched_graph_replay():
    # the three batched forms (each a description kernel plus the segmented
    # or grouped kernels) captured into one HIP graph and replayed
    B, L = 300, 4099
    x = workloads.int_uniform(B * L, seed=95).reshape(B, L)
    xt = to_dev(x)
    r = torch.empty(B, dtype=torch.int64, device=dev())
    y = torch.empty((B, L), dtype=torch.int32, device=dev())
    wr = torch.zeros(desc.desc_reduce_batched_i32_workspace(B, L), dtype=torch.uint8, device=dev())
    wy = torch.zeros(desc.desc_scan_batched_i32_workspace(B, L), dtype=torch.uint8, device=dev())
    G, M, N, K = 6, 96, 80, 70
    g_ = workloads.rng(96)
    A = g_.standard_normal((G, M, K)).astype(np.float32)
    Bm = g_.standard_normal((G, K, N)).astype(np.float32)
    At, Bt = to_dev(A), to_dev(Bm)
    C = torch.empty((G, M, N), dtype=torch.float32, device=dev())
    wg = torch.zeros(desc.desc_gemm_strided_batched_workspace("f32", G, M, N, K, K, N),
                     dtype=torch.uint8, device=dev())
    case("batched eager before capture")
    desc.desc_reduce_batched_i32(xt, r, ws=wr)
    desc.desc_scan_batched_i32(xt, y, ws=wy)
    desc.desc_gemm_strided_batched(At, Bt, C, ws=wg)
    torch.cuda.synchronize()
    want_r, want_y, want_c = r.cpu().numpy(), y.cpu().numpy(), C.cpu().numpy().view(np.uint32)
    assert np.array_equal(want_r, oracle.reduce_segmented_i32(x.ravel(), _offsets(B, L)))
    stream = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        desc.desc_reduce_batched_i32(xt, r, ws=wr)
        desc.desc_scan_batched_i32(xt, y, ws=wy)
        desc.desc_gemm_strided_batched(At, Bt, C, ws=wg)
    for rep in range(3):
        case(f"batched graph replay {rep}")
        r.fill_(-1); y.fill_(-1); C.fill_(float("nan"))
        desc.desc_reduce_batched_i32(xt[:5], torch.empty(5, dtype=torch.int64, device=dev()))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(r.cpu().numpy(), want_r)
        assert np.array_equal(y.cpu().numpy(), want_y)
        assert np.array_equal(C.cpu().numpy().view(np.uint32), want_c)


def test_gemm_strided_batched_bf16x3_long_rows_use_planes():
    # lda past the fused split source's limit (2^24 elements): the split-BF16
    # mode stages these problems through planes sized into the workspace
    G, M, N, K, lda = 2, 3, 50, 5, (1 << 24) + 7
    g = workloads.rng(97)
    A = g.standard_normal((G, M, K)).astype(np.float32)
    B = g.standard_normal((G, K, N)).astype(np.float32)
    buf = torch.zeros(G * M * lda, dtype=torch.float32, device=dev())
    At = buf.as_strided((G, M, K), (M * lda, lda, 1))
    At.copy_(torch.from_numpy(A))
    Bt = to_dev(B)
    C = torch.full((G, M, N), float("nan"), dtype=torch.float32, device=dev())
    need = desc.desc_gemm_strided_batched_workspace("bf16x3", G, M, N, K, lda, N)
    assert need > desc.desc_gemm_strided_batched_workspace("bf16x3", G, M, N, K, K, N)
    case("gemm_strided_batched bf16x3 lda = 2^24 + 7")
    desc.desc_gemm_strided_batched(At, Bt, C, mode="bf16x3")
    out = C.cpu().numpy()
    for b in range(G):
        ii, jj = np.meshgrid(np.arange(M), np.arange(N), indexing="ij")
        R, D = oracle.gemm_ref_sampled(A[b], B[b], ii.ravel(), jj.ravel())
        err = np.abs(out[b].ravel() - R) / np.maximum(D, 1e-300)
        assert err.max() <= bf16x3_bound(K), b
