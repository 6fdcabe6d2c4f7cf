"""Parity of the grouped GEMM with the FP64 oracle through the C ABI: 512
problems with M, N, K uniform over {64, ..., 1024} (seed 12, entries N(0,1)
seed 13, 64 sampled entries per problem seed 14) within the componentwise
bound; exactness on small-integer operands; degenerate shapes; a single
problem equal bit for bit to the plain GEMM (same tile shape); graph
replay."""
import numpy as np
import pytest
import torch

import oracle
import paper_2305_03448_amd as desc
import workloads
from gpu_util import case, dev, needs_gpu, to_dev

pytestmark = [pytest.mark.gpu, needs_gpu]

TOL = 1e-5


def _problems(shapes, seed, integer=False):
    g = workloads.rng(seed)
    out = []
    for M, N, K in shapes:
        if integer:
            A = g.integers(-4, 5, (M, K)).astype(np.float32)
            B = g.integers(-4, 5, (K, N)).astype(np.float32)
        else:
            A = g.standard_normal((M, K)).astype(np.float32)
            B = g.standard_normal((K, N)).astype(np.float32)
        out.append((A, B))
    return out


def _run(pairs, pad=0):
    dev_pairs = []
    for A, B in pairs:
        M, K = A.shape
        N = B.shape[1]
        if pad:
            At = to_dev(np.pad(A, ((0, 0), (0, pad))))[:, :K]
        else:
            At = to_dev(A)
        C = torch.full((M, N), float("nan"), dtype=torch.float32, device=dev())
        dev_pairs.append((At, to_dev(B), C))
    d = desc.grouped_descriptors(dev_pairs, dev())
    desc.desc_gemm_grouped(d)
    torch.cuda.synchronize()
    return [c.cpu().numpy() for _, _, c in dev_pairs], dev_pairs, d


@pytest.fixture
def grouped_config(request):
    """Force one tile configuration of the grouped GEMM for the test."""
    cfg = request.param
    for cls in range(4):
        desc.desc_config_set("gemm_grouped", cls, cfg)
    yield cfg
    for cls in range(4):
        desc.desc_config_set("gemm_grouped", cls, -1)


CONFIGS = [0, 1]   # tile128_or_64, tile64


@pytest.mark.parametrize("grouped_config", CONFIGS, indirect=True)
def test_grouped_integer_exact_mixed_shapes(grouped_config):
    shapes = [(64, 64, 64), (1, 1, 1), (300, 257, 65), (256, 256, 16), (1024, 64, 128),
              (70, 513, 3), (257, 300, 129), (5, 7, 0)]
    case(f"grouped integer {len(shapes)} problems config {grouped_config}")
    pairs = _problems(shapes, 3, integer=True)
    outs, _, _ = _run(pairs)
    for (A, B), C in zip(pairs, outs):
        exact = (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float32)
        assert np.array_equal(C, exact), A.shape


def test_grouped_strided_and_empty():
    case("grouped strided lda, empty problems")
    pairs = _problems([(33, 45, 77), (0, 5, 5), (5, 0, 5), (100, 100, 100)], 4)
    outs, _, _ = _run(pairs, pad=3)
    for (A, B), C in zip(pairs, outs):
        if C.size:
            ii, jj = np.meshgrid(np.arange(C.shape[0]), np.arange(C.shape[1]), indexing="ij")
            R, D = oracle.gemm_ref_sampled(A, B, ii.ravel(), jj.ravel())
            err = np.abs(C.ravel() - R) / np.maximum(D, 1e-300)
            assert err.max() <= TOL


@pytest.mark.parametrize("M,N,K", [(100, 90, 80), (512, 384, 256)])
def test_grouped_single_equals_plain(M, N, K):
    case(f"grouped single vs plain {M}x{N}x{K}")
    pairs = _problems([(M, N, K)], 5)
    outs, dp, _ = _run(pairs)
    C2 = torch.empty((M, N), dtype=torch.float32, device=dev())
    desc.desc_gemm(dp[0][0], dp[0][1], C2)
    assert np.array_equal(outs[0], C2.cpu().numpy())


def test_grouped_graph_replay():
    pairs = _problems([(200, 100, 300), (64, 640, 64), (512, 512, 64)], 6)
    outs, dp, d = _run(pairs)
    ws = torch.empty(desc.desc_gemm_grouped_workspace(len(pairs)), dtype=torch.uint8, device=dev())
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s):
        desc.desc_gemm_grouped(d, ws=ws)
    for rep in range(3):
        case(f"grouped graph replay {rep}")
        for _, _, C in dp:
            C.fill_(0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for (_, _, C), want in zip(dp, outs):
            assert np.array_equal(C.cpu().numpy(), want)


@pytest.mark.parametrize("grouped_config", CONFIGS, indirect=True)
def test_grouped_workload_512(grouped_config):
    assert desc.desc_config_count("gemm_grouped") == len(CONFIGS)
    case(f"grouped 512 problems (seeds 12/13/14) config {grouped_config}")
    shapes = workloads.grouped_shapes()
    pairs = workloads.grouped_operands(shapes)
    outs, _, _ = _run(pairs)
    worst = 0.0
    for p, ((A, B), C) in enumerate(zip(pairs, outs)):
        ii, jj = workloads.sample_pairs(C.shape[0], C.shape[1], 64, seed=14 + p)
        R, D = oracle.gemm_ref_sampled(A, B, ii, jj)
        err = np.abs(C[ii, jj] - R) / np.maximum(D, 1e-300)
        worst = max(worst, float(err.max()))
    print(f"[result] grouped 512 worst componentwise error {worst:.3e}")
    assert worst <= TOL
