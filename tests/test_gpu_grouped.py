"""Parity of the grouped GEMM with the FP64 oracle through the C ABI, in the
FP32 and the split-BF16 modes: 512 problems with M, N, K uniform over
{64, ..., 1024} (seed 12, entries N(0,1) seed 13, 64 sampled entries per
problem seed 14) within the componentwise bound; exactness on small-integer
operands; degenerate shapes; a single FP32 problem equal bit for bit to the
plain GEMM (same tile shape); graph replay; the split-BF16 mode's device-side
refusal of a workspace too small for its planes."""
import numpy as np
import pytest
import torch

import oracle
import paper_2305_03448_amd as desc
import workloads
from gpu_util import bf16x3_bound, case, dev, needs_gpu, to_dev

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


def _run(pairs, pad=0, mode="f32"):
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
    desc.desc_gemm_grouped(d, mode=mode)
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


CONFIGS = [0, 1, 2]   # tile128_or_64, tile64, tile64_rm_d2
BF16_CONFIGS = [0, 1, 2, 3]   # tile64, tile128, fused64, fused128


@pytest.fixture
def bf16_config(request):
    """Force one tile configuration of the split-BF16 grouped GEMM."""
    cfg = request.param
    for cls in range(4):
        desc.desc_config_set("gemm_grouped_bf16x3", cls, cfg)
    yield cfg
    for cls in range(4):
        desc.desc_config_set("gemm_grouped_bf16x3", cls, -1)


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


@pytest.mark.parametrize("grouped_config", [1], indirect=True)   # tile64: the plain GEMM's
@pytest.mark.parametrize("M,N,K", [(100, 90, 80), (512, 384, 256)])  # m64n64k16 tile form
def test_grouped_single_equals_plain(M, N, K, grouped_config):
    case(f"grouped single vs plain {M}x{N}x{K}")
    for cls in range(4):
        desc.desc_config_set("gemm_f32", cls, 3)                        # m64n64k16
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


# ----------------------------------------------------------------- split-BF16 mode
def _tol_bf16x3(K):
    return TOL if K >= 64 else bf16x3_bound(K)


def _check_all(pairs, outs):
    """Every entry against the oracle; returns the worst error as a fraction
    of each problem's tolerance, and the worst error of the K >= 64 problems."""
    worst_frac, worst_long = 0.0, 0.0
    for (A, B), C in zip(pairs, outs):
        if C.size == 0:
            continue
        K = A.shape[1]
        ii, jj = np.meshgrid(np.arange(C.shape[0]), np.arange(C.shape[1]), indexing="ij")
        R, D = oracle.gemm_ref_sampled(A, B, ii.ravel(), jj.ravel())
        err = np.abs(C.ravel() - R) / np.maximum(D, 1e-300)
        print(f"[result] bf16x3 {A.shape[0]}x{C.shape[1]}x{K} worst {err.max():.3e}")
        worst_frac = max(worst_frac, float(err.max()) / _tol_bf16x3(K))
        if K >= 64:
            worst_long = max(worst_long, float(err.max()))
    return worst_frac, worst_long


MIXED = [(64, 64, 64), (1, 1, 1), (300, 257, 65), (256, 256, 16), (1024, 64, 128),
         (70, 513, 3), (257, 300, 129), (5, 7, 0), (0, 5, 5), (5, 0, 5), (63, 65, 1000)]


@pytest.mark.parametrize("bf16_config", BF16_CONFIGS, indirect=True)
def test_grouped_bf16x3_integer_exact_mixed_shapes(bf16_config):
    # entries in {-4..4} are bf16 numbers: hi = a, lo = 0, every product exact
    case(f"grouped bf16x3 integer {len(MIXED)} problems config {bf16_config}")
    pairs = _problems(MIXED, 3, integer=True)
    outs, _, _ = _run(pairs, mode="bf16x3")
    for (A, B), C in zip(pairs, outs):
        exact = (A.astype(np.int64) @ B.astype(np.int64)).astype(np.float32)
        assert np.array_equal(C, exact), A.shape


@pytest.mark.parametrize("bf16_config", BF16_CONFIGS, indirect=True)
def test_grouped_bf16x3_strided_mixed_shapes(bf16_config):
    case(f"grouped bf16x3 strided lda, {len(MIXED)} problems config {bf16_config}")
    pairs = _problems(MIXED, 7)
    outs, _, _ = _run(pairs, pad=3, mode="bf16x3")
    frac, long_k = _check_all(pairs, outs)
    print(f"[result] grouped bf16x3 mixed: worst K >= 64 error {long_k:.3e}, "
          f"worst fraction of the tolerance {frac:.3f}")
    assert frac <= 1.0


@pytest.mark.parametrize("bf16_config", [1], indirect=True)   # a configuration with planes
def test_grouped_bf16x3_workspace_too_small_sets_error(bf16_config):
    pairs = _problems([(100, 90, 80), (64, 64, 64)], 8)
    dev_pairs = [(to_dev(A), to_dev(B),
                  torch.full((A.shape[0], B.shape[1]), float("nan"), dtype=torch.float32,
                             device=dev())) for A, B in pairs]
    d = desc.grouped_descriptors(dev_pairs, dev())
    need = desc.desc_gemm_grouped_workspace_for("bf16x3", d.cpu())
    case("grouped bf16x3 workspace 256 bytes short of the planes")
    small = torch.zeros(need - 256, dtype=torch.uint8, device=dev())
    desc.desc_gemm_grouped(d, mode="bf16x3", ws=small)
    assert desc.workspace_status(small) == 2   # DESC_DEV_PLANES, reset by the read
    assert desc.workspace_status(small) == 0
    for _, _, C in dev_pairs:
        assert torch.isnan(C).all()           # nothing computed
    case("grouped bf16x3 workspace of the full size")
    ws = torch.full((need,), 0xAB, dtype=torch.uint8, device=dev())
    desc.desc_gemm_grouped(d, mode="bf16x3", ws=ws)
    assert desc.workspace_status(ws) == 0
    assert _check_all(pairs, [C.cpu().numpy() for _, _, C in dev_pairs])[0] <= 1.0


@pytest.mark.parametrize("bf16_config", BF16_CONFIGS, indirect=True)
def test_grouped_bf16x3_graph_replay(bf16_config):
    pairs = _problems([(200, 100, 300), (64, 640, 64), (512, 512, 64), (3, 5, 0)], 6)
    outs, dp, d = _run(pairs, mode="bf16x3")
    need = desc.desc_gemm_grouped_workspace_for("bf16x3", d.cpu())
    ws = torch.empty(need, dtype=torch.uint8, device=dev())
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s):
        desc.desc_gemm_grouped(d, mode="bf16x3", ws=ws)
    for rep in range(3):
        case(f"grouped bf16x3 graph replay {rep} config {bf16_config}")
        for _, _, C in dp:
            C.fill_(0)
        ws.fill_(0x5A)                        # planes and plan rewritten by every replay
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        for (_, _, C), want in zip(dp, outs):
            assert np.array_equal(C.cpu().numpy(), want)


@pytest.mark.parametrize("bf16_config", BF16_CONFIGS, indirect=True)
def test_grouped_bf16x3_workload_512(bf16_config):
    assert desc.desc_config_count("gemm_grouped_bf16x3") == len(BF16_CONFIGS)
    case(f"grouped bf16x3 512 problems (seeds 12/13/14) config {bf16_config}")
    shapes = workloads.grouped_shapes()
    pairs = workloads.grouped_operands(shapes)
    outs, _, _ = _run(pairs, mode="bf16x3")
    worst = 0.0
    for p, ((A, B), C) in enumerate(zip(pairs, outs)):
        ii, jj = workloads.sample_pairs(C.shape[0], C.shape[1], 64, seed=14 + p)
        R, D = oracle.gemm_ref_sampled(A, B, ii, jj)
        err = np.abs(C[ii, jj] - R) / np.maximum(D, 1e-300)
        worst = max(worst, float(err.max()))
    print(f"[result] grouped bf16x3 512 worst componentwise error {worst:.3e}")
    assert worst <= TOL


@pytest.mark.parametrize("bf16_config", [2, 3], indirect=True)
def test_grouped_bf16x3_fused_routes_long_strides_through_planes(bf16_config):
    # a B stride past the split source's limit (2^24 elements): that problem
    # goes through the planes while the other is staged from FP32
    case(f"grouped bf16x3 ldb = 2^24 + 7 next to a plain problem, config {bf16_config}")
    g = workloads.rng(30)
    M, N, K, ldb = 70, 50, 3, (1 << 24) + 7
    A1 = g.standard_normal((M, K)).astype(np.float32)
    B1 = g.standard_normal((K, N)).astype(np.float32)
    Bbig = torch.zeros((K, ldb), dtype=torch.float32, device=dev())
    Bbig[:, :N] = torch.from_numpy(B1).to(dev())
    A2, B2 = _problems([(130, 90, 70)], 31)[0]
    C1 = torch.full((M, N), float("nan"), dtype=torch.float32, device=dev())
    C2 = torch.full((130, 90), float("nan"), dtype=torch.float32, device=dev())
    # the operands stay referenced until the call has finished: the
    # descriptors hold raw addresses, and freed blocks can become the workspace
    ops = [(to_dev(A1), Bbig[:, :N], C1), (to_dev(A2), to_dev(B2), C2)]
    d = desc.grouped_descriptors(ops, dev())
    desc.desc_gemm_grouped(d, mode="bf16x3")
    torch.cuda.synchronize()
    frac, _ = _check_all([(A1, B1), (A2, B2)], [C1.cpu().numpy(), C2.cpu().numpy()])
    assert frac <= 1.0
