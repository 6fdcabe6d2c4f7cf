"""The hand-indexed twin kernels (the baseline of the view-layer comparison)
give the library's results bit for bit: compared with the oracle at ragged
sizes and with the view kernels at the sizes of the comparison."""
import os
import sys

import numpy as np
import pytest
import torch

import oracle
import paper_2305_03448_amd as desc
import workloads
from gpu_util import case, dev, needs_gpu, to_dev

sys.path.insert(0, os.path.join(os.path.dirname(os.path.abspath(__file__)), "handwritten"))
import handlib  # noqa: E402

pytestmark = [pytest.mark.gpu, needs_gpu]


@pytest.mark.parametrize("n", [1, 4097, 65535, 65536, 65537, 1_000_003])
def test_hand_reduce_scan_vs_oracle(n):
    case(f"hand reduce/scan n={n}")
    x = workloads.int_uniform(n, seed=300 + n % 89)
    xt = to_dev(x)
    out = torch.empty(1, dtype=torch.int64, device=dev())
    handlib.reduce_i32(xt, out)
    y = torch.empty_like(xt)
    handlib.scan_i32(xt, y)
    assert int(out.item()) == oracle.reduce_i32(x)
    assert np.array_equal(y.cpu().numpy(), oracle.scan_i32(x))


@pytest.mark.parametrize("shape", [(1, 1), (128, 128), (333, 517), (260, 1028)])
def test_hand_transpose_vs_oracle(shape):
    case(f"hand transpose {shape}")
    m = workloads.matrix_f32(*shape, seed=301)
    t = torch.empty((shape[1], shape[0]), dtype=torch.float32, device=dev())
    handlib.transpose_f32(to_dev(m), t)
    assert np.array_equal(t.cpu().numpy().view(np.uint32), oracle.transpose_u32(m).view(np.uint32))


def test_hand_equals_view_at_comparison_sizes():
    # the smallest size of the comparison (256 MB of memory per operation)
    n = 1 << 25
    case(f"hand vs view reduce/scan n={n}")
    x = torch.from_numpy(workloads.int_uniform(n, seed=2)).to(dev())
    o1 = torch.empty(1, dtype=torch.int64, device=dev())
    o2 = torch.empty(1, dtype=torch.int64, device=dev())
    desc.desc_reduce_i32(x, o1)
    handlib.reduce_i32(x, o2)
    y1, y2 = torch.empty_like(x), torch.empty_like(x)
    desc.desc_scan_i32(x, y1)
    handlib.scan_i32(x, y2)
    assert int(o1.item()) == int(o2.item())
    assert torch.equal(y1, y2)
    case("hand vs view transpose 4096x8192")
    m = torch.from_numpy(workloads.matrix_f32(4096, 8192, seed=3)).to(dev())
    t1 = torch.empty((8192, 4096), dtype=torch.float32, device=dev())
    t2 = torch.empty_like(t1)
    desc.desc_transpose_f32(m, t1)
    handlib.transpose_f32(m, t2)
    assert torch.equal(t1.view(torch.int32), t2.view(torch.int32))


@pytest.mark.parametrize("M,N,K", [(256, 128, 16), (300, 200, 50), (1000, 1000, 1000),
                                   (513, 129, 257), (4, 4, 4)])
def test_hand_gemm_equals_the_view_gemm(M, N, K):
    # same tile, same k assignment, same accumulation order: bit-equal
    case(f"hand vs view gemm f32 {M}x{N}x{K}")
    A = to_dev(workloads.matrix_f32(M, K, seed=302)); B = to_dev(workloads.matrix_f32(K, N, seed=303))
    C1 = torch.full((M, N), float("nan"), dtype=torch.float32, device=dev())
    C2 = torch.full((M, N), float("nan"), dtype=torch.float32, device=dev())
    cls = desc.desc_size_class("gemm_f32", M * N * K)
    cfg = [desc.desc_config_name("gemm_f32", i) for i in range(desc.desc_config_count("gemm_f32"))]
    try:
        desc.desc_config_set("gemm_f32", cls, cfg.index(handlib.VIEW_CONFIGS["gemm_f32"]))
        desc.desc_gemm(A, B, C1, mode="f32")
    finally:
        desc.desc_config_set("gemm_f32", cls, -1)
    handlib.gemm_f32(A, B, C2)
    torch.cuda.synchronize()
    assert torch.equal(C1.view(torch.int32), C2.view(torch.int32))
    Ai = workloads.rng(304).integers(-4, 5, (M, K)).astype(np.float32)
    Bi = workloads.rng(305).integers(-4, 5, (K, N)).astype(np.float32)
    handlib.gemm_f32(to_dev(Ai), to_dev(Bi), C2)
    assert np.array_equal(C2.cpu().numpy(), (Ai.astype(np.int64) @ Bi.astype(np.int64)).astype(np.float32))


def test_hardware_e4m3_matches_encoder_on_every_input():
    # the quantisers use the hardware conversion only where this holds
    case("e4m3 hardware vs software over all 2^32 inputs")
    inside, outside = handlib.e4m3_all_inputs()
    assert inside == 0
    assert outside > 0   # NaN codes from 464 up: why larger magnitudes use the software path


def test_hardware_bf16_matches_rounding_on_every_input():
    # the split uses the hardware conversion for every input
    case("bf16 hardware vs software over all 2^32 inputs")
    numbers, nans = handlib.bf16_all_inputs()
    print(f"[result] bf16 hardware disagreements: {numbers} numbers, {nans} NaNs")
    assert numbers == 0 and nans == 0
