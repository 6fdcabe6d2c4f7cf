"""The paper's own forms of the reduction and the scan (Sec. 5): the
block-wide reduction (one exact int64 per chunk of E elements, a
split/synchronise tree inside each block) and the two-kernel scan, bit for
bit against the oracle through the C ABI, at ragged sizes, unaligned starts,
extreme values and the 2^28 workload (where the two scans must agree)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2305_03448_amd as desc
import workloads
from gpu_util import case, dev, needs_gpu, to_dev

pytestmark = [pytest.mark.gpu, needs_gpu]


def _chunk_sums(x, E):
    return np.array([oracle.reduce_i32(x[b:b + E]) for b in range(0, x.size, E)], np.int64)


@pytest.mark.parametrize("E", [1024, 4096, 65536])
@pytest.mark.parametrize("n", [1, 1023, 1024, 4097, 300_001, (1 << 20) + 5])
def test_reduce_blocks_vs_oracle(n, E):
    case(f"reduce_blocks n={n} E={E}")
    x = workloads.int_uniform(n, seed=500 + n % 13)
    out = torch.full(((n + E - 1) // E,), 7, dtype=torch.int64, device=dev())
    desc.desc_reduce_blocks_i32(to_dev(x), E, out)
    assert np.array_equal(out.cpu().numpy(), _chunk_sums(x, E))


@pytest.mark.parametrize("offset", [1, 3])
def test_reduce_blocks_unaligned_and_extremes(offset):
    n, E = 70_000, 2048
    case(f"reduce_blocks unaligned offset={offset}")
    x = np.full(n, 2**31 - 1, np.int32)
    x[::5] = -2**31
    out = torch.empty(((n + E - 1) // E,), dtype=torch.int64, device=dev())
    desc.desc_reduce_blocks_i32(to_dev(x, offset), E, out)
    assert np.array_equal(out.cpu().numpy(), _chunk_sums(x, E))


@pytest.mark.parametrize("n", [1, 5, 65535, 65536, 65537, 131072 + 9, 1_000_003, (1 << 22) + 7])
def test_scan_two_pass_vs_oracle(n):
    case(f"scan_two_pass n={n}")
    x = workloads.int_uniform(n, seed=600 + n % 11)
    y = torch.full((n,), -3, dtype=torch.int32, device=dev())
    desc.desc_scan_two_pass_i32(to_dev(x), y)
    assert np.array_equal(y.cpu().numpy(), oracle.scan_i32(x))


def test_scan_two_pass_unaligned_and_wrap():
    n = 300_001
    case("scan_two_pass unaligned, wrapping")
    x = np.full(n, 2**31 - 1, np.int32)
    y = torch.empty(n + 1, dtype=torch.int32, device=dev())[1:]
    desc.desc_scan_two_pass_i32(to_dev(x, 1), y)
    assert np.array_equal(y.cpu().numpy(), oracle.scan_i32(x))


def test_two_scans_agree_at_2_28():
    n = 1 << 28
    case("scan single-pass vs two-pass 2^28")
    x = torch.from_numpy(workloads.int_uniform(n, seed=2)).to(dev())
    y1, y2 = torch.empty_like(x), torch.empty_like(x)
    desc.desc_scan_i32(x, y1)
    desc.desc_scan_two_pass_i32(x, y2)
    assert torch.equal(y1, y2)
