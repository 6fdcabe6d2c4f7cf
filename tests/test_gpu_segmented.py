"""Parity of the segmented reduce and scan with the CPU oracle, bit for bit,
through the C ABI: each segment equals the unsegmented definition on its
slice, including empty, length-1, unit-boundary and 2^20-long segments,
positions outside every segment stay untouched, and the 4096-segment
workload (lengths log-uniform in [1, 2^20], seed 10; values seed 11) runs at
full size."""
import numpy as np
import pytest
import torch

import oracle
import paper_2305_03448_amd as desc
import workloads
from gpu_util import case, dev, needs_gpu, to_dev

pytestmark = [pytest.mark.gpu, needs_gpu]

UNIT = 8192


def _both(x, off, fill=-7):
    xt = to_dev(x)
    ot = to_dev(off)
    S = off.size - 1
    r = torch.full((S,), 123, dtype=torch.int64, device=dev())
    y = torch.full((x.size,), fill, dtype=torch.int32, device=dev())
    desc.desc_reduce_segmented_i32(xt, ot, r)
    desc.desc_scan_segmented_i32(xt, ot, y)
    return r.cpu().numpy(), y.cpu().numpy()


LENGTH_SETS = {
    "mixed": [0, 1, 5, 0, 64, 65, 1000, 0, 3, UNIT - 1, UNIT, UNIT + 1, 2 * UNIT + 7, 1, 0],
    "one_long": [(1 << 20) + 3],
    "all_empty": [0, 0, 0],
    "unit_multiples": [UNIT] * 5 + [3 * UNIT],
    "many_small": list(workloads.rng(3).integers(0, 40, 3000)),
}


@pytest.mark.parametrize("name", sorted(LENGTH_SETS))
def test_segments_match_oracle(name):
    case(f"segmented {name}")
    lengths = np.array(LENGTH_SETS[name], np.int64)
    off = workloads.offsets_from_lengths(lengths)
    x = workloads.int_uniform(int(off[-1]), seed=17)
    r, y = _both(x, off)
    assert np.array_equal(r, oracle.reduce_segmented_i32(x, off))
    assert np.array_equal(y, oracle.scan_segmented_i32(x, off))


def test_gaps_untouched_and_subrange():
    case("segmented gaps")
    x = workloads.int_uniform(50_000, seed=19)
    off = np.array([3, 10, 10, 9000, 9001, 30_000], np.int64)   # starts late, ends early
    r, y = _both(x, off, fill=-99)
    assert np.array_equal(r, oracle.reduce_segmented_i32(x, off))
    assert np.array_equal(y, oracle.scan_segmented_i32(x, off, fill=-99))


def test_extreme_values_exact():
    case("segmented extremes")
    lengths = np.array([1, (1 << 20), 17, UNIT * 3 + 1], np.int64)
    off = workloads.offsets_from_lengths(lengths)
    x = np.full(int(off[-1]), 2**31 - 1, np.int32)
    x[::3] = -2**31
    r, y = _both(x, off)
    assert np.array_equal(r, oracle.reduce_segmented_i32(x, off))
    assert np.array_equal(y, oracle.scan_segmented_i32(x, off))


def test_repeated_calls_and_graph_replay():
    lengths = workloads.segment_lengths(300, seed=10, max_len=1 << 16)
    off = workloads.offsets_from_lengths(lengths)
    x = workloads.int_uniform(int(off[-1]), seed=11)
    xt, ot = to_dev(x), to_dev(off)
    S = off.size - 1
    want_r = oracle.reduce_segmented_i32(x, off)
    want_y = oracle.scan_segmented_i32(x, off)
    r = torch.empty(S, dtype=torch.int64, device=dev())
    y = torch.empty(x.size, dtype=torch.int32, device=dev())
    wr = torch.empty(desc.desc_reduce_segmented_i32_workspace(x.size, S), dtype=torch.uint8,
                     device=dev())
    wy = torch.empty(desc.desc_scan_segmented_i32_workspace(x.size, S), dtype=torch.uint8,
                     device=dev())
    for rep in range(3):
        case(f"segmented eager rep {rep}")
        desc.desc_reduce_segmented_i32(xt, ot, r, ws=wr)
        desc.desc_scan_segmented_i32(xt, ot, y, ws=wy)
        assert np.array_equal(r.cpu().numpy(), want_r)
        assert np.array_equal(y.cpu().numpy(), want_y)
    case("segmented graph capture")
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s):
        desc.desc_reduce_segmented_i32(xt, ot, r, ws=wr)
        desc.desc_scan_segmented_i32(xt, ot, y, ws=wy)
    for rep in range(3):
        case(f"segmented graph replay {rep}")
        r.fill_(0); y.fill_(0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(r.cpu().numpy(), want_r)
        assert np.array_equal(y.cpu().numpy(), want_y)


def test_workload_4096_segments():
    case("segmented 4096 segments (seeds 10/11)")
    x, off = workloads.segmented_input()
    assert off[-1] == 315_525_003
    r, y = _both(x, off)
    assert np.array_equal(r, oracle.reduce_segmented_i32(x, off))
    assert np.array_equal(y, oracle.scan_segmented_i32(x, off))
