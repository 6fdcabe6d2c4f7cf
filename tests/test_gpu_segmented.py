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

UNIT = 8192                    # units of work
TILES = (8192, 16384, 32768)   # power-of-two block sizes that edge cases straddle


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


def test_one_workspace_across_sizes_and_forms():
    """One zeroed workspace per operation for a sequence of calls whose
    sizes, segment counts and forms differ (one persistent launch up to 8192
    segments, plan + main kernel above): every call equals the oracle, so
    state words an earlier call left never count for a later one."""
    g = workloads.rng(23)
    sets = [
        [3 * UNIT + 5, 1, 0, 2 * UNIT],                            # persistent, long segments
        list(g.integers(0, 200, 9000)),                            # 9000 segments: two launches
        [0, 7, UNIT, 1],                                           # persistent, short
        list(g.integers(0, 3 * UNIT, 40)),                         # persistent, many units
        list(g.integers(0, 50, 8192)),                             # the largest persistent count
        [5 * UNIT + 3],
    ]
    cases = []
    for lengths in sets:
        off = workloads.offsets_from_lengths(np.array(lengths, np.int64))
        cases.append((workloads.int_uniform(int(off[-1]), seed=29), off))
    wr_bytes = max(desc.desc_reduce_segmented_i32_workspace(x.size, off.size - 1) for x, off in cases)
    ws_bytes = max(desc.desc_scan_segmented_i32_workspace(x.size, off.size - 1) for x, off in cases)
    wr = torch.zeros(wr_bytes, dtype=torch.uint8, device=dev())
    wy = torch.zeros(ws_bytes, dtype=torch.uint8, device=dev())
    for rep in range(2):
        for i, (x, off) in enumerate(cases):
            case(f"segmented shared workspace rep {rep} case {i} (S = {off.size - 1})")
            xt, ot = to_dev(x), to_dev(off)
            r = torch.full((off.size - 1,), 123, dtype=torch.int64, device=dev())
            y = torch.full((x.size,), -7, dtype=torch.int32, device=dev())
            desc.desc_reduce_segmented_i32(xt, ot, r, ws=wr)
            desc.desc_scan_segmented_i32(xt, ot, y, ws=wy)
            assert np.array_equal(r.cpu().numpy(), oracle.reduce_segmented_i32(x, off)), i
            assert np.array_equal(y.cpu().numpy(), oracle.scan_segmented_i32(x, off)), i
    assert desc.workspace_status(wr) == 0 and desc.workspace_status(wy) == 0


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
    # zero-filled once, as the workspace contract asks
    wr = torch.zeros(desc.desc_reduce_segmented_i32_workspace(x.size, S), dtype=torch.uint8,
                     device=dev())
    wy = torch.zeros(desc.desc_scan_segmented_i32_workspace(x.size, S), dtype=torch.uint8,
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


def _tile_edge_lengths():
    # boundaries on, just before and just after every tile edge of every
    # configuration, a segment spanning many tiles, and dense short segments
    lengths = []
    for t in TILES:
        lengths += [t, t - 1, 1, t + 1, 0, 2 * t, 3]
    lengths += [5 * 32768 + 11]
    lengths += list(workloads.rng(5).integers(0, 9, 2000))
    lengths += [1] * 300 + [0] * 5 + [70_000]
    return np.array(lengths, np.int64)


@pytest.fixture
def restore_seg_configs():
    yield
    for op in ("seg_scan_i32", "seg_reduce_i32"):
        for cls in range(4):
            desc.desc_config_set(op, cls, -1)


@pytest.mark.parametrize("offset", [0, 1])
def test_every_config_tile_edges(offset, restore_seg_configs):
    lengths = _tile_edge_lengths()
    off = workloads.offsets_from_lengths(lengths)
    n = int(off[-1])
    x = workloads.int_uniform(n, seed=23)
    want = oracle.scan_segmented_i32(x, off)
    xt, ot = to_dev(x, offset), to_dev(off)   # offset 1: unaligned input, scalar path
    cls = desc.desc_size_class("seg_scan_i32", n)
    want_r = oracle.reduce_segmented_i32(x, off)
    for cfg in range(desc.desc_config_count("seg_scan_i32")):
        name = desc.desc_config_name("seg_scan_i32", cfg)
        case(f"segmented scan/reduce config {name} n={n} offset={offset}")
        desc.desc_config_set("seg_scan_i32", cls, cfg)
        # the reduce has fewer configurations; past its last, keep its last
        rcfg = min(cfg, desc.desc_config_count("seg_reduce_i32") - 1)
        desc.desc_config_set("seg_reduce_i32", cls, rcfg)
        y = torch.full((n,), -5, dtype=torch.int32, device=dev())
        desc.desc_scan_segmented_i32(xt, ot, y)
        r = torch.full((off.size - 1,), 9, dtype=torch.int64, device=dev())
        desc.desc_reduce_segmented_i32(xt, ot, r)
        assert np.array_equal(y.cpu().numpy(), want), name
        assert np.array_equal(r.cpu().numpy(), want_r), name


def test_every_config_gaps_and_workload_slice(restore_seg_configs):
    # starts late and ends early (positions outside every segment untouched),
    # and a 2^22-element slice of the 4096-segment workload's lengths
    x = workloads.int_uniform(200_000, seed=29)
    off_gap = np.array([9000, 9000, 40_000, 40_001, 150_000, 150_000], np.int64)
    lengths = workloads.segment_lengths(400, seed=10, max_len=1 << 14)
    off_w = workloads.offsets_from_lengths(lengths)
    xw = workloads.int_uniform(int(off_w[-1]), seed=11)
    for cfg in range(desc.desc_config_count("seg_scan_i32")):
        name = desc.desc_config_name("seg_scan_i32", cfg)
        for xx, off, fill in ((x, off_gap, -77), (xw, off_w, 0)):
            n = xx.size
            case(f"segmented scan config {name} n={n} S={off.size - 1}")
            for cls in range(4):
                desc.desc_config_set("seg_scan_i32", cls, cfg)
            for cls in range(4):
                desc.desc_config_set("seg_reduce_i32", cls,
                                     min(cfg, desc.desc_config_count("seg_reduce_i32") - 1))
            y = torch.full((n,), fill, dtype=torch.int32, device=dev())
            r = torch.full((off.size - 1,), 9, dtype=torch.int64, device=dev())
            desc.desc_scan_segmented_i32(to_dev(xx), to_dev(off), y)
            desc.desc_reduce_segmented_i32(to_dev(xx), to_dev(off), r)
            assert np.array_equal(y.cpu().numpy(), oracle.scan_segmented_i32(xx, off, fill=fill)), name
            assert np.array_equal(r.cpu().numpy(), oracle.reduce_segmented_i32(xx, off)), name
