"""Parity of the HIP min/max and fixed-order float sum with the CPU oracle,
called through the C ABI.

Min/max is compared bit for bit.  The float sum is compared two ways: with
the exact sum (the oracle) within the bound of the documented order,
d 2^-53 sum|x| (d the longest chain of additions), and bit for bit with a
numpy model of that order (tests/sum_order_model.py), which also checks
that the result does not depend on the input's address or on the run.
Sizes span one lane, one chunk (4096), ragged tails, more chunks than
blocks, and the 2^28-element workload in the benchmark's configuration."""
import math
import struct

import numpy as np
import pytest
import torch

import oracle
import paper_2305_03448_amd as desc
import workloads
from gpu_util import case, dev, needs_gpu, to_dev
from sum_order_model import chain_bound, fixed_order_sum

pytestmark = [pytest.mark.gpu, needs_gpu]

SIZES = [1, 2, 3, 4, 5, 63, 255, 256, 1023, 1024, 1025, 4095, 4096, 4097, 8191, 8193,
         3 * 4096 + 17, 65537, 1_000_003, 2048 * 4096, 2048 * 4096 + 1,
         2048 * 4096 + 3 * 4096 + 11, (1 << 22) + 5]


def _bits(v: float) -> int:
    return struct.unpack("<Q", struct.pack("<d", v))[0]


def _minmax(xt):
    out = torch.full((2,), 7, dtype=torch.int32, device=dev())
    desc.desc_reduce_minmax_i32(xt, out)
    lo, hi = out.cpu().tolist()
    return lo, hi


def _sum(xt):
    out = torch.full((1,), -1.0, dtype=torch.float64, device=dev())
    desc.desc_reduce_sum_f32(xt, out)
    return float(out.item())


def _bound(x):
    return chain_bound(x.size) * 2.0 ** -53 * float(np.abs(x.astype(np.float64)).sum())


# ------------------------------------------------------------------ min / max
@pytest.mark.parametrize("n", [0] + SIZES)
def test_minmax_sizes(n):
    case(f"minmax n={n}")
    x = workloads.int_uniform(n, seed=200 + n % 89, lo=-(1 << 31), hi=(1 << 31) - 1)
    assert _minmax(to_dev(x)) == oracle.minmax_i32(x)


@pytest.mark.parametrize("offset", [1, 2, 3])
@pytest.mark.parametrize("n", [5, 4097, 300_001])
def test_minmax_unaligned(n, offset):
    case(f"minmax unaligned n={n} offset={offset}")
    x = workloads.int_uniform(n, seed=9)
    assert _minmax(to_dev(x, offset)) == oracle.minmax_i32(x)


@pytest.mark.parametrize("n", [1, 4097, 2048 * 4096 + 5])
def test_minmax_extremes_at_the_ends(n):
    for where in ("first", "last", "tail"):
        case(f"minmax extremes n={n} at {where}")
        x = np.zeros(n, np.int32)
        i_lo, i_hi = {"first": (0, n - 1), "last": (n - 1, 0),
                      "tail": (n - 1, max(n - 2, 0))}[where]
        x[i_hi] = (1 << 31) - 1
        x[i_lo] = -(1 << 31)
        assert _minmax(to_dev(x)) == oracle.minmax_i32(x)
    case(f"minmax constant n={n}")
    x = np.full(n, -17, np.int32)
    assert _minmax(to_dev(x)) == (-17, -17)


# ------------------------------------------------------------------ float sum
@pytest.mark.parametrize("n", SIZES)
def test_sum_f32_sizes(n):
    case(f"sum_f32 n={n}")
    x = workloads.wide_f32(n, seed=300 + n % 83)
    got = _sum(to_dev(x))
    assert abs(got - oracle.sum_f32(x)) <= _bound(x)
    assert _bits(got) == _bits(fixed_order_sum(x))


def test_sum_f32_empty_is_zero():
    case("sum_f32 n=0")
    assert _sum(torch.empty(0, dtype=torch.float32, device=dev())) == 0.0


@pytest.mark.parametrize("n", [5, 4097, 300_001, 2048 * 4096 + 3])
def test_sum_f32_same_bits_at_every_address_and_run(n):
    x = workloads.wide_f32(n, seed=17)
    want = _bits(fixed_order_sum(x))
    for offset in (0, 1, 2, 3, 5):
        case(f"sum_f32 n={n} offset={offset}")
        xt = to_dev(x, offset)
        assert _bits(_sum(xt)) == want
        assert _bits(_sum(xt)) == want


def test_sum_f32_denormals_and_cancellation():
    n = 3 * 4096 + 7
    x = np.zeros(n, np.float32)
    x[::3] = np.float32(2.0 ** -149)                 # the smallest denormal
    x[1::3] = np.float32(-(2.0 ** -140))
    x[5], x[4096 * 2 + 9] = 2.0 ** 100, -(2.0 ** 100)
    case("sum_f32 denormals and cancellation")
    got = _sum(to_dev(x))
    assert _bits(got) == _bits(fixed_order_sum(x))
    assert abs(got - oracle.sum_f32(x)) <= _bound(x)
    y = np.full(4096 * 5 + 1, np.float32(2.0 ** -149))
    case("sum_f32 denormals only")
    assert _sum(to_dev(y)) == oracle.sum_f32(y) == y.size * 2.0 ** -149


def test_sum_f32_non_finite():
    x = workloads.wide_f32(10_000, seed=18)
    for put, check in ([((7, np.inf),), lambda v: v == math.inf],
                       [((9999, -np.inf),), lambda v: v == -math.inf],
                       [((3, np.inf), (8000, -np.inf)), math.isnan],
                       [((5000, np.nan),), math.isnan]):
        y = x.copy()
        for i, v in put:
            y[i] = v
        case(f"sum_f32 non-finite {put}")
        got = _sum(to_dev(y))
        assert check(got) and check(oracle.sum_f32(y))


def test_sum_f32_shares_workspace_with_minmax():
    ws = torch.zeros(desc.desc_reduce_op_workspace(1 << 20), dtype=torch.uint8, device=dev())
    for rep, n in enumerate((1 << 20, 4097, 1, 1 << 20, 0, 65537)):
        case(f"shared workspace rep {rep} n={n}")
        xf = workloads.wide_f32(n, seed=50 + rep)
        xi = workloads.int_uniform(n, seed=60 + rep)
        s = torch.empty(1, dtype=torch.float64, device=dev())
        m = torch.empty(2, dtype=torch.int32, device=dev())
        desc.desc_reduce_sum_f32(to_dev(xf), s, ws=ws)
        desc.desc_reduce_minmax_i32(to_dev(xi), m, ws=ws)
        assert _bits(float(s.item())) == _bits(fixed_order_sum(xf))
        assert tuple(m.cpu().tolist()) == oracle.minmax_i32(xi)
    assert int(ws[4:8].view(torch.int32).item()) == 0   # no inconsistency recorded


def test_reduce_ops_workload_2_28():
    # the benchmark's 2^28-element inputs and launch configuration
    n = 1 << 28
    case("minmax 2^28")
    xi = workloads.int_uniform(n, seed=workloads.SEEDS["scan"], lo=-(1 << 31), hi=(1 << 31) - 1)
    assert _minmax(to_dev(xi)) == oracle.minmax_i32(xi)
    del xi
    case("sum_f32 2^28")
    xf = workloads.wide_f32(n, seed=workloads.SEEDS["reduce_f32"])
    xt = to_dev(xf)
    got = _sum(xt)
    assert _bits(_sum(xt)) == _bits(got)
    assert abs(got - oracle.sum_f32(xf)) <= _bound(xf)
    assert _bits(got) == _bits(fixed_order_sum(xf))


def test_reduce_ops_graph_replay():
    # min/max and the float sum captured into one HIP graph; each replay,
    # with eager calls on other workspaces in between, gives the eager bits
    n = (1 << 22) + 5
    xf = workloads.wide_f32(n, seed=90)
    xi = workloads.int_uniform(n, seed=91, lo=-(1 << 31), hi=(1 << 31) - 1)
    xft, xit = to_dev(xf), to_dev(xi)
    ws = torch.zeros(desc.desc_reduce_op_workspace(n), dtype=torch.uint8, device=dev())
    s = torch.empty(1, dtype=torch.float64, device=dev())
    m = torch.empty(2, dtype=torch.int32, device=dev())
    case("reduce ops eager before capture")
    desc.desc_reduce_sum_f32(xft, s, ws=ws)
    desc.desc_reduce_minmax_i32(xit, m, ws=ws)
    want_s, want_m = _bits(float(s.item())), tuple(m.cpu().tolist())
    assert want_s == _bits(fixed_order_sum(xf)) and want_m == oracle.minmax_i32(xi)
    stream = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=stream):
        desc.desc_reduce_sum_f32(xft, s, ws=ws)
        desc.desc_reduce_minmax_i32(xit, m, ws=ws)
    other = torch.zeros(desc.desc_reduce_op_workspace(4097), dtype=torch.uint8, device=dev())
    y = to_dev(workloads.wide_f32(4097, seed=92))
    for rep in range(3):
        case(f"reduce ops graph replay {rep}")
        s.fill_(-1.0); m.fill_(7)
        desc.desc_reduce_sum_f32(y, torch.empty(1, dtype=torch.float64, device=dev()), ws=other)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert _bits(float(s.item())) == want_s
        assert tuple(m.cpu().tolist()) == want_m
