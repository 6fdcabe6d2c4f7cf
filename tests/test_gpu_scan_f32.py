"""Parity of the HIP fixed-order float scan with the CPU oracle (the exact
prefix sums), called through the C ABI.

Every output is checked against the exact prefix S_i within the documented
bound 2^-24 |S_i| + 2^-149 + d 2^-53 sum_{k<=i} |x_k| (d = ceil(T / 64) + 160,
T the number of 65536-element tiles): the final rounding to float32 plus the
FP64 additions of the order, so each output is one of the two float32
neighbours of a value within d 2^-53 sum|x| of the exact prefix.  A dropped
or repeated element, or a wrong carry, moves an output by about |x_k|, far
outside the bound.  Outputs are also compared bit for bit across runs and
input addresses (aligned and unaligned load paths), which is what the fixed
order promises.  Sizes span one lane, one tile (65536), one group of 64
tiles, ragged tails in several groups, and the 2^28-element workload
(checked at sampled positions)."""
import numpy as np
import pytest
import torch

import oracle
import workloads
import paper_2305_03448_amd as desc
from gpu_util import case, dev, needs_gpu, to_dev

pytestmark = [pytest.mark.gpu, needs_gpu]

TILE, GROUP = 65536, 64
SIZES = [1, 2, 5, 63, 4095, 4097, 65535, 65536, 65537, 3 * 65536 + 5, GROUP * 65536,
         GROUP * 65536 + 1, 130 * 65536 + 77]


def _scan(xt, ws=None):
    out = torch.full_like(xt, float("nan"))
    desc.desc_scan_f32(xt, out, ws=ws)
    return out.cpu().numpy()


def _check(x, y, idx=None):
    n = x.size
    T = -(-n // TILE)
    d = -(-T // GROUP) + 160
    cum = np.cumsum(np.abs(x.astype(np.float64))) * (1 + 1e-6)
    if idx is None:
        idx = np.arange(n, dtype=np.int64)
    exact = oracle.scan_f32(x, idx)
    got = y[idx].astype(np.float64)
    bound = 2.0 ** -24 * np.abs(exact) + 2.0 ** -149 + d * 2.0 ** -53 * cum[idx]
    err = np.abs(got - exact)
    bad = np.flatnonzero(~(err <= bound))
    assert bad.size == 0, (f"{bad.size} outputs outside the bound; first at {idx[bad[0]]}: "
                           f"got {got[bad[0]]!r}, exact {exact[bad[0]]!r}")


@pytest.mark.parametrize("n", SIZES)
def test_scan_f32_sizes(n):
    case(f"scan_f32 n={n}")
    x = workloads.wide_f32(n, seed=400 + n % 79)
    _check(x, _scan(to_dev(x)))


def test_scan_f32_normal_values_and_cancellation():
    n = 5 * 65536 + 3
    x = workloads.normal_f32(n, seed=41)
    case("scan_f32 normal")
    _check(x, _scan(to_dev(x)))
    y = np.zeros(n, np.float32)
    y[::2], y[1::2] = 3.0e30, -3.0e30          # prefixes alternate 3e30, 0
    y[7] = 1.0
    case("scan_f32 cancellation")
    _check(y, _scan(to_dev(y)))


def test_scan_f32_denormals():
    n = 2 * 65536 + 9
    x = np.full(n, np.float32(2.0 ** -149))
    x[1::5] = np.float32(-(2.0 ** -147))
    case("scan_f32 denormals")
    got = _scan(to_dev(x))
    # every prefix is a small multiple of 2^-149: exact in FP64 and float32
    assert np.array_equal(got.astype(np.float64), oracle.scan_f32(x))


@pytest.mark.parametrize("n", [7, 65537, GROUP * 65536 + 3])
def test_scan_f32_same_bits_at_every_address_and_run(n):
    x = workloads.wide_f32(n, seed=19)
    ref = None
    for offset in (0, 1, 2, 3, 4):
        case(f"scan_f32 n={n} offset={offset}")
        xt = to_dev(x, offset)
        a = _scan(xt).view(np.uint32)
        b = _scan(xt).view(np.uint32)
        assert np.array_equal(a, b)
        if ref is None:
            ref = a
            _check(x, a.view(np.float32))
        assert np.array_equal(a, ref)


def test_scan_f32_non_finite():
    x = workloads.normal_f32(3 * 65536, seed=42)
    y = x.copy()
    y[70000] = np.inf
    case("scan_f32 +inf")
    got = _scan(to_dev(y))
    assert np.all(np.isfinite(got[:70000])) and np.all(got[70000:] == np.inf)
    y[150000] = -np.inf
    case("scan_f32 +inf then -inf")
    got = _scan(to_dev(y))
    assert np.all(got[70000:150000] == np.inf) and np.all(np.isnan(got[150000:]))


def test_scan_f32_workspace_reuse_and_empty():
    ws = torch.zeros(desc.desc_scan_f32_workspace(GROUP * 65536 * 2), dtype=torch.uint8,
                     device=dev())
    for rep, n in enumerate((GROUP * 65536 * 2, 65537, 1, GROUP * 65536 + 5, 3)):
        case(f"scan_f32 shared workspace rep {rep} n={n}")
        x = workloads.wide_f32(n, seed=70 + rep)
        _check(x, _scan(to_dev(x), ws=ws))
    assert int(ws[4:8].view(torch.int32).item()) == 0   # no inconsistency recorded
    case("scan_f32 n=0")
    e = torch.empty(0, dtype=torch.float32, device=dev())
    desc.desc_scan_f32(e, torch.empty_like(e))


def test_scan_f32_workload_2_28_sampled():
    n = 1 << 28
    case("scan_f32 2^28")
    x = workloads.wide_f32(n, seed=workloads.SEEDS["reduce_f32"])
    xt = to_dev(x)
    out = torch.empty_like(xt)
    desc.desc_scan_f32(xt, out)
    g = np.random.default_rng(43)
    idx = np.unique(np.concatenate([g.integers(0, n, 4096), np.arange(0, n, TILE),
                                    np.arange(TILE - 1, n, TILE), [n - 1]])).astype(np.int64)
    y = out[torch.from_numpy(idx).to(dev())].cpu().numpy()
    full = np.empty(n, np.float32)
    full[idx] = y
    _check(x, full, idx)
    out2 = torch.empty_like(xt)
    desc.desc_scan_f32(xt, out2)
    assert torch.equal(out.view(torch.int32), out2.view(torch.int32))


def test_scan_f32_graph_replay():
    # the float scan captured into a HIP graph: every replay, with eager
    # scans on another workspace in between, gives the eager bits
    n = 3 * 65536 + 11
    x = workloads.wide_f32(n, seed=93)
    xt = to_dev(x)
    ws = torch.zeros(desc.desc_scan_f32_workspace(n), dtype=torch.uint8, device=dev())
    y = torch.empty_like(xt)
    case("scan_f32 eager before capture")
    desc.desc_scan_f32(xt, y, ws=ws)
    want = y.cpu().numpy().view(np.uint32).copy()
    _check(x, y.cpu().numpy())
    stream = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=stream):
        desc.desc_scan_f32(xt, y, ws=ws)
    other = torch.zeros(desc.desc_scan_f32_workspace(70000), dtype=torch.uint8, device=dev())
    z = to_dev(workloads.wide_f32(70000, seed=94))
    for rep in range(3):
        case(f"scan_f32 graph replay {rep}")
        y.fill_(float("nan"))
        desc.desc_scan_f32(z, torch.empty_like(z), ws=other)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(y.cpu().numpy().view(np.uint32), want)
