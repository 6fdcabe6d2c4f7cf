"""Parity of the HIP reduce, scan and transpose with the CPU oracle, bit for
bit, called through the C ABI (the Python binding marshals arguments only).

Sizes span one wave, one tile, many tiles and ragged tails; the full
workload sizes (2^22 reduce, 2^28 scan, 8192 x 8192 transpose) run in the
same launch configuration as the benchmark."""
import numpy as np
import pytest
import torch

import oracle
import paper_2305_03448_amd as desc
import workloads
from gpu_util import case, dev, needs_gpu, to_dev

pytestmark = [pytest.mark.gpu, needs_gpu]

EDGE_SIZES = [1, 2, 3, 4, 5, 63, 64, 65, 255, 256, 257, 1023, 1024, 1025, 4095, 4096, 4097,
              8191, 8192, 8193, 12289, 65535, 65536, 65537, 1_000_003, (1 << 20) + 7]


# ------------------------------------------------------------------ reduce
@pytest.mark.parametrize("n", [0] + EDGE_SIZES)
def test_reduce_edge_sizes(n):
    case(f"reduce n={n}")
    x = workloads.int_uniform(n, seed=100 + n % 97)
    out = torch.full((1,), -1, dtype=torch.int64, device=dev())
    desc.desc_reduce_i32(to_dev(x), out)
    assert int(out.item()) == oracle.reduce_i32(x)


@pytest.mark.parametrize("offset", [1, 2, 3])
@pytest.mark.parametrize("n", [5, 4097, 300_001])
def test_reduce_unaligned(n, offset):
    case(f"reduce unaligned n={n} offset={offset}")
    x = workloads.int_uniform(n, seed=7)
    out = torch.empty(1, dtype=torch.int64, device=dev())
    desc.desc_reduce_i32(to_dev(x, offset), out)
    assert int(out.item()) == oracle.reduce_i32(x)


def test_reduce_extremes_exact():
    n = (1 << 20) + 3
    for v in (2**31 - 1, -2**31):
        case(f"reduce extremes v={v}")
        x = np.full(n, v, np.int32)
        out = torch.empty(1, dtype=torch.int64, device=dev())
        desc.desc_reduce_i32(to_dev(x), out)
        assert int(out.item()) == oracle.reduce_i32(x) == n * v


def test_reduce_workload_and_reuse():
    # the 2^22 workload (seed 1), then repeated calls on the same workspace
    x = workloads.int_uniform(1 << 22, seed=1)
    xt = to_dev(x)
    want = oracle.reduce_i32(x)
    out = torch.empty(1, dtype=torch.int64, device=dev())
    for rep in range(5):
        case(f"reduce 2^22 rep {rep}")
        desc.desc_reduce_i32(xt, out)
        assert int(out.item()) == want
    small = xt[:1000]
    desc.desc_reduce_i32(small, out)
    assert int(out.item()) == oracle.reduce_i32(x[:1000])


def test_reduce_large_2_28():
    case("reduce 2^28")
    x = workloads.int_uniform(1 << 28, seed=2)
    out = torch.empty(1, dtype=torch.int64, device=dev())
    desc.desc_reduce_i32(to_dev(x), out)
    assert int(out.item()) == oracle.reduce_i32(x)


# ------------------------------------------------------------------ scan
@pytest.mark.parametrize("n", EDGE_SIZES)
def test_scan_edge_sizes(n):
    case(f"scan n={n}")
    x = workloads.int_uniform(n, seed=200 + n % 89)
    y = torch.full((n,), 7, dtype=torch.int32, device=dev())
    desc.desc_scan_i32(to_dev(x), y)
    assert np.array_equal(y.cpu().numpy(), oracle.scan_i32(x))


@pytest.mark.parametrize("offset", [1, 3])
@pytest.mark.parametrize("n", [7, 4097, 300_001])
def test_scan_unaligned(n, offset):
    case(f"scan unaligned n={n} offset={offset}")
    x = workloads.int_uniform(n, seed=9)
    y = torch.empty(n + offset, dtype=torch.int32, device=dev())[offset:]
    desc.desc_scan_i32(to_dev(x, offset), y)
    assert np.array_equal(y.cpu().numpy(), oracle.scan_i32(x))


def test_scan_wraps_modulo_2_32():
    case("scan wrap")
    n = 1 << 20
    x = np.full(n, 2**31 - 1000, np.int32)
    y = torch.empty(n, dtype=torch.int32, device=dev())
    desc.desc_scan_i32(to_dev(x), y)
    want, wrapped, _ = oracle.scan_i32(x, return_info=True)
    assert wrapped
    assert np.array_equal(y.cpu().numpy(), want)


def test_scan_workspace_reuse_varying_sizes():
    # generation tags: consecutive calls of different sizes on one workspace
    ws = torch.zeros(desc.desc_scan_i32_workspace(1 << 22), dtype=torch.uint8, device=dev())
    for rep, n in enumerate([1 << 22, 5000, (1 << 21) + 17, 1, 1 << 22, 123457]):
        case(f"scan reuse rep={rep} n={n}")
        x = workloads.int_uniform(n, seed=300 + rep)
        y = torch.empty(n, dtype=torch.int32, device=dev())
        desc.desc_scan_i32(to_dev(x), y, ws=ws)
        assert np.array_equal(y.cpu().numpy(), oracle.scan_i32(x))


def test_scan_workload_2_28():
    case("scan 2^28 (seed 2)")
    x = workloads.int_uniform(1 << 28, seed=2)
    y = torch.empty(1 << 28, dtype=torch.int32, device=dev())
    xt = to_dev(x)
    desc.desc_scan_i32(xt, y)
    want = oracle.scan_i32(x)
    assert np.array_equal(y.cpu().numpy(), want)
    # again on the same workspace (the benchmark calls it back to back)
    y.fill_(0)
    desc.desc_scan_i32(xt, y)
    assert np.array_equal(y.cpu().numpy(), want)


# ------------------------------------------------------------------ transpose
SHAPES = [(1, 1), (1, 37), (37, 1), (4, 4), (64, 64), (65, 129), (300, 7), (128, 256),
          (256, 64), (63, 65), (1000, 4), (4, 1000), (129, 4100)]


@pytest.mark.parametrize("rows,cols", SHAPES)
def test_transpose_self_describing(rows, cols):
    case(f"transpose {rows}x{cols}")
    m = workloads.self_describing_u32(rows, cols)
    t = torch.empty((cols, rows), dtype=torch.int32, device=dev())
    desc.desc_transpose_f32(to_dev(m.view(np.int32)), t)
    assert np.array_equal(t.cpu().numpy().view(np.uint32), oracle.transpose_u32(m))


def test_transpose_bits_and_involution():
    case("transpose bit patterns")
    g = workloads.rng(5)
    m = g.integers(0, 2**32, size=(192, 320), dtype=np.uint64).astype(np.uint32)
    m[0, :6] = [0x7FC00001, 0xFFBADBAD, 0x80000000, 0x00000001, 0x7F800000, 0xFF800000]
    a = to_dev(m.view(np.float32))
    t = torch.empty((320, 192), dtype=torch.float32, device=dev())
    desc.desc_transpose_f32(a, t)
    assert np.array_equal(t.cpu().numpy().view(np.uint32), oracle.transpose_u32(m))
    back = torch.empty_like(a)
    desc.desc_transpose_f32(t, back)
    assert np.array_equal(back.cpu().numpy().view(np.uint32), m)


@pytest.mark.parametrize("offset", [1, 2])
def test_transpose_unaligned(offset):
    case(f"transpose unaligned offset={offset}")
    m = workloads.matrix_f32(200, 136, seed=3)
    t = torch.empty(136 * 200 + offset, dtype=torch.float32, device=dev())[offset:].view(136, 200)
    desc.desc_transpose_f32(to_dev(m, offset), t)
    assert np.array_equal(t.cpu().numpy(), oracle.transpose_u32(m))


def test_transpose_batched():
    case("transpose batched 5 x 130 x 70")
    ms = workloads.matrix_f32(5 * 130, 70, seed=4).reshape(5, 130, 70)
    t = torch.empty((5, 70, 130), dtype=torch.float32, device=dev())
    desc.desc_transpose_batched_f32(to_dev(ms), t)
    got = t.cpu().numpy()
    for b in range(5):
        assert np.array_equal(got[b], oracle.transpose_u32(ms[b]))


def test_transpose_workload_8192():
    case("transpose 8192x8192 (seed 3)")
    m = workloads.matrix_f32(8192, 8192, seed=3)
    t = torch.empty((8192, 8192), dtype=torch.float32, device=dev())
    desc.desc_transpose_f32(to_dev(m), t)
    assert np.array_equal(t.cpu().numpy(), oracle.transpose_u32(m))


# ------------------------------------------------------------------ every configuration
def _each_config(op):
    for cfg in range(desc.desc_config_count(op)):
        yield cfg, desc.desc_config_name(op, cfg)


@pytest.fixture
def restore_configs():
    yield
    for op in ("scan_i32", "transpose_32", "copy_32", "reduce_i32"):
        for cls in range(4):
            desc.desc_config_set(op, cls, -1)


@pytest.mark.parametrize("n", [1, 4097, 8191, 8193, 16385, 300_001, (1 << 22) + 5])
def test_scan_every_config(n, restore_configs):
    x = workloads.int_uniform(n, seed=400 + n % 7)
    want = oracle.scan_i32(x)
    xt = to_dev(x)
    cls = desc.desc_size_class("scan_i32", n)
    for cfg, name in _each_config("scan_i32"):
        case(f"scan config {name} n={n}")
        desc.desc_config_set("scan_i32", cls, cfg)
        y = torch.empty(n, dtype=torch.int32, device=dev())
        desc.desc_scan_i32(xt, y)
        assert np.array_equal(y.cpu().numpy(), want), name


@pytest.mark.parametrize("offset", [0, 3])
@pytest.mark.parametrize("n", [1, 4097, 16383, 16384, 16385, 300_001, (1 << 22) + 5,
                               (1 << 24) + 16383])
def test_reduce_every_config(n, offset, restore_configs):
    x = workloads.int_uniform(n, seed=410 + n % 11, lo=-(1 << 31), hi=(1 << 31) - 1)
    want = oracle.reduce_i32(x)
    xt = to_dev(x, offset)
    cls = desc.desc_size_class("reduce_i32", n)
    for cfg, name in _each_config("reduce_i32"):
        case(f"reduce config {name} n={n} offset={offset}")
        desc.desc_config_set("reduce_i32", cls, cfg)
        out = torch.full((1,), -1, dtype=torch.int64, device=dev())
        desc.desc_reduce_i32(xt, out)
        assert int(out.item()) == want, name


@pytest.mark.parametrize("rows,cols", [(37, 1), (64, 64), (200, 136), (130, 260), (1024, 516)])
def test_transpose_every_config(rows, cols, restore_configs):
    m = workloads.self_describing_u32(rows, cols)
    want = oracle.transpose_u32(m)
    mt = to_dev(m.view(np.int32))
    cls = desc.desc_size_class("transpose_32", rows * cols)
    for cfg, name in _each_config("transpose_32"):
        case(f"transpose config {name} {rows}x{cols}")
        desc.desc_config_set("transpose_32", cls, cfg)
        t = torch.empty((cols, rows), dtype=torch.int32, device=dev())
        desc.desc_transpose_f32(mt, t)
        assert np.array_equal(t.cpu().numpy().view(np.uint32), want), name


@pytest.mark.parametrize("n", [1, 5, 1023, 4096 * 4 + 3, 1_000_001])
def test_copy_every_config(n, restore_configs):
    x = workloads.int_uniform(n, seed=5)
    xt = to_dev(x)
    cls = desc.desc_size_class("copy_32", n)
    for cfg, name in _each_config("copy_32"):
        case(f"copy config {name} n={n}")
        desc.desc_config_set("copy_32", cls, cfg)
        y = torch.empty(n, dtype=torch.int32, device=dev())
        desc.desc_copy_32(xt, y)
        assert np.array_equal(y.cpu().numpy(), x), name


# ------------------------------------------------------------------ exclusive scan
@pytest.mark.parametrize("n", [0] + EDGE_SIZES)
def test_scan_exclusive_edge_sizes(n):
    case(f"exclusive scan n={n}")
    x = workloads.int_uniform(n, seed=500 + n % 89)
    y = torch.full((n,), 7, dtype=torch.int32, device=dev())
    desc.desc_scan_exclusive_i32(to_dev(x), y)
    assert np.array_equal(y.cpu().numpy(), oracle.scan_exclusive_i32(x))


@pytest.mark.parametrize("offset", [1, 3])
@pytest.mark.parametrize("n", [5, 65537, 300_001])
def test_scan_exclusive_unaligned(n, offset):
    case(f"exclusive scan unaligned n={n} offset={offset}")
    x = workloads.int_uniform(n, seed=9)
    y = torch.empty(n, dtype=torch.int32, device=dev())
    desc.desc_scan_exclusive_i32(to_dev(x, offset), y)
    assert np.array_equal(y.cpu().numpy(), oracle.scan_exclusive_i32(x))


@pytest.mark.parametrize("n", [8193, (1 << 22) + 5])
def test_scan_exclusive_every_config(n, restore_configs):
    x = workloads.int_uniform(n, seed=600 + n % 7)
    want = oracle.scan_exclusive_i32(x)
    xt = to_dev(x)
    cls = desc.desc_size_class("scan_i32", n)
    for cfg, name in _each_config("scan_i32"):
        case(f"exclusive scan config {name} n={n}")
        desc.desc_config_set("scan_i32", cls, cfg)
        y = torch.empty(n, dtype=torch.int32, device=dev())
        desc.desc_scan_exclusive_i32(xt, y)
        assert np.array_equal(y.cpu().numpy(), want), name


def test_scan_exclusive_workload_2_28_shares_workspace():
    # the benchmark's 2^28 input, alternating with the inclusive scan on one
    # workspace (the generation tags keep the calls apart)
    x = workloads.int_uniform(1 << 28, seed=2)
    xt = to_dev(x)
    ws = torch.zeros(desc.desc_scan_i32_workspace(1 << 28), dtype=torch.uint8, device=dev())
    y = torch.empty(1 << 28, dtype=torch.int32, device=dev())
    case("exclusive scan 2^28")
    desc.desc_scan_exclusive_i32(xt, y, ws=ws)
    assert np.array_equal(y.cpu().numpy(), oracle.scan_exclusive_i32(x))
    case("inclusive scan 2^28 after it")
    desc.desc_scan_i32(xt, y, ws=ws)
    assert np.array_equal(y.cpu().numpy(), oracle.scan_i32(x))


# ------------------------------------------------------------------ 1-, 2-, 8-byte transpose
ELEM_DTYPES = [(1, torch.uint8, np.uint8), (2, torch.int16, np.uint16), (8, torch.float64, np.uint64)]


def _bits(shape, dtype_np, seed):
    g = workloads.rng(seed)
    return g.integers(0, np.iinfo(dtype_np).max, size=shape, dtype=dtype_np, endpoint=True)


@pytest.mark.parametrize("es,tdt,ndt", ELEM_DTYPES)
@pytest.mark.parametrize("rows,cols", [(1, 1), (37, 1), (1, 45), (64, 64), (128, 128), (129, 130),
                                       (200, 136), (256, 512), (1000, 17), (513, 1024)])
def test_transpose_elem_sizes(es, tdt, ndt, rows, cols):
    case(f"transpose {es}-byte {rows}x{cols}")
    m = _bits((rows, cols), ndt, seed=700 + rows % 13 + cols % 7)
    x = torch.from_numpy(m).view(tdt).to(dev())
    y = torch.empty((cols, rows), dtype=tdt, device=dev())
    desc.desc_transpose_batched(x, y)
    got = y.cpu().view(torch.uint8).numpy().view(ndt)
    assert np.array_equal(got, oracle.transpose_bytes(m))


@pytest.mark.parametrize("es,tdt,ndt", ELEM_DTYPES)
def test_transpose_elem_batched_unaligned(es, tdt, ndt):
    # a batch of 3, then a start one element past a 16-byte boundary
    m = _bits((3, 70, 250), ndt, seed=710)
    x = torch.from_numpy(m).view(tdt).to(dev())
    y = torch.empty((3, 250, 70), dtype=tdt, device=dev())
    case(f"transpose {es}-byte batch 3")
    desc.desc_transpose_batched(x, y)
    got = y.cpu().view(torch.uint8).numpy().view(ndt)
    for b in range(3):
        assert np.array_equal(got[b], oracle.transpose_bytes(m[b]))
    buf = torch.empty(64 * 96 + 1, dtype=tdt, device=dev())
    xs = buf[1:].view(64, 96)
    m2 = _bits((64, 96), ndt, seed=711)
    xs.copy_(torch.from_numpy(m2).view(tdt).to(dev()))
    y2 = torch.empty((96, 64), dtype=tdt, device=dev())
    case(f"transpose {es}-byte unaligned start")
    desc.desc_transpose_batched(xs, y2)
    assert np.array_equal(y2.cpu().view(torch.uint8).numpy().view(ndt), oracle.transpose_bytes(m2))


def test_transpose_f64_bit_patterns():
    # the paper's example type: NaN payloads, -0.0, subnormals, infinities
    pats = np.array([0x7FF8000000000001, 0xFFF0DEADBEEF0001, 0x8000000000000000,
                     0x0000000000000001, 0x7FF0000000000000, 0x3FF0000000000000], dtype=np.uint64)
    m = np.tile(pats, (128, 22))[:, :128]                               # 128 x 128, full tiles
    x = torch.from_numpy(m).view(torch.float64).to(dev())
    y = torch.empty((128, 128), dtype=torch.float64, device=dev())
    case("transpose f64 bit patterns")
    desc.desc_transpose_batched(x, y)
    assert np.array_equal(y.cpu().view(torch.uint8).numpy().view(np.uint64), m.T)


# ------------------------------------------------------------------ reversal (reverse view)
@pytest.mark.parametrize("n", [0] + EDGE_SIZES)
def test_reverse_edge_sizes(n):
    case(f"reverse n={n}")
    x = workloads.int_uniform(n, seed=800 + n % 71)
    y = torch.full((n,), -7, dtype=torch.int32, device=dev())
    desc.desc_reverse_u32(to_dev(x), y)
    assert np.array_equal(y.cpu().numpy(), oracle.reverse_u32(x))


@pytest.mark.parametrize("offset", [1, 2, 3])
@pytest.mark.parametrize("n", [7, 65536, 300_004])
def test_reverse_unaligned(n, offset):
    case(f"reverse unaligned n={n} offset={offset}")
    x = workloads.int_uniform(n, seed=810)
    y = torch.empty(n, dtype=torch.int32, device=dev())
    desc.desc_reverse_u32(to_dev(x, offset), y)
    assert np.array_equal(y.cpu().numpy(), oracle.reverse_u32(x))


def test_reverse_2_28_involution():
    case("reverse 2^28 twice")
    x = workloads.int_uniform(1 << 28, seed=2)
    xt = to_dev(x)
    y = torch.empty_like(xt)
    desc.desc_reverse_u32(xt, y)
    assert np.array_equal(y.cpu().numpy(), oracle.reverse_u32(x))
    z = torch.empty_like(xt)
    desc.desc_reverse_u32(y, z)
    assert torch.equal(z, xt)
