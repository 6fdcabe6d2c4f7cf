"""State kept in workspaces between calls, and the device status word.

* No word of an earlier call survives to match a later call's tag: the
  reductions clear every block slot they read, and the look-back scans clear
  what a larger earlier call left past their own tiles.  The tests read the
  workspace back after each call and check that every word after the header
  is zero or carries the last call's tag, then run the sequence that a
  repeating tag would break (a large call, many small ones, a large one).
* Failures seen only on the GPU reach the caller through
  desc_workspace_status: a debug wait limit of zero polls makes every bounded
  wait give up at once (no kernel waits, so each ends normally), which must
  be reported and cleared by the read; the grouped BF16X3 refusal is reported
  the same way.
* The binding's default workspaces are per stream, and a replaced one stays
  alive for the graphs captured with it.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2305_03448_amd as desc
import workloads
from gpu_util import case, dev, needs_gpu, to_dev

pytestmark = [pytest.mark.gpu, needs_gpu]

HDR = 64   # bytes of the workspace header


def words_after_header(ws: torch.Tensor) -> np.ndarray:
    return ws.cpu().numpy()[HDR:].view(np.uint64)


def header(ws: torch.Tensor):
    h = ws.cpu().numpy()[:HDR]
    gen = int(h[0:4].view(np.uint32)[0])
    err = int(h[4:8].view(np.uint32)[0])
    hw = int(h[8:16].view(np.uint64)[0])
    return gen, err, hw


def test_reduce_clears_every_slot_it_reads():
    x = workloads.int_uniform(1 << 24, seed=41)
    xt = to_dev(x)
    want = oracle.reduce_i32(x)
    ws = torch.zeros(desc.desc_reduce_i32_workspace(1 << 28), dtype=torch.uint8, device=dev())
    out = torch.empty(1, dtype=torch.int64, device=dev())
    for n in (1 << 24, 1 << 22, 12345, (1 << 24) - 3):
        case(f"reduce slots cleared n={n}")
        desc.desc_reduce_i32(xt[:n], out, ws=ws)
        assert int(out.item()) == (want if n == 1 << 24 else oracle.reduce_i32(x[:n]))
        assert not words_after_header(ws).any(), "a block slot kept its tag"
    assert header(ws)[1] == 0


def test_reduce_large_small_large_on_one_workspace():
    # a 2^28 call fills 2047 slots, 8190 calls at 2^22 use a quarter of them,
    # then a 2^28 call of other data: with 13-bit tags that is the call whose
    # tag repeats the first one's
    big1 = workloads.int_uniform(1 << 28, seed=42)
    big2 = workloads.int_uniform(1 << 28, seed=43)
    small = workloads.int_uniform(1 << 22, seed=44)
    w1, w2, ws_ = oracle.reduce_i32(big1), oracle.reduce_i32(big2), oracle.reduce_i32(small)
    ws = torch.zeros(desc.desc_reduce_i32_workspace(1 << 28), dtype=torch.uint8, device=dev())
    out = torch.empty(8192, dtype=torch.int64, device=dev())
    case("reduce 2^28 (seed 42)")
    t = to_dev(big1)
    desc.desc_reduce_i32(t, out[0:1], ws=ws)
    del t
    case("reduce 8190 x 2^22 on the same workspace")
    st = to_dev(small)
    for i in range(8190):
        desc.desc_reduce_i32(st, out[1 + i:2 + i], ws=ws)
    case("reduce 2^28 (seed 43)")
    t = to_dev(big2)
    desc.desc_reduce_i32(t, out[8191:8192], ws=ws)
    r = out.cpu().numpy()
    assert r[0] == w1 and r[8191] == w2
    assert (r[1:8191] == ws_).all()
    assert not words_after_header(ws).any()
    gen, err, _ = header(ws)
    assert gen == 8192 and err == 0


def test_reduce_op_clears_every_slot_it_reads():
    x = workloads.int_uniform((1 << 23) + 5, seed=45)
    f = workloads.normal_f32((1 << 23) + 5, seed=46)
    xt, ft = to_dev(x), to_dev(f)
    ws = torch.zeros(desc.desc_reduce_op_workspace(1 << 24), dtype=torch.uint8, device=dev())
    mm = torch.empty(2, dtype=torch.int32, device=dev())
    s = torch.empty(1, dtype=torch.float64, device=dev())
    for n in (x.size, 4097, 1 << 20, 1):
        case(f"reduce_op slots cleared n={n}")
        desc.desc_reduce_minmax_i32(xt[:n], mm, ws=ws)
        assert not words_after_header(ws).any()
        assert tuple(mm.cpu().numpy()) == tuple(oracle.minmax_i32(x[:n]))
        desc.desc_reduce_sum_f32(ft[:n], s, ws=ws)
        assert not words_after_header(ws).any()


@pytest.mark.parametrize("exclusive", [False, True])
def test_scan_leaves_only_its_own_tiles_tagged(exclusive):
    ws = torch.zeros(desc.desc_scan_i32_workspace(1 << 26), dtype=torch.uint8, device=dev())
    fn = desc.desc_scan_exclusive_i32 if exclusive else desc.desc_scan_i32
    for rep, n in enumerate([1 << 26, 70000, 1 << 22, 1, (1 << 24) + 3]):
        case(f"scan tags exclusive={exclusive} n={n}")
        x = workloads.int_uniform(n, seed=500 + rep)
        y = torch.empty(n, dtype=torch.int32, device=dev())
        fn(to_dev(x), y, ws=ws)
        want = oracle.scan_i32(x)
        if exclusive:
            want = np.concatenate([[0], want[:-1]]).astype(np.int32)
        assert np.array_equal(y.cpu().numpy(), want)
        gen, err, hw = header(ws)
        w = words_after_header(ws)
        assert err == 0 and gen == rep + 1
        assert hw > 0 and not w[hw:].any(), "a word past the call's tiles kept a tag"
        tags = (w[:hw] >> np.uint64(32)) & np.uint64(0x3FFFFFFF)
        flags = w[:hw] >> np.uint64(62)
        assert (flags == 2).all() and (tags == rep).all()


def test_scan_large_small_large_on_one_workspace():
    big = workloads.int_uniform(1 << 28, seed=47)
    small = workloads.int_uniform(1 << 16, seed=48)
    ws = torch.zeros(desc.desc_scan_i32_workspace(1 << 28), dtype=torch.uint8, device=dev())
    bt, st = to_dev(big), to_dev(small)
    y = torch.empty(1 << 28, dtype=torch.int32, device=dev())
    ys = torch.empty(1 << 16, dtype=torch.int32, device=dev())
    case("scan 2^28, then 200 x 2^16, then 2^28 on one workspace")
    desc.desc_scan_i32(bt, y, ws=ws)
    for _ in range(200):
        desc.desc_scan_i32(st, ys, ws=ws)
    assert np.array_equal(ys.cpu().numpy(), oracle.scan_i32(small))
    _, _, hw = header(ws)
    assert not words_after_header(ws)[hw:].any()
    y.fill_(0)
    desc.desc_scan_i32(bt, y, ws=ws)
    assert np.array_equal(y.cpu().numpy(), oracle.scan_i32(big))


def test_scan_f32_leaves_only_its_own_region_tagged():
    ws = torch.zeros(desc.desc_scan_f32_workspace(1 << 25), dtype=torch.uint8, device=dev())
    for rep, n in enumerate([1 << 25, 65536 * 70 + 3, 1000, 65536 * 64]):
        case(f"scan_f32 tags n={n}")
        x = workloads.normal_f32(n, seed=600 + rep)
        y = torch.empty(n, dtype=torch.float32, device=dev())
        desc.desc_scan_f32(to_dev(x), y, ws=ws)
        T = -(-n // 65536)
        used = 2 * T + 2 * (-(-T // 64))
        gen, err, hw = header(ws)
        w = words_after_header(ws)
        assert err == 0 and hw == used
        assert not w[used:].any()
        assert ((w[:used] >> np.uint64(32)) == rep + 1).all(), "a word of the region unwritten"


def _zero_wait_gives_error(ws, run, what):
    case(f"{what}: wait limit 0")
    desc.desc_workspace_set_wait_limit(ws, 0)
    run()
    st = desc.workspace_status(ws)
    assert st == 1, f"{what}: status {st}"
    assert desc.workspace_status(ws) == 0, "the read resets the word"
    desc.desc_workspace_set_wait_limit(ws, -1)


def test_wait_limit_zero_is_reported_and_cleared():
    n = 1 << 22
    x = workloads.int_uniform(n, seed=49)
    xt = to_dev(x)
    out = torch.empty(1, dtype=torch.int64, device=dev())
    y = torch.empty(n, dtype=torch.int32, device=dev())

    wr = torch.zeros(desc.desc_reduce_i32_workspace(n), dtype=torch.uint8, device=dev())
    _zero_wait_gives_error(wr, lambda: desc.desc_reduce_i32(xt, out, ws=wr), "reduce")
    desc.desc_reduce_i32(xt, out, ws=wr)
    assert int(out.item()) == oracle.reduce_i32(x) and desc.workspace_status(wr) == 0

    wo = torch.zeros(desc.desc_reduce_op_workspace(n), dtype=torch.uint8, device=dev())
    mm = torch.empty(2, dtype=torch.int32, device=dev())
    _zero_wait_gives_error(wo, lambda: desc.desc_reduce_minmax_i32(xt, mm, ws=wo), "min/max")
    desc.desc_reduce_minmax_i32(xt, mm, ws=wo)
    assert tuple(mm.cpu().numpy()) == tuple(oracle.minmax_i32(x)) and desc.workspace_status(wo) == 0

    wsc = torch.zeros(desc.desc_scan_i32_workspace(n), dtype=torch.uint8, device=dev())
    _zero_wait_gives_error(wsc, lambda: desc.desc_scan_i32(xt, y, ws=wsc), "scan")
    desc.desc_scan_i32(xt, y, ws=wsc)
    assert np.array_equal(y.cpu().numpy(), oracle.scan_i32(x)) and desc.workspace_status(wsc) == 0

    f = workloads.normal_f32(n, seed=50)
    ft, fy = to_dev(f), torch.empty(n, dtype=torch.float32, device=dev())
    wf = torch.zeros(desc.desc_scan_f32_workspace(n), dtype=torch.uint8, device=dev())
    _zero_wait_gives_error(wf, lambda: desc.desc_scan_f32(ft, fy, ws=wf), "float scan")
    desc.desc_scan_f32(ft, fy, ws=wf)
    assert desc.workspace_status(wf) == 0

    off = np.array([0, 5, n // 2, n], dtype=np.int64)
    ot = to_dev(off)
    wg = torch.zeros(desc.desc_scan_segmented_i32_workspace(n, 3), dtype=torch.uint8, device=dev())
    _zero_wait_gives_error(wg, lambda: desc.desc_scan_segmented_i32(xt, ot, y, ws=wg), "segmented")
    desc.desc_scan_segmented_i32(xt, ot, y, ws=wg)
    assert np.array_equal(y.cpu().numpy(), oracle.scan_segmented_i32(x, off))
    assert desc.workspace_status(wg) == 0

    wb = torch.zeros(desc.desc_scan_batched_i32_workspace(4, n // 4), dtype=torch.uint8,
                     device=dev())
    x2, y2 = xt.view(4, n // 4), y.view(4, n // 4)
    _zero_wait_gives_error(wb, lambda: desc.desc_scan_batched_i32(x2, y2, ws=wb), "batched")
    desc.desc_scan_batched_i32(x2, y2, ws=wb)
    want = np.concatenate([oracle.scan_i32(x[i * (n // 4):(i + 1) * (n // 4)]) for i in range(4)])
    assert np.array_equal(y.cpu().numpy(), want) and desc.workspace_status(wb) == 0


def test_status_read_is_stream_ordered_and_capturable():
    n = 1 << 20
    x = workloads.int_uniform(n, seed=51)
    xt = to_dev(x)
    y = torch.empty(n, dtype=torch.int32, device=dev())
    ws = torch.zeros(desc.desc_scan_i32_workspace(n), dtype=torch.uint8, device=dev())
    st = torch.full((1,), -7, dtype=torch.int32, device=dev())
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        desc.desc_scan_i32(xt, y, ws=ws)
        desc.desc_workspace_status(ws, st)
    s.synchronize()
    assert int(st.item()) == 0
    case("scan + status read captured and replayed")
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        desc.desc_scan_i32(xt, y, ws=ws)
        desc.desc_workspace_status(ws, st)
    for rep in range(3):
        y.fill_(0)
        st.fill_(-7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert int(st.item()) == 0
        assert np.array_equal(y.cpu().numpy(), oracle.scan_i32(x))
        desc.desc_scan_i32(xt, y, ws=ws)       # eager work between replays
        torch.cuda.synchronize()


def test_default_workspaces_are_per_stream_and_outlive_replacement():
    desc.lib()
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    a = desc.workspace("probe", 1024, dev(), s1)
    b = desc.workspace("probe", 1024, dev(), s2)
    assert a.data_ptr() != b.data_ptr()
    assert desc.workspace("probe", 512, dev(), s1).data_ptr() == a.data_ptr()

    n_small, n_big = 1 << 16, 1 << 24
    xs = workloads.int_uniform(n_small, seed=52)
    xb = workloads.int_uniform(n_big, seed=53)
    xst, xbt = to_dev(xs), to_dev(xb)
    ys = torch.empty(n_small, dtype=torch.int32, device=dev())
    yb = torch.empty(n_big, dtype=torch.int32, device=dev())
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        desc.desc_scan_i32(xst, ys)               # creates the stream's cached workspace
    s.synchronize()
    case("capture with the default workspace, then a larger eager call, then replay")
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        desc.desc_scan_i32(xst, ys)
    with torch.cuda.stream(s):
        desc.desc_scan_i32(xbt, yb)               # replaces the cached workspace
    s.synchronize()
    assert np.array_equal(yb.cpu().numpy(), oracle.scan_i32(xb))
    junk = [torch.full((1 << 20,), -1, dtype=torch.int32, device=dev()) for _ in range(8)]
    for rep in range(3):
        ys.fill_(0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert np.array_equal(ys.cpu().numpy(), oracle.scan_i32(xs)), f"replay {rep}"
    del junk
