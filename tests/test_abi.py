"""The C-ABI boundary on a machine without a GPU: the library loads, exports
every entry point include/desc.h declares (and the binding knows each one),
and the argument checks reject bad calls before anything is launched.

The checks are driven through the pointer-classifier hook: addresses in a
fake "device" range classify as GPU memory, everything else as host memory.
No case here passes every check, so nothing is ever launched."""
import ctypes
import os
import re

import pytest

import paper_2305_03448_amd as desc

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "desc.h")

OK, NULL, SIZE, HOST, ALIAS, WS, UNSUP, HIP, ALIGN = 0, -1, -2, -3, -4, -5, -6, -7, -8


def declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(desc_[a-z0-9_]+)\s*\(", src)))


def test_every_declared_symbol_is_exported_and_bound():
    names = declared()
    assert len(names) >= 10
    L = desc.lib()
    for name in names:
        assert hasattr(L, name), f"{name} not exported"
        assert name in desc.SIGNATURES, f"{name} missing from the binding"


def test_status_strings():
    for s in (OK, NULL, SIZE, HOST, ALIAS, WS, UNSUP, HIP, ALIGN):
        assert desc.desc_status_string(s).startswith("DESC_")
    assert desc.desc_version() >= 100


DEV_LO, DEV_HI = 0x7F0000000000, 0x7F8000000000   # fake GPU address range

_CLASSIFIER = ctypes.CFUNCTYPE(ctypes.c_int, ctypes.c_void_p)


@_CLASSIFIER
def _fake_classifier(p):
    if p is None:
        return -1
    return 0 if DEV_LO <= p < DEV_HI else 1


@pytest.fixture
def fake_pointers():
    L = desc.lib()
    L.desc_set_pointer_classifier(ctypes.cast(_fake_classifier, ctypes.c_void_p))
    yield L
    L.desc_set_pointer_classifier(None)


def D(off):   # a fake device address
    return ctypes.c_void_p(DEV_LO + off)


HOSTP = ctypes.c_void_p(0x1000)


def test_reduce_checks(fake_pointers):
    L = fake_pointers
    wsb = L.desc_reduce_i32_workspace(100)
    st = lambda *a: L.desc_reduce_i32(*a, None)
    assert st(D(0), 100, None, D(1 << 20), wsb) == NULL
    assert st(None, 100, D(4096), D(1 << 20), wsb) == NULL
    assert st(D(0), 100, D(4096), None, wsb) == NULL
    assert st(D(0), -1, D(4096), D(1 << 20), wsb) == SIZE
    assert st(D(0), 1 << 62, D(4096), D(1 << 20), wsb) == SIZE
    assert st(HOSTP, 100, D(4096), D(1 << 20), wsb) == HOST
    assert st(D(0), 100, HOSTP, D(1 << 20), wsb) == HOST
    assert st(D(2), 100, D(4096), D(1 << 20), wsb) == ALIGN
    assert st(D(0), 100, D(4), D(1 << 20), wsb) == ALIGN
    assert st(D(0), 100, D(200), D(1 << 20), wsb) == ALIAS         # out inside in
    assert st(D(0), 100, D(4096), D(64), wsb) == ALIAS             # ws overlaps in
    assert st(D(0), 100, D(4096), D(1 << 20), wsb - 1) == WS


@pytest.mark.parametrize("entry,out_align", [("desc_reduce_minmax_i32", 4),
                                              ("desc_reduce_sum_f32", 8)])
def test_reduce_op_checks(fake_pointers, entry, out_align):
    L = fake_pointers
    wsb = L.desc_reduce_op_workspace(100)
    assert wsb == 64 + 16 and L.desc_reduce_op_workspace(1 << 28) == 64 + 16 * 2048
    assert L.desc_reduce_op_workspace(0) == L.desc_reduce_op_workspace(-5) == 64 + 16
    st = lambda *a: getattr(L, entry)(*a, None)
    assert st(D(0), 100, None, D(1 << 20), wsb) == NULL
    assert st(None, 100, D(4096), D(1 << 20), wsb) == NULL
    assert st(D(0), 100, D(4096), None, wsb) == NULL
    assert st(D(0), -1, D(4096), D(1 << 20), wsb) == SIZE
    assert st(D(0), 1 << 62, D(4096), D(1 << 20), wsb) == SIZE
    assert st(HOSTP, 100, D(4096), D(1 << 20), wsb) == HOST
    assert st(D(0), 100, HOSTP, D(1 << 20), wsb) == HOST
    assert st(D(0), 100, D(4096), HOSTP, wsb) == HOST
    assert st(D(2), 100, D(4096), D(1 << 20), wsb) == ALIGN
    assert st(D(0), 100, D(4096 + out_align // 2), D(1 << 20), wsb) == ALIGN
    assert st(D(0), 100, D(4096), D((1 << 20) + 4), wsb) == ALIGN
    assert st(D(0), 100, D(392), D(1 << 20), wsb) == ALIAS          # out overlaps in's end
    assert st(D(0), 100, D(4096), D(96), wsb) == ALIAS              # ws overlaps in
    assert st(D(0), 100, D(4096), D(4096 - 16), wsb) == ALIAS       # ws overlaps out
    assert st(D(0), 100, D(4096), D(1 << 20), wsb - 1) == WS


def test_scan_f32_checks(fake_pointers):
    L = fake_pointers
    wsb = L.desc_scan_f32_workspace(100)
    assert wsb == 64 + 16 + 16
    assert L.desc_scan_f32_workspace((1 << 28) + 1) == 64 + 16 * 4097 + 16 * 65
    st = lambda *a: L.desc_scan_f32(*a, None)
    assert st(D(0), D(4096), 100, None, wsb) == NULL
    assert st(None, D(4096), 100, D(1 << 20), wsb) == NULL
    assert st(D(0), None, 100, D(1 << 20), wsb) == NULL
    assert st(D(0), D(4096), -1, D(1 << 20), wsb) == SIZE
    assert st(D(0), D(4096), 1 << 62, D(1 << 20), wsb) == SIZE
    assert st(HOSTP, D(4096), 100, D(1 << 20), wsb) == HOST
    assert st(D(0), HOSTP, 100, D(1 << 20), wsb) == HOST
    assert st(D(2), D(4096), 100, D(1 << 20), wsb) == ALIGN
    assert st(D(0), D(4098), 100, D(1 << 20), wsb) == ALIGN
    assert st(D(0), D(4096), 100, D((1 << 20) + 4), wsb) == ALIGN
    assert st(D(0), D(200), 100, D(1 << 20), wsb) == ALIAS
    assert st(D(0), D(4096), 100, D(4096 + 200), wsb) == ALIAS
    assert st(D(0), D(4096), 100, D(1 << 20), wsb - 1) == WS
    assert st(None, None, 0, D(1 << 20), 0) == 0         # n = 0: nothing to check or launch


def test_batched_reduce_scan_checks(fake_pointers):
    L = fake_pointers
    for entry, wsf in (("desc_reduce_batched_i32", L.desc_reduce_batched_i32_workspace),
                       ("desc_scan_batched_i32", L.desc_scan_batched_i32_workspace)):
        wsb = wsf(10, 10)
        assert wsb > 0 and wsf(-1, 5) == 0 and wsf(1 << 40, 1 << 40) == 0
        if entry == "desc_reduce_batched_i32":
            st = lambda i, b, l, o, w, n: L.desc_reduce_batched_i32(i, b, l, o, w, n, None)
        else:
            st = lambda i, b, l, o, w, n: L.desc_scan_batched_i32(i, o, b, l, w, n, None)
        assert st(D(0), 10, 10, None, D(1 << 20), wsb) == NULL
        assert st(None, 10, 10, D(4096), D(1 << 20), wsb) == NULL
        assert st(D(0), 10, 10, D(4096), None, wsb) == NULL
        assert st(D(0), -1, 10, D(4096), D(1 << 20), wsb) == SIZE
        assert st(D(0), 10, -1, D(4096), D(1 << 20), wsb) == SIZE
        assert st(D(0), 1 << 40, 1 << 40, D(4096), D(1 << 20), wsb) == SIZE
        assert st(HOSTP, 10, 10, D(4096), D(1 << 20), wsb) == HOST
        assert st(D(0), 10, 10, HOSTP, D(1 << 20), wsb) == HOST
        assert st(D(2), 10, 10, D(4096), D(1 << 20), wsb) == ALIGN
        assert st(D(0), 10, 10, D(4096), D((1 << 20) + 4), wsb) == ALIGN
        assert st(D(0), 10, 10, D(200), D(1 << 20), wsb) == ALIAS
        assert st(D(0), 10, 10, D(4096), D(0), wsb) == ALIAS
        assert st(D(0), 10, 10, D(4096), D(1 << 20), wsb - 1) == WS
        assert st(None, 0, 10, None, None, 0) == 0              # batch = 0: nothing to do
    assert L.desc_reduce_batched_i32(D(0), 10, 10, D(4100), D(1 << 20), 1 << 16, None) == ALIGN


def test_strided_batched_gemm_checks(fake_pointers):
    L = fake_pointers
    F32, BF = 0, 1
    wsb = L.desc_gemm_strided_batched_workspace(F32, 4, 8, 8, 8, 8, 8)
    assert wsb > 0 and L.desc_gemm_strided_batched_workspace(2, 4, 8, 8, 8, 8, 8) == 0
    assert L.desc_gemm_strided_batched_workspace(BF, 4, 8, 8, 8, 8, 8) > 0
    A, B, C, W = D(0), D(1 << 16), D(1 << 17), D(1 << 20)
    st = lambda mode=F32, G=4, M=8, N=8, K=8, a=A, lda=8, sa=64, b=B, ldb=8, sb=64, c=C, ldc=8, \
        sc=64, w=W, n=wsb: L.desc_gemm_strided_batched(mode, G, M, N, K, a, lda, sa, b, ldb, sb,
                                                       c, ldc, sc, w, n, None)
    assert st(mode=2) == -6                                      # FP8 is not offered here
    assert st(G=-1) == SIZE and st(sa=-1) == SIZE
    assert st(G=0, a=None) == 0 and st(M=0, a=None) == 0         # nothing to do
    assert st(c=None) == NULL and st(a=None) == NULL and st(w=None) == NULL
    assert st(K=0, a=None, b=None, n=0) == WS                    # K = 0 needs no operands
    assert st(lda=7) == SIZE and st(ldc=7) == SIZE
    assert st(a=HOSTP) == HOST and st(w=HOSTP) == HOST
    assert st(a=D(2)) == ALIGN and st(w=D((1 << 20) + 64)) == ALIGN
    assert st(c=D(100)) == ALIAS                                 # C overlaps A's batches
    assert st(sc=63) == ALIAS                                    # two batches of C overlap
    assert st(w=D((1 << 17) + 256)) == ALIAS                     # workspace overlaps C
    assert st(n=wsb - 1) == WS


@pytest.mark.parametrize("entry", ["desc_scan_i32", "desc_scan_exclusive_i32"])
def test_scan_checks(fake_pointers, entry):
    L = fake_pointers
    n = 10_000
    wsb = L.desc_scan_i32_workspace(n)
    assert wsb >= 64 + 8
    fn = getattr(L, entry)
    st = lambda *a: fn(*a, None)
    assert st(D(0), D(1 << 20), 0, D(1 << 24), wsb) == OK           # empty: nothing to do
    assert st(None, D(1 << 20), n, D(1 << 24), wsb) == NULL
    assert st(D(0), D(1 << 20), -5, D(1 << 24), wsb) == SIZE
    assert st(D(0), HOSTP, n, D(1 << 24), wsb) == HOST
    assert st(D(0), D(1 << 20), n, HOSTP, wsb) == HOST
    assert st(D(1), D(1 << 20), n, D(1 << 24), wsb) == ALIGN
    assert st(D(0), D(4 * n - 4), n, D(1 << 24), wsb) == ALIAS      # last word overlaps
    assert st(D(0), D(4 * n), n, D(4 * n - 8), wsb) == ALIAS        # ws overlaps in
    assert st(D(0), D(1 << 20), n, D(1 << 24), wsb - 8) == WS
    # larger n needs a larger workspace
    assert L.desc_scan_i32_workspace(1 << 28) > L.desc_scan_i32_workspace(1 << 20)


def test_reduce_blocks_checks(fake_pointers):
    L = fake_pointers
    st = lambda *a: L.desc_reduce_blocks_i32(*a, None)
    n = 10_000                                                       # 3 chunks of 4096
    assert st(D(0), 0, 4096, D(1 << 20)) == OK                       # empty: nothing to do
    assert st(None, n, 4096, D(1 << 20)) == NULL
    assert st(D(0), n, 4096, None) == NULL
    assert st(D(0), -1, 4096, D(1 << 20)) == SIZE
    assert st(D(0), n, 1000, D(1 << 20)) == SIZE                     # not a multiple of 1024
    assert st(D(0), n, 0, D(1 << 20)) == SIZE
    assert st(HOSTP, n, 4096, D(1 << 20)) == HOST
    assert st(D(0), n, 4096, HOSTP) == HOST
    assert st(D(2), n, 4096, D(1 << 20)) == ALIGN
    assert st(D(0), n, 4096, D((1 << 20) + 4)) == ALIGN
    assert st(D(0), n, 4096, D(4 * n - 16)) == ALIAS                 # 3 outputs reach into in


def test_scan_two_pass_checks(fake_pointers):
    L = fake_pointers
    n = 100_000                                                      # 2 tiles of 65536
    wsb = L.desc_scan_two_pass_i32_workspace(n)
    assert wsb == 8
    st = lambda *a: L.desc_scan_two_pass_i32(*a, None)
    assert st(D(0), D(1 << 20), 0, D(1 << 24), wsb) == OK
    assert st(D(0), D(1 << 20), n, None, wsb) == NULL
    assert st(D(0), D(1 << 20), -1, D(1 << 24), wsb) == SIZE
    assert st(D(0), D(1 << 20), n, HOSTP, wsb) == HOST
    assert st(D(0), D(1 << 20), n, D((1 << 24) + 2), wsb) == ALIGN
    assert st(D(0), D(4 * n - 4), n, D(1 << 24), wsb) == ALIAS
    assert st(D(0), D(1 << 20), n, D(4 * n - 4), wsb) == ALIAS       # ws overlaps in
    assert st(D(0), D(1 << 20), n, D(1 << 24), wsb - 1) == WS


def test_transpose_checks(fake_pointers):
    L = fake_pointers
    st = L.desc_transpose_batched_f32
    assert st(D(0), D(1 << 24), 1, 0, 5, None) == OK
    assert st(D(0), D(1 << 24), 0, 5, 5, None) == OK
    assert st(None, D(1 << 24), 1, 5, 5, None) == NULL
    assert st(D(0), D(1 << 24), 1, -1, 5, None) == SIZE
    assert st(D(0), D(1 << 24), 1, 1 << 40, 1 << 40, None) == SIZE
    assert st(D(0), HOSTP, 1, 5, 5, None) == HOST
    assert st(D(2), D(1 << 24), 1, 5, 5, None) == ALIGN
    assert st(D(0), D(96), 1, 5, 5, None) == ALIAS                  # 25 words from 0
    assert st(D(0), D(1 << 24), 70000, 5, 5, None) == UNSUP         # batch beyond grid z
    assert L.desc_transpose_f32(D(0), HOSTP, 3, 3, None) == HOST


def test_reverse_checks(fake_pointers):
    L = fake_pointers
    st = lambda *a: L.desc_reverse_u32(*a, None)
    assert st(D(0), D(1 << 20), 0) == OK                               # nothing to move
    assert st(None, D(1 << 20), 5) == NULL
    assert st(D(0), None, 5) == NULL
    assert st(D(0), D(1 << 20), -1) == SIZE
    assert st(D(0), D(1 << 20), 1 << 62) == SIZE
    assert st(HOSTP, D(1 << 20), 5) == HOST
    assert st(D(2), D(1 << 20), 5) == ALIGN
    assert st(D(0), D(16), 5) == ALIAS                                 # out starts inside in


def test_transpose_any_element_size_checks(fake_pointers):
    L = fake_pointers
    st = lambda *a: L.desc_transpose_batched(*a, None)
    for es in (3, 0, 16, -8):
        assert st(D(0), D(1 << 24), es, 1, 5, 5) == UNSUP
    for es in (1, 2, 8):
        assert st(D(0), D(1 << 24), es, 1, 0, 5) == OK                 # nothing to move
        assert st(None, D(1 << 24), es, 1, 5, 5) == NULL
        assert st(D(0), D(1 << 24), es, 1, -1, 5) == SIZE
        assert st(D(0), D(1 << 24), es, 1, 1 << 40, 1 << 40) == SIZE
        assert st(D(0), HOSTP, es, 1, 5, 5) == HOST
        assert st(D(0), D(1 << 24), es, 70000, 5, 5) == UNSUP          # batch beyond grid z
        # 25 elements from 0 end at byte 25 es; out starting inside overlaps
        assert st(D(0), D(24 * es), es, 1, 5, 5) == ALIAS
    assert st(D(1), D(1 << 24), 2, 1, 5, 5) == ALIGN
    assert st(D(4), D(1 << 24), 8, 1, 5, 5) == ALIGN
    assert st(D(0), D(1 << 24), 8, 1, 64 * 65535 + 1, 5) == UNSUP      # rows beyond the grid
    assert st(D(0), D(2), 4, 1, 5, 5) == ALIGN                          # the 32-bit path


def _problems_host(shapes):
    """A host desc_gemm_problem array (nine int64 words each) with the given
    M, N, K and placeholder strides and pointers."""
    words = []
    for M, N, K in shapes:
        words += [M, N, K, max(K, 1), max(N, 1), max(N, 1), 0, 0, 0]
    return (ctypes.c_int64 * max(len(words), 1))(*words)


def _problems_host_ld(rows):
    """Like _problems_host, with explicit (M, N, K, lda, ldb) per problem."""
    words = []
    for M, N, K, lda, ldb in rows:
        words += [M, N, K, lda, ldb, max(N, 1), 0, 0, 0]
    return (ctypes.c_int64 * max(len(words), 1))(*words)


def test_grouped_workspace_for():
    L = desc.lib()
    F32, BF16X3, FP8 = 0, 1, 2
    # bf16x3: a head of 256 bytes + four 256-aligned arrays of G + 1 int64 +
    # one 256-aligned array of G int32 (the fused order),
    # then, for each problem staged through planes, four bf16 planes
    # (Ma + Na) x Kp with M, N rounded up to multiples of 128 (either tile
    # size fits) and K to a multiple of 64 (at least 64); empty problems
    # take nothing
    shapes = [(100, 90, 80), (0, 5, 5), (5, 7, 0), (64, 64, 64), (1, 1, 1000)]
    head = 256 + 4 * 256 + 256
    planes = [4 * (128 + 128) * 128, 0, 4 * (128 + 128) * 64, 4 * (128 + 128) * 64,
              4 * (128 + 128) * 1024]
    op = desc.OPS["gemm_grouped_bf16x3"]
    try:
        for cfg, name in enumerate(["tile64", "tile128"]):
            assert desc.desc_config_name(op, cfg) == name
            L.desc_config_set(op, 0, cfg)                 # G < 2^24: size class 0
            assert L.desc_gemm_grouped_workspace_for(BF16X3, 5, _problems_host(shapes)) == \
                head + sum(planes)
        for cfg in (2, 3):                                # fused: planes only past 2^24 strides
            L.desc_config_set(op, 0, cfg)
            assert L.desc_gemm_grouped_workspace_for(BF16X3, 5, _problems_host(shapes)) == head
            rows = [(100, 90, 80, 80, 1 << 24), (100, 90, 80, 80, (1 << 24) + 1),
                    (100, 90, 80, (1 << 24) + 1, 90)]
            assert L.desc_gemm_grouped_workspace_for(BF16X3, 3, _problems_host_ld(rows)) == \
                head + 2 * planes[0]
    finally:
        L.desc_config_set(op, 0, -1)
    assert L.desc_gemm_grouped_workspace_for(BF16X3, 0, None) == 256 + 4 * 256
    big_G = 100                      # (101 * 8) rounded to 256 = 1024; 400 rounded = 512
    assert L.desc_gemm_grouped_workspace_for(BF16X3, big_G, _problems_host(
        [(0, 0, 0)] * big_G)) == 256 + 4 * 1024 + 512
    assert L.desc_gemm_grouped_workspace_for(F32, 7, None) == L.desc_gemm_grouped_workspace(7)
    assert L.desc_gemm_grouped_workspace_for(FP8, 1, _problems_host(shapes[:1])) == 0
    assert L.desc_gemm_grouped_workspace_for(BF16X3, -1, None) == 0
    assert L.desc_gemm_grouped_workspace_for(BF16X3, 2, None) == 0
    assert L.desc_gemm_grouped_workspace_for(BF16X3, 1, _problems_host([(64, 64, 1 << 41)])) == 0
    assert L.desc_gemm_grouped_workspace_for(BF16X3, 1, _problems_host([(1 << 40, 64, 64)])) == 0


def test_grouped_checks(fake_pointers):
    L = fake_pointers
    F32, BF16X3, FP8 = 0, 1, 2
    G = 3                                         # 3 x 72 descriptor bytes at D(0)
    wsb = L.desc_gemm_grouped_workspace(G)
    head3 = 256 + 4 * 256                         # (G + 1) * 8 = 32 bytes per array
    st = lambda *a: L.desc_gemm_grouped(*a, None)
    assert st(F32, 0, None, None, 0) == OK        # nothing to do
    assert st(F32, -1, D(0), D(1 << 20), wsb) == SIZE
    assert st(FP8, G, D(0), D(1 << 20), wsb) == UNSUP
    assert st(F32, G, None, D(1 << 20), wsb) == NULL
    assert st(F32, G, D(0), None, wsb) == NULL
    assert st(F32, G, HOSTP, D(1 << 20), wsb) == HOST
    assert st(F32, G, D(0), HOSTP, wsb) == HOST
    assert st(F32, G, D(4), D(1 << 20), wsb) == ALIGN
    assert st(F32, G, D(0), D((1 << 20) + 32), wsb) == ALIGN
    assert st(BF16X3, G, D(0), D((1 << 20) + 64), 1 << 20) == ALIGN    # 256 needed
    assert st(F32, G, D(0), D(192), wsb) == ALIAS  # ws starts inside the descriptors
    assert st(F32, G, D(0), D(1 << 20), wsb - 1) == WS
    assert st(BF16X3, G, D(0), D(1 << 20), head3 - 1) == WS


def test_tuning_table_names_known_configurations():
    # every line of the shipped table names a registered operation and one of
    # its configurations, and loading it selects exactly that configuration
    L = desc.lib()
    assert L.desc_config_load(desc.TUNE_FILE.encode()) == 0
    seen = 0
    with open(desc.TUNE_FILE) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            op, cls, name = line.split()
            assert op in desc.OPS, op
            names = [desc.desc_config_name(op, c) for c in range(desc.desc_config_count(op))]
            assert name in names, (op, name, names)
            assert desc.desc_config_get(op, int(cls)) == names.index(name), line
            seen += 1
    assert seen == 4 * len(desc.OPS)          # four size classes for every operation


def test_workspace_status_checks(fake_pointers):
    L = fake_pointers
    st = D(1 << 20)
    assert L.desc_workspace_status(None, 64, st, None) == NULL
    assert L.desc_workspace_status(D(0), 64, None, None) == NULL
    assert L.desc_workspace_status(HOSTP, 64, st, None) == HOST
    assert L.desc_workspace_status(D(0), 64, HOSTP, None) == HOST
    assert L.desc_workspace_status(D(4), 64, st, None) == ALIGN       # ws 8-byte aligned
    assert L.desc_workspace_status(D(0), 64, D(2), None) == ALIGN     # status 4-byte aligned
    assert L.desc_workspace_status(D(0), 64, D(4), None) == ALIAS     # status inside ws
    assert L.desc_workspace_status(D(0), 63, st, None) == WS          # no room for the header
    assert L.desc_workspace_set_wait_limit(None, 64, 0, None) == NULL
    assert L.desc_workspace_set_wait_limit(D(0), 64, (1 << 32) - 1, None) == SIZE
    assert L.desc_workspace_set_wait_limit(HOSTP, 64, 0, None) == HOST
    assert L.desc_workspace_set_wait_limit(D(4), 64, 0, None) == ALIGN
    assert L.desc_workspace_set_wait_limit(D(0), 32, 0, None) == WS


def test_batched_workspaces_put_the_segmented_header_first():
    # the segmented workspace (header with the status word at byte 4) is the
    # front part of a batched one; the offsets follow, 256-byte aligned
    L = desc.lib()
    for B, n in ((1, 5), (300, 4099), (4096, 1 << 16)):
        seg_r = L.desc_reduce_segmented_i32_workspace(B * n, B)
        seg_s = L.desc_scan_segmented_i32_workspace(B * n, B)
        offs = (8 * (B + 1) + 255) // 256 * 256
        assert L.desc_reduce_batched_i32_workspace(B, n) == (seg_r + 255) // 256 * 256 + offs
        assert L.desc_scan_batched_i32_workspace(B, n) == (seg_s + 255) // 256 * 256 + offs
    F32, BF = 0, 1
    for mode in (F32, BF):
        for G in (1, 7, 512):
            descs = (72 * G + 255) // 256 * 256
            total = L.desc_gemm_strided_batched_workspace(mode, G, 100, 60, 30, 30, 60)
            assert total > descs and (total - descs) % 256 == 0
            if mode == F32:
                assert total - descs >= L.desc_gemm_grouped_workspace(G)


def test_scan_noalloc_checks(fake_pointers):
    L = fake_pointers
    LIMIT = -9
    big = (1 << 31) + 1
    assert L.desc_scan_i32_noalloc(None, D(0), 5, None) == NULL
    assert L.desc_scan_i32_noalloc(D(0), D(1 << 20), -1, None) == SIZE
    assert L.desc_scan_i32_noalloc(HOSTP, D(1 << 20), 5, None) == HOST
    assert L.desc_scan_i32_noalloc(D(2), D(1 << 20), 5, None) == ALIGN
    assert L.desc_scan_i32_noalloc(D(0), D(8), 5, None) == ALIAS
    # above the fixed scratch: refused after the pointer checks, before any launch
    assert L.desc_scan_i32_noalloc(D(0), D(1 << 36), big, None) == LIMIT
    assert L.desc_scan_i32_noalloc(D(0), D(1 << 20), 0, None) == OK     # n = 0: nothing to do
    assert "allocation-free" in desc.desc_status_string(LIMIT)
