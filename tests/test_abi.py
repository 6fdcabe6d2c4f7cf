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


def test_scan_checks(fake_pointers):
    L = fake_pointers
    n = 10_000
    wsb = L.desc_scan_i32_workspace(n)
    assert wsb >= 64 + 8
    st = lambda *a: L.desc_scan_i32(*a, None)
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
