"""The view / execution-resource layer on the host (no GPU): the index maps
of the paper's worked examples and of every kernel are enumerated by a C++
program compiled with g++ against the same headers the kernels include, and
the rule that a split resource cannot synchronise is checked at compile
time (a kernel that calls sync inside split must not compile)."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2305_03448_amd", "csrc")
SRC = os.path.join(ROOT, "tests", "view_checks.cpp")

EXPECTED = [
    "listing1_racy_index_collides", "listing1_corrected_index_is_bijection",
    "group_by_row_32_4_is_listing1_corrected", "group8_transpose_thread_t_gets_t_t8_t16_t24",
    "listing2_with_tmp_transpose_is_transposition", "listing2_as_printed_moves_tiles_only",
    "narrowing_group32_block_thread_is_bijection", "narrowing_without_block_selection_conflicts",
    "reverse_per_block_read_write_conflict", "split_Y_at_1_gives_two_single_block_groups",
    "scan_wave_striped_groups_bijection_and_coalesced", "scan_wave_striped_elements_bijection",
    "reduce_block_striped_bijection", "transpose_kernel_maps_T32", "transpose_kernel_maps_T64",
    "transpose_kernel_maps_T128", "gemm_lds_xor_swizzle_bkb32", "gemm_lds_xor_swizzle_bkb64",
    "gemm_lds_xor_swizzle_bkb128", "transpose_f64_lds_swizzle", "transpose_u16_lds_swizzle",
    # access checking (tests/access_check.hpp): clean kernels, and the
    # conflicts the paper's type system rejects
    "access_check_listing1_racy_conflicts_corrected_clean", "access_check_rev_per_block_needs_barrier",
    "access_check_transpose_kernel_clean", "access_check_transpose_without_barrier_races",
    "access_check_reduce_tree_clean", "access_check_reduce_tree_without_barriers_races",
    "access_check_scan_stores_clean",
    # layouts of the min/max and float-sum kernel and the transposes' tile order
    "reduce_ops_chunk_groups_bijection", "transpose_diagonal_tile_order_bijection",
    # the fused split staging's buffer windows (gemm_nt.hpp SplitSource)
    "split_staging_buffer_windows",
    # the FP32 GEMM's LDS double buffer under its two-stages-ahead schedule
    "access_check_gemm_double_buffer_clean",
    "access_check_gemm_double_buffer_without_a_barrier_races",
    "access_check_gemm16_double_buffer_clean",
    "access_check_gemm16_double_buffer_without_a_barrier_races",
    "segmented_units_cover_every_segment_once",
    "segmented_lookback_windows_stay_in_segment",
    "access_check_segmented_scan_clean",
    "access_check_segmented_reduce_clean",
    "access_check_segmented_reduce_plain_stores_race",
    "access_check_segmented_persistent_reduce_clean",
    "grouped_tile_walk_takes_every_tile_once",
    "access_check_grouped_walk_clean",
    "access_check_grouped_walk_without_the_end_barrier_races",
    "float_scan_handover_waits_on_earlier_tiles_only",
    "access_check_float_scan_handover_clean",
    "float_scan_handover_leaves_no_older_word",
]


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("views") / "view_checks")
    subprocess.run(["g++", "-std=c++17", "-O1", "-I", CSRC, "-I", os.path.dirname(SRC), SRC, "-o",
                    exe], check=True)
    return exe


def test_view_maps(checker):
    r = subprocess.run([checker], capture_output=True, text=True, timeout=120)
    lines = {}
    for line in r.stdout.splitlines():
        status, rest = line.split(" ", 1)
        lines[rest.split(":")[0]] = status
    for name in EXPECTED:
        assert lines.get(name) == "OK", f"{name}: {lines.get(name)}\n{r.stdout}"
    assert r.returncode == 0, r.stdout


def test_select_extent_mismatch_is_rejected(checker):
    r = subprocess.run([checker, "select_mismatch"], capture_output=True, text=True, timeout=60)
    assert r.returncode != 0


SYNC_IN_SPLIT = r'''
#include "view.hpp"
using namespace desc;
__global__ void k(int* p) {
  auto t = thread_x<256>();
  split(t, 32, [&](auto h) { sync(h); p[0] = 1; }, [&](auto h) { p[1] = 2; });
}
'''
SYNC_WHOLE = r'''
#include "view.hpp"
using namespace desc;
__global__ void k(int* p) {
  auto t = thread_x<256>();
  p[t.index()] = 1;
  sync(t);
}
'''


def _hip_syntax(src: str):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    with tempfile.TemporaryDirectory() as d:
        f = os.path.join(d, "k.hip")
        open(f, "w").write(src)
        return subprocess.run([hipcc, "--offload-arch=gfx950", "-std=c++17", "-fsyntax-only",
                               "--cuda-device-only", "-I", CSRC, f],
                              capture_output=True, text=True, timeout=120)


def test_sync_inside_split_does_not_compile():
    r = _hip_syntax(SYNC_IN_SPLIT)
    assert r.returncode != 0
    assert "sync inside a split" in r.stderr


def test_sync_of_whole_block_compiles():
    r = _hip_syntax(SYNC_WHOLE)
    assert r.returncode == 0, r.stderr
