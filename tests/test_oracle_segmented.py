"""Pins of the segmented oracle: each segment equals the unsegmented
definition on its slice, segment sums add up to the total, empty segments are
zero and leave the output untouched, brute force on tiny inputs."""
import itertools

import numpy as np

import oracle
import workloads


def test_segments_equal_slices():
    lengths = np.array([0, 1, 5, 0, 64, 65, 1000, 0, 3], np.int64)
    off = workloads.offsets_from_lengths(lengths)
    x = workloads.int_uniform(int(off[-1]), seed=5)
    r = oracle.reduce_segmented_i32(x, off)
    y = oracle.scan_segmented_i32(x, off)
    for s in range(lengths.size):
        sl = slice(off[s], off[s + 1])
        assert r[s] == oracle.reduce_i32(x[sl])
        assert np.array_equal(y[sl], oracle.scan_i32(x[sl]))
        if lengths[s]:
            assert int(y[off[s + 1] - 1]) == r[s]  # no wrap at these sizes
    assert int(r.sum()) == oracle.reduce_i32(x)


def test_brute_force_tiny():
    vals = (-1, 0, 2)
    for lens in itertools.product(range(3), repeat=3):
        off = workloads.offsets_from_lengths(lens)
        n = int(off[-1])
        for xs in itertools.product(vals, repeat=n):
            x = np.array(xs, np.int32)
            r = oracle.reduce_segmented_i32(x, off)
            y = oracle.scan_segmented_i32(x, off)
            want_y = []
            for s in range(3):
                seg = xs[off[s]:off[s + 1]]
                assert r[s] == sum(seg)
                want_y += [sum(seg[: k + 1]) for k in range(len(seg))]
            assert y.tolist() == want_y


def test_gap_positions_untouched():
    # offsets need not cover the whole buffer from the front when callers
    # pass a sub-range; positions outside every segment keep their fill.
    off = np.array([2, 4, 7], np.int64)
    x = np.arange(10, dtype=np.int32)
    y = oracle.scan_segmented_i32(x, off, fill=-99)
    assert y.tolist() == [-99, -99, 2, 5, 4, 9, 15, -99, -99, -99]


def test_workload_recipe():
    lengths = workloads.segment_lengths(4096, seed=10)
    assert lengths.min() >= 1 and lengths.max() <= 1 << 20
    assert int(lengths.sum()) == 315525003
    # log-uniform: about a tenth of the segments in each of the ten 2-bit bands
    counts = np.histogram(np.log2(lengths), bins=10, range=(0, 20))[0]
    assert counts.min() > 300 and counts.max() < 520
