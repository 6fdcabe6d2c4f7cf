"""Benchmark of the hot path on one MI355X.

A step is one pass over the HBM-bound workload: the inclusive int32 scan of
2^28 elements (uniform in [-1024, 1024], seed 2) followed by the
out-of-place FP32 transpose of an 8192 x 8192 matrix (N(0,1), seed 3).
Inputs are resident in HBM before timing starts.  `value` is the
algorithmic bytes of a step (read + write of both operations:
8 * 2^28 + 8 * 8192^2 bytes) divided by the mean step time.

The JSON line also carries:
  roofline      the scan kernel (the dominant one): algorithmic bytes per
                launch over its mean launch time, taken with HIP events on
                the stream the kernel runs on, against the 8 TB/s HBM peak;
  cpu_baseline  the plain CPU oracle on the same workload, on this host;
  ops           the other rows of the path measured in the same run: the
                copy ceiling, the 2^22 reduction, the GEMM modes (TFLOP/s
                and error against the FP64 oracle on sampled entries), the
                segmented reduce/scan and the grouped GEMM.

Small kernels are timed as HIP-graph replays of many back-to-back launches,
so that host launch overhead does not enter their time.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--ops LIST]
  --ops: comma list of copy,reduce,gemm,gemm8192,segmented,grouped,views,variants
         ('' for none)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PEAK_TFLOPS = {"f32": 157.3, "bf16": 2500.0, "fp8": 5000.0}
METRIC = "GB/s & % HBM peak (reduce/scan/transpose); GEMM TFLOP/s BF16x3 vs FP32"

SCAN_N = 1 << 28
T_ROWS = T_COLS = 8192
SCAN_BYTES = 8 * SCAN_N                   # read n int32 + write n int32
TRANSPOSE_BYTES = 8 * T_ROWS * T_COLS     # read + write rows*cols words
STEP_BYTES = SCAN_BYTES + TRANSPOSE_BYTES

# HBM traffic of one scan launch from rocprofv3 FETCH_SIZE / WRITE_SIZE,
# each scaled by what the counter reads for the copy kernel of known size
# (FETCH_SIZE x 2.0, WRITE_SIZE x 1.0), taken for ScanCfg<1024, 16, true>
# built from the sources whose hash is SCAN_TRAFFIC_SRC_HASH; reported as
# None once the kernel's sources (or its configuration) have changed.
SCAN_TRAFFIC_BYTES = 2151897620
SCAN_TRAFFIC_CONFIG = "b1024_r16_nt"
SCAN_TRAFFIC_SRC_HASH = "70f36618b525c0db"
SCAN_SOURCES = ("scan.hip", "lookback.hpp", "common.hpp", "layouts.hpp", "view.hpp", "wave.hpp")


def scan_source_hash() -> str:
    """SHA-256 (first 16 hex digits) of the scan kernel's source files."""
    import hashlib
    h = hashlib.sha256()
    for name in SCAN_SOURCES:
        with open(os.path.join(ROOT, "paper_2305_03448_amd", "csrc", name), "rb") as f:
            h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def log(msg: str) -> None:
    print(f"bench: {msg}", file=sys.stderr, flush=True)


def _load_library():
    import paper_2305_03448_amd as desc
    if not os.path.exists(desc.LIB_PATH):
        import __graft_entry__
        __graft_entry__.build()
    desc.lib()
    return desc


class Timer:
    """HIP events on the current stream around a sequence of launches."""

    def __init__(self, torch):
        self.torch = torch
        self.pairs = []

    def start(self):
        e = self.torch.cuda.Event(enable_timing=True)
        e.record()
        return e

    def stop(self, s):
        e = self.torch.cuda.Event(enable_timing=True)
        e.record()
        self.pairs.append((s, e))

    def mean_ms(self):
        self.torch.cuda.synchronize()
        return sum(s.elapsed_time(e) for s, e in self.pairs) / max(1, len(self.pairs))

    def spread_us(self):
        """p10, median and p90 of the launch durations, in microseconds."""
        self.torch.cuda.synchronize()
        d = sorted(s.elapsed_time(e) * 1e3 for s, e in self.pairs)
        if not d:
            return {}
        pick = lambda q: round(d[min(len(d) - 1, int(q * (len(d) - 1) + 0.5))], 2)
        return {"p10_us": pick(0.1), "median_us": pick(0.5), "p90_us": pick(0.9)}


def graph_time_ms(torch, fn, reps: int = 50, warm: int = 3) -> float:
    """Mean time of fn() from a HIP graph holding `reps` back-to-back calls."""
    for _ in range(warm):
        fn()
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        for _ in range(reps):
            fn()
    g.replay()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    g.replay()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def events_time_ms(torch, fn, reps: int = 10, warm: int = 2) -> float:
    for _ in range(warm):
        fn()
    t = Timer(torch)
    for _ in range(reps):
        s = t.start(); fn(); t.stop(s)
    return t.mean_ms()


def op_views(desc, torch, workloads, reps: int = 100):
    """The evaluation of Sec. 5 on this GPU: the library's view kernels against
    their hand-indexed twins (same algorithm and configuration, indices
    written by hand; the library is set to the twins' configurations for the
    comparison), for 256 MB, 512 MB and 1 GB of memory per operation (for
    the FP32 GEMM: n x n operands with 3 n^2 words within that size, n =
    4608, 6528, 9216), 100 runs each, alternating the two; reported as median
    kernel times and the relative runtime hand / view (above 1: the view
    kernel is faster)."""
    import statistics
    sys.path.insert(0, os.path.join(ROOT, "tests", "handwritten"))
    import handlib
    # the library runs the configuration each twin mirrors, in every size class
    # (the tuned choices are put back afterwards)
    saved = {(op, cls): desc.desc_config_get(op, cls) for op in handlib.VIEW_CONFIGS
             for cls in range(4)}
    for op, name in handlib.VIEW_CONFIGS.items():
        cfg = [desc.desc_config_name(op, c) for c in range(desc.desc_config_count(op))].index(name)
        for cls in range(4):
            desc.desc_config_set(op, cls, cfg)

    def median_ms(timer):
        return statistics.median(a.elapsed_time(b) for a, b in timer.pairs)

    results = []
    for mb in (256, 512, 1024):
        words = mb << 18                      # 32-bit words in `mb` MiB
        half = words // 2                     # scan and transpose: input + output
        x = torch.from_numpy(workloads.int_uniform(words, seed=2)).cuda()
        xs = x[:half]
        rows = 8192 if mb == 1024 else 4096 * mb // 256
        m = xs.view(torch.float32).view(rows, half // rows)
        r1, r2 = torch.empty(1, dtype=torch.int64, device="cuda"), torch.empty(1, dtype=torch.int64,
                                                                                device="cuda")
        y1, y2 = torch.empty_like(xs), torch.empty_like(xs)
        t1 = torch.empty((m.shape[1], m.shape[0]), dtype=torch.float32, device="cuda")
        t2 = torch.empty_like(t1)
        # matrix multiplication: A, B, C of n x n FP32 taking the memory size
        gn = {256: 4608, 512: 6528, 1024: 9216}[mb]
        ga = torch.from_numpy(workloads.matrix_f32(gn, gn, seed=4)).cuda()
        gb = torch.from_numpy(workloads.matrix_f32(gn, gn, seed=5)).cuda()
        gc1, gc2 = torch.empty_like(ga), torch.empty_like(ga)
        cases = [
            ("gemm_f32", lambda: desc.desc_gemm(ga, gb, gc1, mode="f32"),
             lambda: handlib.gemm_f32(ga, gb, gc2),
             lambda: torch.equal(gc1.view(torch.int32), gc2.view(torch.int32))),
            ("reduce", lambda: desc.desc_reduce_i32(x, r1), lambda: handlib.reduce_i32(x, r2),
             lambda: torch.equal(r1, r2)),
            ("scan", lambda: desc.desc_scan_i32(xs, y1), lambda: handlib.scan_i32(xs, y2),
             lambda: torch.equal(y1, y2)),
            ("transpose", lambda: desc.desc_transpose_f32(m, t1),
             lambda: handlib.transpose_f32(m, t2),
             lambda: torch.equal(t1.view(torch.int32), t2.view(torch.int32))),
        ]
        for name, fv, fh, check in cases:
            for _ in range(3):
                fv(); fh()
            tv, th = Timer(torch), Timer(torch)
            for i in range(reps):
                # alternate which of the pair runs first, so neither gains
                # from the other's warm-up of clocks and caches
                order = ((tv, fv), (th, fh)) if i % 2 == 0 else ((th, fh), (tv, fv))
                for tm, fn in order:
                    e = tm.start(); fn(); tm.stop(e)
            torch.cuda.synchronize()
            mv, mh = median_ms(tv), median_ms(th)
            r = {"op": name, "memory_MB": mb, "view_us": round(mv * 1e3, 2),
                 **({"n": gn} if name == "gemm_f32" else {}),
                 "hand_us": round(mh * 1e3, 2), "hand_over_view": round(mh / mv, 4),
                 "equal": bool(check())}
            log(f"views {r}")
            results.append(r)
        del x, xs, m, y1, y2, t1, t2, ga, gb, gc1, gc2
        torch.cuda.empty_cache()
    for (op, cls), cfg in saved.items():
        desc.desc_config_set(op, cls, cfg)
    return results


def op_variants(desc, torch, workloads, reps: int = 20):
    """The paper's forms against the single-pass ones at 2^28 int32: the scan
    as two kernels (tile sums, then carry and scan: 12 B per element) against
    the single pass (8 B), and the block-wide reduction (one int64 per chunk of
    E elements) against the full reduction.  Median times of `reps` runs."""
    import statistics
    n = 1 << 28
    x = torch.from_numpy(workloads.int_uniform(n, seed=2)).cuda()
    y1, y2 = torch.empty_like(x), torch.empty_like(x)
    r = torch.empty(1, dtype=torch.int64, device="cuda")
    blocks = {E: torch.empty((n + E - 1) // E, dtype=torch.int64, device="cuda")
              for E in (4096, 65536)}

    def median_us(fn):
        for _ in range(3):
            fn()
        t = Timer(torch)
        for _ in range(reps):
            e = t.start(); fn(); t.stop(e)
        torch.cuda.synchronize()
        return statistics.median(a.elapsed_time(b) for a, b in t.pairs) * 1e3

    out = {}
    single = median_us(lambda: desc.desc_scan_i32(x, y1))
    two = median_us(lambda: desc.desc_scan_two_pass_i32(x, y2))
    out["scan_single_pass"] = {"us": round(single, 2), "GBs": round(8 * n / single / 1e3, 1)}
    out["scan_two_kernels"] = {"us": round(two, 2), "GBs_algorithmic": round(8 * n / two / 1e3, 1),
                               "GBs_moved": round(12 * n / two / 1e3, 1),
                               "equal": bool(torch.equal(y1, y2))}
    excl = median_us(lambda: desc.desc_scan_exclusive_i32(x, y2))
    y1_last = int(y1[-1].item()); y2_last = int(y2[-1].item()); x_last = int(x[-1].item())
    out["scan_exclusive_single_pass"] = {
        "us": round(excl, 2), "GBs": round(8 * n / excl / 1e3, 1),
        "consistent": bool(int(y2[0].item()) == 0 and
                           (y2_last + x_last - y1_last) % (1 << 32) == 0)}
    full = median_us(lambda: desc.desc_reduce_i32(x, r))
    out["reduce_full"] = {"us": round(full, 2), "GBs": round(4 * n / full / 1e3, 1)}
    for E, o in blocks.items():
        t = median_us(lambda o=o, E=E: desc.desc_reduce_blocks_i32(x, E, o))
        out[f"reduce_blocks_E{E}"] = {"us": round(t, 2), "GBs": round(4 * n / t / 1e3, 1),
                                      "sum_equal": bool(int(o.sum().item()) == int(r.item()))}
    del x, y1, y2
    torch.cuda.empty_cache()
    return out


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(x_np, m_np, budget_s: float = 20.0):
    """Time the oracle's scan and transpose on the same workload (1 thread),
    then the same loops over every host core (OpenMP, oracle/cpu_parallel.c)."""
    import numpy as np
    import oracle
    oracle.lib()
    reps, t_scan, t_tr = 0, 0.0, 0.0
    t_end = time.perf_counter() + budget_s
    while reps < 3 and (reps == 0 or time.perf_counter() < t_end):
        t0 = time.perf_counter()
        oracle.scan_i32(x_np)
        t1 = time.perf_counter()
        oracle.transpose_u32(m_np)
        t2 = time.perf_counter()
        t_scan += t1 - t0
        t_tr += t2 - t1
        reps += 1
    step_s = (t_scan + t_tr) / reps
    res = {
        "value": round(STEP_BYTES / step_s / 1e9, 3),
        "unit": "GB/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"the full step workload (scan 2^28 + transpose 8192^2), {reps} rep(s), "
                  f"single-thread C oracle: scan {t_scan / reps:.3f} s, "
                  f"transpose {t_tr / reps:.3f} s per rep",
        "host_cpus": os.cpu_count(),
        "cpu_model": _cpu_model(),
    }
    # The same loops over all host cores: median of 5 full steps.
    threads = oracle.omp_threads()
    y = np.empty_like(x_np)
    times = []
    for _ in range(5):
        t0 = time.perf_counter()
        y = oracle.omp_scan_i32(x_np)
        t1 = time.perf_counter()
        oracle.omp_transpose_u32(m_np)
        t2 = time.perf_counter()
        times.append((t1 - t0, t2 - t1))
    times.sort(key=lambda t: t[0] + t[1])
    ts, tt = times[len(times) // 2]
    res["all_cores"] = {
        "value": round(STEP_BYTES / (ts + tt) / 1e9, 3), "unit": "GB/s", "cores": threads,
        "kind": "openmp loops of the oracle (oracle/cpu_parallel.c)",
        "sample": f"the full step workload, median of 5: scan {ts:.4f} s, transpose {tt:.4f} s",
    }
    del y
    return res


# ------------------------------------------------------------------ per-op measurements
def op_transpose_elems(desc, torch):
    """Transposes of 1-, 2- and 8-byte elements, 256 MiB in and 256 MiB out
    each (the paper's 512 MB size): graph-replay time and algorithmic GB/s."""
    out = {}
    for name, dtype, rows, cols in (("u8", torch.uint8, 16384, 16384),
                                    ("u16", torch.int16, 16384, 8192),
                                    ("f64", torch.float64, 8192, 4096)):
        x = torch.zeros((rows, cols), dtype=dtype, device="cuda")
        y = torch.empty((cols, rows), dtype=dtype, device="cuda")
        ms = graph_time_ms(torch, lambda: desc.desc_transpose_batched(x, y), reps=10)
        nbytes = 2 * x.numel() * x.element_size()
        out[name] = {"shape": [rows, cols], "us": round(ms * 1e3, 1),
                     "GBs": round(nbytes / ms / 1e6, 1), "frac": round(nbytes / ms / 1e6 / HBM_PEAK_GBS, 4)}
        del x, y
    torch.cuda.empty_cache()
    return out


def op_reverse(desc, torch):
    """Reversal of 2^28 words (the copy through the reverse view) beside the copy."""
    n = 1 << 28
    x = torch.zeros(n, dtype=torch.int32, device="cuda")
    y = torch.empty_like(x)
    ms_r = graph_time_ms(torch, lambda: desc.desc_reverse_u32(x, y), reps=10)
    ms_c = graph_time_ms(torch, lambda: desc.desc_copy_32(x, y), reps=10)
    del x, y
    torch.cuda.empty_cache()
    return {"reverse_us": round(ms_r * 1e3, 1), "reverse_GBs": round(8 * n / ms_r / 1e6, 1),
            "copy_us": round(ms_c * 1e3, 1), "copy_GBs": round(8 * n / ms_c / 1e6, 1)}


def op_copy(desc, torch):
    n = 1 << 28
    x = torch.empty(n, dtype=torch.int32, device="cuda")
    y = torch.empty_like(x)
    ms = events_time_ms(torch, lambda: desc.desc_copy_32(x, y))
    return {"n_words": n, "us": round(ms * 1e3, 2), "GBs": round(8 * n / ms / 1e6, 1),
            "frac": round(8 * n / ms / 1e6 / HBM_PEAK_GBS, 4)}


def op_reduce(desc, torch, workloads):
    """Reduction of 2^22 int32 (seed 1): L2/MALL-resident (warm) and after a
    512 MiB write that evicts it (cold), both as graph replays; then a cold
    sweep over 2^22 .. 2^28 elements."""
    x_np = workloads.int_uniform(1 << 22, seed=1)
    x = torch.from_numpy(x_np).cuda()
    out = torch.empty(1, dtype=torch.int64, device="cuda")
    ws = torch.zeros(desc.desc_reduce_i32_workspace(x.numel()), dtype=torch.uint8, device="cuda")
    flush = torch.empty(512 << 20, dtype=torch.uint8, device="cuda")
    warm = graph_time_ms(torch, lambda: desc.desc_reduce_i32(x, out, ws=ws), reps=100)
    both = graph_time_ms(torch, lambda: (flush.fill_(1), desc.desc_reduce_i32(x, out, ws=ws)),
                         reps=20)
    fl = graph_time_ms(torch, lambda: flush.fill_(1), reps=20)
    cold = max(both - fl, 1e-6)
    torch.cuda.synchronize()
    ok = int(out.item()) == int(x_np.sum(dtype="int64"))
    nbytes = 4 * (1 << 22) + 8
    # sweep: where the latency of one launch stops dominating (cold, after the flush)
    sweep = []
    for lg in (22, 24, 26, 28):
        n = 1 << lg
        xs_np = workloads.int_uniform(n, seed=1)
        xs = torch.from_numpy(xs_np).cuda()
        wss = torch.zeros(desc.desc_reduce_i32_workspace(n), dtype=torch.uint8, device="cuda")
        t_both = graph_time_ms(torch, lambda: (flush.fill_(1),
                                               desc.desc_reduce_i32(xs, out, ws=wss)), reps=10)
        t = max(t_both - fl, 1e-6)
        torch.cuda.synchronize()
        sweep.append({"n": n, "cold_us": round(t * 1e3, 2),
                      "cold_GBs": round((4 * n + 8) / t / 1e6, 1),
                      "check": int(out.item()) == int(xs_np.sum(dtype="int64"))})
        del xs, wss
    return {"n": 1 << 22, "bytes": nbytes, "check": ok,
            "warm_us": round(warm * 1e3, 2), "warm_GBs": round(nbytes / warm / 1e6, 1),
            "cold_us": round(cold * 1e3, 2), "cold_GBs": round(nbytes / cold / 1e6, 1),
            "sweep_cold": sweep}


def op_reduce_ops(desc, torch, workloads, oracle):
    """Min/max of 2^28 int32, the fixed-order FP64 sum and the fixed-order
    scan of 2^28 float32 (wide exponent range, seed 15), beside the int32 sum
    of the same size, as graph replays; each result checked against the
    oracle (the scan at 2048 sampled positions)."""
    import numpy as np
    n = 1 << 28
    xi_np = workloads.int_uniform(n, seed=2, lo=-(1 << 31), hi=(1 << 31) - 1)
    xi = torch.from_numpy(xi_np).cuda()
    mm = torch.empty(2, dtype=torch.int32, device="cuda")
    si = torch.empty(1, dtype=torch.int64, device="cuda")
    ws = torch.zeros(desc.desc_reduce_op_workspace(n), dtype=torch.uint8, device="cuda")
    wsi = torch.zeros(desc.desc_reduce_i32_workspace(n), dtype=torch.uint8, device="cuda")
    ms_mm = graph_time_ms(torch, lambda: desc.desc_reduce_minmax_i32(xi, mm, ws=ws), reps=10)
    ms_si = graph_time_ms(torch, lambda: desc.desc_reduce_i32(xi, si, ws=wsi), reps=10)
    ok_mm = tuple(mm.cpu().tolist()) == oracle.minmax_i32(xi_np)
    ok_si = int(si.item()) == oracle.reduce_i32(xi_np)
    del xi, xi_np
    xf_np = workloads.wide_f32(n, seed=15)
    xf = torch.from_numpy(xf_np).cuda()
    sf = torch.empty(1, dtype=torch.float64, device="cuda")
    ms_sf = graph_time_ms(torch, lambda: desc.desc_reduce_sum_f32(xf, sf, ws=ws), reps=10)
    got = float(sf.item())
    chunks = n // 4096
    G = min(chunks, 2048)
    d = 16 * (-(-chunks // G)) + (-(-G // 256)) + 16
    bound = d * 2.0 ** -53 * float(np.abs(xf_np.astype(np.float64)).sum())
    exact = oracle.sum_f32(xf_np)
    # the fixed-order float scan of the same input, beside the int32 scan
    yf = torch.empty_like(xf)
    wss = torch.zeros(desc.desc_scan_f32_workspace(n), dtype=torch.uint8, device="cuda")
    ms_scf = graph_time_ms(torch, lambda: desc.desc_scan_f32(xf, yf, ws=wss), reps=10)
    idx = np.unique(np.random.default_rng(44).integers(0, n, 2048)).astype(np.int64)
    ys = yf[torch.from_numpy(idx).cuda()].cpu().numpy().astype(np.float64)
    ex = oracle.scan_f32(xf_np, idx)
    cum = np.cumsum(np.abs(xf_np.astype(np.float64)))[idx]
    d_scan = -(-(n // 65536) // 64) + 160
    ok_scf = bool(np.all(np.abs(ys - ex) <= 2.0 ** -24 * np.abs(ex) + 2.0 ** -149
                         + d_scan * 2.0 ** -53 * cum * (1 + 1e-6)))
    del xf, xf_np, ws, wsi, yf, wss
    torch.cuda.empty_cache()
    gbs = lambda ms: round(4 * n / ms / 1e6, 1)
    return {"n": n,
            "minmax_us": round(ms_mm * 1e3, 1), "minmax_GBs": gbs(ms_mm), "minmax_check": ok_mm,
            "sum_f32_us": round(ms_sf * 1e3, 1), "sum_f32_GBs": gbs(ms_sf),
            "sum_f32_err": abs(got - exact), "sum_f32_bound": bound,
            "sum_f32_check": abs(got - exact) <= bound,
            "sum_i32_us": round(ms_si * 1e3, 1), "sum_i32_GBs": gbs(ms_si), "sum_i32_check": ok_si,
            "scan_f32_us": round(ms_scf * 1e3, 1), "scan_f32_GBs": round(8 * n / ms_scf / 1e6, 1),
            "scan_f32_check": ok_scf}


def op_gemm(desc, torch, workloads, oracle, n, seeds, modes):
    import numpy as np
    A_np = workloads.matrix_f32(n, n, seed=seeds[0])
    B_np = workloads.matrix_f32(n, n, seed=seeds[1])
    ii, jj = workloads.sample_pairs(n, n, 4096, seed=seeds[2])
    R, D = oracle.gemm_ref_sampled(A_np, B_np, ii, jj)
    A = torch.from_numpy(A_np).cuda()
    B = torch.from_numpy(B_np).cuda()
    C = torch.empty(n, n, device="cuda")
    out = {}
    for mode in modes:
        need = desc.desc_gemm_workspace(mode, n, n, n)
        ws = torch.empty(max(need, 256), dtype=torch.uint8, device="cuda")
        ms = graph_time_ms(torch, lambda: desc.desc_gemm(A, B, C, mode=mode, ws=ws), reps=5)
        Cs = C.cpu().numpy()[ii, jj].astype(np.float64)
        comp = np.abs(Cs - R) / D
        rel = np.abs(Cs - R) / np.maximum(np.abs(R), 1e-300)
        tflops = 2 * n ** 3 / ms / 1e9
        peak = PEAK_TFLOPS["f32" if mode == "f32" else ("bf16" if mode == "bf16x3" else "fp8")]
        issued = 3 * tflops if mode == "bf16x3" else tflops
        out[mode] = {"us": round(ms * 1e3, 1), "TFLOPs": round(tflops, 2),
                     "peak_TFLOPs": peak, "mfma_frac": round(issued / peak, 4),
                     "err_componentwise_max": float(f"{comp.max():.3e}"),
                     "err_componentwise_mean": float(f"{comp.mean():.3e}"),
                     "err_elementwise_max": float(f"{rel.max():.3e}"),
                     "err_elementwise_median": float(f"{np.median(rel):.3e}"),
                     "err_normwise": float(f"{np.abs(Cs - R).max() / np.abs(R).max():.3e}"),
                     "within_1e-5": bool(comp.max() <= 1e-5)}
    # context, not this library: the vendor FP32 GEMM behind torch.mm (hipBLASLt / rocBLAS)
    torch.backends.cuda.matmul.allow_tf32 = False
    ms = graph_time_ms(torch, lambda: torch.mm(A, B, out=C), reps=5)
    Cs = C.cpu().numpy()[ii, jj].astype(np.float64)
    out["vendor_sgemm_context"] = {"us": round(ms * 1e3, 1), "TFLOPs": round(2 * n ** 3 / ms / 1e9, 2),
                                   "err_componentwise_max": float(f"{(np.abs(Cs - R) / D).max():.3e}")}
    del A, B, C
    torch.cuda.empty_cache()
    return out


def op_segmented(desc, torch, workloads):
    import numpy as np
    x_np, off_np = workloads.segmented_input()
    T, S = int(off_np[-1]), off_np.size - 1
    x = torch.from_numpy(x_np).cuda()
    off = torch.from_numpy(off_np).cuda()
    r = torch.empty(S, dtype=torch.int64, device="cuda")
    y = torch.empty_like(x)
    wr = torch.zeros(desc.desc_reduce_segmented_i32_workspace(T, S), dtype=torch.uint8,
                     device="cuda")
    wy = torch.zeros(desc.desc_scan_segmented_i32_workspace(T, S), dtype=torch.uint8,
                     device="cuda")
    red = graph_time_ms(torch, lambda: desc.desc_reduce_segmented_i32(x, off, r, ws=wr), reps=10)
    scn = graph_time_ms(torch, lambda: desc.desc_scan_segmented_i32(x, off, y, ws=wy), reps=10)
    torch.cuda.synchronize()
    # spot check against the definition on a few segments
    r_h = r.cpu().numpy()
    ok = all(int(r_h[s]) == int(x_np[off_np[s]:off_np[s + 1]].sum(dtype=np.int64))
             for s in (0, 1, S // 2, S - 1))
    ends = [int(off_np[s + 1]) - 1 for s in (0, 1, S // 2, S - 1) if off_np[s + 1] > off_np[s]]
    y_h = y[torch.tensor(ends, device="cuda")].cpu().numpy()
    ok = ok and all(int(v) == int(np.int64(r_h[s]).astype(np.int32))
                    for v, s in zip(y_h, [s for s in (0, 1, S // 2, S - 1)
                                          if off_np[s + 1] > off_np[s]]))
    rb = 4 * T + 8 * (S + 1) + 8 * S
    sb = 8 * T + 8 * (S + 1)
    del x, y
    torch.cuda.empty_cache()
    return {"segments": S, "elements": T, "check": ok,
            "reduce_us": round(red * 1e3, 1), "reduce_GBs": round(rb / red / 1e6, 1),
            "reduce_frac": round(rb / red / 1e6 / HBM_PEAK_GBS, 4),
            "scan_us": round(scn * 1e3, 1), "scan_GBs": round(sb / scn / 1e6, 1),
            "scan_frac": round(sb / scn / 1e6 / HBM_PEAK_GBS, 4)}


def op_grouped(desc, torch, workloads):
    shapes = workloads.grouped_shapes()
    pairs = workloads.grouped_operands(shapes)
    dev_pairs = []
    flops = 0
    roof_s = 0.0
    for (A, B), (M, N, K) in zip(pairs, shapes):
        M, N, K = int(M), int(N), int(K)
        dev_pairs.append((torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda(),
                          torch.empty(M, N, device="cuda")))
        flops += 2 * M * N * K
        roof_s += max(2 * M * N * K / (PEAK_TFLOPS["f32"] * 1e12),
                      4 * (M * K + K * N + M * N) / (HBM_PEAK_GBS * 1e9))
    d = desc.grouped_descriptors(dev_pairs, torch.device("cuda"))
    ws = torch.empty(desc.desc_gemm_grouped_workspace(len(pairs)), dtype=torch.uint8,
                     device="cuda")
    ms = graph_time_ms(torch, lambda: desc.desc_gemm_grouped(d, ws=ws), reps=5)
    # split-BF16 mode: three bf16 products on the matrix cores, the operands
    # split while they are staged; its floor is the larger of 3 x 2MNK at the
    # bf16 peak and the bytes of reading A and B once and writing C
    ws3 = torch.empty(desc.desc_gemm_grouped_workspace_for("bf16x3", d.cpu()),
                      dtype=torch.uint8, device="cuda")
    ms3 = graph_time_ms(torch, lambda: desc.desc_gemm_grouped(d, mode="bf16x3", ws=ws3), reps=5)
    roof3_s = 0.0
    for M, N, K in shapes:
        M, N, K = int(M), int(N), int(K)
        roof3_s += max(6 * M * N * K / (PEAK_TFLOPS["bf16"] * 1e12),
                       4 * (M * K + K * N + M * N) / (HBM_PEAK_GBS * 1e9))
    return {"problems": len(pairs), "flop": flops, "us": round(ms * 1e3, 1),
            "TFLOPs": round(flops / ms / 1e9, 2), "roofline_us": round(roof_s * 1e6, 1),
            "roofline_frac": round(roof_s * 1e3 / ms, 4),
            "bf16x3_us": round(ms3 * 1e3, 1), "bf16x3_TFLOPs": round(flops / ms3 / 1e9, 2),
            "bf16x3_roofline_us": round(roof3_s * 1e6, 1),
            "bf16x3_roofline_frac": round(roof3_s * 1e3 / ms3, 4)}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--ops", default="copy,reduce,gemm,gemm8192,segmented,grouped,views,variants,"
                                     "transpose_elems,reverse,reduce_ops",
                    help="extra per-op measurements ('' for none)")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py: the library runs on one GPU; --gpus {args.gpus} is not supported "
              "(the kernels have no multi-GPU path)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import workloads
    desc = _load_library()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    log("generating inputs")
    x_np = workloads.int_uniform(SCAN_N, seed=2)
    m_np = workloads.matrix_f32(T_ROWS, T_COLS, seed=3)
    x = torch.from_numpy(x_np).to(dev)
    y = torch.empty_like(x)
    m = torch.from_numpy(m_np).to(dev)
    mt = torch.empty_like(m)
    ws = torch.zeros(desc.desc_scan_i32_workspace(SCAN_N), dtype=torch.uint8, device=dev)

    def step(timer_scan=None, timer_tr=None):
        s = timer_scan.start() if timer_scan else None
        desc.desc_scan_i32(x, y, ws=ws)
        if timer_scan:
            timer_scan.stop(s)
        s = timer_tr.start() if timer_tr else None
        desc.desc_transpose_f32(m, mt)
        if timer_tr:
            timer_tr.stop(s)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    log(f"timing {args.steps} steps")

    t_scan, t_tr = Timer(torch), Timer(torch)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    ev0.record()
    for _ in range(args.steps):
        step(t_scan, t_tr)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - w0
    ms_per_step = ev0.elapsed_time(ev1) / args.steps
    scan_ms, tr_ms = t_scan.mean_ms(), t_tr.mean_ms()

    # the last step's outputs, checked on samples against the definitions
    ok_scan = bool(int(y[-1].item()) == int(np.int64(x_np.sum(dtype=np.int64)).astype(np.int32)))
    ok_tr = bool(torch.equal(mt[:64, :64].cpu(), m[:64, :64].t().cpu()))

    value = STEP_BYTES / (ms_per_step * 1e-3) / 1e9
    scan_cfg = desc.desc_config_name(
        "scan_i32", desc.desc_config_get("scan_i32", desc.desc_size_class("scan_i32", SCAN_N)))
    traffic = (SCAN_TRAFFIC_BYTES if scan_cfg == SCAN_TRAFFIC_CONFIG
               and scan_source_hash() == SCAN_TRAFFIC_SRC_HASH else None)
    scan_gbs = SCAN_BYTES / (scan_ms * 1e-3) / 1e9
    tr_gbs = TRANSPOSE_BYTES / (tr_ms * 1e-3) / 1e9
    result = {
        "metric": METRIC,
        "value": round(value, 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i32",
        "data": "synthetic",
        "config": {"workload": "int32 inclusive scan of 2^28 (U[-1024,1024], seed 2) + "
                               "FP32 transpose 8192x8192 (N(0,1), seed 3)",
                   "scan_n": SCAN_N, "transpose_shape": [T_ROWS, T_COLS],
                   "bytes_per_step": STEP_BYTES},
        "hbm_frac": round(value / HBM_PEAK_GBS, 4),
        "wall_s": round(wall, 3),
        "roofline": {"bound": "hbm", "kernel": f"scan_i32_kernel {scan_cfg}",
                     "achieved": round(scan_gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(scan_gbs / HBM_PEAK_GBS, 4),
                     "bytes_per_launch": SCAN_BYTES, "launch_us": round(scan_ms * 1e3, 2),
                     "traffic": traffic},
        "ops": {"scan_2^28": {"us": round(scan_ms * 1e3, 2), "GBs": round(scan_gbs, 1),
                              "frac": round(scan_gbs / HBM_PEAK_GBS, 4), "check": ok_scan,
                              **t_scan.spread_us()},
                "transpose_8192": {"us": round(tr_ms * 1e3, 2), "GBs": round(tr_gbs, 1),
                                   "frac": round(tr_gbs / HBM_PEAK_GBS, 4), "check": ok_tr,
                                   **t_tr.spread_us()}},
    }
    extra = [o for o in args.ops.split(",") if o]
    if extra:
        import oracle
        del x, y, m, mt, ws
        torch.cuda.empty_cache()
    if "variants" in extra:
        log("paper's forms: two-kernel scan, block-wide reduction")
        result["ops"]["paper_forms_2^28"] = op_variants(desc, torch, workloads)
    if "views" in extra:
        log("view kernels against hand-indexed twins")
        result["ops"]["views_vs_hand"] = op_views(desc, torch, workloads)
    if "reverse" in extra:
        log("reversal through the reverse view")
        result["ops"]["reverse_2^28"] = op_reverse(desc, torch)
    if "transpose_elems" in extra:
        log("transposes of 1-, 2- and 8-byte elements")
        result["ops"]["transpose_elems_512MB"] = op_transpose_elems(desc, torch)
    if "copy" in extra:
        log("copy ceiling")
        result["ops"]["copy_2^28"] = op_copy(desc, torch)
    if "reduce" in extra:
        log("reduce 2^22")
        result["ops"]["reduce_2^22"] = op_reduce(desc, torch, workloads)
    if "reduce_ops" in extra:
        log("min/max and fixed-order float sum 2^28")
        result["ops"]["reduce_ops_2^28"] = op_reduce_ops(desc, torch, workloads, oracle)
    if "gemm" in extra:
        log("gemm 4096^3")
        result["ops"]["gemm_4096"] = op_gemm(desc, torch, workloads, oracle, 4096, (4, 5, 6),
                                             ("f32", "bf16x3", "fp8"))
    if "gemm8192" in extra:
        log("gemm 8192^3")
        result["ops"]["gemm_8192"] = op_gemm(desc, torch, workloads, oracle, 8192, (7, 8, 9),
                                             ("f32", "bf16x3", "fp8"))
    if "segmented" in extra:
        log("segmented 4096 segments")
        result["ops"]["segmented_4096"] = op_segmented(desc, torch, workloads)
    if "grouped" in extra:
        log("grouped gemm 512 problems")
        result["ops"]["grouped_512"] = op_grouped(desc, torch, workloads)
    if not args.no_cpu:
        log("CPU oracle baseline")
        result["cpu_baseline"] = cpu_baseline(x_np, m_np)
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
