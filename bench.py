"""Benchmark of the hot path on one MI355X.

A step is one pass over the HBM-bound workload: the inclusive int32 scan of
2^28 elements (seed 2) followed by the out-of-place FP32 transpose of an
8192 x 8192 matrix (seed 3).  Inputs are resident in HBM before timing
starts.  `value` is the algorithmic bytes of a step (read + write of both
operations: 8 * 2^28 + 8 * 8192^2 bytes) divided by the mean step time.

The JSON line also carries:
  roofline      the scan kernel (the dominant one): algorithmic bytes per
                launch over its mean launch time, taken with HIP events on
                the stream the kernel runs on, against the 8 TB/s HBM peak;
  cpu_baseline  the plain CPU oracle on the same workload, on this host;
  ops           per-operation figures measured in the same run.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu] [--ops LIST]
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
METRIC = "GB/s & % HBM peak (reduce/scan/transpose); GEMM TFLOP/s BF16x3 vs FP32"

SCAN_N = 1 << 28
T_ROWS = T_COLS = 8192
SCAN_BYTES = 8 * SCAN_N                   # read n int32 + write n int32
TRANSPOSE_BYTES = 8 * T_ROWS * T_COLS     # read + write rows*cols words
STEP_BYTES = SCAN_BYTES + TRANSPOSE_BYTES

# rocprofv3 summaries whose FETCH_SIZE / WRITE_SIZE give the scan's HBM
# traffic per launch (null until counters for the current kernel are taken).
SCAN_TRAFFIC_BYTES = None


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


def cpu_baseline(x_np, m_np, budget_s: float = 20.0):
    """Time the oracle's scan and transpose on the same workload (1 thread)."""
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
    return {
        "value": round(STEP_BYTES / step_s / 1e9, 3),
        "unit": "GB/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"full workload (scan 2^28 + transpose 8192^2), {reps} rep(s), "
                  f"single-thread C oracle; scan {t_scan / reps:.3f} s, "
                  f"transpose {t_tr / reps:.3f} s per rep",
        "host_cpus": os.cpu_count(),
    }


def bench_reduce(desc, torch, workloads, reps=50):
    """Reduce of 2^22 int32 (seed 1): warm (L2/MALL-resident) and cold."""
    x = torch.from_numpy(workloads.int_uniform(1 << 22, seed=1)).cuda()
    out = torch.empty(1, dtype=torch.int64, device="cuda")
    flush = torch.empty(512 << 20, dtype=torch.uint8, device="cuda")
    for _ in range(5):
        desc.desc_reduce_i32(x, out)
    warm = Timer(torch)
    for _ in range(reps):
        s = warm.start(); desc.desc_reduce_i32(x, out); warm.stop(s)
    cold = Timer(torch)
    for _ in range(reps):
        flush.fill_(1)
        s = cold.start(); desc.desc_reduce_i32(x, out); cold.stop(s)
    nbytes = 4 * (1 << 22) + 8
    w, c = warm.mean_ms(), cold.mean_ms()
    return {"n": 1 << 22, "bytes": nbytes,
            "warm_us": round(w * 1e3, 2), "warm_GBs": round(nbytes / w / 1e6, 1),
            "cold_us": round(c * 1e3, 2), "cold_GBs": round(nbytes / c / 1e6, 1)}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--ops", default="reduce", help="extra per-op measurements ('' for none)")
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              "(the kernels have no multi-GPU path)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import workloads
    desc = _load_library()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    print("bench: generating inputs", file=sys.stderr, flush=True)
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
    print(f"bench: timing {args.steps} steps", file=sys.stderr, flush=True)

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

    # the last step's outputs, checked on a sample against the definition
    ok_scan = bool(int(y[-1].item()) == int(np.int64(x_np.sum(dtype=np.int64)).astype(np.int32)))
    ok_tr = bool(torch.equal(mt[:64, :64].cpu(), m[:64, :64].t().cpu()))

    value = STEP_BYTES / (ms_per_step * 1e-3) / 1e9
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
        "roofline": {"bound": "hbm", "kernel": "scan_i32_kernel",
                     "achieved": round(scan_gbs, 2), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(scan_gbs / HBM_PEAK_GBS, 4),
                     "bytes_per_launch": SCAN_BYTES, "launch_us": round(scan_ms * 1e3, 2),
                     "traffic": SCAN_TRAFFIC_BYTES},
        "ops": {"scan_2^28": {"us": round(scan_ms * 1e3, 2), "GBs": round(scan_gbs, 1),
                              "frac": round(scan_gbs / HBM_PEAK_GBS, 4), "check": ok_scan},
                "transpose_8192": {"us": round(tr_ms * 1e3, 2), "GBs": round(tr_gbs, 1),
                                   "frac": round(tr_gbs / HBM_PEAK_GBS, 4), "check": ok_tr}},
    }
    extra = [o for o in args.ops.split(",") if o]
    if "reduce" in extra:
        print("bench: reduce 2^22", file=sys.stderr, flush=True)
        result["ops"]["reduce_2^22"] = bench_reduce(desc, torch, workloads)
    if not args.no_cpu:
        print("bench: CPU oracle baseline", file=sys.stderr, flush=True)
        result["cpu_baseline"] = cpu_baseline(x_np, m_np)
    print(json.dumps(result), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
