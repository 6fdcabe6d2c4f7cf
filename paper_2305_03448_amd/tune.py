"""Offline tuner: times every compiled configuration of each operation on
representative problems of each size class and writes the fastest into a
table file that the library loads at start-up (tune_gfx950.txt next to the
library; format: "<op name> <size class> <config name>" per line).

Usage:  python -m paper_2305_03448_amd.tune [--ops scan_i32,transpose_32,...]
                                            [--out PATH] [--reps N]
Prints one JSON object per (op, class) with the median time of each config.
"""
from __future__ import annotations

import argparse
import json
import os
import sys

import torch

import paper_2305_03448_amd as desc


def _time(fn, reps: int, warmup: int = 3) -> float:
    """Median of `reps` timings (ms) of fn() with HIP events on the current stream."""
    for _ in range(warmup):
        fn()
    times = []
    for _ in range(reps):
        s = torch.cuda.Event(enable_timing=True)
        e = torch.cuda.Event(enable_timing=True)
        s.record()
        fn()
        e.record()
        e.synchronize()
        times.append(s.elapsed_time(e))
    times.sort()
    return times[len(times) // 2]


def _problems(op: str, dev):
    """(size class, label, bytes moved, callable) for each representative problem."""
    g = torch.Generator(device=dev).manual_seed(0)
    out = []
    if op in ("scan_i32", "reduce_i32", "copy_32"):
        for n in (1 << 14, 1 << 18, 1 << 22, 1 << 28):
            x = torch.randint(-1024, 1025, (n,), dtype=torch.int32, device=dev, generator=g)
            if op == "scan_i32":
                y = torch.empty_like(x)
                ws = torch.zeros(desc.desc_scan_i32_workspace(n), dtype=torch.uint8, device=dev)
                fn = (lambda x=x, y=y, ws=ws: desc.desc_scan_i32(x, y, ws=ws))
                nbytes = 8 * n
            elif op == "reduce_i32":
                o = torch.empty(1, dtype=torch.int64, device=dev)
                ws = torch.zeros(desc.desc_reduce_i32_workspace(n), dtype=torch.uint8, device=dev)
                fn = (lambda x=x, o=o, ws=ws: desc.desc_reduce_i32(x, o, ws=ws))
                nbytes = 4 * n
            else:
                y = torch.empty_like(x)
                fn = (lambda x=x, y=y: desc.desc_copy_32(x, y))
                nbytes = 8 * n
            out.append((desc.desc_size_class(op, n), f"n={n}", nbytes, fn))
    elif op == "transpose_32":
        for r, c in ((96, 160), (512, 1024), (2048, 2048), (8192, 8192)):
            m = torch.randn(r, c, device=dev, generator=g)
            t = torch.empty(c, r, device=dev)
            fn = (lambda m=m, t=t: desc.desc_transpose_f32(m, t))
            out.append((desc.desc_size_class(op, r * c), f"{r}x{c}", 8 * r * c, fn))
    elif op in ("gemm_f32", "gemm_bf16x3", "gemm_fp8"):
        mode = op.split("_")[1]
        for n in (128, 512, 2048, 4096):
            A = torch.randn(n, n, device=dev, generator=g)
            B = torch.randn(n, n, device=dev, generator=g)
            C = torch.empty(n, n, device=dev)
            need = desc.desc_gemm_workspace(mode, n, n, n)
            ws = torch.empty(max(need, 256), dtype=torch.uint8, device=dev)
            fn = (lambda A=A, B=B, C=C, ws=ws, mode=mode: desc.desc_gemm(A, B, C, mode=mode, ws=ws))
            # "bytes" here is the flop count (2 n^3); the GBs column then reads GFLOP/s
            out.append((desc.desc_size_class(op, n ** 3), f"{n}^3", 2 * n ** 3, fn))
    elif op in ("seg_scan_i32", "seg_reduce_i32"):
        # log-uniform segment lengths in [1, max_len]; the last problem is the
        # size of the 4096-segment workload (about 3.2e8 elements)
        for S, max_len in ((8, 1 << 12), (64, 1 << 14), (256, 1 << 16), (4096, 1 << 20)):
            u = torch.rand(S, device=dev, generator=g, dtype=torch.float64)
            lengths = torch.floor(2.0 ** (u * torch.log2(torch.tensor(max_len + 1.0)))).long()
            off = torch.zeros(S + 1, dtype=torch.int64, device=dev)
            off[1:] = torch.cumsum(lengths, 0)
            n = int(off[-1].item())
            x = torch.randint(-1024, 1025, (n,), dtype=torch.int32, device=dev, generator=g)
            if op == "seg_scan_i32":
                y = torch.empty_like(x)
                ws = torch.zeros(desc.desc_scan_segmented_i32_workspace(n, S), dtype=torch.uint8,
                                 device=dev)
                fn = (lambda x=x, off=off, y=y, ws=ws:
                      desc.desc_scan_segmented_i32(x, off, y, ws=ws))
                nbytes = 8 * n
            else:
                r = torch.empty(S, dtype=torch.int64, device=dev)
                ws = torch.zeros(desc.desc_reduce_segmented_i32_workspace(n, S),
                                 dtype=torch.uint8, device=dev)
                fn = (lambda x=x, off=off, r=r, ws=ws:
                      desc.desc_reduce_segmented_i32(x, off, r, ws=ws))
                nbytes = 4 * n
            out.append((desc.desc_size_class(op, n), f"n={n} S={S}", nbytes, fn))
    elif op in ("gemm_grouped", "gemm_grouped_bf16x3"):
        # G problems with M, N, K uniform over {64, 128, ..., 1024}
        mode = "f32" if op == "gemm_grouped" else "bf16x3"
        for G in (64, 512):
            dims = torch.randint(1, 17, (G, 3), device=dev, generator=g) * 64
            probs = []
            flops = 0
            for M, N, K in dims.tolist():
                probs.append((torch.randn(M, K, device=dev, generator=g),
                              torch.randn(K, N, device=dev, generator=g),
                              torch.empty(M, N, device=dev)))
                flops += 2 * M * N * K
            d = desc.grouped_descriptors(probs, dev)
            if mode == "f32":
                need = desc.desc_gemm_grouped_workspace(G)
            else:
                # the workspace depends on the configuration: size it for the largest
                cls = desc.desc_size_class(op, G)
                need = 0
                for cfg in range(desc.desc_config_count(op)):
                    desc.desc_config_set(op, cls, cfg)
                    need = max(need, desc.desc_gemm_grouped_workspace_for(mode, d.cpu()))
                desc.desc_config_set(op, cls, -1)
            ws = torch.empty(need, dtype=torch.uint8, device=dev)
            fn = (lambda d=d, ws=ws, probs=probs, mode=mode:
                  desc.desc_gemm_grouped(d, mode=mode, ws=ws))
            out.append((desc.desc_size_class(op, G), f"G={G}", flops, fn))
    else:
        raise ValueError(f"no tuning problems for {op}")
    return out


def tune(ops, reps: int = 20):
    dev = torch.device("cuda:0")
    table = {}
    for op in ops:
        ncfg = desc.desc_config_count(op)
        for cls, label, nbytes, fn in _problems(op, dev):
            res = {}
            for cfg in range(ncfg):
                desc.desc_config_set(op, cls, cfg)
                ms = _time(fn, reps)
                res[desc.desc_config_name(op, cfg)] = {"us": round(ms * 1e3, 2),
                                                        "GBs": round(nbytes / ms / 1e6, 1)}
            desc.desc_config_set(op, cls, -1)
            best = min(res, key=lambda k: res[k]["us"])
            table[(op, cls)] = best
            print(json.dumps({"op": op, "class": cls, "problem": label, "best": best,
                              "configs": res}), flush=True)
    return table


def write_table(table, path: str) -> None:
    with open(path, "w") as f:
        f.write("# op size_class config -- timed per size class by paper_2305_03448_amd/tune.py\n")
        for (op, cls), cfg in sorted(table.items()):
            f.write(f"{op} {cls} {cfg}\n")


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--ops", default="copy_32,scan_i32,transpose_32,reduce_i32,seg_scan_i32,seg_reduce_i32")
    ap.add_argument("--out", default=None, help="table file to write")
    ap.add_argument("--reps", type=int, default=20)
    args = ap.parse_args(argv)
    table = tune([o for o in args.ops.split(",") if o], args.reps)
    if args.out:
        write_table(table, args.out)
    return 0


if __name__ == "__main__":
    sys.exit(main())
