"""Build and ctypes binding of the hand-indexed twin kernels (hand.hip) and
of the exhaustive check of the e4m3 conversion the quantisers rely on.

The twins are the baseline of the view-layer comparison: the same reduce,
scan and transpose algorithms as the library's view kernels, with the index
arithmetic written out by hand.  They are measurement infrastructure used by
the tests and by bench.py, not part of the library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2305_03448_amd import build as _pkg_build  # noqa: E402

SRC = os.path.join(HERE, "hand.hip")
LIB_PATH = os.path.join(HERE, "libdesc_hand.so")

# The one configuration of each library kernel that the twins mirror; the
# comparison sets the library to these.
VIEW_CONFIGS = {"reduce_i32": "b256_u4_nt", "scan_i32": "b1024_r16_nt", "transpose_32": "t128",
                "gemm_f32": "m128n128k16_rm_d2_x16"}


def build() -> str:
    tmp = LIB_PATH + ".tmp%d" % os.getpid()
    cmd = [_pkg_build.HIPCC, *_pkg_build.HIP_FLAGS, "-I", _pkg_build.CSRC, "-shared", SRC,
           "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed for {SRC}:\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built (run __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        c = ctypes
        for name, res, args in (
            ("hand_reduce_i32_workspace", c.c_size_t, [c.c_int64]),
            ("hand_reduce_i32", c.c_int, [c.c_void_p, c.c_int64, c.c_void_p, c.c_void_p,
                                          c.c_void_p]),
            ("hand_scan_i32_workspace", c.c_size_t, [c.c_int64]),
            ("hand_scan_i32", c.c_int, [c.c_void_p, c.c_void_p, c.c_int64, c.c_void_p,
                                        c.c_void_p]),
            ("hand_transpose_f32", c.c_int, [c.c_void_p, c.c_void_p, c.c_int64, c.c_int64,
                                             c.c_void_p]),
            ("hand_gemm_f32", c.c_int, [c.c_void_p, c.c_int64, c.c_void_p, c.c_int64,
                                        c.c_void_p, c.c_int64, c.c_int64, c.c_int64, c.c_int64,
                                        c.c_void_p]),
            ("hand_e4m3_all_inputs", c.c_int, [c.c_void_p, c.c_void_p]),
            ("hand_bf16_all_inputs", c.c_int, [c.c_void_p, c.c_void_p]),
        ):
            f = getattr(L, name)
            f.restype, f.argtypes = res, args
        _lib = L
    return _lib


def _stream(t):
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _check(rc: int, name: str) -> None:
    if rc != 0:
        raise RuntimeError(f"{name}: hipError {rc}")


def _contig(t, dtype, name):
    import torch
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous {dtype} tensor on the GPU")


_ws = {}


def _workspace(kind, nbytes, device):
    import torch
    w = _ws.get(kind)
    if w is None or w.numel() < nbytes:
        w = torch.zeros(max(nbytes, 256), dtype=torch.uint8, device=device)
        _ws[kind] = w
    return w


def reduce_i32(x, out):
    _contig(x, __import__("torch").int32, "x")
    w = _workspace("reduce", lib().hand_reduce_i32_workspace(x.numel()), x.device)
    _check(lib().hand_reduce_i32(x.data_ptr(), x.numel(), out.data_ptr(), w.data_ptr(),
                                 _stream(x)), "hand_reduce_i32")
    return out


def scan_i32(x, out):
    _contig(x, __import__("torch").int32, "x")
    if out.numel() != x.numel():
        raise ValueError("out must have as many elements as x")
    w = _workspace("scan", lib().hand_scan_i32_workspace(x.numel()), x.device)
    _check(lib().hand_scan_i32(x.data_ptr(), out.data_ptr(), x.numel(), w.data_ptr(),
                               _stream(x)), "hand_scan_i32")
    return out


def transpose_f32(x, out):
    _contig(x, __import__("torch").float32, "x")
    if x.dim() != 2 or tuple(out.shape) != (x.shape[1], x.shape[0]):
        raise ValueError("x must be (rows, cols) and out (cols, rows)")
    _check(lib().hand_transpose_f32(x.data_ptr(), out.data_ptr(), x.shape[0], x.shape[1],
                                    _stream(x)), "hand_transpose_f32")
    return out


def gemm_f32(A, B, C):
    """C = A @ B (contiguous row-major float32 GPU tensors) with the twin of
    the library's 256 x 128 x 16 row-major FP32 tile."""
    import torch
    for t, name in ((A, "A"), (B, "B"), (C, "C")):
        _contig(t, torch.float32, name)
    M, K = A.shape
    N = B.shape[1]
    if tuple(B.shape) != (K, N) or tuple(C.shape) != (M, N):
        raise ValueError("shapes must be A (M,K), B (K,N), C (M,N)")
    _check(lib().hand_gemm_f32(A.data_ptr(), K, B.data_ptr(), N, C.data_ptr(), N, M, N, K,
                               _stream(A)), "hand_gemm_f32")
    return C


def e4m3_all_inputs():
    """(disagreements at finite |x| <= 448, other disagreements) between the
    hardware e4m3 conversion and the library's software encoder over all
    2^32 binary32 inputs."""
    import torch
    counts = torch.zeros(2, dtype=torch.int64, device="cuda")
    _check(lib().hand_e4m3_all_inputs(counts.data_ptr(), _stream(counts)), "hand_e4m3_all_inputs")
    torch.cuda.synchronize()
    return int(counts[0].item()), int(counts[1].item())


def bf16_all_inputs():
    """(disagreements on non-NaN inputs, disagreements on NaNs) between the
    hardware bf16 conversion and the library's software rounding over all
    2^32 binary32 inputs, each in both halves of the packed pair."""
    import torch
    counts = torch.zeros(2, dtype=torch.int64, device="cuda")
    _check(lib().hand_bf16_all_inputs(counts.data_ptr(), _stream(counts)), "hand_bf16_all_inputs")
    torch.cuda.synchronize()
    return int(counts[0].item()), int(counts[1].item())
