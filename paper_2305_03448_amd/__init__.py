"""Python binding of the MI355X kernel library (``libdesc.so``).

Argument marshalling only: each function has the name of the C entry point it
calls (declared in ``include/desc.h``), takes ``torch.Tensor`` arguments that
live in GPU memory, passes their addresses, sizes and the current HIP stream,
and turns a non-zero status into :class:`DescError`.  Every step of the
computation runs in the library's HIP kernels; there is no other path, and
importing this module fails loudly when the library has not been built.

Workspaces: calls that keep state in a workspace get one from a cache keyed
by device, operation and stream when ``ws`` is omitted.  The cache hands out
zero-filled buffers and keeps them for later calls on the same stream, which
is the contract the library expects (zero before the first use, reused by
ordered calls afterwards).  Failures seen only on the GPU are read from a
workspace's device status word with ``desc_workspace_status``.
"""
from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdesc.so")

__all__ = [
    "DescError", "lib", "desc_status_string", "desc_version",
    "desc_workspace_status", "workspace_status", "desc_workspace_set_wait_limit", "DEV_STATUS",
    "desc_reduce_i32_workspace", "desc_reduce_i32",
    "desc_reduce_op_workspace", "desc_reduce_minmax_i32", "desc_reduce_sum_f32",
    "desc_scan_f32_workspace", "desc_scan_f32",
    "desc_scan_i32_workspace", "desc_scan_i32", "desc_scan_exclusive_i32", "desc_reduce_blocks_i32",
    "desc_scan_i32_noalloc",
    "desc_scan_two_pass_i32_workspace", "desc_scan_two_pass_i32",
    "desc_transpose_f32", "desc_transpose_batched_f32", "desc_transpose_batched", "desc_copy_32", "desc_reverse_u32",
    "desc_config_count", "desc_config_name", "desc_op_name", "desc_size_class",
    "desc_config_set", "desc_config_get", "desc_config_load", "OPS",
    "desc_gemm_workspace", "desc_gemm", "GEMM_MODES",
    "desc_split_bf16_rows", "desc_split_bf16_cols", "desc_quant_e4m3_rows",
    "desc_quant_e4m3_cols_workspace", "desc_quant_e4m3_cols",
    "desc_reduce_segmented_i32_workspace", "desc_reduce_segmented_i32",
    "desc_scan_segmented_i32_workspace", "desc_scan_segmented_i32",
    "desc_gemm_grouped_workspace", "desc_gemm_grouped_workspace_for", "desc_gemm_grouped",
    "grouped_descriptors",
    "desc_gemm_strided_batched_workspace", "desc_gemm_strided_batched",
    "desc_reduce_batched_i32_workspace", "desc_reduce_batched_i32",
    "desc_scan_batched_i32_workspace", "desc_scan_batched_i32",
]

_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_SZ = ctypes.c_size_t
_ST = ctypes.c_int

# name -> (restype, argtypes) of every exported entry point.
SIGNATURES = {
    "desc_status_string": (ctypes.c_char_p, [_ST]),
    "desc_workspace_status": (_ST, [_P, _SZ, _P, _P]),
    "desc_workspace_set_wait_limit": (_ST, [_P, _SZ, _I64, _P]),
    "desc_last_hip_error": (ctypes.c_int, []),
    "desc_version": (ctypes.c_int, []),
    "desc_set_pointer_classifier": (None, [_P]),
    "desc_reduce_i32_workspace": (_SZ, [_I64]),
    "desc_reduce_i32": (_ST, [_P, _I64, _P, _P, _SZ, _P]),
    "desc_reduce_op_workspace": (_SZ, [_I64]),
    "desc_reduce_minmax_i32": (_ST, [_P, _I64, _P, _P, _SZ, _P]),
    "desc_reduce_sum_f32": (_ST, [_P, _I64, _P, _P, _SZ, _P]),
    "desc_scan_f32_workspace": (_SZ, [_I64]),
    "desc_scan_f32": (_ST, [_P, _P, _I64, _P, _SZ, _P]),
    "desc_scan_i32_workspace": (_SZ, [_I64]),
    "desc_scan_i32": (_ST, [_P, _P, _I64, _P, _SZ, _P]),
    "desc_scan_exclusive_i32": (_ST, [_P, _P, _I64, _P, _SZ, _P]),
    "desc_scan_i32_noalloc": (_ST, [_P, _P, _I64, _P]),
    "desc_reduce_blocks_i32": (_ST, [_P, _I64, _I64, _P, _P]),
    "desc_scan_two_pass_i32_workspace": (_SZ, [_I64]),
    "desc_scan_two_pass_i32": (_ST, [_P, _P, _I64, _P, _SZ, _P]),
    "desc_transpose_f32": (_ST, [_P, _P, _I64, _I64, _P]),
    "desc_transpose_batched_f32": (_ST, [_P, _P, _I64, _I64, _I64, _P]),
    "desc_transpose_batched": (_ST, [_P, _P, _I64, _I64, _I64, _I64, _P]),
    "desc_copy_32": (_ST, [_P, _P, _I64, _P]),
    "desc_reverse_u32": (_ST, [_P, _P, _I64, _P]),
    "desc_config_count": (ctypes.c_int, [ctypes.c_int]),
    "desc_config_name": (ctypes.c_char_p, [ctypes.c_int, ctypes.c_int]),
    "desc_op_name": (ctypes.c_char_p, [ctypes.c_int]),
    "desc_size_class": (ctypes.c_int, [ctypes.c_int, _I64]),
    "desc_config_set": (_ST, [ctypes.c_int, ctypes.c_int, ctypes.c_int]),
    "desc_config_get": (ctypes.c_int, [ctypes.c_int, ctypes.c_int]),
    "desc_config_load": (_ST, [ctypes.c_char_p]),
    "desc_gemm_workspace": (_SZ, [ctypes.c_int, _I64, _I64, _I64]),
    "desc_gemm": (_ST, [ctypes.c_int, _I64, _I64, _I64, _P, _I64, _P, _I64, _P, _I64, _P, _SZ,
                        _P]),
    "desc_split_bf16_rows": (_ST, [_P, _I64, _I64, _I64, _P, _P, _I64, _P]),
    "desc_split_bf16_cols": (_ST, [_P, _I64, _I64, _I64, _P, _P, _I64, _P]),
    "desc_quant_e4m3_rows": (_ST, [_P, _I64, _I64, _I64, _P, _I64, _P, _P]),
    "desc_quant_e4m3_cols_workspace": (_SZ, [_I64, _I64]),
    "desc_quant_e4m3_cols": (_ST, [_P, _I64, _I64, _I64, _P, _I64, _P, _P, _SZ, _P]),
    "desc_reduce_segmented_i32_workspace": (_SZ, [_I64, _I64]),
    "desc_reduce_segmented_i32": (_ST, [_P, _I64, _P, _I64, _P, _P, _SZ, _P]),
    "desc_scan_segmented_i32_workspace": (_SZ, [_I64, _I64]),
    "desc_scan_segmented_i32": (_ST, [_P, _P, _I64, _P, _I64, _P, _SZ, _P]),
    "desc_gemm_grouped_workspace": (_SZ, [_I64]),
    "desc_gemm_grouped_workspace_for": (_SZ, [ctypes.c_int, _I64, _P]),
    "desc_gemm_grouped": (_ST, [ctypes.c_int, _I64, _P, _P, _SZ, _P]),
    "desc_gemm_strided_batched_workspace": (_SZ, [ctypes.c_int, _I64, _I64, _I64, _I64, _I64, _I64]),
    "desc_gemm_strided_batched": (_ST, [ctypes.c_int, _I64, _I64, _I64, _I64, _P, _I64, _I64, _P,
                                        _I64, _I64, _P, _I64, _I64, _P, _SZ, _P]),
    "desc_reduce_batched_i32_workspace": (_SZ, [_I64, _I64]),
    "desc_reduce_batched_i32": (_ST, [_P, _I64, _I64, _P, _P, _SZ, _P]),
    "desc_scan_batched_i32_workspace": (_SZ, [_I64, _I64]),
    "desc_scan_batched_i32": (_ST, [_P, _P, _I64, _I64, _P, _SZ, _P]),
}

# desc_gemm_mode values
GEMM_MODES = {"f32": 0, "bf16x3": 1, "fp8": 2}

# desc_op values (include/desc.h)
OPS = {"reduce_i32": 0, "scan_i32": 1, "transpose_32": 2, "copy_32": 3, "gemm_f32": 4,
       "gemm_bf16x3": 5, "gemm_fp8": 6, "seg_reduce_i32": 7, "seg_scan_i32": 8,
       "gemm_grouped": 9, "gemm_grouped_bf16x3": 10}
TUNE_FILE = os.path.join(HERE, "tune_gfx950.txt")

_lib = None


def lib() -> ctypes.CDLL:
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it first (python -c "
                "'import __graft_entry__ as g; g.build()')")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
        if os.path.exists(TUNE_FILE):
            _check(L.desc_config_load(TUNE_FILE.encode()), "desc_config_load")
    return _lib


class DescError(RuntimeError):
    def __init__(self, status: int, where: str):
        self.status = status
        msg = lib().desc_status_string(status).decode()
        if status == -7:
            msg += f" (hipError {lib().desc_last_hip_error()})"
        super().__init__(f"{where}: {msg}")


def _check(status: int, where: str) -> None:
    if status != 0:
        raise DescError(status, where)


def desc_status_string(status: int) -> str:
    return lib().desc_status_string(status).decode()


def desc_version() -> int:
    return lib().desc_version()


# ------------------------------------------------------------------ plumbing
def _stream(t: torch.Tensor, stream):
    if stream is None:
        stream = torch.cuda.current_stream(t.device)
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _dev(t: torch.Tensor, dtype: torch.dtype, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be in GPU memory (got {t.device})")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype} (got {t.dtype})")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


def _ptr(t: torch.Tensor | None):
    return ctypes.c_void_p(t.data_ptr() if t is not None and t.numel() > 0 else 0)


_ws_cache: dict = {}
# Cached workspaces that a larger one has replaced.  They stay allocated: a
# graph captured with one, or a kernel still running on another stream, may
# use it later, and the caching allocator could otherwise hand its memory to
# a new tensor.
_ws_retired: list = []


def _stream_of(device: torch.device, stream):
    """The torch stream object for `stream` (None: the current stream)."""
    if stream is None:
        return torch.cuda.current_stream(device)
    if isinstance(stream, torch.cuda.Stream):
        return stream
    return torch.cuda.ExternalStream(int(stream), device=device)


def workspace(kind: str, nbytes: int, device, stream=None) -> torch.Tensor:
    """A zero-filled workspace of at least ``nbytes`` kept per (device, kind,
    stream): calls that share a workspace must be ordered, which calls on one
    stream are.  A new buffer is allocated and zeroed on that stream, so the
    fill is ordered before the call that uses it."""
    device = torch.device(device)
    idx = device.index if device.index is not None else torch.cuda.current_device()
    device = torch.device("cuda", idx)
    s = _stream_of(device, stream)
    key = (idx, kind, s.cuda_stream)
    ws = _ws_cache.get(key)
    if ws is None or ws.numel() < nbytes:
        with torch.cuda.stream(s):
            new = torch.zeros(max(nbytes, 256), dtype=torch.uint8, device=device)
        if ws is not None:
            _ws_retired.append(ws)
        _ws_cache[key] = new
        ws = new
    return ws


def _ws(kind, nbytes, ref: torch.Tensor, ws, stream=None):
    if ws is None:
        return workspace(kind, nbytes, ref.device, stream)
    return _dev(ws, torch.uint8, "ws")


# ------------------------------------------------------------------ device status word
DEV_STATUS = {0: "ok", 1: "wait limit reached", 2: "bf16 planes do not fit"}


def desc_workspace_status(ws: torch.Tensor, out: torch.Tensor | None = None,
                          stream=None) -> torch.Tensor:
    """Copies the device status word of ``ws`` into ``out`` (int32[1] on the
    GPU, allocated if omitted) and resets it, in stream order."""
    _dev(ws, torch.uint8, "ws")
    if out is None:
        out = torch.empty(1, dtype=torch.int32, device=ws.device)
    _dev(out, torch.int32, "out")
    if out.numel() != 1:
        raise ValueError("out must hold one int32")
    _check(lib().desc_workspace_status(_ptr(ws), ws.numel(), _ptr(out), _stream(ws, stream)),
           "desc_workspace_status")
    return out


def workspace_status(ws: torch.Tensor, stream=None) -> int:
    """The device status word of ``ws`` as a host int (synchronises), reset to 0."""
    out = desc_workspace_status(ws, stream=stream)
    return int(out.item())


def desc_workspace_set_wait_limit(ws: torch.Tensor, max_polls: int, stream=None) -> None:
    """Debugging: every bounded wait of later calls on ``ws`` gives up after
    ``max_polls`` polls (0: at once); a negative value restores the default."""
    _dev(ws, torch.uint8, "ws")
    _check(lib().desc_workspace_set_wait_limit(_ptr(ws), ws.numel(), int(max_polls),
                                               _stream(ws, stream)),
           "desc_workspace_set_wait_limit")


# ------------------------------------------------------------------ reduce
def desc_reduce_i32_workspace(n: int) -> int:
    return lib().desc_reduce_i32_workspace(n)


def desc_reduce_i32(x: torch.Tensor, out: torch.Tensor, ws: torch.Tensor | None = None,
                    stream=None) -> torch.Tensor:
    """out[0] = exact int64 sum of int32 ``x``."""
    _dev(x, torch.int32, "x"); _dev(out, torch.int64, "out")
    if out.numel() != 1:
        raise ValueError("out must hold one int64")
    n = x.numel()
    w = _ws("reduce_i32", desc_reduce_i32_workspace(n), x, ws, stream)
    _check(lib().desc_reduce_i32(_ptr(x), n, _ptr(out), _ptr(w), w.numel(), _stream(x, stream)),
           "desc_reduce_i32")
    return out


# ------------------------------------------------------------------ min/max, float sum
def desc_reduce_op_workspace(n: int) -> int:
    return lib().desc_reduce_op_workspace(n)


def desc_reduce_minmax_i32(x: torch.Tensor, out: torch.Tensor, ws: torch.Tensor | None = None,
                           stream=None) -> torch.Tensor:
    """out = [min, max] of int32 ``x`` ([INT32_MAX, INT32_MIN] when empty)."""
    _dev(x, torch.int32, "x"); _dev(out, torch.int32, "out")
    if out.numel() != 2:
        raise ValueError("out must hold two int32")
    n = x.numel()
    w = _ws("reduce_op", desc_reduce_op_workspace(n), x, ws, stream)
    _check(lib().desc_reduce_minmax_i32(_ptr(x), n, _ptr(out), _ptr(w), w.numel(),
                                        _stream(x, stream)), "desc_reduce_minmax_i32")
    return out


def desc_reduce_sum_f32(x: torch.Tensor, out: torch.Tensor, ws: torch.Tensor | None = None,
                        stream=None) -> torch.Tensor:
    """out[0] = FP64 sum of float32 ``x`` in the order fixed by the indices and n."""
    _dev(x, torch.float32, "x"); _dev(out, torch.float64, "out")
    if out.numel() != 1:
        raise ValueError("out must hold one float64")
    n = x.numel()
    w = _ws("reduce_op", desc_reduce_op_workspace(n), x, ws, stream)
    _check(lib().desc_reduce_sum_f32(_ptr(x), n, _ptr(out), _ptr(w), w.numel(),
                                     _stream(x, stream)), "desc_reduce_sum_f32")
    return out


# ------------------------------------------------------------------ fixed-order float scan
def desc_scan_f32_workspace(n: int) -> int:
    return lib().desc_scan_f32_workspace(n)


def desc_scan_f32(x: torch.Tensor, out: torch.Tensor, ws: torch.Tensor | None = None,
                  stream=None) -> torch.Tensor:
    """Inclusive scan of float32 ``x`` into ``out``, FP64 accumulation in the
    order fixed by the indices and n, rounded once to float32."""
    _dev(x, torch.float32, "x"); _dev(out, torch.float32, "out")
    if out.numel() != x.numel():
        raise ValueError("out must have as many elements as x")
    n = x.numel()
    w = _ws("scan_f32", desc_scan_f32_workspace(n), x, ws, stream)
    _check(lib().desc_scan_f32(_ptr(x), _ptr(out), n, _ptr(w), w.numel(), _stream(x, stream)),
           "desc_scan_f32")
    return out


# ------------------------------------------------------------------ scan
def desc_scan_i32_workspace(n: int) -> int:
    return lib().desc_scan_i32_workspace(n)


def desc_scan_i32(x: torch.Tensor, out: torch.Tensor, ws: torch.Tensor | None = None,
                  stream=None) -> torch.Tensor:
    """Inclusive scan of int32 ``x`` into ``out`` (wrapping modulo 2^32)."""
    _dev(x, torch.int32, "x"); _dev(out, torch.int32, "out")
    if out.numel() != x.numel():
        raise ValueError("out must have as many elements as x")
    n = x.numel()
    w = _ws("scan_i32", desc_scan_i32_workspace(n), x, ws, stream)
    _check(lib().desc_scan_i32(_ptr(x), _ptr(out), n, _ptr(w), w.numel(), _stream(x, stream)),
           "desc_scan_i32")
    return out


def desc_scan_i32_noalloc(x: torch.Tensor, out: torch.Tensor, stream=None) -> torch.Tensor:
    """Inclusive scan of int32 ``x`` into ``out`` through the entry point that
    allocates nothing (the library's fixed per-GPU scratch; n <= 2^31)."""
    _dev(x, torch.int32, "x"); _dev(out, torch.int32, "out")
    if out.numel() != x.numel():
        raise ValueError("out must have as many elements as x")
    _check(lib().desc_scan_i32_noalloc(_ptr(x), _ptr(out), x.numel(), _stream(x, stream)),
           "desc_scan_i32_noalloc")
    return out


def desc_scan_exclusive_i32(x: torch.Tensor, out: torch.Tensor, ws: torch.Tensor | None = None,
                            stream=None) -> torch.Tensor:
    """Exclusive scan of int32 ``x`` into ``out``: out[0] = 0, out[i] = x[0] + ... + x[i-1]
    (wrapping modulo 2^32)."""
    _dev(x, torch.int32, "x"); _dev(out, torch.int32, "out")
    if out.numel() != x.numel():
        raise ValueError("out must have as many elements as x")
    n = x.numel()
    w = _ws("scan_i32", desc_scan_i32_workspace(n), x, ws, stream)
    _check(lib().desc_scan_exclusive_i32(_ptr(x), _ptr(out), n, _ptr(w), w.numel(),
                                         _stream(x, stream)), "desc_scan_exclusive_i32")
    return out


# ------------------------------------------------------------------ the paper's forms
def desc_reduce_blocks_i32(x: torch.Tensor, E: int, out: torch.Tensor, stream=None) -> torch.Tensor:
    """out[b] = exact int64 sum of x[b*E : (b+1)*E] (E a multiple of 1024)."""
    _dev(x, torch.int32, "x"); _dev(out, torch.int64, "out")
    n = x.numel()
    if E > 0 and out.numel() != (n + E - 1) // E:
        raise ValueError("out must hold ceil(n / E) int64")
    _check(lib().desc_reduce_blocks_i32(_ptr(x), n, E, _ptr(out), _stream(x, stream)),
           "desc_reduce_blocks_i32")
    return out


def desc_scan_two_pass_i32_workspace(n: int) -> int:
    return lib().desc_scan_two_pass_i32_workspace(n)


def desc_scan_two_pass_i32(x: torch.Tensor, out: torch.Tensor, ws: torch.Tensor | None = None,
                           stream=None) -> torch.Tensor:
    """Inclusive scan of int32 ``x`` into ``out`` by the two-kernel method."""
    _dev(x, torch.int32, "x"); _dev(out, torch.int32, "out")
    if out.numel() != x.numel():
        raise ValueError("out must have as many elements as x")
    n = x.numel()
    w = _ws("scan_two_pass_i32", desc_scan_two_pass_i32_workspace(n), x, ws, stream)
    _check(lib().desc_scan_two_pass_i32(_ptr(x), _ptr(out), n, _ptr(w), w.numel(),
                                        _stream(x, stream)), "desc_scan_two_pass_i32")
    return out


# ------------------------------------------------------------------ transpose
def _as_f32(t: torch.Tensor, name: str) -> torch.Tensor:
    if t.dtype in (torch.int32, torch.uint32) and t.device.type == "cuda":
        t = t.view(torch.float32)
    return _dev(t, torch.float32, name)


def desc_transpose_f32(x: torch.Tensor, out: torch.Tensor, stream=None) -> torch.Tensor:
    """out (cols x rows) = transpose of the row-major rows x cols ``x``."""
    x = _as_f32(x, "x"); o = _as_f32(out, "out")
    if x.dim() != 2 or o.dim() != 2 or tuple(o.shape) != (x.shape[1], x.shape[0]):
        raise ValueError("x must be (rows, cols) and out (cols, rows)")
    _check(lib().desc_transpose_f32(_ptr(x), _ptr(o), x.shape[0], x.shape[1],
                                    _stream(x, stream)), "desc_transpose_f32")
    return out


def desc_transpose_batched_f32(x: torch.Tensor, out: torch.Tensor, stream=None) -> torch.Tensor:
    """out[b] = transpose of x[b] for a (batch, rows, cols) ``x``."""
    x = _as_f32(x, "x"); o = _as_f32(out, "out")
    if x.dim() != 3 or tuple(o.shape) != (x.shape[0], x.shape[2], x.shape[1]):
        raise ValueError("x must be (batch, rows, cols) and out (batch, cols, rows)")
    _check(lib().desc_transpose_batched_f32(_ptr(x), _ptr(o), x.shape[0], x.shape[1],
                                            x.shape[2], _stream(x, stream)),
           "desc_transpose_batched_f32")
    return out


def desc_transpose_batched(x: torch.Tensor, out: torch.Tensor, stream=None) -> torch.Tensor:
    """out[b] = transpose of x[b] for a (rows, cols) or (batch, rows, cols) ``x`` of 1-, 2-,
    4- or 8-byte elements (bit patterns moved; any dtype of that size)."""
    if x.device.type != "cuda" or out.device.type != "cuda":
        raise ValueError("x and out must be in GPU memory")
    if not (x.is_contiguous() and out.is_contiguous()) or x.element_size() != out.element_size():
        raise ValueError("x and out must be contiguous with the same element size")
    xs = x.shape if x.dim() == 3 else (1,) + tuple(x.shape)
    if x.dim() not in (2, 3) or tuple(out.shape) != tuple(x.shape[:-2]) + (x.shape[-1], x.shape[-2]):
        raise ValueError("x must be (rows, cols) or (batch, rows, cols), out the transposes")
    _check(lib().desc_transpose_batched(_ptr(x), _ptr(out), x.element_size(), xs[0], xs[1], xs[2],
                                        _stream(x, stream)), "desc_transpose_batched")
    return out


def desc_reverse_u32(x: torch.Tensor, out: torch.Tensor, stream=None) -> torch.Tensor:
    """out[i] = x[n - 1 - i] for contiguous tensors of n 32-bit elements."""
    if x.device.type != "cuda" or out.device.type != "cuda":
        raise ValueError("x and out must be in GPU memory")
    if x.element_size() != 4 or out.element_size() != 4 or x.numel() != out.numel():
        raise ValueError("x and out must hold the same number of 32-bit elements")
    if not (x.is_contiguous() and out.is_contiguous()):
        raise ValueError("x and out must be contiguous")
    _check(lib().desc_reverse_u32(_ptr(x), _ptr(out), x.numel(), _stream(x, stream)),
           "desc_reverse_u32")
    return out


# ------------------------------------------------------------------ copy
def desc_copy_32(x: torch.Tensor, out: torch.Tensor, stream=None) -> torch.Tensor:
    """out = x, for tensors of 32-bit elements (the bandwidth ceiling)."""
    if x.device.type != "cuda" or out.device.type != "cuda":
        raise ValueError("x and out must be in GPU memory")
    if x.element_size() != 4 or out.element_size() != 4 or x.numel() != out.numel():
        raise ValueError("x and out must hold the same number of 32-bit elements")
    if not (x.is_contiguous() and out.is_contiguous()):
        raise ValueError("x and out must be contiguous")
    _check(lib().desc_copy_32(_ptr(x), _ptr(out), x.numel(), _stream(x, stream)),
           "desc_copy_32")
    return out


# ------------------------------------------------------------------ configurations
def _op(op) -> int:
    return OPS[op] if isinstance(op, str) else int(op)


def desc_config_count(op) -> int:
    return lib().desc_config_count(_op(op))


def desc_config_name(op, cfg: int):
    r = lib().desc_config_name(_op(op), cfg)
    return r.decode() if r else None


def desc_op_name(op):
    r = lib().desc_op_name(_op(op))
    return r.decode() if r else None


def desc_size_class(op, size: int) -> int:
    return lib().desc_size_class(_op(op), size)


def desc_config_set(op, size_class: int, cfg: int) -> None:
    _check(lib().desc_config_set(_op(op), size_class, cfg), "desc_config_set")


def desc_config_get(op, size_class: int) -> int:
    return lib().desc_config_get(_op(op), size_class)


def desc_config_load(path: str) -> None:
    _check(lib().desc_config_load(path.encode()), "desc_config_load")


# ------------------------------------------------------------------ GEMM
def _mode(mode) -> int:
    return GEMM_MODES[mode] if isinstance(mode, str) else int(mode)


def desc_gemm_workspace(mode, M: int, N: int, K: int) -> int:
    return lib().desc_gemm_workspace(_mode(mode), M, N, K)


def _rows(t: torch.Tensor, name: str):
    """(rows, cols, row stride) of a 2-D float32 GPU tensor with unit column stride."""
    if t.device.type != "cuda" or t.dtype != torch.float32 or t.dim() != 2:
        raise ValueError(f"{name} must be a 2-D float32 GPU tensor")
    rows, cols = t.shape
    if t.numel() == 0:
        return rows, cols, max(cols, 1)
    if cols > 1 and t.stride(1) != 1:
        raise ValueError(f"{name} must have unit column stride (row-major)")
    return rows, cols, t.stride(0) if rows > 1 else max(cols, 1)


def desc_gemm(A: torch.Tensor, B: torch.Tensor, C: torch.Tensor, mode="f32",
              ws: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """C = A @ B (row-major FP32 operands; strided rows allowed)."""
    M, K, lda = _rows(A, "A")
    K2, N, ldb = _rows(B, "B")
    M2, N2, ldc = _rows(C, "C")
    if K2 != K or M2 != M or N2 != N:
        raise ValueError("shapes must be A (M,K), B (K,N), C (M,N)")
    m = _mode(mode)
    need = desc_gemm_workspace(m, M, N, K)
    w = None
    if need:
        w = _ws(f"gemm{m}", need, A, ws, stream)
    _check(lib().desc_gemm(m, M, N, K, _ptr(A), lda, _ptr(B), ldb, _ptr(C), ldc, _ptr(w),
                           w.numel() if w is not None else 0, _stream(A, stream)), "desc_gemm")
    return C


# ------------------------------------------------------------------ operand preparation
def _u(t: torch.Tensor, dtype, name):
    if t.device.type != "cuda" or t.dtype != dtype or t.dim() != 2 or not t.is_contiguous():
        raise ValueError(f"{name} must be a contiguous 2-D {dtype} GPU tensor")
    return t


def desc_split_bf16_rows(A: torch.Tensor, hi: torch.Tensor, lo: torch.Tensor, stream=None):
    """hi, lo (int16 bit patterns, M x K) of the rows of float32 A (M x K)."""
    M, K, lda = _rows(A, "A")
    _u(hi, torch.int16, "hi"); _u(lo, torch.int16, "lo")
    if tuple(hi.shape) != (M, K) or tuple(lo.shape) != (M, K):
        raise ValueError("hi and lo must be (M, K)")
    _check(lib().desc_split_bf16_rows(_ptr(A), M, K, lda, _ptr(hi), _ptr(lo), max(K, 1),
                                      _stream(A, stream)), "desc_split_bf16_rows")


def desc_split_bf16_cols(B: torch.Tensor, hi_t: torch.Tensor, lo_t: torch.Tensor, stream=None):
    """hi^T, lo^T (int16 bit patterns, N x K) of the columns of float32 B (K x N)."""
    K, N, ldb = _rows(B, "B")
    _u(hi_t, torch.int16, "hi_t"); _u(lo_t, torch.int16, "lo_t")
    if tuple(hi_t.shape) != (N, K) or tuple(lo_t.shape) != (N, K):
        raise ValueError("hi_t and lo_t must be (N, K)")
    _check(lib().desc_split_bf16_cols(_ptr(B), K, N, ldb, _ptr(hi_t), _ptr(lo_t), max(K, 1),
                                      _stream(B, stream)), "desc_split_bf16_cols")


def desc_quant_e4m3_rows(A: torch.Tensor, q: torch.Tensor, scale: torch.Tensor, stream=None):
    """e4m3 codes (uint8, M x K) and scales alpha_i / 448 of the rows of A."""
    M, K, lda = _rows(A, "A")
    _u(q, torch.uint8, "q")
    if tuple(q.shape) != (M, K) or scale.numel() != M or scale.dtype != torch.float32:
        raise ValueError("q must be (M, K) and scale float32[M]")
    _check(lib().desc_quant_e4m3_rows(_ptr(A), M, K, lda, _ptr(q), max(K, 1), _ptr(scale),
                                      _stream(A, stream)), "desc_quant_e4m3_rows")


def desc_quant_e4m3_cols_workspace(K: int, N: int) -> int:
    return lib().desc_quant_e4m3_cols_workspace(K, N)


def desc_quant_e4m3_cols(B: torch.Tensor, q_t: torch.Tensor, scale: torch.Tensor,
                         ws: torch.Tensor | None = None, stream=None):
    """Transposed e4m3 codes (uint8, N x K) and scales beta_j / 448 of B's columns."""
    K, N, ldb = _rows(B, "B")
    _u(q_t, torch.uint8, "q_t")
    if tuple(q_t.shape) != (N, K) or scale.numel() != N or scale.dtype != torch.float32:
        raise ValueError("q_t must be (N, K) and scale float32[N]")
    need = desc_quant_e4m3_cols_workspace(K, N)
    w = ws if ws is not None else torch.empty(max(need, 4), dtype=torch.uint8, device=B.device)
    _check(lib().desc_quant_e4m3_cols(_ptr(B), K, N, ldb, _ptr(q_t), max(K, 1), _ptr(scale),
                                      _ptr(w), w.numel(), _stream(B, stream)),
           "desc_quant_e4m3_cols")


# ------------------------------------------------------------------ segmented
def desc_reduce_segmented_i32_workspace(n: int, num_segments: int) -> int:
    return lib().desc_reduce_segmented_i32_workspace(n, num_segments)


def desc_scan_segmented_i32_workspace(n: int, num_segments: int) -> int:
    return lib().desc_scan_segmented_i32_workspace(n, num_segments)


def desc_reduce_segmented_i32(x: torch.Tensor, offsets: torch.Tensor, out: torch.Tensor,
                              ws: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """out[s] = exact int64 sum of x[offsets[s]:offsets[s+1]]."""
    _dev(x, torch.int32, "x"); _dev(offsets, torch.int64, "offsets"); _dev(out, torch.int64, "out")
    S = offsets.numel() - 1
    if S < 0 or out.numel() != S:
        raise ValueError("offsets must hold S + 1 entries and out S")
    n = x.numel()
    w = _ws("reduce_segmented_i32", desc_reduce_segmented_i32_workspace(n, S), x, ws, stream)
    _check(lib().desc_reduce_segmented_i32(_ptr(x), n, _ptr(offsets), S, _ptr(out), _ptr(w),
                                           w.numel(), _stream(x, stream)),
           "desc_reduce_segmented_i32")
    return out


def desc_scan_segmented_i32(x: torch.Tensor, offsets: torch.Tensor, out: torch.Tensor,
                            ws: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Inclusive scan of x restarted at every offsets[s] (wrapping modulo 2^32)."""
    _dev(x, torch.int32, "x"); _dev(offsets, torch.int64, "offsets"); _dev(out, torch.int32, "out")
    S = offsets.numel() - 1
    if S < 0 or out.numel() != x.numel():
        raise ValueError("offsets must hold S + 1 entries and out as many elements as x")
    n = x.numel()
    w = _ws("scan_segmented_i32", desc_scan_segmented_i32_workspace(n, S), x, ws, stream)
    _check(lib().desc_scan_segmented_i32(_ptr(x), _ptr(out), n, _ptr(offsets), S, _ptr(w),
                                         w.numel(), _stream(x, stream)),
           "desc_scan_segmented_i32")
    return out


# ------------------------------------------------------------------ grouped GEMM
def desc_gemm_grouped_workspace(G: int) -> int:
    return lib().desc_gemm_grouped_workspace(G)


def grouped_descriptors(problems, device) -> torch.Tensor:
    """Device array of desc_gemm_problem for a list of (A, B, C) float32 GPU
    tensors (row-major, unit column stride): nine int64 words per problem,
    M, N, K, lda, ldb, ldc and the three addresses."""
    rows = []
    for A, B, C in problems:
        M, K, lda = _rows(A, "A")
        K2, N, ldb = _rows(B, "B")
        M2, N2, ldc = _rows(C, "C")
        if (K2, M2, N2) != (K, M, N):
            raise ValueError("shapes must be A (M,K), B (K,N), C (M,N)")
        rows.append([M, N, K, lda, ldb, ldc, A.data_ptr(), B.data_ptr(), C.data_ptr()])
    return torch.tensor(rows, dtype=torch.int64).reshape(-1, 9).to(device)


def desc_gemm_grouped_workspace_for(mode, descriptors_host: torch.Tensor) -> int:
    """Workspace bytes of a grouped call in `mode`, from a host copy of the
    descriptor array (G x 9 int64); 0 for a refused mode or shape."""
    d = descriptors_host
    if d.device.type != "cpu" or d.dtype != torch.int64 or d.dim() != 2 or d.shape[1] != 9:
        raise ValueError("descriptors_host must be a CPU int64 tensor of shape (G, 9)")
    d = d.contiguous()
    return lib().desc_gemm_grouped_workspace_for(_mode(mode), d.shape[0], d.data_ptr())


def desc_gemm_grouped(descriptors: torch.Tensor, mode="f32", ws: torch.Tensor | None = None,
                      stream=None, descriptors_host: torch.Tensor | None = None) -> None:
    """C_g = A_g @ B_g for every problem of a descriptor array (see
    grouped_descriptors); the tensors it points to must stay alive.  In mode
    "bf16x3" the workspace depends on the shapes: pass `ws` sized by
    desc_gemm_grouped_workspace_for, or `descriptors_host` (else the
    descriptors are copied to the host to size it)."""
    _dev(descriptors, torch.int64, "descriptors")
    G = descriptors.shape[0]
    if _mode(mode) == _mode("f32"):
        need = desc_gemm_grouped_workspace(G)
    elif ws is None or descriptors_host is not None:
        host = descriptors_host if descriptors_host is not None else descriptors.cpu()
        need = desc_gemm_grouped_workspace_for(mode, host)
        if need == 0 and G > 0:
            raise ValueError("a grouped problem has a shape the bf16x3 mode refuses")
        if ws is not None and ws.numel() < need:
            # the device would refuse the call and only set the error word
            raise ValueError(f"workspace of {ws.numel()} bytes, the current configuration "
                             f"needs {need}")
    else:
        need = ws.numel()
    w = ws if ws is not None else torch.empty(max(need, 256), dtype=torch.uint8,
                                              device=descriptors.device)
    _check(lib().desc_gemm_grouped(_mode(mode), G, _ptr(descriptors), _ptr(w), w.numel(),
                                   _stream(descriptors, stream)), "desc_gemm_grouped")


# ------------------------------------------------------------------ uniform batched forms
def desc_reduce_batched_i32_workspace(batch: int, length: int) -> int:
    return lib().desc_reduce_batched_i32_workspace(batch, length)


def desc_scan_batched_i32_workspace(batch: int, length: int) -> int:
    return lib().desc_scan_batched_i32_workspace(batch, length)


def desc_reduce_batched_i32(x: torch.Tensor, out: torch.Tensor, ws: torch.Tensor | None = None,
                            stream=None) -> torch.Tensor:
    """out[b] = exact int64 sum of row b of the 2-D int32 ``x``."""
    _dev(x, torch.int32, "x"); _dev(out, torch.int64, "out")
    if x.dim() != 2 or out.numel() != x.shape[0]:
        raise ValueError("x must be 2-D and out hold one int64 per row")
    B, L = x.shape
    w = _ws("batched_reduce", desc_reduce_batched_i32_workspace(B, L), x, ws, stream)
    _check(lib().desc_reduce_batched_i32(_ptr(x), B, L, _ptr(out), _ptr(w), w.numel(),
                                         _stream(x, stream)), "desc_reduce_batched_i32")
    return out


def desc_scan_batched_i32(x: torch.Tensor, out: torch.Tensor, ws: torch.Tensor | None = None,
                          stream=None) -> torch.Tensor:
    """Inclusive scan of every row of the 2-D int32 ``x`` (wrapping modulo 2^32)."""
    _dev(x, torch.int32, "x"); _dev(out, torch.int32, "out")
    if x.dim() != 2 or out.shape != x.shape:
        raise ValueError("x must be 2-D and out of the same shape")
    B, L = x.shape
    w = _ws("batched_scan", desc_scan_batched_i32_workspace(B, L), x, ws, stream)
    _check(lib().desc_scan_batched_i32(_ptr(x), _ptr(out), B, L, _ptr(w), w.numel(),
                                       _stream(x, stream)), "desc_scan_batched_i32")
    return out


def _strided3(t: torch.Tensor, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or t.device.type != "cuda" or t.dtype != torch.float32:
        raise TypeError(f"{name} must be a float32 tensor in GPU memory")
    if t.dim() != 3 or (t.numel() > 0 and t.stride(2) != 1):
        raise ValueError(f"{name} must be 3-D with unit stride in its last dimension")
    return t


def desc_gemm_strided_batched_workspace(mode, G: int, M: int, N: int, K: int, lda: int,
                                        ldb: int) -> int:
    return lib().desc_gemm_strided_batched_workspace(_mode(mode), G, M, N, K, lda, ldb)


def desc_gemm_strided_batched(A: torch.Tensor, B: torch.Tensor, C: torch.Tensor, mode="f32",
                              ws: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """C[g] = A[g] @ B[g] for 3-D float32 tensors with unit stride in the last
    dimension (any batch and row strides, e.g. padded views)."""
    _strided3(A, "A"); _strided3(B, "B"); _strided3(C, "C")
    G, M, K = A.shape
    N = B.shape[2]
    if B.shape[:2] != (G, K) or tuple(C.shape) != (G, M, N):
        raise ValueError("shapes must be A (G, M, K), B (G, K, N), C (G, M, N)")
    lda, ldb, ldc = A.stride(1), B.stride(1), C.stride(1)
    need = desc_gemm_strided_batched_workspace(mode, G, M, N, K, lda, ldb)
    if need == 0 and G > 0 and M > 0 and N > 0:
        raise ValueError("shape refused by this mode")
    w = _ws("strided_batched_" + str(mode), need, C, ws, stream)
    _check(lib().desc_gemm_strided_batched(_mode(mode), G, M, N, K, _ptr(A), lda, A.stride(0),
                                           _ptr(B), ldb, B.stride(0), _ptr(C), ldc, C.stride(0),
                                           _ptr(w), w.numel(), _stream(C, stream)),
           "desc_gemm_strided_batched")
    return C
