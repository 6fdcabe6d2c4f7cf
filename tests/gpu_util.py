"""Helpers of the GPU tests (no arithmetic of the operations here)."""
import sys

import pytest
import torch

needs_gpu = pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")


def dev():
    return torch.device("cuda:0")


def case(msg: str) -> None:
    """Name the case on stdout before it touches the GPU."""
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def to_dev(a, offset_elems: int = 0):
    """Copy a numpy array to the GPU, optionally at an element offset inside a
    larger buffer (to exercise unaligned starts)."""
    t = torch.from_numpy(a.copy())
    if offset_elems == 0:
        return t.to(dev())
    flat = t.reshape(-1)
    buf = torch.empty(flat.numel() + offset_elems, dtype=t.dtype, device=dev())
    view = buf[offset_elems:]
    view.copy_(flat)
    return view.view(t.shape)


def bf16x3_bound(K: int) -> float:
    """A-priori componentwise bound of the split-BF16 product (relative to
    sum_k |a_ik| |b_kj|): two round-to-nearest bf16 planes (8 significant
    bits each) leave |a - hi - lo| <= 2^-16 |a| per operand, the dropped
    lo*lo term is at most 2^-16 |a b|, and the FP32 accumulation of the 3K
    exact products adds at most 3K * 2^-24.  For short sums this exceeds the
    1e-5 target, which random signs of the per-term errors only reach for
    longer ones; the tests take 1e-5 for K >= 64 and this bound below."""
    return 3 * 2.0 ** -16 + 3 * K * 2.0 ** -24
