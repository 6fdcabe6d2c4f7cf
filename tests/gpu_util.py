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
