"""The allocation-free scan entry point (desc_scan_i32_noalloc) against the
scan that takes a caller's workspace (desc_scan_i32), through the C ABI.

Two calls in a row on the shared per-GPU scratch, the second smaller than
the first (so the second must not pick up state the first left behind),
each bit-equal to desc_scan_i32 on the same input and to the oracle.  (The
refusal of sizes above the fixed limit is checked on the CPU, in
test_abi.py.)  Named to be collected last: it leaves the per-GPU scratch
set up, which no other test depends on, and passes alone or after them."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import paper_2305_03448_amd as desc
import workloads
from gpu_util import case, dev, needs_gpu, to_dev

pytestmark = [pytest.mark.gpu, needs_gpu]



def _noalloc(x: torch.Tensor, y: torch.Tensor) -> int:
    L = desc.lib()
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return L.desc_scan_i32_noalloc(ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                   x.numel(), s)


def test_noalloc_scan_matches_the_workspace_scan_twice_shrinking():
    for rep, n in enumerate([(1 << 26) + 12345, 70001]):
        case(f"noalloc scan rep {rep} n={n}")
        x = workloads.int_uniform(n, seed=800 + rep)
        xt = to_dev(x)
        y_na = torch.full((n,), 7, dtype=torch.int32, device=dev())
        y_ws = torch.full((n,), 9, dtype=torch.int32, device=dev())
        assert _noalloc(xt, y_na) == 0
        ws = torch.zeros(desc.desc_scan_i32_workspace(n), dtype=torch.uint8, device=dev())
        L = desc.lib()
        assert L.desc_scan_i32(ctypes.c_void_p(xt.data_ptr()), ctypes.c_void_p(y_ws.data_ptr()),
                               n, ctypes.c_void_p(ws.data_ptr()), ws.numel(),
                               ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)) == 0
        torch.cuda.synchronize()
        a, b = y_na.cpu().numpy(), y_ws.cpu().numpy()
        assert np.array_equal(a, b)
        assert np.array_equal(a, oracle.scan_i32(x))
