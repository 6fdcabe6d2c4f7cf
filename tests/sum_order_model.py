"""A numpy model of the FP64 summation order that desc_reduce_sum_f32
documents (chunks of 4096 elements; lane j of block b adds elements
1024u + 4j + e of chunks b, b + G, ...; a fixed tree over the block's lanes;
the last block gathers the G block values, lane t those of blocks t, t + 256,
..., and combines them with the same tree).  Every step is one IEEE FP64
addition, so the model reproduces the documented result bit for bit.

It is a model of the library's stated contract, written from that statement
alone; it is not the oracle (the oracle is the exact sum), and it shares no
code with the library."""
from __future__ import annotations

import numpy as np

CHUNK, LANES, WAVE = 4096, 256, 64
MAX_BLOCKS = 2048


def grid(n: int) -> int:
    chunks = -(-n // CHUNK)
    return min(max(chunks, 1), MAX_BLOCKS)


def chain_bound(n: int) -> int:
    """Longest chain of additions in the order, d in |err| <= d 2^-53 sum|x|."""
    chunks, G = -(-n // CHUNK), grid(n)
    return 16 * (-(-chunks // G)) + 8 + (-(-G // LANES)) + 8


def _tree(v: np.ndarray) -> np.ndarray:
    """[B, 256] lane values -> [B] block values: butterfly inside each wave
    (lane i adds lane i ^ m, m = 32, 16, ..., 1), then (w0 + w1) + (w2 + w3)."""
    v = v.reshape(v.shape[0], LANES // WAVE, WAVE)
    lane = np.arange(WAVE)
    m = 32
    while m >= 1:
        v = v + v[:, :, lane ^ m]
        m >>= 1
    w = v[:, :, 0]
    return (w[:, 0] + w[:, 1]) + (w[:, 2] + w[:, 3])


def fixed_order_sum(x) -> float:
    x = np.ascontiguousarray(x, dtype=np.float32)
    n = x.size
    G = grid(n)
    nfull = n // CHUNK
    full = x[: nfull * CHUNK].reshape(nfull, 4, LANES, 4)   # [c][u][j][e]
    acc = np.zeros((G, LANES), np.float64)
    b = np.arange(G)
    for k in range(-(-nfull // G)):
        c = k * G + b
        live = c < nfull
        cs = c[live]
        for u in range(4):
            for e in range(4):
                acc[live] = acc[live] + full[cs, u, :, e].astype(np.float64)
    if nfull * CHUNK < n:                      # the partial chunk, skipped past n
        owner = nfull % G
        idx = nfull * CHUNK + 4 * np.arange(LANES)
        for u in range(4):
            for e in range(4):
                i = idx + 1024 * u + e
                ok = i < n
                acc[owner, ok] = acc[owner, ok] + x[i[ok]].astype(np.float64)
    blocks = _tree(acc)                        # [G]
    q = np.zeros(LANES, np.float64)
    t = np.arange(LANES)
    for k in range(-(-G // LANES)):
        bb = k * LANES + t
        ok = bb < G
        q[ok] = q[ok] + blocks[bb[ok]]
    return float(_tree(q[None, :])[0])
