"""Compression codec of the feature vectors, in the precision the paper's
codec fixes.  Test infrastructure only.

Paper, Section 8 (compression results): the feature vectors of every block,
E = U_c^T v (c coefficients per coordinate axis), are quantised uniformly
with q_c bits (q_c = 12); the rate is counted in bits per vertex.

Readings (listed in the design notes):
  * The quantiser's range is not given.  Each block and coordinate axis
    uses the range [lo, hi] of its own c coefficients, with 2^q levels
    lo + k * step, step = (hi - lo) / (2^q - 1); a coefficient takes the
    nearest level (ties to even).  A constant axis (hi = lo) has step 0 and
    every code 0.
  * The paper's bpv = 3 q_c c k / n_d counts k blocks of n_d vertices; for
    blocks of different sizes the rate is 3 q_c sum_b c_b / n, with n the
    mesh's vertex count.
  * Codes decide integers from floating point, so the oracle takes them in
    FP32 with every operation rounded on its own, as the GPU does.
"""
from __future__ import annotations

import numpy as np


def quantize_block(E: np.ndarray, c: int, qbits: int):
    """Codes (uint16, c x 3), per-axis (lo, step) and the dequantised
    coefficients (float32) of one block's first c feature vectors."""
    E = np.asarray(E, dtype=np.float32)[:c]
    levels = np.float32((1 << qbits) - 1)
    codes = np.zeros((c, 3), dtype=np.uint16)
    deq = np.zeros((c, 3), dtype=np.float32)
    lo = np.zeros(3, dtype=np.float32)
    step = np.zeros(3, dtype=np.float32)
    for k in range(3):
        col = E[:, k]
        l = np.float32(col.min()) if c > 0 else np.float32(0.0)
        h = np.float32(col.max()) if c > 0 else np.float32(0.0)
        s = np.float32(np.float32(h - l) / levels)
        lo[k], step[k] = l, s
        for j in range(c):
            q = np.float32(0.0)
            if s > 0:
                q = np.float32(np.rint(np.float32(np.float32(col[j] - l) / s)))
                q = np.float32(min(max(q, np.float32(0.0)), levels))
            codes[j, k] = np.uint16(q)
            deq[j, k] = np.float32(l + np.float32(q * s))
    return codes, lo, step, deq


def bits_per_vertex(qbits: int, c: np.ndarray, n_vertices: int) -> float:
    """Rate of the quantised feature vectors: 3 coordinates x q bits x the
    kept coefficients of every block, per mesh vertex."""
    return 3.0 * qbits * float(np.sum(c)) / float(n_vertices)
