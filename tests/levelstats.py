"""Per-level statistics of an oracle trace, computed on the host with numpy.

Used by the GPU parity tests to show that an input reaches a particular
branch of the GPU kernels (test helper; no partitioning arithmetic).
"""
import numpy as np

import oracle


def _bits(x):
    """Number of significant bits of each non-negative int64 value (0 for 0)."""
    x = np.asarray(x, dtype=np.int64)
    out = np.zeros(x.shape, dtype=np.int64)
    v = x.copy()
    while np.any(v):
        nz = v > 0
        out[nz] += 1
        v >>= 1
    return out


def wide_counter_nodes(tr, hedge_w, omega):
    """Node-levels whose rating needs 64-bit (hist, c) counters: nodes of
    size < Omega (the ones that are rated) with
    bits(sum of w(e) over incident hedges) + bits(|in(n)|) > 32."""
    hw = np.asarray(hedge_w, dtype=np.int64)
    count = 0
    for l in range(tr.levels):
        hoff = tr.get(oracle.LV_HOFF, l).astype(np.int64)
        hpin = tr.get(oracle.LV_HPIN, l).astype(np.int64) & 0xFFFFFFFF
        size = tr.get(oracle.LV_SIZE, l).astype(np.int64)
        n = size.shape[0]
        ids = hpin & 0x7FFFFFFF
        dst = (hpin >> 31) & 1
        e_of = np.repeat(np.arange(len(hoff) - 1), np.diff(hoff))
        total = np.bincount(ids, weights=hw[e_of], minlength=n).astype(np.int64)
        indeg = np.bincount(ids, weights=dst, minlength=n).astype(np.int64)
        wide = (_bits(total) + _bits(indeg) > 32) & (size < omega)
        count += int(wide.sum())
    return count
