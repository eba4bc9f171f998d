"""Philox4x32-10 counter-based generator, written from its published definition.

Reference: J. K. Salmon, M. A. Moraes, R. O. Dror, D. E. Shaw, "Parallel
random numbers: as easy as 1, 2, 3", SC'11.  Philox4x32 keeps a 4-word
counter and a 2-word key.  One round multiplies counter words 0 and 2 by
the constants M0 = 0xD2511F53 and M1 = 0xCD9E8D57, producing 64-bit
products (hi, lo); the new counter is (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1,
lo0).  Between rounds the key is bumped by the Weyl constants
0x9E3779B9 and 0xBB67AE85.  Ten rounds are applied.

The paper asks for a random subselection but names no generator; the
counter-based choice makes every particle's draw a pure function of
(seed, snapshot, particle id), so any evaluation order gives the same bits.

TEST INFRASTRUCTURE ONLY (see the package docstring).  Pinned by the
published known-answer vectors (tests/golden/philox4x32_10_kat.txt) and by
uniformity statistics.
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint64(0x9E3779B9)
W1 = np.uint64(0xBB67AE85)
_MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Return the four output words (uint32 arrays) for counters/keys (broadcast)."""
    c0, c1, c2, c3, k0, k1 = (np.asarray(v, dtype=np.uint64) & _MASK
                              for v in (c0, c1, c2, c3, k0, k1))
    c0, c1, c2, c3, k0, k1 = np.broadcast_arrays(c0, c1, c2, c3, k0, k1)
    c0, c1, c2, c3 = c0.copy(), c1.copy(), c2.copy(), c3.copy()
    k0, k1 = k0.copy(), k1.copy()
    for rnd in range(10):
        if rnd:
            k0 = (k0 + W0) & _MASK
            k1 = (k1 + W1) & _MASK
        p0 = M0 * c0
        p1 = M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return tuple(v.astype(np.uint32) for v in (c0, c1, c2, c3))


def particle_uniform(pid, snap, seed):
    """U = word0(Philox4x32-10(ctr=(id lo, id hi, snapshot, 0), key=(seed lo, seed hi))) + 1.

    Returns uint64 values in [1, 2**32]; u = U / 2**32 lies in (0, 1].
    """
    pid = np.asarray(pid, dtype=np.uint64)
    snap = np.asarray(snap, dtype=np.uint64)
    seed = int(seed)
    r0, _, _, _ = philox4x32_10(pid & _MASK, pid >> np.uint64(32), snap, 0,
                                seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    return r0.astype(np.uint64) + np.uint64(1)
