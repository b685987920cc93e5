"""32-bit MurmurHash3 finaliser (fmix32), written from Appleby's published
definition: xor-shift 16, multiply 0x85ebca6b, xor-shift 13, multiply
0xc2b2ae35, xor-shift 16, all modulo 2^32.

Test infrastructure only (see the package docstring).  The aggregation uses
it to give every node of a level a pseudo-random priority."""
from __future__ import annotations

import numpy as np

_M32 = np.uint64(0xFFFFFFFF)


def fmix32(h):
    h = np.asarray(h, dtype=np.uint64) & _M32
    h = h ^ (h >> np.uint64(16))
    h = (h * np.uint64(0x85EBCA6B)) & _M32
    h = h ^ (h >> np.uint64(13))
    h = (h * np.uint64(0xC2B2AE35)) & _M32
    h = h ^ (h >> np.uint64(16))
    return h


def level_salt(level: int) -> int:
    """Per-level salt xor-ed into the node index before hashing."""
    return (int(level) * 0x9E3779B9) & 0xFFFFFFFF


def priority(n: int, level: int) -> np.ndarray:
    """uint64 array of 32-bit priorities fmix32(i xor salt(level))."""
    idx = np.arange(n, dtype=np.uint64)
    return fmix32(idx ^ np.uint64(level_salt(level)))
