"""Philox4x32-10, written from its published definition (Salmon, Moraes, Dror, Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC'11, section 4.2).

State: four 32-bit counter words and two 32-bit key words.  One round multiplies
counter words 0 and 2 by two fixed odd constants into 64-bit products, and
produces (hi(c2*M1) ^ c1 ^ k0, lo(c2*M1), hi(c0*M0) ^ c3 ^ k1, lo(c0*M0)).  The
key is advanced by two Weyl constants between rounds; ten rounds.

Counter layout used by the GEM depth sampler (a reading; the paper is silent on
how its random depth samples are drawn):
  c0 = pixel index on the level's grid (row-major),
  c1 = slot group g (slots 3+4g .. 3+4g+3 use the four output words),
  c2 = (iteration << 8) | (level << 4) | purpose,
  c3 = window id;
  key = (seed & 0xffffffff, seed >> 32).
A 32-bit word x maps to u = (x >> 8) * 2^-24 in [0, 1), exact in FP32 and FP64.

Test infrastructure: see the package docstring.
"""
import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint64(0x9E3779B9)
W1 = np.uint64(0xBB67AE85)
MASK = np.uint64(0xFFFFFFFF)
S32 = np.uint64(32)

PURPOSE_INIT = 0
PURPOSE_CAND = 1


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Ten Philox rounds on arrays of 32-bit values (held in uint64)."""
    c0, c1, c2, c3 = (np.asarray(x, dtype=np.uint64) & MASK for x in (c0, c1, c2, c3))
    k0 = np.asarray(k0, dtype=np.uint64) & MASK
    k1 = np.asarray(k1, dtype=np.uint64) & MASK
    for r in range(10):
        if r:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        p0 = M0 * c0           # < 2^64: no wrap
        p1 = M1 * c2
        c0, c1, c2, c3 = ((p1 >> S32) ^ c1 ^ k0, p1 & MASK, (p0 >> S32) ^ c3 ^ k1, p0 & MASK)
    return c0, c1, c2, c3


def to_unit(x):
    """u = (x >> 8) / 2^24."""
    return (np.asarray(x, dtype=np.uint64) >> np.uint64(8)).astype(np.float64) * 2.0 ** -24


def word2(it, level, purpose):
    return (int(it) << 8) | (int(level) << 4) | int(purpose)


def key_of(seed):
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return seed & 0xFFFFFFFF, seed >> 32


def uniforms(pix, group, it, level, purpose, window_id, seed):
    """Four uniforms per pixel index in `pix` for one slot group: array [len(pix), 4]."""
    k0, k1 = key_of(seed)
    pix = np.asarray(pix, dtype=np.uint64)
    out = philox4x32_10(pix, np.full_like(pix, group), np.full_like(pix, word2(it, level, purpose)),
                        np.full_like(pix, int(window_id) & 0xFFFFFFFF), k0, k1)
    return np.stack([to_unit(o) for o in out], axis=-1)
