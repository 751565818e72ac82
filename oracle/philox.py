"""Philox4x32-10 in numpy, written from its published definition.

Reference: J. K. Salmon, M. A. Moraes, R. O. Dror, D. E. Shaw, "Parallel random
numbers: as easy as 1, 2, 3", SC'11. Philox-4x32 with R = 10 rounds maps a
128-bit counter (four 32-bit words) and a 64-bit key (two words) to four
32-bit output words. One round multiplies words 0 and 2 by the two constants,
splits each 64-bit product into high and low halves, and permutes:

    out0 = hi(M1*x2) ^ x1 ^ k0
    out1 = lo(M1*x2)
    out2 = hi(M0*x0) ^ x3 ^ k1
    out3 = lo(M0*x0)

and between rounds the key is bumped by the two Weyl constants.

The paper itself used MRG32k3a and xorshift with skip-ahead (Parallel Random
Number Generation subsection); a counter-based generator makes the streams of
every particle, step and purpose independent and reproducible with no stored
state, which is what the GPU/CPU bit-identity of the draws needs.

Counter layout shared (by specification, not by code) with the GPU path:

    c0 = index  (particle, chain or pair; 0 for per-step scalars)
    c1 = block  (which group of four words for this index)
    c2 = step   (tempering step or PT iteration)
    c3 = (purpose << 24) | move
    key = (seed & 0xffffffff, seed >> 32)
"""

from __future__ import annotations

import numpy as np

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85
_MASK = np.uint64(0xFFFFFFFF)

# purposes (counter word 3, bits 24..31)
PRIOR = 1
PROP = 2
ACC = 3
RESAMP = 4
EXCH = 5
PARITY = 6

TWO_PI = 6.283185307179586          # the double nearest 2*pi
TWO_POW_M32 = 2.0 ** -32


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32-10. Inputs are integers or integer arrays holding
    32-bit values (broadcast together); returns four uint64 arrays of words."""
    x0, x1, x2, x3, key0, key1 = np.broadcast_arrays(
        *[np.asarray(v, dtype=np.uint64) & _MASK for v in (c0, c1, c2, c3, k0, k1)])
    x0, x1, x2, x3 = (a.copy() for a in (x0, x1, x2, x3))
    key0 = key0.copy()
    key1 = key1.copy()
    m0 = np.uint64(M0)
    m1 = np.uint64(M1)
    w0 = np.uint64(W0)
    w1 = np.uint64(W1)
    s32 = np.uint64(32)
    for r in range(10):
        if r:
            key0 = (key0 + w0) & _MASK
            key1 = (key1 + w1) & _MASK
        p0 = x0 * m0            # < 2^64: exact in uint64
        p1 = x2 * m1
        x0, x1, x2, x3 = ((p1 >> s32) ^ x1 ^ key0, p1 & _MASK,
                          (p0 >> s32) ^ x3 ^ key1, p0 & _MASK)
    return x0, x1, x2, x3


def key_of(seed: int):
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    return seed & 0xFFFFFFFF, seed >> 32


def words(seed, index, block, step, purpose, move=0):
    """The four Philox words for (index, block, step, purpose, move) under ``seed``."""
    k0, k1 = key_of(seed)
    c3 = (int(purpose) << 24) | (int(move) & 0xFFFFFF)
    return philox4x32_10(index, block, step, c3, k0, k1)


def u01_open(w) -> np.ndarray:
    """(w + 1/2) * 2^-32: a uniform strictly inside (0, 1), exact in FP64."""
    return (np.asarray(w, dtype=np.float64) + 0.5) * TWO_POW_M32


def u01_left_closed(w) -> np.ndarray:
    """w * 2^-32: a uniform in [0, 1), exact in FP64 (systematic-resampling offset)."""
    return np.asarray(w, dtype=np.float64) * TWO_POW_M32


def u01_53(wa, wb) -> np.ndarray:
    """A 53-bit uniform in [0, 1) from two words: (wa * 2^21 + (wb >> 11)) * 2^-53,
    exact in FP64 (per-particle offsets of stratified and multinomial resampling)."""
    hi = np.asarray(wa, dtype=np.uint64) << np.uint64(21)
    lo = np.asarray(wb, dtype=np.uint64) >> np.uint64(11)
    return (hi | lo).astype(np.float64) * 2.0 ** -53


def box_muller(wa, wb):
    """Two standard normals from two words (Box & Muller, 1958), FP64."""
    u0 = u01_open(wa)
    u1 = u01_open(wb)
    r = np.sqrt(-2.0 * np.log(u0))
    ang = TWO_PI * u1
    return r * np.cos(ang), r * np.sin(ang)


def normals(seed, index, step, purpose, move, count):
    """``count`` standard normals per index, shape (count, len(index)).

    Coordinate c uses block c // 4 of the stream, and within the block the
    words (0, 1) give coordinates 4b, 4b+1 and the words (2, 3) give 4b+2, 4b+3.
    """
    index = np.asarray(index, dtype=np.uint64)
    nb = (count + 3) // 4
    out = np.empty((4 * nb,) + index.shape, dtype=np.float64)
    for b in range(nb):
        w0, w1, w2, w3 = words(seed, index, b, step, purpose, move)
        out[4 * b + 0], out[4 * b + 1] = box_muller(w0, w1)
        out[4 * b + 2], out[4 * b + 3] = box_muller(w2, w3)
    return out[:count]


def uniforms_open(seed, index, step, purpose, move=0):
    """One open-interval uniform per index (word 0 of block 0)."""
    w0, _, _, _ = words(seed, index, 0, step, purpose, move)
    return u01_open(w0)
