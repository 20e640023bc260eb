"""Philox4x32-10 counter-based generator, written from its published definition.

Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3" (SC'11): a 4-word
(32-bit) counter and a 2-word key; each of the 10 rounds forms the 64-bit products of words 0
and 2 with two fixed odd multipliers and outputs
(hi(M1*x2) ^ x1 ^ k0, lo(M1*x2), hi(M0*x0) ^ x3 ^ k1, lo(M0*x0)); between rounds the key is
bumped by the two Weyl constants (golden ratio and sqrt(3)-1 in 32-bit fixed point).

TEST INFRASTRUCTURE ONLY (see oracle/__init__.py).  The photon and read noise of the sensor
model (the paper mentions calibration "(noise)", Sec. 2.5) draw their uniforms from these words.
"""

import numpy as np

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK32 = 0xFFFFFFFF
ROUNDS = 10


def philox4x32_10_scalar(counter, key):
    """One block with Python integers: counter = 4 words, key = 2 words -> 4 words."""
    x = [int(c) & MASK32 for c in counter]
    k0, k1 = int(key[0]) & MASK32, int(key[1]) & MASK32
    for r in range(ROUNDS):
        if r > 0:
            k0 = (k0 + W0) & MASK32
            k1 = (k1 + W1) & MASK32
        p0 = M0 * x[0]
        p1 = M1 * x[2]
        x = [(p1 >> 32) ^ x[1] ^ k0, p1 & MASK32, (p0 >> 32) ^ x[3] ^ k1, p0 & MASK32]
    return x


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised blocks over broadcastable integer arrays -> 4 uint64 arrays holding words."""
    m32 = np.uint64(MASK32)
    s32 = np.uint64(32)
    x0, x1, x2, x3 = (np.asarray(c, dtype=np.uint64) & m32
                      for c in np.broadcast_arrays(c0, c1, c2, c3))
    k0 = int(k0) & MASK32
    k1 = int(k1) & MASK32
    for r in range(ROUNDS):
        if r > 0:
            k0 = (k0 + W0) & MASK32
            k1 = (k1 + W1) & MASK32
        p0 = x0 * np.uint64(M0)  # < 2**64: exact in uint64
        p1 = x2 * np.uint64(M1)
        x0, x1, x2, x3 = ((p1 >> s32) ^ x1 ^ np.uint64(k0), p1 & m32,
                          (p0 >> s32) ^ x3 ^ np.uint64(k1), p0 & m32)
    return x0, x1, x2, x3


def uniforms_from_words(w):
    """u = ((w >> 8) + 1/2) * 2^-24 in (0, 1): the top 24 bits of a 32-bit word, centred."""
    w = np.asarray(w, dtype=np.uint64)
    return ((w >> np.uint64(8)).astype(np.float64) + 0.5) * 2.0 ** -24
