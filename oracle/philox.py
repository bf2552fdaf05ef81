"""Philox4x32-10 and the maps from its words to integers and uniforms.

Philox4x32-10 is the counter-based generator of Salmon, Moraes, Dror and Shaw,
"Parallel Random Numbers: As Easy as 1, 2, 3" (SC'11): ten rounds of two
32x32->64-bit multiplications with fixed multipliers, XOR of the high halves
with the other counter words and the round key, and a Weyl increment of the
key between rounds.  The paper under study only asks that every executor get
the same initial seed (one-shot evaluation, Sec. III-C); the counter-based
generator makes every random choice a pure function of
(seed, stream, generation, individual, word), so the GPU path and this oracle
can draw the same numbers without sharing state.

Counter layout (this implementation's convention):
    key = (seed & 0xffffffff, seed >> 32)
    ctr = (block, individual, phase, stream)
word w of an individual is output word (w % 4) of block w // 4.
``phase`` is the generation number, or INIT_PHASE for the initial population.
"""
from __future__ import annotations

import numpy as np

M0 = 0xD2511F53
M1 = 0xCD9E8D57
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK32 = 0xFFFFFFFF

INIT_PHASE = 0xFFFFFFFF
OUTER_STREAM_BIT = 0x80000000


def philox4x32_10(ctr, key):
    """Philox4x32-10 on arrays.

    ctr: integer array [..., 4] (uint32 range); key: integer array [..., 2].
    Returns uint32 array [..., 4].
    """
    ctr = np.asarray(ctr, dtype=np.uint64)
    key = np.asarray(key, dtype=np.uint64)
    c0, c1, c2, c3 = (ctr[..., k].copy() for k in range(4))
    k0 = np.broadcast_to(key[..., 0], c0.shape).copy()
    k1 = np.broadcast_to(key[..., 1], c0.shape).copy()
    m0 = np.uint64(M0)
    m1 = np.uint64(M1)
    mask = np.uint64(MASK32)
    sh = np.uint64(32)
    for rnd in range(10):
        p0 = m0 * c0            # exact: both factors < 2^32
        p1 = m1 * c2
        hi0, lo0 = p0 >> sh, p0 & mask
        hi1, lo1 = p1 >> sh, p1 & mask
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
        if rnd < 9:
            k0 = (k0 + np.uint64(W0)) & mask
            k1 = (k1 + np.uint64(W1)) & mask
    return np.stack([c0, c1, c2, c3], axis=-1).astype(np.uint32)


def seed_key(seed: int):
    seed = int(seed)
    return np.array([seed & MASK32, (seed >> 32) & MASK32], dtype=np.uint64)


def words(seed: int, individual, phase: int, stream: int, n_words: int):
    """First n_words Philox words of each individual (array of indices).

    Returns uint32 [len(individual), n_words].
    """
    ind = np.atleast_1d(np.asarray(individual, dtype=np.uint64))
    n_blocks = (n_words + 3) // 4
    blk = np.arange(n_blocks, dtype=np.uint64)
    ctr = np.zeros((ind.shape[0], n_blocks, 4), dtype=np.uint64)
    ctr[:, :, 0] = blk[None, :]
    ctr[:, :, 1] = ind[:, None]
    ctr[:, :, 2] = np.uint64(int(phase) & MASK32)
    ctr[:, :, 3] = np.uint64(int(stream) & MASK32)
    out = philox4x32_10(ctr, seed_key(seed))
    return out.reshape(ind.shape[0], n_blocks * 4)[:, :n_words]


def word_at(seed: int, individual: int, phase: int, stream: int, w: int) -> int:
    """Single Philox word w of one individual."""
    ctr = np.array([w // 4, individual, int(phase) & MASK32, int(stream) & MASK32], dtype=np.uint64)
    return int(philox4x32_10(ctr, seed_key(seed))[w % 4])


def lemire(w, m):
    """floor(w * m / 2^32): an integer in [0, m) from one 32-bit word (no rejection)."""
    w = np.asarray(w, dtype=np.uint64)
    m = np.asarray(m, dtype=np.uint64)
    return ((w * m) >> np.uint64(32)).astype(np.int64)


def unit_open_closed(w):
    """Uniform in (0, 1] with 24-bit resolution, exactly representable in float32."""
    w = np.asarray(w, dtype=np.uint64)
    return (((w >> np.uint64(8)) + np.uint64(1)).astype(np.float64) * 2.0 ** -24).astype(np.float32)


def unit_closed_open64(w):
    """Uniform in [0, 1) with 24-bit resolution, as float64 (exact)."""
    w = np.asarray(w, dtype=np.uint64)
    return (w >> np.uint64(8)).astype(np.float64) * 2.0 ** -24
