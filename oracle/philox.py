"""Counter-based thermal noise, FP64 (Results "A replica-batched engine" and
Methods "Replica batching": a device-side counter-based Philox stream keyed by
seed, replica-and-cell index and step, drawn once per step and reused by the
predictor and the corrector).

Generator: Philox4x32-10 as published by Salmon, Moraes, Dror & Shaw (SC'11,
"Parallel random numbers: as easy as 1, 2, 3"): a 4x32-bit counter and a
2x32-bit key, ten rounds of two 32x32->64 multiplications with the published
multipliers, xor-mixing of the high halves with the other counter words and the
round key, and a Weyl increment of the key between rounds.

Reading of the key/counter mapping (the paper does not fix it): key = the
replica's 64-bit seed (low word, high word); counter = (cell index within the
replica, step low word, step high word, trial generation g), with g = 0
except for the refilled trials of the retire/refill scheme.  Uniforms u = (x + 1/2) 2^-32;
Box-Muller on (u0, u1) and (u2, u3) gives four normals, of which the first three
are the x, y, z components of eta.
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = 0x9E3779B9
W1 = 0xBB67AE85
LO = np.uint64(0xFFFFFFFF)
S32 = np.uint64(32)


def philox4x32_10(ctr, key):
    """ctr: uint64 array (..., 4) holding 32-bit words; key: (..., 2).
    Returns (..., 4) uint64 holding the 32-bit output words."""
    c = [np.asarray(ctr[..., i], dtype=np.uint64) & LO for i in range(4)]
    k0 = np.asarray(key[..., 0], dtype=np.uint64) & LO
    k1 = np.asarray(key[..., 1], dtype=np.uint64) & LO
    for rnd in range(10):
        p0 = M0 * c[0]
        p1 = M1 * c[2]
        hi0, lo0 = p0 >> S32, p0 & LO
        hi1, lo1 = p1 >> S32, p1 & LO
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
        k0 = (k0 + np.uint64(W0)) & LO
        k1 = (k1 + np.uint64(W1)) & LO
    return np.stack(c, axis=-1)


def raw_words(seeds, ncell, step, gen=0):
    """Raw Philox output words (R, ncell, 4) for cells 0..ncell-1 of each
    replica key in ``seeds`` (R,) at ``step`` (trial generation ``gen``)."""
    seeds = np.atleast_1d(np.asarray(seeds, dtype=np.uint64))
    step = int(step)
    R = seeds.size
    ctr = np.zeros((R, ncell, 4), dtype=np.uint64)
    ctr[:, :, 0] = np.arange(ncell, dtype=np.uint64)[None, :]
    ctr[:, :, 1] = step & 0xFFFFFFFF
    ctr[:, :, 2] = (step >> 32) & 0xFFFFFFFF
    ctr[:, :, 3] = int(gen) & 0xFFFFFFFF
    key = np.zeros((R, ncell, 2), dtype=np.uint64)
    key[:, :, 0] = (seeds & np.uint64(0xFFFFFFFF))[:, None]
    key[:, :, 1] = (seeds >> np.uint64(32))[:, None]
    return philox4x32_10(ctr, key)


def gaussian_eta(seeds, ncell, step, gen=0):
    """eta (R, 3, ncell) ~ N(0, 1) i.i.d. for the replica keys ``seeds`` at
    ``step`` (trial generation ``gen``)."""
    x = raw_words(seeds, ncell, step, gen).astype(np.float64)
    u = (x + 0.5) * 2.0 ** -32
    r01 = np.sqrt(-2.0 * np.log(u[..., 0]))
    r23 = np.sqrt(-2.0 * np.log(u[..., 2]))
    n0 = r01 * np.cos(2.0 * np.pi * u[..., 1])
    n1 = r01 * np.sin(2.0 * np.pi * u[..., 1])
    n2 = r23 * np.cos(2.0 * np.pi * u[..., 3])
    return np.stack([n0, n1, n2], axis=1)
