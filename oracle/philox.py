"""Philox4x32-10 counter-based generator and Box-Muller normals (oracle side).

Written from the published definition (Salmon, Moraes, Dror, Shaw, "Parallel
random numbers: as easy as 1, 2, 3", SC'11, Sec. 4): each of the ten rounds
multiplies counter words 0 and 2 by the two Philox multipliers, mixes the
high halves with the other two words and the round key, and the key advances
by the two Weyl constants between rounds.

Thermostat noise (the O step of PILE-L) is indexed by
counter = (global index of (system, normal mode, atom), half, step lo, step hi)
and key = (seed lo, seed hi); half is 0 for the O step before the force
evaluation and 1 for the one after it.
"""
import numpy as np

M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK = 0xFFFFFFFF


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Ten Philox rounds on uint64 arrays that hold 32-bit values."""
    c0, c1, c2, c3 = (np.asarray(x, dtype=np.uint64) & MASK for x in (c0, c1, c2, c3))
    k0 = np.uint64(k0 & MASK)
    k1 = np.uint64(k1 & MASK)
    for _ in range(10):
        p0 = np.uint64(M0) * c0
        p1 = np.uint64(M1) * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & np.uint64(MASK)
        hi1, lo1 = p1 >> np.uint64(32), p1 & np.uint64(MASK)
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
        k0 = (k0 + np.uint64(W0)) & np.uint64(MASK)
        k1 = (k1 + np.uint64(W1)) & np.uint64(MASK)
    return c0, c1, c2, c3


def noise_words(seed, step, half, n):
    """The four uint32 words for global indices 0..n-1."""
    idx = np.arange(n, dtype=np.uint64)
    step = int(step)
    return philox4x32_10(idx, np.full(n, half), np.full(n, step & MASK), np.full(n, step >> 32),
                         seed & MASK, (seed >> 32) & MASK)


def words_to_normals(x0, x1, x2, x3):
    """u = (x + 1/2) 2^-32 in (0, 1); Box-Muller on (u0, u1) and (u2, u3);
    returns three normals (the fourth is unused)."""
    u = [(w.astype(np.float64) + 0.5) * 2.0 ** -32 for w in (x0, x1, x2, x3)]
    r0 = np.sqrt(-2.0 * np.log(u[0]))
    r1 = np.sqrt(-2.0 * np.log(u[2]))
    return np.stack([r0 * np.cos(2 * np.pi * u[1]), r0 * np.sin(2 * np.pi * u[1]),
                     r1 * np.cos(2 * np.pi * u[3])], axis=-1)


def thermostat_noise(seed, step, half, n):
    """Normals [n, 3] for the O step `half` of step `step`."""
    return words_to_normals(*noise_words(seed, step, half, n))
