"""Oracle: the counter-based Gaussian generator the library draws its random
matrices with, written from its published definition.

Test infrastructure only (see ``oracle/__init__``).

Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
as 1, 2, 3", SC'11): a 4 x 32-bit counter is mixed by ten rounds of

    (x0, x1, x2, x3) -> (hi(M1 x2) ^ x1 ^ k0, lo(M1 x2), hi(M0 x0) ^ x3 ^ k1, lo(M0 x0))

with M0 = 0xD2511F53, M1 = 0xCD9E8D57 and the key (k0, k1) advanced by the
Weyl increments (0x9E3779B9, 0xBB67AE85) after every round.

The library's Gaussian stream (the mapping documented with its
``rp4d_philox_normal``): pair q of a stream keyed by a 64-bit seed s uses the
counter (q mod 2^32, q >> 32, 0, 0) and the key (s mod 2^32, s >> 32); the
output words give two 53-bit integers a = ((x0 << 21) ^ (x1 >> 11)) mod 2^53
and b = ((x2 << 21) ^ (x3 >> 11)) mod 2^53, the uniforms u1 = (a + 1) 2^-53 in
(0, 1] and u2 = b 2^-53, and by Box-Muller the normals
r cos(2 pi u2), r sin(2 pi u2) with r = sqrt(-2 ln u1).
"""
import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = 0x9E3779B9
W1 = 0xBB67AE85
MASK32 = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr, key):
    """ctr: (..., 4) integer array of 32-bit words; key: pair of 32-bit words.
    Returns the (..., 4) uint64 array of output words."""
    x = np.asarray(ctr, dtype=np.uint64) & MASK32
    x0, x1, x2, x3 = (x[..., i].copy() for i in range(4))
    k0, k1 = int(key[0]) & 0xFFFFFFFF, int(key[1]) & 0xFFFFFFFF
    for _ in range(10):
        p0 = M0 * x0                      # < 2^64: exact in uint64
        p1 = M1 * x2
        y0 = (p1 >> np.uint64(32)) ^ x1 ^ np.uint64(k0)
        y1 = p1 & MASK32
        y2 = (p0 >> np.uint64(32)) ^ x3 ^ np.uint64(k1)
        y3 = p0 & MASK32
        x0, x1, x2, x3 = y0, y1, y2, y3
        k0 = (k0 + W0) & 0xFFFFFFFF
        k1 = (k1 + W1) & 0xFFFFFFFF
    return np.stack([x0, x1, x2, x3], axis=-1)


def normal(seed, count):
    """`count` standard normals of the stream keyed by `seed` (see the module
    docstring), as float64."""
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    npairs = (int(count) + 1) // 2
    q = np.arange(npairs, dtype=np.uint64)
    ctr = np.stack([q & MASK32, q >> np.uint64(32), np.zeros_like(q), np.zeros_like(q)], axis=-1)
    x = philox4x32_10(ctr, (seed & 0xFFFFFFFF, seed >> 32))
    m53 = np.uint64((1 << 53) - 1)
    a = ((x[:, 0] << np.uint64(21)) ^ (x[:, 1] >> np.uint64(11))) & m53
    b = ((x[:, 2] << np.uint64(21)) ^ (x[:, 3] >> np.uint64(11))) & m53
    u1 = (a.astype(np.float64) + 1.0) * 2.0 ** -53
    u2 = b.astype(np.float64) * 2.0 ** -53
    r = np.sqrt(-2.0 * np.log(u1))
    z = np.empty(2 * npairs)
    z[0::2] = r * np.cos(2.0 * np.pi * u2)
    z[1::2] = r * np.sin(2.0 * np.pi * u2)
    return z[:count]


def gaussian_matrix(seed, rows, cols):
    """A rows x cols Gaussian matrix, row-major, as the library lays out a
    drawn block (Omega is n x l, grid point major)."""
    return normal(seed, rows * cols).reshape(rows, cols)
