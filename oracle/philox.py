"""Counter-based random numbers for the fluctuating LB oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Philox4x32-10 as published by Salmon, Moraes, Dror and Shaw, "Parallel
random numbers: as easy as 1, 2, 3" (SC'11): a 4 x 32-bit counter and a
2 x 32-bit key; each of ten rounds multiplies counter words 0 and 2 by
0xD2511F53 and 0xCD9E8D57 (64-bit products split into high and low halves),
mixes the high halves with the other counter words and the key, and the key
is advanced by the Weyl increments 0x9E3779B9 and 0xBB67AE85 between rounds.
Vectorised over numpy arrays of counters.

Uniforms: u = (x + 1/2) 2^-32 in (0, 1).  Normals: the Box-Muller transform
(Box and Muller 1958) on consecutive pairs, z0 = r cos(2 pi u1),
z1 = r sin(2 pi u1), r = sqrt(-2 ln u0).
"""
from __future__ import annotations

import numpy as np

M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK = 0xFFFFFFFF


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Counter words c0..c3 (arrays or ints, < 2^32) and key k0, k1 -> four uint64 arrays of 32-bit outputs."""
    c = [np.asarray(x, dtype=np.uint64) & MASK for x in (c0, c1, c2, c3)]
    c = np.broadcast_arrays(*c)
    c = [x.copy() for x in c]
    k0 = np.uint64(k0 & MASK)
    k1 = np.uint64(k1 & MASK)
    m0, m1 = np.uint64(M0), np.uint64(M1)
    s32, mask = np.uint64(32), np.uint64(MASK)
    for r in range(10):
        p0 = m0 * c[0]
        p1 = m1 * c[2]
        hi0, lo0 = p0 >> s32, p0 & mask
        hi1, lo1 = p1 >> s32, p1 & mask
        c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
        k0 = np.uint64((int(k0) + W0) & MASK)
        k1 = np.uint64((int(k1) + W1) & MASK)
    return c


def uniform(x):
    """32-bit integers -> (x + 1/2) 2^-32 (exact in FP64)."""
    return (np.asarray(x, dtype=np.float64) + 0.5) * 2.0 ** -32


def box_muller(x0, x1):
    """Two 32-bit integers -> two independent standard normals."""
    u0, u1 = uniform(x0), uniform(x1)
    r = np.sqrt(-2.0 * np.log(u0))
    t = 2.0 * np.pi * u1
    return r * np.cos(t), r * np.sin(t)


def normals(c0, c1, c2, c3_base, ncalls, k0, k1):
    """4 * ncalls normals per counter: call j uses counter word 3 = c3_base | j; the pairs
    (x0, x1) and (x2, x3) of each call give normals 4 j .. 4 j + 3 in that order."""
    out = []
    for j in range(ncalls):
        x = philox4x32_10(c0, c1, c2, np.asarray(c3_base, dtype=np.uint64) | np.uint64(j), k0, k1)
        a, b = box_muller(x[0], x[1])
        c, d = box_muller(x[2], x[3])
        out += [a, b, c, d]
    return out
