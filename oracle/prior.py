"""Prior draw and prior log-density.

Paper: Sec. 1 (the trivial / prior distribution, point-wise independent) and the
example parameter file (prior = Normal{Float32}(0, 1)): every site is an
independent standard normal in FP32, so

    log r(z) = -1/2 sum_n z(n)^2 - (V/2) ln(2 pi).

The random numbers are realised with the counter-based generator Philox4x32-10
(Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3",
SC'11) followed by the Box-Muller transform (Box & Muller, 1958).  Both are
written here from their published definitions; the HIP library implements the
same definitions independently.

Stream layout (shared definition, not shared code): for sample b of a draw with
base counter c0 and a 64-bit key k, the 4 sites 4j..4j+3 take the Philox output
for counter (j, lo32(c0+b), hi32(c0+b), 0) under key (lo32(k), hi32(k)).  Each
32-bit word x becomes u = (floor(x / 2^9) + 1/2) / 2^23, exactly representable in
FP32 (at most 24 significant bits) and strictly inside (0, 1).  Words (u0,u1) give sites 4j and 4j+1, words
(u2,u3) give 4j+2 and 4j+3, via z_a = sqrt(-2 ln u_a) cos(2 pi u_b),
z_b = sqrt(-2 ln u_a) sin(2 pi u_b).

Pinned by: the Philox known-answer vectors, the Box-Muller radius identity
z_a^2 + z_b^2 = -2 ln u_a, a KS test against N(0,1), and scipy's normal logpdf.
"""
from __future__ import annotations

import numpy as np

_M0 = 0xD2511F53
_M1 = 0xCD9E8D57
_W0 = 0x9E3779B9
_W1 = 0xBB67AE85
_MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """Philox4x32 with 10 rounds on uint64 arrays holding 32-bit words.

    ctr: tuple of 4 arrays (broadcastable), key: tuple of 2 arrays.  Returns 4 arrays.
    One round multiplies words 0 and 2 by the two constants (64-bit products), and
    the new words are (hi(M1*c2) ^ c1 ^ k0, lo(M1*c2), hi(M0*c0) ^ c3 ^ k1, lo(M0*c0));
    the key is bumped by the Weyl constants between rounds.
    """
    c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint64) & np.uint64(_MASK) for c in ctr)
    k0, k1 = (np.asarray(k, dtype=np.uint64) & np.uint64(_MASK) for k in key)
    for r in range(10):
        if r > 0:
            k0 = (k0 + np.uint64(_W0)) & np.uint64(_MASK)
            k1 = (k1 + np.uint64(_W1)) & np.uint64(_MASK)
        p0 = np.uint64(_M0) * c0
        p1 = np.uint64(_M1) * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & np.uint64(_MASK)
        hi1, lo1 = p1 >> np.uint64(32), p1 & np.uint64(_MASK)
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def words_to_unit(x):
    """32-bit word -> u in (0,1): top 23 bits plus one half, scaled by 2^-23 (exact in FP32)."""
    x = np.asarray(x, dtype=np.uint64)
    return ((x >> np.uint64(9)).astype(np.float64) + 0.5) * 2.0 ** -23


def box_muller(ua, ub):
    """Box-Muller pair in FP64."""
    r = np.sqrt(-2.0 * np.log(ua))
    ang = 2.0 * np.pi * ub
    return r * np.cos(ang), r * np.sin(ang)


def prior_uniforms(key: int, counter0: int, B: int, V: int):
    """The four uniform streams u0..u3 [B, V/4] of the prior draw."""
    assert V % 4 == 0
    b = np.arange(B, dtype=np.uint64)[:, None] + np.uint64(counter0)
    j = np.arange(V // 4, dtype=np.uint64)[None, :]
    ctr = (j, b & np.uint64(_MASK), b >> np.uint64(32), np.zeros_like(j))
    key_t = (np.uint64(key & _MASK), np.uint64((key >> 32) & _MASK))
    return [words_to_unit(w) for w in philox4x32_10(ctr, key_t)]


def prior_normal(key: int, counter0: int, B: int, V: int) -> np.ndarray:
    """FP64 standard normals [B, V] as defined in the module header."""
    u0, u1, u2, u3 = prior_uniforms(key, counter0, B, V)
    za, zb = box_muller(u0, u1)
    zc, zd = box_muller(u2, u3)
    z = np.empty((B, V), dtype=np.float64)
    z[:, 0::4], z[:, 1::4], z[:, 2::4], z[:, 3::4] = za, zb, zc, zd
    return z


def log_prior(z) -> np.ndarray:
    """log r(z) for z of shape [B, ...]: independent N(0,1) per site, FP64."""
    z = np.asarray(z, dtype=np.float64).reshape(len(z), -1)
    V = z.shape[1]
    return -0.5 * np.sum(z * z, axis=1) - 0.5 * V * np.log(2.0 * np.pi)
