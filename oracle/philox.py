"""Counter-based Gaussian draws for the Lanczos start vectors.

The estimator of the wanted threshold needs random start vectors.  So that the
oracle and the HIP path draw the *same* vectors without sharing code, both
implement Philox4x32-10 from its published definition (Salmon, Moraes, Dror,
Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC'11) and the
Box-Muller transform.  This file is the oracle's own implementation.

Stream layout (identical on both sides): entry i of vector ``stream`` uses the
pair index p = i // 2; counter = (p mod 2^32, p >> 32, stream, 0),
key = (seed mod 2^32, seed >> 32).  The four output words give two 53-bit
uniforms u1 = ((w0 >> 5) 2^26 + (w1 >> 6) + 1/2) / 2^53 and u2 likewise from
(w2, w3); entry 2p is sqrt(-2 ln u1) cos(2 pi u2), entry 2p+1 the sine.
"""
import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint64(0x9E3779B9)
W1 = np.uint64(0xBB67AE85)
MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr, key):
    """Philox4x32 with 10 rounds.  ctr: (..., 4) uint32-valued, key: (..., 2)."""
    c = [np.asarray(ctr[..., i], dtype=np.uint64) for i in range(4)]
    k0 = np.asarray(key[..., 0], dtype=np.uint64)
    k1 = np.asarray(key[..., 1], dtype=np.uint64)
    for r in range(10):
        p0 = M0 * c[0]
        p1 = M1 * c[2]
        hi0, lo0 = p0 >> np.uint64(32), p0 & MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & MASK
        c = [(hi1 ^ c[1] ^ k0) & MASK, lo1, (hi0 ^ c[3] ^ k1) & MASK, lo0]
        if r < 9:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
    return np.stack(c, axis=-1).astype(np.uint32)


def gaussian(seed, stream, n):
    """n standard normal draws of the given stream (layout in the module docstring)."""
    npair = (n + 1) // 2
    p = np.arange(npair, dtype=np.uint64)
    ctr = np.zeros((npair, 4), dtype=np.uint64)
    ctr[:, 0] = p & MASK
    ctr[:, 1] = p >> np.uint64(32)
    ctr[:, 2] = np.uint64(stream) & MASK
    seed = np.uint64(seed)
    key = np.zeros((npair, 2), dtype=np.uint64)
    key[:, 0] = seed & MASK
    key[:, 1] = seed >> np.uint64(32)
    w = philox4x32_10(ctr, key).astype(np.uint64)
    scale = 2.0 ** -53
    u1 = ((w[:, 0] >> np.uint64(5)).astype(np.float64) * 67108864.0
          + (w[:, 1] >> np.uint64(6)).astype(np.float64) + 0.5) * scale
    u2 = ((w[:, 2] >> np.uint64(5)).astype(np.float64) * 67108864.0
          + (w[:, 3] >> np.uint64(6)).astype(np.float64) + 0.5) * scale
    rad = np.sqrt(-2.0 * np.log(u1))
    z = np.empty(2 * npair)
    z[0::2] = rad * np.cos(2.0 * np.pi * u2)
    z[1::2] = rad * np.sin(2.0 * np.pi * u2)
    return z[:n]
