"""Philox4x32-10 counter-based generator and the Box-Muller normals drawn from it.

Test infrastructure: only tests, the smoke check and the CPU-baseline timing use
this package.

Philox4x32-10 follows its published definition (Salmon, Moraes, Dror & Shaw,
"Parallel random numbers: as easy as 1, 2, 3", SC'11): a 4-word counter and a
2-word key; each of the 10 rounds multiplies counter words 0 and 2 by the
constants 0xD2511F53 and 0xCD9E8D57 into 64-bit products, and the new counter is
(hi(P1) ^ c1 ^ k0, lo(P1), hi(P0) ^ c3 ^ k1, lo(P0)); the key is bumped by the
Weyl constants (0x9E3779B9, 0xBB67AE85) between rounds.

The paper does not say how the correlated-noise draw gets its randomness; the
reading used here (also implemented, separately, by the device code):

* key = (seed & 0xffffffff, segment id),
  counter = (Fourier mode k, iter & 0xffffffff, iter >> 32, seed >> 32);
* u_i = (x_i + 1/2) 2^-32 for the four output words;
* Box-Muller: z0 + i z1 = sqrt(-2 ln u0) exp(2 pi i u1), z2 + i z3 likewise from
  (u2, u3).
"""
import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint64(0x9E3779B9)
W1 = np.uint64(0xBB67AE85)
MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32-10.  All arguments broadcast; returns 4 uint32 arrays."""
    c0, c1, c2, c3, k0, k1 = [np.asarray(a, dtype=np.uint64) & MASK
                              for a in np.broadcast_arrays(c0, c1, c2, c3, k0, k1)]
    for rnd in range(10):
        p0 = M0 * c0
        p1 = M1 * c2
        n0 = (p1 >> np.uint64(32)) ^ c1 ^ k0
        n1 = p1 & MASK
        n2 = (p0 >> np.uint64(32)) ^ c3 ^ k1
        n3 = p0 & MASK
        c0, c1, c2, c3 = n0 & MASK, n1, n2 & MASK, n3
        if rnd < 9:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
    return [c.astype(np.uint32) for c in (c0, c1, c2, c3)]


def mode_words(seed, seg, it, k):
    """The four Philox words for Fourier modes ``k`` of segment ``seg``."""
    seed = int(seed)
    it = int(it)
    k = np.asarray(k, dtype=np.uint64)
    return philox4x32_10(k, it & 0xFFFFFFFF, (it >> 32) & 0xFFFFFFFF,
                         (seed >> 32) & 0xFFFFFFFF, seed & 0xFFFFFFFF, int(seg))


def uniforms(words):
    return [(w.astype(np.float64) + 0.5) * 2.0 ** -32 for w in words]


def box_muller(u0, u1):
    rad = np.sqrt(-2.0 * np.log(u0))
    return rad * np.cos(2.0 * np.pi * u1), rad * np.sin(2.0 * np.pi * u1)


def mode_normals(seed, seg, it, k):
    """Four standard normals (z0, z1, z2, z3) per mode k."""
    u0, u1, u2, u3 = uniforms(mode_words(seed, seg, it, k))
    z0, z1 = box_muller(u0, u1)
    z2, z3 = box_muller(u2, u3)
    return z0, z1, z2, z3
