"""Counter-based normal generator of the training data, CPU side.

TEST INFRASTRUCTURE ONLY (oracle): only the tests, the smoke check and the
benchmark's CPU-baseline leg may import it.  It shares no code with the GPU
library; both sides implement the same published generator from its
definition, so that the random x of the training triples (section 3.4,
eq. 3.8: x drawn from a normal distribution) can be drawn on the device and
reproduced here.

Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as
easy as 1, 2, 3", SC 2011): a 128-bit counter (four 32-bit words) and a
64-bit key; each of ten rounds multiplies words 0 and 2 by the constants
0xD2511F53 and 0xCD9E8D57 into 64-bit products, and the new counter is
(hi(word 2 product) ^ word 1 ^ key 0, lo(word 2 product),
 hi(word 0 product) ^ word 3 ^ key 1, lo(word 0 product));
between rounds the key words grow by 0x9E3779B9 and 0xBB67AE85.

Normals of sample s at point p: the block of counter (p, s_lo, s_hi, 0)
under key (seed_lo, seed_hi); its words a, c give u1 = (a + 1) 2^-32 in
(0, 1] and u2 = c 2^-32, and Box-Muller gives
Re x = sqrt(-2 ln u1) cos(2 pi u2), Im x = sqrt(-2 ln u1) sin(2 pi u2).
"""
from __future__ import annotations

import numpy as np

M0, M1 = np.uint64(0xD2511F53), np.uint64(0xCD9E8D57)
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr, key):
    """ctr: uint32-valued array [..., 4]; key: (k0, k1) ints.  Returns the
    uint32 output block [..., 4] (as uint64 values)."""
    c = [np.asarray(ctr, dtype=np.uint64)[..., i] & MASK for i in range(4)]
    k0, k1 = int(key[0]) & 0xFFFFFFFF, int(key[1]) & 0xFFFFFFFF
    for r in range(10):
        if r > 0:
            k0 = (k0 + W0) & 0xFFFFFFFF
            k1 = (k1 + W1) & 0xFFFFFFFF
        p0 = M0 * c[0]
        p1 = M1 * c[2]
        c = [(p1 >> np.uint64(32)) ^ c[1] ^ np.uint64(k0), p1 & MASK,
             (p0 >> np.uint64(32)) ^ c[3] ^ np.uint64(k1), p0 & MASK]
    return np.stack(c, axis=-1)


def normals(seed, index, npts):
    """complex128 [npts]: the complex normal x of sample `index` at points
    0 .. npts - 1 (FP64 Box-Muller)."""
    p = np.arange(npts, dtype=np.uint64)
    s = int(index)
    ctr = np.stack([p, np.full_like(p, s & 0xFFFFFFFF), np.full_like(p, (s >> 32) & 0xFFFFFFFF),
                    np.zeros_like(p)], axis=-1)
    o = philox4x32_10(ctr, (int(seed) & 0xFFFFFFFF, (int(seed) >> 32) & 0xFFFFFFFF))
    u1 = (o[:, 0].astype(np.float64) + 1.0) * 2.0 ** -32
    u2 = o[:, 1].astype(np.float64) * 2.0 ** -32
    rad = np.sqrt(-2.0 * np.log(u1))
    return rad * np.cos(2.0 * np.pi * u2) + 1j * rad * np.sin(2.0 * np.pi * u2)


def sample_x(seed, index, n):
    """The [n, n] complex x of one training sample, rounded to complex64 as
    the device stores it."""
    z = normals(seed, index, n * n).reshape(n, n)
    return (z.real.astype(np.float32) + 1j * z.imag.astype(np.float32)).astype(np.complex64)
