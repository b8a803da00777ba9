"""FP64 reference of the seeded sensor-noise deviates (test infrastructure only).

Only the test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this module.  It shares no code with the GPU library.

Paper section III.A: the multichannel signals of the training set get additive
Gaussian sensor noise at a drawn signal-to-noise ratio.  The noise is a random
draw; for the GPU and this oracle to draw the same numbers, each side
implements one counter-based generator from its published definition:

* Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as
  easy as 1, 2, 3", SC 2011): a 128-bit counter (four 32-bit words) and a
  64-bit key (two words) pass through ten rounds.  A round multiplies word 0
  by 0xD2511F53 and word 2 by 0xCD9E8D57 into 64-bit products and returns
  (hi(word 2 product) ^ word 1 ^ key 0, lo(word 2 product),
   hi(word 0 product) ^ word 3 ^ key 1, lo(word 0 product));
  the key is raised by the Weyl constants (0x9E3779B9, 0xBB67AE85) between
  rounds.
* Box and Muller (1958): two uniforms u1 in (0, 1], u2 in [0, 1) give the two
  independent standard normals sqrt(-2 ln u1) cos(2 pi u2) and
  sqrt(-2 ln u1) sin(2 pi u2).

The library's convention (include/ism.h, ism_normal_deviates): the deviates of
room r, microphone m, samples 4j .. 4j+3 come from the Philox output words
(x0, x1, x2, x3) of counter (j, m, r, 0) and key (seed mod 2^32, seed >> 32);
a word x becomes the uniform ((x >> 9) + 1/2) 2^-23 (23 bits and the half: exact
in FP32); (x0, x1) give samples 4j, 4j+1 (cos, sin) and (x2, x3) samples 4j+2,
4j+3.  The deviates are therefore bounded by sqrt(48 ln 2) = 5.77 in magnitude.
"""
from __future__ import annotations

import numpy as np

M0, M1 = 0xD2511F53, 0xCD9E8D57
W0, W1 = 0x9E3779B9, 0xBB67AE85
MASK = 0xFFFFFFFF


def philox4x32_10(ctr, key):
    """Philox4x32 with 10 rounds (SC 2011 definition).  ctr: (N, 4) integers < 2^32;
    key: two integers < 2^32.  Returns (N, 4) uint64 holding the 32-bit output words."""
    c = np.array(ctr, dtype=np.uint64).reshape(-1, 4)
    c0, c1, c2, c3 = (c[:, i].copy() for i in range(4))
    k0, k1 = int(key[0]) & MASK, int(key[1]) & MASK
    for rnd in range(10):
        if rnd > 0:
            k0 = (k0 + W0) & MASK
            k1 = (k1 + W1) & MASK
        p0 = c0 * np.uint64(M0)        # exact: both factors below 2^32
        p2 = c2 * np.uint64(M1)
        hi0, lo0 = p0 >> np.uint64(32), p0 & np.uint64(MASK)
        hi2, lo2 = p2 >> np.uint64(32), p2 & np.uint64(MASK)
        c0, c1, c2, c3 = hi2 ^ c1 ^ np.uint64(k0), lo2, hi0 ^ c3 ^ np.uint64(k1), lo0
    return np.stack([c0, c1, c2, c3], axis=1)


def uniforms(words):
    """Uniforms in (0, 1) from 32-bit words: ((x >> 9) + 1/2) 2^-23 (exact in FP64 and FP32)."""
    return ((np.asarray(words, dtype=np.uint64) >> np.uint64(9)).astype(np.float64) + 0.5) * 2.0 ** -23


def box_muller(u1, u2):
    """Box-Muller pair (cos, sin) of standard normals from uniforms u1 in (0, 1], u2 in [0, 1)
    (the open interval (0, 1) here)."""
    rad = np.sqrt(-2.0 * np.log(u1))
    return rad * np.cos(2.0 * np.pi * u2), rad * np.sin(2.0 * np.pi * u2)


def deviates(seed, room, n_mics, n_samples):
    """Standard normal sensor-noise deviates z[m][n] of one room (m < n_mics, n < n_samples), in
    the library's counter layout (module docstring); FP64."""
    seed = int(seed)
    key = (seed & MASK, (seed >> 32) & MASK)
    nblk = (int(n_samples) + 3) // 4
    z = np.empty((int(n_mics), 4 * nblk))
    j = np.arange(nblk)
    for m in range(int(n_mics)):
        ctr = np.stack([j, np.full(nblk, m), np.full(nblk, int(room)), np.zeros(nblk, dtype=np.int64)], axis=1)
        u = uniforms(philox4x32_10(ctr, key))
        a, b = box_muller(u[:, 0], u[:, 1])
        c, d = box_muller(u[:, 2], u[:, 3])
        z[m, 0::4], z[m, 1::4], z[m, 2::4], z[m, 3::4] = a, b, c, d
    return z[:, :int(n_samples)]
