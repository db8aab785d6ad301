"""Counter-based white noise, float64 (oracle).

Test infrastructure only (see the package header).

The paper draws the initial Gaussian modes from a seed (design section:
derivatives are taken with respect to these modes).  Where the noise cannot
be handed to both sides as an array (a served request carries only its
seed), each side implements the same counter-based generator from its
published definition:

  Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
  easy as 1, 2, 3", SC 2011): a 4 x 64-bit counter and a 2 x 64-bit key;
  each of 10 rounds multiplies counter words 0 and 2 by two fixed odd
  constants into 128-bit products and mixes their halves with words 1, 3
  and the key; the key is advanced by two Weyl constants between rounds.

Recipe of the noise (shared with the device kernel):
  key   = (seed mod 2^64, seed >> 64)
  block c (c = 0, 1, ...) uses counter (c + 1, 0, 0, 0) and gives words
        w0..w3; this is the order of numpy's Philox(key=seed).random_raw()
  uniforms u_j = (w_j >> 11) 2^-53 in [0, 1)
  Box-Muller: r = sqrt(-2 ln(1 - u0)), z[4c] = r cos(2 pi u1),
        z[4c+1] = r sin(2 pi u1); the same with (u2, u3) for z[4c+2],
        z[4c+3]
  element i of the Np^3 lattice (C order) is z[i].

Pins (tests/test_oracle_rng.py): raw words bitwise equal to numpy's
Philox random_raw for several keys; mean, variance and a flat power
spectrum of the normals.
"""
from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2E7470EE14C6C93)
M1 = np.uint64(0xCA5A826395121157)
W0 = np.uint64(0x9E3779B97F4A7C15)
W1 = np.uint64(0xBB67AE8584CAA73B)
_LO32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def _mulhilo(a, b):
    """128-bit product of uint64 arrays a * b (b scalar): (hi, lo)."""
    a_lo, a_hi = a & _LO32, a >> _S32
    b_lo, b_hi = b & _LO32, b >> _S32
    ll = a_lo * b_lo
    lh = a_lo * b_hi
    hl = a_hi * b_lo
    hh = a_hi * b_hi
    mid = (ll >> _S32) + (lh & _LO32) + (hl & _LO32)
    lo = (ll & _LO32) | ((mid & _LO32) << _S32)
    hi = hh + (lh >> _S32) + (hl >> _S32) + (mid >> _S32)
    return hi, lo


def philox4x64(counter, key, rounds=10):
    """Philox4x64 over a batch: counter uint64 [4][n], key (k0, k1)."""
    c0, c1, c2, c3 = (np.array(v, dtype=np.uint64) for v in counter)
    k0, k1 = np.uint64(key[0]), np.uint64(key[1])
    with np.errstate(over="ignore"):
        for r in range(rounds):
            if r > 0:
                k0 = k0 + W0
                k1 = k1 + W1
            hi0, lo0 = _mulhilo(c0, M0)
            hi1, lo1 = _mulhilo(c2, M1)
            c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def raw_words(seed: int, n: int) -> np.ndarray:
    """The first n 64-bit words of the stream keyed by seed."""
    nblk = (n + 3) // 4
    c = np.arange(1, nblk + 1, dtype=np.uint64)
    z = np.zeros(nblk, dtype=np.uint64)
    key = (seed & 0xFFFFFFFFFFFFFFFF, seed >> 64)
    w = philox4x64((c, z, z, z), key)
    return np.stack(w, axis=1).reshape(-1)[:n]


def white_noise(np_side: int, seed: int) -> np.ndarray:
    """N(0,1) noise [Np][Np][Np] by the recipe above, float64."""
    n = np_side ** 3
    w = raw_words(seed, ((n + 3) // 4) * 4).reshape(-1, 4)
    u = (w >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    out = np.empty((w.shape[0], 4))
    for a, b in ((0, 1), (2, 3)):
        r = np.sqrt(-2.0 * np.log1p(-u[:, a]))
        out[:, a] = r * np.cos(2.0 * np.pi * u[:, b])
        out[:, b] = r * np.sin(2.0 * np.pi * u[:, b])
    return out.reshape(-1)[:n].reshape((np_side,) * 3)
