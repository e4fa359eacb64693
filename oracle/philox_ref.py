"""Philox counter-based generator and the Gaussian noise drawn from it.

Test infrastructure only (see the package docstring).

Philox4xW-R is the generator of Salmon, Moraes, Dror and Shaw, "Parallel
random numbers: as easy as 1, 2, 3" (SC'11): a 4-word counter is mixed with a
2-word key by R rounds; each round multiplies words 0 and 2 by fixed odd
constants, keeps the high and low halves of the double-width products, XORs
the high halves with words 1/3 and the key, and permutes; the key is bumped
by two Weyl constants between rounds.  The constants below are the ones that
paper gives for W = 32 and W = 64.

The W = 64 instance is the same algorithm that ``numpy.random.Philox``
implements, which is what pins this code (the tests compare raw outputs).

Noise reading (the paper does not specify its generator): the Gaussian
increment of bead ``i`` at step ``t`` uses counter (i, t mod 2^32, t >> 32, 0)
and key (seed mod 2^32, seed >> 32) with Philox4x32-10; the four 32-bit words
become uniforms u_j = (w_j + 1/2) 2^-32 in (0, 1), and Box-Muller gives
xi_x, xi_y from (u0, u1) and xi_z from (u2, u3).
"""

from __future__ import annotations

import numpy as np

_CONSTANTS = {
    32: dict(mul=(0xD2511F53, 0xCD9E8D57), weyl=(0x9E3779B9, 0xBB67AE85)),
    64: dict(mul=(0xD2E7470EE14C6C93, 0xCA5A826395121157),
             weyl=(0x9E3779B97F4A7C15, 0xBB67AE8584CAA73B)),
}
_M32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def _mulhilo(a: np.ndarray, b: int, width: int):
    """High and low words of the 2W-bit product a*b (a: uint64 array holding W-bit words)."""
    a = a.astype(np.uint64)
    if width == 32:
        p = a * np.uint64(b)
        return p >> _S32, p & _M32
    # 64-bit words: schoolbook product on 32-bit halves (numpy wraps modulo 2^64)
    a0, a1 = a & _M32, a >> _S32
    b0, b1 = np.uint64(b & 0xFFFFFFFF), np.uint64(b >> 32)
    p00, p01, p10, p11 = a0 * b0, a0 * b1, a1 * b0, a1 * b1
    mid = (p00 >> _S32) + (p01 & _M32) + (p10 & _M32)
    hi = p11 + (p01 >> _S32) + (p10 >> _S32) + (mid >> _S32)
    lo = (mid << _S32) | (p00 & _M32)
    return hi, lo


def philox4(counter, key, width: int = 32, rounds: int = 10) -> np.ndarray:
    """Philox4xW-R block function.

    counter: (n, 4) unsigned words; key: (2,) words.  Returns (n, 4) uint64
    arrays holding W-bit words.
    """
    c = np.array(counter, dtype=np.uint64).reshape(-1, 4)
    mask = np.uint64((1 << width) - 1) if width < 64 else np.uint64(0xFFFFFFFFFFFFFFFF)
    c0, c1, c2, c3 = (c[:, j].copy() & mask for j in range(4))
    k0 = int(key[0]) & int(mask)
    k1 = int(key[1]) & int(mask)
    m0, m1 = _CONSTANTS[width]["mul"]
    w0, w1 = _CONSTANTS[width]["weyl"]
    full = (1 << width) - 1
    for r in range(rounds):
        if r > 0:
            k0 = (k0 + w0) & full
            k1 = (k1 + w1) & full
        hi0, lo0 = _mulhilo(c0, m0, width)
        hi1, lo1 = _mulhilo(c2, m1, width)
        c0, c1, c2, c3 = ((hi1 ^ c1 ^ np.uint64(k0)) & mask, lo1 & mask,
                          (hi0 ^ c3 ^ np.uint64(k1)) & mask, lo0 & mask)
    return np.stack([c0, c1, c2, c3], axis=1)


def philox4x32(counter, key) -> np.ndarray:
    """Philox4x32-10; returns (n, 4) uint32."""
    return philox4(counter, key, 32, 10).astype(np.uint32)


def noise_counters(ids: np.ndarray, step: int) -> np.ndarray:
    ids = np.asarray(ids, dtype=np.uint64)
    n = ids.shape[0]
    ctr = np.zeros((n, 4), dtype=np.uint64)
    ctr[:, 0] = ids & _M32
    ctr[:, 1] = np.uint64(step & 0xFFFFFFFF)
    ctr[:, 2] = np.uint64((step >> 32) & 0xFFFFFFFF)
    return ctr


def uniforms(words: np.ndarray) -> np.ndarray:
    """Map 32-bit words to (0, 1): u = (w + 1/2) / 2^32 (exact in float64)."""
    return (words.astype(np.float64) + 0.5) * (2.0 ** -32)


def gaussian_noise(ids: np.ndarray, step: int, seed: int) -> np.ndarray:
    """Unit Gaussian increments xi (n, 3) for beads ``ids`` at step ``step``."""
    key = (seed & 0xFFFFFFFF, (seed >> 32) & 0xFFFFFFFF)
    w = philox4x32(noise_counters(ids, step), key)
    u = uniforms(w)
    r01 = np.sqrt(-2.0 * np.log(u[:, 0]))
    r23 = np.sqrt(-2.0 * np.log(u[:, 2]))
    xi = np.empty((w.shape[0], 3))
    xi[:, 0] = r01 * np.cos(2.0 * np.pi * u[:, 1])
    xi[:, 1] = r01 * np.sin(2.0 * np.pi * u[:, 1])
    xi[:, 2] = r23 * np.cos(2.0 * np.pi * u[:, 3])
    return xi
