"""Counter-based Gaussian numbers for the sampling matrices (oracle side).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The method draws a Gaussian Omega (Section 3).  Both the oracle and the HIP
library implement the same published generator on their own, so that a whole
solve can be compared with identical random numbers:
  * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
    easy as 1, 2, 3", SC 2011): 10 rounds of two 32x32->64 multiplies by
    0xD2511F53 and 0xCD9E8D57 with a Weyl key schedule 0x9E3779B9, 0xBB67AE85;
  * two 53-bit uniforms per call, u = (a>>5 * 2^26 + b>>6) * 2^-53;
  * the Box-Muller transform (Box & Muller 1958): r = sqrt(-2 ln(1 - u1)),
    n0 = r cos(2 pi u2), n1 = r sin(2 pi u2).
Element (i, c) of a K x s matrix is normal number e = i*s + c of the stream:
counter (e >> 1, stream, 0, 0), key (seed_lo, seed_hi), branch e & 1.
"""
import numpy as np

_M0 = np.uint64(0xD2511F53)
_M1 = np.uint64(0xCD9E8D57)
_W0 = 0x9E3779B9
_W1 = 0xBB67AE85
_MASK = np.uint64(0xFFFFFFFF)


def philox4x32(c0, c1, c2, c3, k0, k1):
    """Philox4x32-10 on uint64 arrays holding 32-bit values."""
    c0, c1, c2, c3 = (np.asarray(x, np.uint64) & _MASK for x in (c0, c1, c2, c3))
    k0 = int(k0) & 0xFFFFFFFF
    k1 = int(k1) & 0xFFFFFFFF
    for _ in range(10):
        p0 = _M0 * c0
        p1 = _M1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ np.uint64(k0)), lo1, (hi0 ^ c3 ^ np.uint64(k1)), lo0
        k0 = (k0 + _W0) & 0xFFFFFFFF
        k1 = (k1 + _W1) & 0xFFFFFFFF
    return c0, c1, c2, c3


def philox_normal(K, s, seed, stream):
    """K x s standard normal matrix, element (i, c) = normal number i*s + c."""
    e = np.arange(K * s, dtype=np.uint64)
    ctr = e >> np.uint64(1)
    seed = int(seed) & 0xFFFFFFFFFFFFFFFF
    x0, x1, x2, x3 = philox4x32(ctr & _MASK, ctr >> np.uint64(32), np.uint64(stream), 0,
                                seed & 0xFFFFFFFF, seed >> 32)
    u1 = ((x0 >> np.uint64(5)).astype(np.float64) * 67108864.0 + (x1 >> np.uint64(6)).astype(np.float64)) * (2.0 ** -53)
    u2 = ((x2 >> np.uint64(5)).astype(np.float64) * 67108864.0 + (x3 >> np.uint64(6)).astype(np.float64)) * (2.0 ** -53)
    r = np.sqrt(-2.0 * np.log(1.0 - u1))
    th = 2.0 * np.pi * u2
    odd = (e & np.uint64(1)).astype(bool)
    out = np.where(odd, r * np.sin(th), r * np.cos(th))
    return out.reshape(K, s)
