"""Philox4x64-10 counter-based generator, written from its published definition.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper starts each run from "slightly fluctuating initial conditions"
(Sec. 2.2, the paragraph after Eq. (5)) without naming a generator.  The noise
is drawn from Philox4x64 with 10 rounds (J. K. Salmon et al., "Parallel random
numbers: as easy as 1, 2, 3", SC'11): a 4x64-bit counter and a 2x64-bit key
go through ten rounds of two 64x64->128-bit multiplies with the Weyl key
schedule.  Pinned against ``numpy.random.Philox`` in the tests.

All arithmetic is vectorised numpy ``uint64``; the 128-bit product is formed
from 32-bit limbs.
"""
import numpy as np

M0 = np.uint64(0xD2E7470EE14C6C93)
M1 = np.uint64(0xCA5A826395121157)
W0 = np.uint64(0x9E3779B97F4A7C15)
W1 = np.uint64(0xBB67AE8584CAA73B)
_M32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def _mulhilo(a, b):
    """Return (hi, lo) of the 128-bit product of uint64 arrays a*b."""
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    a0, a1 = a & _M32, a >> _S32
    b0, b1 = b & _M32, b >> _S32
    p00 = a0 * b0
    p01 = a0 * b1
    p10 = a1 * b0
    p11 = a1 * b1
    mid = (p00 >> _S32) + (p01 & _M32) + (p10 & _M32)
    hi = p11 + (p01 >> _S32) + (p10 >> _S32) + (mid >> _S32)
    with np.errstate(over="ignore"):
        lo = a * b
    return hi, lo


def philox4x64_10(ctr, key):
    """One Philox4x64-10 block.

    ctr: sequence of 4 uint64 arrays (broadcastable), key: sequence of 2.
    Returns a list of 4 uint64 arrays.
    """
    c0, c1, c2, c3 = (np.asarray(c, dtype=np.uint64) for c in ctr)
    k0, k1 = (np.asarray(k, dtype=np.uint64) for k in key)
    with np.errstate(over="ignore"):
        for rnd in range(10):
            if rnd > 0:
                k0 = k0 + W0
                k1 = k1 + W1
            hi0, lo0 = _mulhilo(M0, c0)
            hi1, lo1 = _mulhilo(M1, c2)
            c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return [c0, c1, c2, c3]


def uniform_open(x):
    """Map uint64 words to doubles in the open interval (0, 1), exactly.

    The top 52 bits plus one half: u = (floor(x / 2^12) + 1/2) * 2^-52.
    Every step is exact in FP64, the smallest value is 2^-53 and the largest
    1 - 2^-53, so log(u) is finite and u never rounds to 1.
    """
    x = np.asarray(x, dtype=np.uint64)
    return ((x >> np.uint64(12)).astype(np.float64) + 0.5) * (2.0 ** -52)


def gaussian_pair(ctr, key):
    """Two independent standard normals per counter (Box-Muller, FP64).

    The first two words of the block give u1, u2; g_re = sqrt(-2 ln u1) cos(2 pi u2),
    g_im = sqrt(-2 ln u1) sin(2 pi u2).
    """
    blk = philox4x64_10(ctr, key)
    u1 = uniform_open(blk[0])
    u2 = uniform_open(blk[1])
    rad = np.sqrt(-2.0 * np.log(u1))
    ang = 2.0 * np.pi * u2
    return rad * np.cos(ang), rad * np.sin(ang)
