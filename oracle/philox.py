"""Counter-based random numbers for the oracle.

The paper draws uniform samples R_f in [0, 1] throughout (Sec. IV: initial
loading by Box-Muller, Eq. (5) free-flight times, the null-collision selection
of Eq. (6), the impact parameter and azimuth of Eq. (10), the sputter yield and
emission laws of Sec. IV.B).  Both this oracle and the GPU path draw them from
one counter-based generator so that a particle's random numbers depend only on
(case, particle id, step, purpose) and not on thread or slot order.

Generator: Philox4x64-10 as published by Salmon, Moraes, Dror and Shaw,
"Parallel Random Numbers: As Easy as 1, 2, 3" (SC'11): ten rounds of two 64x64
-> 128-bit multiplications with the S-box/P-box wiring of the 4x64 variant and a
Weyl-sequence key schedule.  This module is an independent numpy implementation;
its output is pinned to numpy's own ``np.random.Philox`` (the same published
generator, library code) by ``tests/test_oracle_rng.py``.

Counter layout (shared contract with the GPU path, each side written from this
text):  counter = (c0, c1, c2, c3) = (particle id, step or event index as u64,
tag, aux), key = (seed, stream); tag = species * 256 + purpose.

Uniform map: each 64-bit output word w gives two uniforms in (0, 1),
    U_hi = ((w >> 41) + 0.5) * 2^-23,    U_lo = (((w >> 9) & (2^23 - 1)) + 0.5) * 2^-23,
so one call yields 8 uniforms U[0..7] = (hi(w0), lo(w0), hi(w1), ..., lo(w3)).
Every such value is exactly representable in FP32 and FP64, so FP32 and FP64
code see the same number.
"""
import numpy as np

M0 = np.uint64(0xD2E7470EE14C6C93)
M1 = np.uint64(0xCA5A826395121157)
W0 = np.uint64(0x9E3779B97F4A7C15)   # golden ratio
W1 = np.uint64(0xBB67AE8584CAA73B)   # sqrt(3) - 1
_M32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)

# species codes and purposes of the counter's tag word
SP_E, SP_I, SP_AL, SP_YIELD = 0, 1, 2, 3
INIT, SKIP, COLL, PARTNER, ION, CHILD = 1, 2, 3, 4, 5, 6
TP_SRC, TP_EVT = 16, 17
YIELD = 32


def tag(species, purpose):
    return species * 256 + purpose


def _u64(x, n=None):
    a = np.asarray(x)
    if a.dtype != np.uint64:
        a = a.astype(np.int64).astype(np.uint64) if a.dtype.kind == "i" else a.astype(np.uint64)
    if n is not None and a.ndim == 0:
        a = np.full(n, a, dtype=np.uint64)
    return a


def mulhilo64(a, b):
    """(hi, lo) words of the 128-bit product a*b, from four 32x32 partial products."""
    with np.errstate(over="ignore"):
        a0, a1 = a & _M32, a >> _S32
        b0, b1 = b & _M32, b >> _S32
        p00, p01, p10, p11 = a0 * b0, a0 * b1, a1 * b0, a1 * b1
        mid = (p00 >> _S32) + (p01 & _M32) + (p10 & _M32)
        hi = p11 + (p01 >> _S32) + (p10 >> _S32) + (mid >> _S32)
        lo = a * b
    return hi, lo


def philox4x64(c0, c1, c2, c3, k0, k1):
    """Philox4x64-10 block function, vectorised over any broadcastable inputs.

    Returns four uint64 arrays (the output words w0..w3)."""
    c0, c1, c2, c3 = (np.atleast_1d(_u64(c)) for c in (c0, c1, c2, c3))
    c0, c1, c2, c3 = np.broadcast_arrays(c0, c1, c2, c3)
    k0 = _u64(k0)
    k1 = _u64(k1)
    with np.errstate(over="ignore"):
        for r in range(10):
            if r > 0:
                k0 = k0 + W0
                k1 = k1 + W1
            hi0, lo0 = mulhilo64(M0, c0)
            hi1, lo1 = mulhilo64(M1, c2)
            c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def uniforms(words):
    """The 8 uniforms in (0, 1) of one Philox call, as an (n, 8) float64 array."""
    cols = []
    for w in words:
        cols.append(((w >> np.uint64(41)).astype(np.float64) + 0.5) * 2.0 ** -23)
        cols.append((((w >> np.uint64(9)) & np.uint64(0x7FFFFF)).astype(np.float64) + 0.5) * 2.0 ** -23)
    return np.stack(cols, axis=-1)


def draw(ids, index, tg, seed, stream, aux=0):
    """Uniforms for counter (ids, index, tag, aux) under key (seed, stream): (n, 8)."""
    return uniforms(philox4x64(ids, _u64(index), tg, aux, seed, stream))


def box_muller(ua, ub):
    """Two independent standard normals from two uniforms (Box and Muller, 1958)."""
    r = np.sqrt(-2.0 * np.log(ua))
    return r * np.cos(2.0 * np.pi * ub), r * np.sin(2.0 * np.pi * ub)


def maxwell_velocity(U, sigma):
    """3D Maxwellian velocity (n, 3) from uniforms U[:, 0:4]: two Box-Muller pairs,
    the first three normals scaled by sigma = sqrt(k_B T / m)."""
    n0, n1 = box_muller(U[:, 0], U[:, 1])
    n2, _ = box_muller(U[:, 2], U[:, 3])
    return np.stack([n0, n1, n2], axis=-1) * np.asarray(sigma)[..., None]
