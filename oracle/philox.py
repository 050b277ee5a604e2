"""Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
easy as 1, 2, 3", SC'11), written from its published definition.

The paper does not say which generator its random sampling uses; every
random draw of the method (first-pass permutation, second-pass attempts,
factor initialisation, cluster representatives) is taken from this
counter-based generator so that the oracle and the GPU draw identical
numbers from (key, counter) alone.

One round maps counter (c0, c1, c2, c3) under key (k0, k1) to
    (hi(M1*c2) ^ c1 ^ k0,  lo(M1*c2),  hi(M0*c0) ^ c3 ^ k1,  lo(M0*c0))
and the key is bumped by the Weyl constants (W0, W1) between rounds.

Pinned by: bit equality with ``numpy.random.Philox`` raw output
(tests/test_oracle_philox.py).  Two implementations live here, a scalar one
on Python integers (the definition written out) and a vectorised one on
uint64 arrays; both are pinned.
"""
import numpy as np

M0 = 0xD2E7470EE14C6C93
M1 = 0xCA5A826395121157
W0 = 0x9E3779B97F4A7C15
W1 = 0xBB67AE8584CAA73B
MASK64 = (1 << 64) - 1
ROUNDS = 10

# Counter tags: the third counter word separates the method's random streams.
TAG_PASS1 = 1   # first-pass Feistel round function
TAG_PASS2 = 2   # second-pass attempts
TAG_INITX = 3   # initial X of the completion
TAG_INITY = 4   # initial Y of the completion
TAG_REP = 5     # cluster representative pick


def philox4x64(key, ctr, rounds=ROUNDS):
    """Scalar Philox4x64 on Python ints: key (k0, k1), ctr (c0..c3) -> 4 words."""
    k0, k1 = key[0] & MASK64, key[1] & MASK64
    c0, c1, c2, c3 = (c & MASK64 for c in ctr)
    for r in range(rounds):
        if r > 0:
            k0 = (k0 + W0) & MASK64
            k1 = (k1 + W1) & MASK64
        p0 = M0 * c0
        p1 = M1 * c2
        hi0, lo0 = p0 >> 64, p0 & MASK64
        hi1, lo1 = p1 >> 64, p1 & MASK64
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return (c0, c1, c2, c3)


_U32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def _mulhilo64(a, b):
    """Full 64x64 -> 128-bit product of uint64 arrays, as (hi, lo), from
    32-bit limbs (schoolbook multiplication)."""
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    a_lo, a_hi = a & _U32, a >> _S32
    b_lo, b_hi = b & _U32, b >> _S32
    ll = a_lo * b_lo
    lh = a_lo * b_hi
    hl = a_hi * b_lo
    hh = a_hi * b_hi
    mid = (ll >> _S32) + (lh & _U32) + (hl & _U32)
    lo = (ll & _U32) | ((mid & _U32) << _S32)
    hi = hh + (lh >> _S32) + (hl >> _S32) + (mid >> _S32)
    return hi, lo


def philox4x64_vec(k0, k1, c0, c1, c2, c3, rounds=ROUNDS):
    """Vectorised Philox4x64 over broadcastable uint64 arrays."""
    with np.errstate(over="ignore"):
        k0 = np.asarray(k0, dtype=np.uint64) + np.uint64(0)
        k1 = np.asarray(k1, dtype=np.uint64) + np.uint64(0)
        c0, c1, c2, c3 = np.broadcast_arrays(*(np.asarray(c, dtype=np.uint64) for c in (c0, c1, c2, c3)))
        c0, c1, c2, c3 = (c.copy() for c in (c0, c1, c2, c3))
        m0 = np.uint64(M0)
        m1 = np.uint64(M1)
        for r in range(rounds):
            if r > 0:
                k0 = k0 + np.uint64(W0)
                k1 = k1 + np.uint64(W1)
            hi0, lo0 = _mulhilo64(m0, c0)
            hi1, lo1 = _mulhilo64(m1, c2)
            c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


def mulhi64(r, n):
    """floor(r * n / 2^64): maps a uniform 64-bit word onto [0, n)."""
    if isinstance(r, (int, np.integer)) and isinstance(n, (int, np.integer)):
        return (int(r) * int(n)) >> 64
    hi, _ = _mulhilo64(r, n)
    return hi


def u24(r):
    """Top 24 bits of a 64-bit word as an exact float in [0, 1)."""
    if isinstance(r, (int, np.integer)):
        return float(int(r) >> 40) * 2.0 ** -24
    return (np.asarray(r, dtype=np.uint64) >> np.uint64(40)).astype(np.float64) * 2.0 ** -24
