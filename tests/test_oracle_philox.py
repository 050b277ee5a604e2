"""Pins the oracle's Philox4x64-10 against numpy's independent implementation.

numpy's bit generator increments its 256-bit counter BEFORE each block, so
with counter c its first four raw outputs are Philox(key, c + 1); that
convention is derived here from a run starting at counter 0 and checked
again at a counter with a carry between words.
"""
import numpy as np
import pytest

from oracle.philox import mulhi64, philox4x64, philox4x64_vec, u24


def numpy_block(key, ctr_minus_one):
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64),
                          counter=np.array(ctr_minus_one, dtype=np.uint64))
    return tuple(int(v) for v in bg.random_raw(4))


KEYS = [(0, 0), (1, 2), (0xFFFFFFFFFFFFFFFF, 7), (12345, 0xDEADBEEFCAFEF00D)]


@pytest.mark.parametrize("key", KEYS)
def test_scalar_matches_numpy(key):
    rng = np.random.default_rng(5)
    for _ in range(20):
        c = [int(v) for v in rng.integers(0, 2**63, 4, dtype=np.uint64)]
        expect = numpy_block(key, c)
        got = philox4x64(key, (c[0] + 1, c[1], c[2], c[3]))
        assert got == expect


def test_counter_carry_convention():
    # counter word 0 at its maximum: numpy's increment carries into word 1
    key = (3, 4)
    expect = numpy_block(key, [2**64 - 1, 5, 6, 7])
    assert philox4x64(key, (0, 6, 6, 7)) == expect


@pytest.mark.parametrize("key", KEYS)
def test_vector_matches_scalar(key):
    rng = np.random.default_rng(11)
    C = rng.integers(0, 2**64 - 1, (64, 4), dtype=np.uint64)
    out = philox4x64_vec(key[0], key[1], C[:, 0], C[:, 1], C[:, 2], C[:, 3])
    for r in range(64):
        want = philox4x64(key, tuple(int(v) for v in C[r]))
        assert tuple(int(o[r]) for o in out) == want


def test_mulhi_and_u24():
    assert mulhi64(2**63, 10) == 5
    assert mulhi64(2**64 - 1, 7) == 6
    v = np.array([2**63, 2**64 - 1], dtype=np.uint64)
    assert list(mulhi64(v, np.uint64(10))) == [5, 9]
    assert u24(2**64 - 1) == (2**24 - 1) / 2**24
    assert u24(1 << 40) == 2.0 ** -24
