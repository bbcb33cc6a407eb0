"""Pins of the oracle's array digest.

The digest of an array a is the sum over i of the low 64 bits (word0 | word1 << 32)
of the Philox4x32-10 block at counter (i, a_i, 0xD16E57, 0) under the zero key,
modulo 2^64.  The expected values are summed here from rocRAND's Philox (its
host-callable header, compiled for the CPU), which shares nothing with the
oracle; the remaining tests check the properties the check-sum is used for.
"""
import numpy as np
import pytest

import oracle
from tests.test_oracle_philox import _rocrand_blocks

TAG = 0xD16E57


def _expected(vals):
    rows = [[i, int(v) & 0xFFFFFFFF, TAG, 0, 0, 0] for i, v in enumerate(vals)]
    blocks = _rocrand_blocks(rows)
    return sum(b[0] | (b[1] << 32) for b in blocks) % 2**64


def test_digest_matches_rocrand():
    rng = np.random.default_rng(5804)
    u8 = rng.integers(0, 256, size=300, dtype=np.uint8)
    # rocRAND takes counter words 0-1 as one 64-bit offset times 4: values stay below 2^30
    i32 = rng.integers(0, 2**30, size=200, dtype=np.int64).astype(np.int32)
    assert oracle.digest(u8) == _expected(u8)
    assert oracle.digest(i32) == _expected(i32)
    states = rng.integers(0, 3, size=257, dtype=np.uint8)
    assert oracle.digest(states) == _expected(states)


def test_digest_properties():
    assert oracle.digest(np.zeros(0, np.uint8)) == 0
    a = np.arange(1000, dtype=np.int32)
    d = oracle.digest(a)
    # a change in one element changes it
    b = a.copy()
    b[7] = 8
    assert oracle.digest(b) != d
    # index-keyed: swapping two different values changes it
    c = a.copy()
    c[[3, 4]] = c[[4, 3]]
    assert oracle.digest(c) != d
    # uint8 and int32 arrays of the same values agree (values are taken as uint32)
    s = np.array([0, 1, 2, 1, 0], np.uint8)
    assert oracle.digest(s) == oracle.digest(s.astype(np.int32))
    # negative labels use their two's-complement bits
    neg = np.array([-1, 5], np.int32)
    assert oracle.digest(neg) != oracle.digest(np.array([0, 5], np.int32))
    with pytest.raises(TypeError):
        oracle.digest(np.zeros(3, np.float32))
