"""Pins for the oracle's counter-based generator (Philox4x64-10) and normals.

The external pin is numpy's independent Philox4x64-10 implementation: numpy
increments its counter before producing the first block, so a generator
constructed with counter c yields the block of counter c + 1.
"""
import numpy as np
import pytest
from scipy import stats

import oracle as O

M64 = (1 << 64) - 1


def _numpy_block(ctr, key):
    c = list(ctr)
    # step numpy's counter back by one (with borrow) so its pre-increment lands on ctr
    c0 = (c[0] - 1) & M64
    borrow = 1 if c[0] == 0 else 0
    c1 = (c[1] - borrow) & M64
    borrow = 1 if (borrow and c[1] == 0) else 0
    c2 = (c[2] - borrow) & M64
    borrow = 1 if (borrow and c[2] == 0) else 0
    c3 = (c[3] - borrow) & M64
    g = np.random.Philox(counter=np.array([c0, c1, c2, c3], dtype=np.uint64),
                         key=np.array(key, dtype=np.uint64))
    return [int(v) for v in g.random_raw(4)]


@pytest.mark.parametrize("ctr,key", [
    ((0, 0, 0, 0), (0, 0)),
    ((1, 0, 0, 0), (0, 0)),
    ((M64, M64, M64, M64), (M64, M64)),
    ((7, 3, 5, (3 << 8) | 1), (20130406, 1)),
    ((123456789, 42, 17, 4), (1, 0)),
    ((0x243F6A8885A308D3, 0x13198A2E03707344, 0xA4093822299F31D0, 0x082EFA98EC4E6C89),
     (0x452821E638D01377, 0xBE5466CF34E90C6C)),
])
def test_philox_matches_numpy(ctr, key):
    assert O.philox(ctr, key) == _numpy_block(ctr, key)


def test_philox_many_random_counters():
    rng = np.random.default_rng(5)
    for _ in range(200):
        ctr = [int(v) for v in rng.integers(0, 2**63, size=4, dtype=np.int64)]
        key = [int(v) for v in rng.integers(0, 2**63, size=2, dtype=np.int64)]
        assert O.philox(ctr, key) == _numpy_block(ctr, key)


def test_normals_are_standard_normal():
    z = np.concatenate([O.normals(3, 0, p, 1, 2, O.PROPOSAL, 9) for p in range(4000)])
    assert abs(z.mean()) < 4 * (1 / np.sqrt(z.size))
    assert abs(z.var() - 1) < 4 * np.sqrt(2 / z.size)
    assert stats.kstest(z, "norm").pvalue > 1e-3


def test_normals_depend_on_every_coordinate():
    base = O.normals(3, 0, 5, 1, 2, O.PROPOSAL, 4)
    for args in [(4, 0, 5, 1, 2), (3, 1, 5, 1, 2), (3, 0, 6, 1, 2), (3, 0, 5, 2, 2),
                 (3, 0, 5, 1, 3)]:
        assert not np.allclose(O.normals(*args, O.PROPOSAL, 4), base)
    assert not np.allclose(O.normals(3, 0, 5, 1, 2, O.PRIOR, 4), base)
    # prefix property: the first n normals do not depend on how many are asked for
    assert np.array_equal(O.normals(3, 0, 5, 1, 2, O.PROPOSAL, 9)[:4], base)
