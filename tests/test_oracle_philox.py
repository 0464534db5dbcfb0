"""Pins of the oracle's counter-based noise stream.

Philox4x64-10 is checked bit-exactly against the known-answer vectors
published with the Random123 library (tests/golden) and against numpy's
independent implementation; the Gaussian and uniform maps against their
moments.  The paper draws its Brownian forces from uniform doubles (Eq. 2,
Section 4 "Generation of Random Numbers"); the Gaussian form has the same
covariance.
"""
import os

import numpy as np
import pytest
from numpy.random import Philox

from oracle import oracle as o

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x64_10_kat.txt")
M64 = 2**64 - 1


def _kat():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        v = [int(t, 16) for t in line.split()]
        rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,out", _kat())
def test_published_known_answers(ctr, key, out):
    assert [int(w) for w in o.philox(ctr, key)] == out


def _numpy_block(ctr, key):
    # numpy's Philox increments its 256-bit counter before each block, so
    # start it one below the wanted counter.
    c = list(ctr)
    i = 0
    while True:
        if c[i] > 0:
            c[i] -= 1
            break
        c[i] = M64
        i += 1
    g = Philox(counter=np.array(c, dtype=np.uint64), key=np.array(list(key), dtype=np.uint64))
    return [int(w) for w in g.random_raw(4)]


def test_bit_exact_vs_numpy_random_counters():
    rng = np.random.default_rng(7)
    for _ in range(200):
        ctr = [int(v) for v in rng.integers(0, 2**63, size=4, dtype=np.int64)]
        ctr[0] *= 2  # use the full 64-bit range in word 0
        key = [int(v) for v in rng.integers(0, 2**63, size=2, dtype=np.int64)]
        assert [int(w) for w in o.philox(ctr, key)] == _numpy_block(ctr, key)


def test_noise_stream_layout_matches_philox_blocks():
    p = o.make_params(11, seed=12345, chain_id=678)
    n = 3 * p.n_beads
    step = 42
    z = o.noise(p, step, n)
    # uniform mode exposes the raw u01 map: element e = lane e%4 of block e//4
    pu = o.make_params(11, seed=12345, chain_id=678, noise=o.NOISE_UNIFORM_PAPER)
    zu = o.noise(pu, step, n)
    for e in range(n):
        w = _numpy_block([e // 4, step, 0, 0], [12345, 678])[e % 4]
        u = ((w >> 11) + 0.5) * 2.0**-53
        assert zu[e] == 2.0 * u - 1.0
    # Gaussian mode: Box-Muller on lane pairs
    for blk in range((n + 3) // 4):
        w = _numpy_block([blk, step, 0, 0], [12345, 678])
        u = [((v >> 11) + 0.5) * 2.0**-53 for v in w]
        for pr in range(2):
            rad = np.sqrt(-2.0 * np.log(u[2 * pr]))
            ang = 2.0 * np.pi * u[2 * pr + 1]
            for lane, val in ((2 * pr, rad * np.cos(ang)), (2 * pr + 1, rad * np.sin(ang))):
                e = 4 * blk + lane
                if e < n:
                    assert abs(z[e] - val) <= 1e-15 * max(1.0, abs(val))


def test_gaussian_moments():
    p = o.make_params(2, seed=3, chain_id=1)
    n = 2_000_000
    z = o.noise(p, 5, n)
    m, v = z.mean(), z.var()
    k = ((z - m) ** 4).mean() / v**2
    assert abs(m) < 5 * np.sqrt(1.0 / n)
    assert abs(v - 1.0) < 5 * np.sqrt(2.0 / n)
    assert abs(k - 3.0) < 5 * np.sqrt(24.0 / n)


def test_uniform_paper_moments():
    # Eq. 2: components uniform on [-1, 1]: mean 0, variance 1/3
    p = o.make_params(2, seed=3, chain_id=1, noise=o.NOISE_UNIFORM_PAPER)
    n = 1_000_000
    z = o.noise(p, 9, n)
    assert z.min() > -1.0 and z.max() < 1.0
    assert abs(z.mean()) < 5 * np.sqrt((1 / 3) / n)
    assert abs(z.var() - 1 / 3) < 5 * np.sqrt((1 / 5 - 1 / 9) / n)


def test_streams_independent_across_chain_and_step():
    n = 200_000
    a = o.noise(o.make_params(2, seed=1, chain_id=0), 0, n)
    b = o.noise(o.make_params(2, seed=1, chain_id=1), 0, n)
    c = o.noise(o.make_params(2, seed=1, chain_id=0), 1, n)
    for u, v in ((a, b), (a, c), (b, c)):
        r = np.corrcoef(u, v)[0, 1]
        assert abs(r) < 5 / np.sqrt(n)
