"""Pins of the Andersen-thermostat oracle (CPU).

Philox4x64-10 is checked against numpy's independent Philox bit generator
(the same published algorithm: numpy's raw outputs for counter c are the
block of counter c + 1); the collision rule and the Box-Muller normals
against their definitions: probability p per particle and step, standard
normal components, and draws that depend only on (seed, step, id)."""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import thermostat as T


def _numpy_block(key, ctr):
    """The four words numpy's Philox returns first for `ctr` (= block ctr + 1)."""
    bg = np.random.Philox(key=np.array(key, dtype=np.uint64), counter=np.array(ctr, dtype=np.uint64))
    return tuple(int(v) for v in bg.random_raw(4))


@pytest.mark.parametrize("key,ctr", [
    ((0, 0), (0, 0, 0, 0)),
    ((123456789, 987654321), (41, 7, 0, 0)),
    ((2**64 - 1, 2**63 + 5), (2**64 - 1, 3, 9, 2**64 - 1)),   # carry into word 1
    ((0x243F6A8885A308D3, 0x13198A2E03707344), (0xA4093822299F31D0, 0x082EFA98EC4E6C89, 1, 2)),
])
def test_philox_matches_numpy(key, ctr):
    c0, c1, c2, c3 = ctr
    nxt = c0 + 1
    c1 += nxt >> 64
    nxt &= (1 << 64) - 1
    assert T.philox4x64_10((nxt, c1, c2, c3), key) == _numpy_block(key, ctr)


def test_uniform53():
    assert T.uniform53(0) == 0.0
    assert T.uniform53((1 << 64) - 1) == 1.0 - 2.0**-53
    assert T.uniform53(1 << 63) == 0.5


def test_collision_probability_and_normals():
    p = 0.3
    hits, normals = 0, []
    trials = 20000
    for k in range(trials):
        hit, n = T.andersen_draw(seed=11, step=1 + k // 100, pid=k % 100, p=p)
        if hit:
            hits += 1
            normals.extend(n)
    # binomial: within 5 standard deviations
    assert abs(hits - p * trials) < 5 * math.sqrt(trials * p * (1 - p))
    z = np.array(normals)
    assert abs(z.mean()) < 5 / math.sqrt(z.size)
    assert abs(z.var() - 1.0) < 5 * math.sqrt(2.0 / z.size)
    assert stats.kstest(z, "norm").pvalue > 1e-4
    # the three components are uncorrelated
    c = np.corrcoef(z.reshape(-1, 3).T)
    assert np.max(np.abs(c - np.eye(3))) < 5 / math.sqrt(z.size / 3)


def test_never_and_always():
    for k in range(200):
        assert T.andersen_draw(3, 5, k, 0.0)[0] is False
        assert T.andersen_draw(3, 5, k, 1.0)[0] is True


def test_andersen_depends_on_ids_not_rows():
    r = np.random.Generator(np.random.PCG64(4))
    v = r.standard_normal((50, 3))
    ids = r.permutation(50)
    a, ha = T.andersen(v, ids, step=7, temperature=0.5, nu=20.0, dt=0.01, seed=9)
    perm = r.permutation(50)
    b, hb = T.andersen(v[perm], ids[perm], step=7, temperature=0.5, nu=20.0, dt=0.01, seed=9)
    assert ha == hb and 0 < ha < 50
    assert np.array_equal(a[perm], b)
    same = np.all(a == v, axis=1)
    assert same.sum() == 50 - ha          # untouched rows keep their velocity exactly
    # resampled components have variance T/m = 0.5 (loose: 3*ha samples)
    assert abs(np.var(a[~same]) - 0.5) < 0.35
