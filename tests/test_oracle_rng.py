"""Pins of the oracle's counter-based Gaussian generator (oracle/rng.py): the
published Philox4x32-10 known answers, and the distribution of the Box-Muller
normals built on it."""
import os

import numpy as np
from scipy import stats

from oracle import rng

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        w = [int(t, 16) for t in line.split()]
        rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


def test_philox_known_answers():
    rows = _kat()
    assert len(rows) == 3
    for ctr, key, out in rows:
        got = rng.philox4x32_10(np.array(ctr), key)
        assert [int(v) for v in got] == out


def test_philox_vectorised_over_counters():
    rows = _kat()
    ctr = np.array([r[0] for r in rows[:1]] * 3)
    got = rng.philox4x32_10(ctr, rows[0][1])
    assert all([int(v) for v in g] == rows[0][2] for g in got)


def test_normals_are_standard_normal():
    z = rng.normal(1234, 200001)
    assert z.shape == (200001,)
    assert abs(z.mean()) < 5 * (1 / np.sqrt(z.size))
    assert abs(z.var() - 1.0) < 5 * np.sqrt(2.0 / z.size)
    assert stats.kstest(z, "norm").pvalue > 1e-3
    # pairs are independent: the correlation of consecutive draws is at noise level
    c = np.corrcoef(z[0:-1:2], z[1::2])[0, 1]
    assert abs(c) < 5 / np.sqrt(z.size / 2)


def test_streams_differ_by_seed_and_prefix_is_stable():
    a = rng.normal(7, 1001)
    b = rng.normal(7, 64)
    assert np.array_equal(a[:64], b)
    assert not np.allclose(rng.normal(8, 64), b)
    # a 64-bit seed uses both key words
    assert not np.allclose(rng.normal(7 + (1 << 32), 64), b)


def test_gaussian_matrix_is_row_major():
    M = rng.gaussian_matrix(3, 5, 4)
    assert np.array_equal(M.reshape(-1), rng.normal(3, 20))
