"""Pins of the oracle's seeded grain placement (the paper's cluster of 44
grains is known only from a figure, Sec. II; the workloads stand in for it with
seeded clusters): uniform in a sphere by rejection, a minimum separation from
the grains placed before, Philox(g, t, 7, 0) words 0..2 for candidate t of
grain g, proposing c + R (2u - 1) with u = (w + 1/2) 2^-32."""
import numpy as np
import pytest
from scipy import stats

import oracle


def test_first_grain_is_the_first_candidate_inside():
    seed, c, R = 12345, np.array([10.0, 20.0, 30.0]), 4.0
    got = oracle.place_grains(seed, 1, c, R, 0.0)[0]
    key = [seed & 0xffffffff, seed >> 32]
    for t in range(100):
        w = oracle.philox4x32_10([0, t, 7, 0], key)[:3]
        p = c + R * (2.0 * ((np.array(w, float) + 0.5) * 2.0 ** -32) - 1.0)
        if np.sum((p - c) ** 2) <= R * R:
            break
    assert np.array_equal(got, p)


def test_sphere_separation_and_determinism():
    c = np.array([32.0, 32.0, 231.6])
    g = oracle.place_grains(1, 8, c, 10.0, 4.0)
    assert np.all(np.sum((g - c) ** 2, axis=1) <= 100.0)
    d = np.sqrt(((g[:, None] - g[None]) ** 2).sum(-1))
    assert d[~np.eye(8, dtype=bool)].min() >= 4.0
    assert np.array_equal(g, oracle.place_grains(1, 8, c, 10.0, 4.0))
    assert not np.array_equal(g, oracle.place_grains(2, 8, c, 10.0, 4.0))
    # the grains placed first do not depend on how many follow
    assert np.array_equal(g[:5], oracle.place_grains(1, 5, c, 10.0, 4.0))


def test_uniform_in_the_sphere():
    """Without a separation every grain is an independent uniform point in the
    ball: (r/R)^3 is uniform on [0, 1] (Kolmogorov-Smirnov), the mean is the
    centre and the directions are isotropic (3 sigma)."""
    n, c, R = 4000, np.array([5.0, -3.0, 8.0]), 2.5
    g = oracle.place_grains(7, n, c, R, 0.0)
    u = (np.sqrt(np.sum((g - c) ** 2, axis=1)) / R) ** 3
    assert stats.kstest(u, "uniform").pvalue > 1e-3
    sigma = R * np.sqrt(1.0 / 5.0 / n)  # per-axis standard deviation of the mean
    assert np.all(np.abs(g.mean(axis=0) - c) < 3.0 * sigma)


def test_no_room_is_an_error():
    with pytest.raises(ValueError):
        oracle.place_grains(0, 40, np.zeros(3), 1.0, 1.0)
