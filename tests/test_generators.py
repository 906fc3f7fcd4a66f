"""The seeded input generators: determinism and the distributions they are
meant to draw from (CPU only)."""
import math

import numpy as np

import oracle
from paper_2209_04541_amd import gen


def test_deterministic_from_seed():
    for make in (lambda k: gen.rmat(10, 8, gen.seed(9, k)),
                 lambda k: gen.er(500, 3000, gen.seed(9, k)),
                 lambda k: gen.rgg(500, 12, gen.seed(9, k))):
        n1, s1, d1 = make(1)
        n2, s2, d2 = make(1)
        n3, s3, d3 = make(2)
        assert n1 == n2 and np.array_equal(s1, s2) and np.array_equal(d1, d2)
        assert not (len(s1) == len(s3) and np.array_equal(s1, s3) and np.array_equal(d1, d3))
    assert gen.seed(1, 0) != gen.seed(0, 1)


def test_rmat_quadrant_frequencies():
    """Every bit level of a sample picks quadrant (src bit, dst bit) with
    probabilities (a, b, c, d); with 2^20 samples the standard error is
    below 0.0005."""
    n, s, d = gen.rmat(16, 16, gen.seed(9, 2))
    assert n == 1 << 16 and len(s) == 16 << 16
    assert s.min() >= 0 and s.max() < n and d.min() >= 0 and d.max() < n
    for bit in (0, 7, 15):
        q = ((s >> bit) & 1) * 2 + ((d >> bit) & 1)
        freq = np.bincount(q, minlength=4) / len(q)
        assert np.allclose(freq, [0.57, 0.19, 0.19, 0.05], atol=0.004), (bit, freq)


def test_er_exact_distinct_pairs_and_clamp():
    n, s, d = gen.er(3000, 20000, gen.seed(9, 3))
    assert len(s) == 20000
    assert np.all(s != d) and s.min() >= 0 and max(s.max(), d.max()) < n
    keys = np.minimum(s, d).astype(np.int64) * n + np.maximum(s, d)
    assert len(np.unique(keys)) == 20000
    # asking for more than C(n, 2) pairs gives the complete graph
    n, s, d = gen.er(60, 10 ** 6, gen.seed(9, 4))
    assert len(s) == 60 * 59 // 2
    assert oracle.tc(n, s, d) == math.comb(60, 3)


def test_rgg_mean_degree_and_clamp():
    """Two uniform points of the unit square lie within r (r <= 1) with
    probability pi r^2 - 8 r^3 / 3 + r^4 / 2, so the realised mean degree
    is (n - 1) times that, a little below the target d."""
    n, s, d = gen.rgg(4000, 20, gen.seed(9, 1))
    assert np.all(s != d)
    keys = np.minimum(s, d).astype(np.int64) * n + np.maximum(s, d)
    assert len(np.unique(keys)) == len(keys)
    r = gen.rgg_radius(4000, 20)
    p = math.pi * r * r - 8 * r ** 3 / 3 + r ** 4 / 2
    mean = 2 * len(s) / n
    assert abs(mean - (n - 1) * p) < 0.03 * (n - 1) * p
    assert mean < 20
    # a radius of sqrt(2) joins every pair
    n, s, d = gen.rgg(50, 10 ** 6, gen.seed(9, 5))
    assert len(s) == 50 * 49 // 2
    assert oracle.tc(n, s, d) == math.comb(50, 3)


def test_uniform_draws_and_arrivals():
    s = gen.seed(9, 6)
    xs = [gen.uniform_int(s, c, 3, 9) for c in range(4000)]
    assert min(xs) == 3 and max(xs) == 9
    assert abs(np.mean(xs) - 6.0) < 0.15
    us = [gen.unit(s, c) for c in range(4000)]
    assert 0.0 <= min(us) and max(us) < 1.0 and abs(np.mean(us) - 0.5) < 0.02
    t = gen.poisson_arrivals(1000.0, 2.0, gen.seed(9, 4))
    assert np.all(np.diff(t) > 0) and t[-1] < 2.0
    assert abs(len(t) - 2000) < 5 * math.sqrt(2000)
    # exponential gaps: mean 1/rate, standard deviation 1/rate
    g = np.diff(t)
    assert abs(g.mean() - 1e-3) < 1e-4 and abs(g.std() - 1e-3) < 1.5e-4


def test_workload_parameters_in_range():
    for g in range(200):
        fam, n, d = gen.batch_params(g)
        assert fam == ("rgg" if g % 2 == 0 else "er")
        assert 64 <= n <= 8192 and 8 <= d <= 64
    for r in range(200):
        sc, ef = gen.served_params(r)
        assert 10 <= sc <= 22 and 8 <= ef <= 32
