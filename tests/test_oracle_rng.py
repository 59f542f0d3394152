"""Oracle pins: the counter-based SplitMix64 generator and the random vectors."""
import os

import numpy as np

from oracle import rng

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "splitmix64_seed0.txt")


def test_splitmix64_published_sequence():
    want = [int(l, 16) for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    got = rng.counter_u64(0, 0, np.arange(3, dtype=np.uint64))
    assert [int(x) for x in got] == want


def test_counter_is_offset_sequence():
    """u(seed, ctr) is output ctr+1 of the generator started at `seed`:
    shifting the seed by G shifts the counter by one."""
    s = 12345
    a = rng.counter_u64(s, 0, np.arange(1, 10, dtype=np.uint64))
    b = rng.counter_u64((s + rng.G) % 2**64, 0, np.arange(0, 9, dtype=np.uint64))
    assert np.array_equal(a, b)


def test_rademacher_balanced_and_streams_distinct():
    n = 1 << 20
    x = rng.rademacher(0, 0, 12, 0, n)
    assert set(np.unique(x)) == {-1.0, 1.0}
    assert abs(x.mean()) < 5 / np.sqrt(n)
    y = rng.rademacher(0, 0, 12, 1, n)
    z = rng.rademacher(0, 1, 12, 0, n)
    w = rng.rademacher(0, 0, 13, 0, n)
    for o in (y, z, w):
        assert abs(np.dot(x, o)) / n < 5 / np.sqrt(n)


def test_gaussian_moments():
    n = 1 << 20
    re, im = rng.box_muller(7, 3, 10, 5, n)
    for v in (re, im):
        assert abs(v.mean()) < 5 / np.sqrt(n)
        assert abs(v.var() - 1) < 5 * np.sqrt(2 / n)
        assert abs(np.mean(v**4) - 3) < 5 * np.sqrt(96 / n)
    assert abs(np.mean(re * im)) < 5 / np.sqrt(n)


def test_normalisation_and_column_layout():
    dim = 1000
    V, voc, R = rng.random_columns("complex_gaussian", 0, 0, 5, 3, dim)
    assert V.shape == (dim, 6) and R == 3
    assert np.array_equal(voc, [0, 0, 1, 1, 2, 2])
    for r in range(3):
        assert np.sum(V[:, 2 * r:2 * r + 2] ** 2) == np.float64(dim) or \
            abs(np.sum(V[:, 2 * r:2 * r + 2] ** 2) - dim) < 1e-9
    V, voc, R = rng.random_columns("gaussian", 0, 0, 5, 2, dim)
    assert np.allclose((V**2).sum(0), dim, rtol=1e-14)
    V, voc, R = rng.random_columns("basis", 0, 0, 5, 2, 7)
    assert R == 7 and np.array_equal(V, np.eye(7))
