"""Oracle pins: S^z-sector enumeration and combinatorial-number-system ranking."""
import math

import numpy as np
import pytest

from oracle import basis


@pytest.mark.parametrize("N", range(1, 15))
def test_cns_rank_equals_enumeration_index(N):
    for k in range(N + 1):
        s = basis.sector_states(N, k)
        assert s.size == math.comb(N, k)
        assert np.all(np.diff(s.astype(np.int64)) > 0)
        assert np.all(np.bitwise_count(s) == k)
        assert np.array_equal(basis.cns_rank(s, N), np.arange(s.size))


def test_cns_rank_bijection_n20_sz0():
    s = basis.sector_states(20, 10)
    r = basis.cns_rank(s, 20)
    assert np.array_equal(r, np.arange(184756))


def test_unrank_inverts_rank_small_and_large():
    for N, k in [(12, 6), (24, 12), (30, 15), (32, 16), (32, 1), (32, 32)]:
        dim = math.comb(N, k)
        rng = np.random.default_rng(N * 100 + k)
        ranks = np.unique(np.concatenate([[0, dim - 1], rng.integers(0, dim, 50)]))
        for r in ranks:
            w = basis.cns_unrank(int(r), N, k)
            assert bin(w).count("1") == k and w < (1 << N)
            assert basis.cns_rank([w], N)[0] == r


def test_unrank_is_ascending_order_n24():
    s = basis.sector_states(24, 12)
    for r in [0, 1, 2, 1000, 123456, 2704155]:
        assert basis.cns_unrank(r, 24, 12) == int(s[r])
