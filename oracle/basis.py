"""S^z-sector basis of N spin-1/2 sites and its ranking (oracle).

A basis state is an N-bit word s: bit p set <=> spin p points up (s^z_p = +1/2).
The sector with n_up spins up (S^z = n_up - N/2, the quantum number of the
susceptibility formula, Eq. (3)) holds all words of popcount n_up.  The
sector's basis order is ascending integer order.

Two independent ways to get a state's index are provided: brute-force
enumeration + binary search (`sector_states`, `index_of`), and the closed
combinatorial-number-system formula (`cns_rank`): for set-bit positions
p_1 < ... < p_k (0-based), rank(s) = sum_{j=1..k} C(p_j, j).  Tests check that
the two agree; the oracle's Hamiltonian uses only the first.
"""
from __future__ import annotations

import math
from itertools import combinations

import numpy as np


def binomial_table(nmax: int = 64) -> np.ndarray:
    """C[n, j] = n choose j (0 when j > n), int64 (exact for n <= 64, j <= 32)."""
    C = np.zeros((nmax + 1, nmax + 2), dtype=np.int64)
    for n in range(nmax + 1):
        for j in range(n + 1):
            v = math.comb(n, j)
            C[n, j] = v if v < 2**62 else -1
    return C


_C = binomial_table(64)


def sector_dim(N: int, n_up: int) -> int:
    return math.comb(N, n_up) if 0 <= n_up <= N else 0


def sector_states(N: int, n_up: int) -> np.ndarray:
    """All N-bit words with popcount n_up, ascending, as uint64 (brute force)."""
    if not (0 <= n_up <= N):
        return np.zeros(0, dtype=np.uint64)
    if N <= 26:
        w = np.arange(1 << N, dtype=np.uint64)
        return w[np.bitwise_count(w) == n_up]
    if math.comb(N, n_up) > 5_000_000:
        raise ValueError("sector too large for brute-force enumeration")
    out = np.fromiter((sum(1 << p for p in c) for c in combinations(range(N), n_up)),
                      dtype=np.uint64, count=math.comb(N, n_up))
    out.sort()
    return out


def index_of(states: np.ndarray, words) -> np.ndarray:
    """Position of each word in the ascending `states` array (binary search)."""
    words = np.asarray(words, dtype=np.uint64)
    idx = np.searchsorted(states, words)
    if np.any(idx >= states.size) or np.any(states[np.minimum(idx, states.size - 1)] != words):
        raise KeyError("word not in sector")
    return idx.astype(np.int64)


def cns_rank(words, N: int) -> np.ndarray:
    """Combinatorial-number-system rank: sum over set bits p_j (j-th set bit,
    1-based) of C(p_j, j)."""
    s = np.asarray(words, dtype=np.uint64)
    r = np.zeros(s.shape, dtype=np.int64)
    cnt = np.zeros(s.shape, dtype=np.int64)
    for p in range(N):
        bit = ((s >> np.uint64(p)) & np.uint64(1)).astype(bool)
        cnt += bit
        r += np.where(bit, _C[p, np.minimum(cnt, 63)], 0)
    return r


def cns_unrank(rank: int, N: int, n_up: int) -> int:
    """Inverse of `cns_rank` for one rank: greedily take, for j = k..1, the
    largest p with C(p, j) <= remaining rank."""
    r = int(rank)
    if not (0 <= r < math.comb(N, n_up)):
        raise ValueError("rank out of range")
    s = 0
    p = N - 1
    for j in range(n_up, 0, -1):
        while math.comb(p, j) > r:
            p -= 1
        s |= 1 << p
        r -= math.comb(p, j)
        p -= 1
    return s
