"""Spin-s Heisenberg sectors (oracle), the basis of the paper's spin-5/2 Fe10
molecule (Sec. III.B).  Test infrastructure only.

A site carries d = s + m in {0, .., 2s} (m = S^z of the site).  The sector
with total sum d_i = n (S^z = n - N s) holds all digit strings with that sum,
ordered by the value sum_i d_i B^i, B = 2s + 1, ascending; for s = 1/2 this is
the spin-1/2 basis of `basis` (d_i = bit i, value = the word itself).

  H = sum_b J_b (S^z_i S^z_j + (S^+_i S^-_j + S^-_i S^+_j)/2),
  S^+ |m> = sqrt(s(s+1) - m(m+1)) |m+1>.

Two ways to the index of a state are kept apart: brute-force enumeration with
binary search (used by the Hamiltonian), and the counting formula
(`rank_formula`, `rank_many`, inverted by `unrank_formula`): rank = sum over
sites i, from the most significant down, of the number of states that agree
above i and carry a smaller digit at i, cnt(i, r - v) summed over v < d_i,
where cnt(i, r) counts digit strings of length i with sum r and r is the sum
still left for sites 0..i.  `recursion_rows` evaluates single rows of the
Chebyshev vectors of sectors too large for the matrix with the second way.
"""
from __future__ import annotations

import itertools
import math

import numpy as np
import scipy.sparse as sp


def counts(N: int, two_s: int) -> np.ndarray:
    """cnt[i, r]: digit strings of length i (digits 0..2s) with sum r."""
    B = two_s + 1
    cnt = np.zeros((N + 1, two_s * N + 1), dtype=np.int64)
    cnt[0, 0] = 1
    for i in range(1, N + 1):
        for r in range(two_s * i + 1):
            cnt[i, r] = sum(cnt[i - 1, r - v] for v in range(B) if r - v >= 0)
    return cnt


def sector_dim(N: int, two_s: int, n: int) -> int:
    if not (0 <= n <= two_s * N):
        return 0
    return int(counts(N, two_s)[N, n])


def sector_digits(N: int, two_s: int, n: int) -> np.ndarray:
    """All digit strings [dim, N] (column i = site i) with sum n, ascending value
    (brute force over B^N strings when that is small, else a depth-first walk
    from the most significant site with the sum still reachable by the rest)."""
    B = two_s + 1
    if B ** N <= 20_000_000:
        vals = np.arange(B ** N, dtype=np.int64)
        digs = np.stack([(vals // B ** i) % B for i in range(N)], axis=1)
        keep = digs.sum(axis=1) == n
        return digs[keep]
    return _walk_digits(N, two_s, n)


def _walk_digits(N: int, two_s: int, n: int, limit: int = 2_000_000) -> np.ndarray:
    out = []
    d = [0] * N

    def rec(i, left):
        if i < 0:
            if left == 0:
                out.append(list(d))
                if len(out) > limit:
                    raise ValueError("sector too large to enumerate")
            return
        for x in range(0, min(two_s, left) + 1):
            if left - x <= two_s * i:
                d[i] = x
                rec(i - 1, left - x)
        d[i] = 0

    rec(N - 1, n)
    return np.array(out, dtype=np.int64).reshape(-1, N)


def values(digits: np.ndarray, two_s: int) -> np.ndarray:
    B = two_s + 1
    w = B ** np.arange(digits.shape[1], dtype=np.int64)
    return digits.astype(np.int64) @ w


def rank_formula(d, two_s: int) -> int:
    """Index of digit string d in its sector by the counting formula."""
    N = len(d)
    cnt = counts(N, two_s)
    r = int(sum(d))
    rank = 0
    for i in range(N - 1, -1, -1):
        for v in range(int(d[i])):
            if r - v >= 0:
                rank += int(cnt[i, r - v])
        r -= int(d[i])
    return rank


def rank_table(N: int, two_s: int) -> np.ndarray:
    """P[i, r, d] = sum_{v < d} cnt(i, r - v): the term that site i with digit d
    adds to the rank when the sites 0..i carry the sum r."""
    cnt = counts(N, two_s)
    R1, B = two_s * N + 1, two_s + 1
    P = np.zeros((N, R1, B), dtype=np.int64)
    for i in range(N):
        for r in range(R1):
            for d in range(1, B):
                v = d - 1
                P[i, r, d] = P[i, r, d - 1] + (cnt[i, r - v] if r - v >= 0 else 0)
    return P


def rank_many(digits: np.ndarray, two_s: int, n: int, P=None) -> np.ndarray:
    """rank_formula for every row of digits [k, N] at once (digit sum n)."""
    digits = np.asarray(digits, dtype=np.int64)
    N = digits.shape[1]
    if P is None:
        P = rank_table(N, two_s)
    r = np.full(digits.shape[0], n, dtype=np.int64)
    rank = np.zeros(digits.shape[0], dtype=np.int64)
    for i in range(N - 1, -1, -1):
        rank += P[i, r, digits[:, i]]
        r -= digits[:, i]
    return rank


def unrank_formula(rank: int, N: int, two_s: int, n: int, P=None) -> np.ndarray:
    """Digit string of index `rank` in sector n: from the most significant site
    down, the largest digit whose count of smaller strings does not exceed
    what is left of the rank."""
    if P is None:
        P = rank_table(N, two_s)
    d = np.zeros(N, dtype=np.int64)
    r, rem = n, int(rank)
    for i in range(N - 1, -1, -1):
        best = 0
        for x in range(min(two_s, r) + 1):
            if P[i, r, x] <= rem and r - x <= two_s * i:
                best = x
        d[i] = best
        rem -= int(P[i, r, best])
        r -= best
    if rem != 0 or r != 0:
        raise ValueError("rank outside the sector")
    return d


def _ladder(s: float, m: np.ndarray) -> np.ndarray:
    """<m+1| S^+ |m> = sqrt(s(s+1) - m(m+1)) (0 at m = s)."""
    return np.sqrt(np.maximum(s * (s + 1) - m * (m + 1), 0.0))


def sector_hamiltonian(cluster, two_s: int, n: int) -> sp.csr_matrix:
    """H on the sector (n = S^z + N s), CSR in the ascending value order;
    neighbour indices by binary search in the enumerated basis."""
    N = cluster.n_sites
    s = two_s / 2.0
    digs = sector_digits(N, two_s, n)
    vals = values(digs, two_s)
    B = two_s + 1
    dim = vals.size
    m = digs - s
    diag = np.zeros(dim)
    rows, cols, data = [], [], []
    for i, j, Jb in zip(cluster.bond_i, cluster.bond_j, cluster.J):
        i, j = int(i), int(j)
        diag += Jb * m[:, i] * m[:, j]
        # S^+_i S^-_j and S^-_i S^+_j
        for a, b in ((i, j), (j, i)):
            ok = (digs[:, a] < two_s) & (digs[:, b] > 0)
            r = np.nonzero(ok)[0]
            if not r.size:
                continue
            amp = 0.5 * Jb * _ladder(s, m[r, a]) * _ladder(s, -m[r, b])
            t = vals[r] + B ** a - B ** b
            c = np.searchsorted(vals, t)
            assert np.all(vals[c] == t)
            rows.append(r); cols.append(c); data.append(amp)
    rows.append(np.arange(dim)); cols.append(np.arange(dim)); data.append(diag)
    H = sp.coo_matrix((np.concatenate(data), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(dim, dim)).tocsr()
    H.sum_duplicates()
    return H


def spin_matrices(two_s: int):
    """S^x, S^y, S^z in the basis d = 0..2s (m = d - s)."""
    s = two_s / 2.0
    B = two_s + 1
    m = np.arange(B) - s
    Sp = np.zeros((B, B))
    for d in range(B - 1):
        Sp[d + 1, d] = math.sqrt(s * (s + 1) - m[d] * (m[d] + 1))
    Sm = Sp.T
    return (Sp + Sm) / 2, (Sp - Sm) / 2j, np.diag(m)


def full_hamiltonian_kron(cluster, two_s: int) -> np.ndarray:
    """Dense B^N x B^N H from Kronecker products (site i = digit i of the
    value, so the leftmost factor is site N-1)."""
    N = cluster.n_sites
    B = two_s + 1
    ops = spin_matrices(two_s)

    def site(op, p):
        out = np.ones((1, 1))
        for q in range(N - 1, -1, -1):
            out = np.kron(out, op if q == p else np.eye(B))
        return out

    H = np.zeros((B ** N, B ** N), dtype=complex)
    for i, j, Jb in zip(cluster.bond_i, cluster.bond_j, cluster.J):
        for op in ops:
            H += Jb * (site(op, int(i)) @ site(op, int(j)))
    assert np.abs(H.imag).max() < 1e-12
    return H.real


def sectors(cluster, two_s: int, cluster_id: int = 0):
    """(n, dim) of every sector with S^z >= 0 (2n >= 2s N)."""
    N = cluster.n_sites
    lo = (two_s * N + 1) // 2
    return [(n, sector_dim(N, two_s, n)) for n in range(lo, two_s * N + 1)]


def recursion_rows(cluster, two_s: int, n: int, a: float, b: float, kind: str, seed: int, R: int,
                   rows, n_vec: int, cluster_id: int = 0, store=np.float64, norms=None) -> np.ndarray:
    """Rows of v_{n_vec} = T_{n_vec}(H') v_0 (H' = (H - b)/a) of a spin-s sector
    too large to hold as a matrix, from the neighbourhood cones of the rows:
    v_m is needed on every state within n_vec - m exchange moves of a row.
    v_0 comes from the counter generator (the vectors of Eq. (7)); `store`
    rounds every stored vector as the reduced-storage form does."""
    from . import rows as rows_mod

    N = cluster.n_sites
    s = two_s / 2.0
    B = two_s + 1
    dim = int(counts(N, two_s)[N, n])
    P = rank_table(N, two_s)
    bi = np.asarray(cluster.bond_i, dtype=np.int64)
    bj = np.asarray(cluster.bond_j, dtype=np.int64)
    J = np.asarray(cluster.J, dtype=np.float64)
    rows = np.asarray(rows, dtype=np.int64)
    sets = [None] * (n_vec + 1)
    digs_of = [None] * (n_vec + 1)
    sets[n_vec] = np.unique(rows)
    digs_of[n_vec] = np.array([unrank_formula(int(r), N, two_s, n, P) for r in sets[n_vec]]).reshape(-1, N)
    ops = [None] * (n_vec + 1)     # per level: diag, neighbour ranks [k, 2 n_b], amplitudes
    for m in range(n_vec, 0, -1):
        dg = digs_of[m]
        mm = dg - s
        diag = (J[None, :] * mm[:, bi] * mm[:, bj]).sum(axis=1)
        nr, amp, nd = [], [], []
        for src, dst in ((bi, bj), (bj, bi)):      # S^+_src S^-_dst
            ok = (dg[:, src] < two_s) & (dg[:, dst] > 0)
            t = np.repeat(dg[:, None, :], len(J), axis=1)
            k = np.arange(len(J))
            t[:, k, src] += 1
            t[:, k, dst] -= 1
            t = np.where(ok[:, :, None], t, dg[:, None, :])
            nd.append(t.reshape(-1, N))
            nr.append(rank_many(t.reshape(-1, N), two_s, n, P).reshape(ok.shape))
            amp.append(np.where(ok, 0.5 * J[None, :] * _ladder(s, mm[:, src]) * _ladder(s, -mm[:, dst]), 0.0))
        nr = np.concatenate(nr, axis=1)
        amp = np.concatenate(amp, axis=1)
        ops[m] = (diag, nr, amp)
        allr = np.concatenate([sets[m], nr.ravel()])
        sets[m - 1], first = np.unique(allr, return_index=True)
        # nd holds [k * n_b] rows per direction: restore the order of nr.ravel()
        nd_ord = np.concatenate([x.reshape(dg.shape[0], len(J), N) for x in nd], axis=1).reshape(-1, N)
        alld = np.concatenate([dg, nd_ord], axis=0)
        digs_of[m - 1] = alld[first]
    v = [None] * (n_vec + 1)
    v[0] = rows_mod.start_rows(kind, seed, cluster_id, n, R, sets[0], dim, norms).astype(store).astype(np.float64)
    for m in range(1, n_vec + 1):
        diag, nr, amp = ops[m]
        x = v[m - 1]
        pos = np.searchsorted(sets[m - 1], nr)
        self_pos = np.searchsorted(sets[m - 1], sets[m])
        hx = ((diag - b) / a)[:, None] * x[self_pos]
        for k in range(nr.shape[1]):
            hx += (amp[:, k] / a)[:, None] * x[pos[:, k]]
        y = hx if m == 1 else 2.0 * hx - v[m - 2][np.searchsorted(sets[m - 2], sets[m])]
        v[m] = y.astype(store).astype(np.float64)
    return v[n_vec][np.searchsorted(sets[n_vec], rows)]
