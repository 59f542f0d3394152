"""Single rows of the Chebyshev vectors v_n = C_n(H') v_0 (oracle).

For sectors too large to hold the matrix, rows of v_n are computed one at a
time from their neighbourhood cone: with N[S] the set S together with every
state one bond flip away,
    v_0 on N^n[S]  straight from the counter generator (the vectors of Eq. (7)),
    v_1 = H' v_0                on N^(n-1)[S],
    v_m = 2 H' v_{m-1} - v_{m-2} on N^(n-m)[S],   m = 2..n
(the recursion that the paper takes from Weisse et al.).  H' = (H - b)/a as in
Eqs. (4)-(5), with H = sum_b J_b s_i.s_j in the bit basis (Sec. III).  Ranks
are the combinatorial-number-system ranks of the sector (ascending integer
order).  `store` rounds every stored vector as the reduced-storage form does.

Parity pin: for small sectors these rows equal T_n(H') v_0 evaluated with
numpy's Chebyshev series on the dense matrix (tests/test_oracle_rows.py).
"""
from __future__ import annotations

import math

import numpy as np

from . import basis, rng


def _gauss_norms(kind: str, seed: int, cluster_id: int, n_up: int, R: int, dim: int,
                 chunk: int = 1 << 22) -> np.ndarray:
    """<r|r> of every Gaussian vector over the whole sector (Eq. (7) vectors
    are normalised to <r|r> = dim), accumulated in chunks of indices."""
    out = np.zeros(R)
    for r in range(R):
        s = rng.stream_id(cluster_id, n_up, r)
        acc = 0.0
        for i0 in range(0, dim, chunk):
            nu = np.arange(i0, min(dim, i0 + chunk), dtype=np.uint64)
            u1 = rng.uniform01(rng.counter_u64(seed, s, 2 * nu))
            u2 = rng.uniform01(rng.counter_u64(seed, s, 2 * nu + np.uint64(1)))
            rad2 = -2.0 * np.log(u1)
            if kind == "complex_gaussian":
                acc += float(np.sum(rad2))          # Re^2 + Im^2 = rad^2
            else:
                acc += float(np.sum(rad2 * np.cos(2.0 * np.pi * u2) ** 2))
        out[r] = acc
    return out


def start_rows(kind: str, seed: int, cluster_id: int, n_up: int, R: int, idx, dim: int,
               norms=None) -> np.ndarray:
    """Rows `idx` of the start block V0 (the columns of random_columns)."""
    idx = np.asarray(idx, dtype=np.uint64)
    cols = []
    if kind == "rademacher":
        for r in range(R):
            u = rng.counter_u64(seed, rng.stream_id(cluster_id, n_up, r), idx)
            cols.append(np.where((u >> np.uint64(63)) == 0, 1.0, -1.0))
        return np.stack(cols, axis=1)
    if kind in ("gaussian", "complex_gaussian"):
        if norms is None:
            norms = _gauss_norms(kind, seed, cluster_id, n_up, R, dim)
        for r in range(R):
            s = rng.stream_id(cluster_id, n_up, r)
            u1 = rng.uniform01(rng.counter_u64(seed, s, 2 * idx))
            u2 = rng.uniform01(rng.counter_u64(seed, s, 2 * idx + np.uint64(1)))
            rad = np.sqrt(-2.0 * np.log(u1))
            scale = math.sqrt(dim / norms[r])
            cols.append(rad * np.cos(2.0 * np.pi * u2) * scale)
            if kind == "complex_gaussian":
                cols.append(rad * np.sin(2.0 * np.pi * u2) * scale)
        return np.stack(cols, axis=1)
    raise ValueError(kind)


def _flips(cluster, words: np.ndarray):
    """For every state and bond: the flipped word (or the state itself when the
    two bits are equal), the bond's diagonal sign and whether it flips."""
    w = words.astype(np.uint64)[:, None]
    bi = np.asarray(cluster.bond_i, dtype=np.uint64)[None, :]
    bj = np.asarray(cluster.bond_j, dtype=np.uint64)[None, :]
    differ = (((w >> bi) ^ (w >> bj)) & np.uint64(1)).astype(bool)
    mask = (np.uint64(1) << bi) | (np.uint64(1) << bj)
    flipped = np.where(differ, w ^ mask, w)
    return flipped, differ


def recursion_rows(cluster, n_up: int, a: float, b: float, kind: str, seed: int, R: int, rows,
                   n: int, cluster_id: int = 0, store=np.float64, norms=None) -> np.ndarray:
    """v_n[rows, :] (float64 values of `store`-rounded vectors)."""
    N = cluster.n_sites
    dim = math.comb(N, n_up)
    J = np.asarray(cluster.J, dtype=np.float64)
    rows = np.asarray(rows, dtype=np.int64)
    # cones: sets[m] holds the ranks on which v_m is needed (sorted, unique)
    sets = [None] * (n + 1)
    words_of = [None] * (n + 1)
    sets[n] = np.unique(rows)
    words_of[n] = np.array([basis.cns_unrank(int(r), N, n_up) for r in sets[n]], dtype=np.uint64)
    nbr = [None] * (n + 1)   # nbr[m]: (flipped ranks [|S_m|, n_bonds], differ)
    for m in range(n, 0, -1):
        flipped, differ = _flips(cluster, words_of[m])
        fr = basis.cns_rank(flipped.ravel(), N).reshape(flipped.shape)
        nbr[m] = (fr, differ)
        allr = np.concatenate([sets[m], fr.ravel()])
        sets[m - 1], first = np.unique(allr, return_index=True)
        allw = np.concatenate([words_of[m], flipped.ravel()])
        words_of[m - 1] = allw[first]
    v = [None] * (n + 1)
    v[0] = start_rows(kind, seed, cluster_id, n_up, R, sets[0], dim, norms).astype(store).astype(np.float64)
    for m in range(1, n + 1):
        fr, differ = nbr[m]
        pos = np.searchsorted(sets[m - 1], fr)          # every neighbour lies in the cone
        self_pos = np.searchsorted(sets[m - 1], sets[m])
        diag = ((np.where(differ, -0.25, 0.25) * J[None, :]).sum(axis=1) - b) / a
        off = np.where(differ, 0.5 * J[None, :] / a, 0.0)
        x = v[m - 1]
        hx = diag[:, None] * x[self_pos]
        for k in range(fr.shape[1]):
            hx += off[:, k:k + 1] * x[pos[:, k]]
        if m == 1:
            y = hx
        else:
            y = 2.0 * hx - v[m - 2][np.searchsorted(sets[m - 2], sets[m])]
        v[m] = y.astype(store).astype(np.float64)
    return v[n][np.searchsorted(sets[n], rows)]
