"""Sector matrices of the spin-1/2 Heisenberg Hamiltonian (oracle).

H = sum_b J_b s_i . s_j (Sec. III, ladder / ring / sawtooth Hamiltonians, and
any bond list), s = sigma/2.  In the bit basis (bit = 1 <=> up):
  s_i.s_j |s> = (+1/4)|s>                              if bits i, j are equal,
              = (-1/4)|s> + (1/2)|s with i, j flipped>  if they differ.
Duplicated bonds are summed; i == j is rejected.

The rescaled operator of Eqs. (4)-(5): H' = (H - c)/m with
m = (E_max - E_min)/(2 - eps), c = (E_max + E_min)/2; below (a, b) = (m, c).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import basis


def _check_bonds(cluster):
    N = cluster.n_sites
    bi, bj = np.asarray(cluster.bond_i), np.asarray(cluster.bond_j)
    if np.any(bi == bj):
        raise ValueError("bond with i == j")
    if np.any((bi < 0) | (bi >= N) | (bj < 0) | (bj >= N)):
        raise ValueError("bond site out of range")
    if not np.all(np.isfinite(cluster.J)):
        raise ValueError("non-finite coupling")


def sector_hamiltonian(cluster, n_up: int, states=None, J=None) -> sp.csr_matrix:
    """H restricted to the sector with n_up up spins, as CSR in the ascending
    basis order.  Neighbour indices come from binary search in the enumerated
    basis, not from the ranking formula."""
    _check_bonds(cluster)
    if states is None:
        states = basis.sector_states(cluster.n_sites, n_up)
    J = cluster.J if J is None else np.asarray(J, dtype=np.float64)
    dim = states.size
    diag = np.zeros(dim)
    rows, cols, vals = [], [], []
    for i, j, Jb in zip(cluster.bond_i, cluster.bond_j, J):
        bi = (states >> np.uint64(i)) & np.uint64(1)
        bj = (states >> np.uint64(j)) & np.uint64(1)
        differ = bi != bj
        diag += np.where(differ, -0.25, 0.25) * Jb
        r = np.nonzero(differ)[0]
        if r.size:
            t = states[r] ^ np.uint64((1 << int(i)) | (1 << int(j)))
            rows.append(r)
            cols.append(basis.index_of(states, t))
            vals.append(np.full(r.size, 0.5 * Jb))
    rows.append(np.arange(dim)); cols.append(np.arange(dim)); vals.append(diag)
    H = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(dim, dim)).tocsr()
    H.sum_duplicates()
    return H


def bond_operator(cluster, n_up: int, b: int, states=None) -> sp.csr_matrix:
    """h_b = s_i . s_j of bond b restricted to the sector (so dH/dJ_b = h_b)."""
    from workloads import Cluster
    one = Cluster(cluster.n_sites, cluster.bond_i[b:b + 1], cluster.bond_j[b:b + 1], np.ones(1))
    return sector_hamiltonian(one, n_up, states)


def sector_neighbors(cluster, n_up: int, rows, states=None):
    """Per requested row: the list of (neighbour index, bond) for every bond whose
    two bits differ, in bond order, and the diagonal element of H."""
    if states is None:
        states = basis.sector_states(cluster.n_sites, n_up)
    out, diag = [], []
    for r in np.asarray(rows, dtype=np.int64):
        s = int(states[r])
        lst, d = [], 0.0
        for b, (i, j, Jb) in enumerate(zip(cluster.bond_i, cluster.bond_j, cluster.J)):
            if ((s >> int(i)) ^ (s >> int(j))) & 1:
                t = s ^ ((1 << int(i)) | (1 << int(j)))
                lst.append((int(basis.index_of(states, [t])[0]), b))
                d -= 0.25 * Jb
            else:
                d += 0.25 * Jb
        out.append(lst)
        diag.append(d)
    return out, np.array(diag)


_SX = np.array([[0.0, 0.5], [0.5, 0.0]])
_SY = np.array([[0.0, -0.5j], [0.5j, 0.0]])
_SZ = np.array([[-0.5, 0.0], [0.0, 0.5]])   # basis order: |0> = down, |1> = up


def _site_op(op, p, N):
    """Kronecker product with `op` at site p; site p is bit p of the index, so
    the leftmost factor is site N-1."""
    out = np.ones((1, 1))
    for q in range(N - 1, -1, -1):
        out = np.kron(out, op if q == p else np.eye(2))
    return out


def full_hamiltonian_kron(cluster) -> np.ndarray:
    """Dense 2^N x 2^N H from Kronecker products of spin matrices (small N)."""
    N = cluster.n_sites
    H = np.zeros((1 << N, 1 << N), dtype=complex)
    for i, j, Jb in zip(cluster.bond_i, cluster.bond_j, cluster.J):
        for op in (_SX, _SY, _SZ):
            H += Jb * (_site_op(op, int(i), N) @ _site_op(op, int(j), N))
    assert np.abs(H.imag).max() < 1e-12
    return H.real


def scale_from_bounds(e_lo: float, e_hi: float, eps: float):
    """Eq. (5): m = (E_max - E_min)/(2 - eps), c = (E_max + E_min)/2."""
    return (e_hi - e_lo) / (2.0 - eps), 0.5 * (e_hi + e_lo)


def rescaled(H: sp.spmatrix, a: float, b: float) -> sp.csr_matrix:
    """Eq. (4): H' = (H - b)/a."""
    return ((H - b * sp.identity(H.shape[0], format="csr")) / a).tocsr()
