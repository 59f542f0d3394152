"""Oracle pins: sector matrices of H = sum_b J_b s_i.s_j against an independent
Kronecker-product construction, closed-form traces and known spectra."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import basis, hamiltonian


def _random_cluster(N, nb, seed):
    rng = np.random.default_rng(seed)
    bi, bj = [], []
    while len(bi) < nb:
        i, j = rng.integers(0, N, 2)
        if i != j:
            bi.append(i); bj.append(j)
    return W.Cluster(N, np.array(bi), np.array(bj), rng.uniform(-1.5, 1.5, nb))


@pytest.mark.parametrize("cluster", [W.j1j2_chain(8, 1.0, 0.37), W.ladder(8), _random_cluster(7, 12, 3),
                                     W.sawtooth(8)])
def test_sector_matrix_matches_kronecker_build(cluster):
    Hf = hamiltonian.full_hamiltonian_kron(cluster)
    N = cluster.n_sites
    for k in range(N + 1):
        idx = basis.sector_states(N, k).astype(np.int64)
        Hs = hamiltonian.sector_hamiltonian(cluster, k).toarray()
        np.testing.assert_allclose(Hs, Hf[np.ix_(idx, idx)], atol=1e-14, rtol=0)
    # no matrix element leaves the sector (S^z is conserved)
    pc = np.array([bin(i).count("1") for i in range(1 << N)])
    assert np.abs(Hf[pc[:, None] != pc[None, :]]).max() < 1e-14


def test_full_space_traces_closed_form():
    """Tr H = 0 and Tr H^2 = 2^N (3/16) sum_b J_b^2 (distinct bonds)."""
    for cl in [W.ring(12), W.j1j2_chain(10, 1.0, 0.5), W.random_regular_cluster(12, 3, 7, J_range=(0.5, 1.5))]:
        N = cl.n_sites
        tr1 = tr2 = 0.0
        for k in range(N + 1):
            H = hamiltonian.sector_hamiltonian(cl, k)
            tr1 += H.diagonal().sum()
            tr2 += H.multiply(H).sum()
        assert abs(tr1) < 1e-9
        assert tr2 == pytest.approx(2**N * 3 / 16 * np.sum(cl.J**2), rel=1e-12)


def test_sector_trace_closed_form():
    """Tr_k H = sum_b J_b/4 [C(N-2,k-2) + C(N-2,k) - 2 C(N-2,k-1)]."""
    cl = W.random_regular_cluster(11, 3, 5, J_range=(0.5, 1.5))
    N = cl.n_sites
    c = lambda n, k: math.comb(n, k) if 0 <= k <= n else 0
    for k in range(N + 1):
        H = hamiltonian.sector_hamiltonian(cl, k)
        want = np.sum(cl.J) / 4 * (c(N - 2, k - 2) + c(N - 2, k) - 2 * c(N - 2, k - 1))
        assert H.diagonal().sum() == pytest.approx(want, abs=1e-11)


def test_max_eigenvalue_antiferro_is_ferro_energy():
    """With all J_b > 0 the fully polarised multiplet is the top level of every sector."""
    cl = W.random_regular_cluster(10, 3, 1, J_range=(0.5, 1.5))
    for k in range(5, 11):
        e = np.linalg.eigvalsh(hamiltonian.sector_hamiltonian(cl, k).toarray())
        assert e.max() == pytest.approx(np.sum(cl.J) / 4, abs=1e-12)


def test_dimer_spectrum():
    J = 1.3
    d = W.dimer(J)
    e0 = np.linalg.eigvalsh(hamiltonian.sector_hamiltonian(d, 1).toarray())
    e1 = np.linalg.eigvalsh(hamiltonian.sector_hamiltonian(d, 2).toarray())
    np.testing.assert_allclose(e0, [-0.75 * J, 0.25 * J], atol=1e-15)
    np.testing.assert_allclose(e1, [0.25 * J], atol=1e-15)


def test_su2_sector_inclusion():
    """SU(2): spectrum of sector n_up+1 is a sub-multiset of sector n_up (n_up >= N/2)."""
    cl = W.ring(12)
    prev = None
    for k in range(6, 13):
        e = np.sort(np.linalg.eigvalsh(hamiltonian.sector_hamiltonian(cl, k).toarray()))
        if prev is not None:
            avail = list(prev)
            for x in e:
                j = int(np.argmin(np.abs(np.array(avail) - x)))
                assert abs(avail[j] - x) < 1e-9
                avail.pop(j)
        prev = e


def test_duplicate_bonds_sum_and_order_irrelevant():
    a = W.Cluster(6, np.array([0, 1, 2]), np.array([1, 2, 3]), np.array([1.0, 0.5, 0.25]))
    b = W.Cluster(6, np.array([2, 3, 0, 1, 1]), np.array([1, 2, 1, 0, 2]), np.array([0.25, 0.25, 0.4, 0.6, 0.25]))
    for k in range(7):
        np.testing.assert_allclose(hamiltonian.sector_hamiltonian(a, k).toarray(),
                                   hamiltonian.sector_hamiltonian(b, k).toarray(), atol=1e-15)


def test_rejects_self_bond():
    with pytest.raises(ValueError):
        hamiltonian.sector_hamiltonian(W.Cluster(4, np.array([1]), np.array([1]), np.array([1.0])), 2)


def test_neighbor_lists_match_matrix():
    cl = W.random_regular_cluster(12, 3, 11, J_range=(0.5, 1.5))
    st = basis.sector_states(12, 6)
    H = hamiltonian.sector_hamiltonian(cl, 6, st).toarray()
    rows = np.arange(0, st.size, 37)
    lists, diag = hamiltonian.sector_neighbors(cl, 6, rows, st)
    for r, lst, d in zip(rows, lists, diag):
        row = np.zeros(st.size)
        row[r] += d
        for col, b in lst:
            row[col] += 0.5 * cl.J[b]
        np.testing.assert_allclose(row, H[r], atol=1e-14)
