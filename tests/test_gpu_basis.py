"""GPU vs oracle: basis enumeration and matrix-element indexing, bit-exact."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import basis, hamiltonian

pytestmark = pytest.mark.gpu


def _u32(t):
    return t.cpu().numpy().view(np.uint32).astype(np.uint64)


@pytest.mark.parametrize("N", [1, 2, 5, 12, 16, 20])
def test_sector_states_all_k(kpm, N):
    for k in range(N + 1):
        got = _u32(kpm.sector_states(N, k))
        assert np.array_equal(got, basis.sector_states(N, k)), (N, k)


def test_sector_states_n24_full(kpm):
    got = _u32(kpm.sector_states(24, 12))
    assert got.size == 2704156
    assert np.array_equal(got, basis.sector_states(24, 12))


@pytest.mark.parametrize("N,k", [(30, 15), (32, 16), (32, 31), (28, 20)])
def test_sector_states_large_sampled(kpm, N, k):
    dim = math.comb(N, k)
    t = kpm.sector_states(N, k)
    rng = np.random.default_rng(N * 64 + k)
    ranks = np.unique(np.concatenate([[0, 1, dim - 2, dim - 1], rng.integers(0, dim, 400)]))
    got = t.cpu().numpy().view(np.uint32)[ranks].astype(np.int64)
    want = np.array([basis.cns_unrank(int(r), N, k) for r in ranks])
    assert np.array_equal(got, want)
    del t


def _check_rows(kpm, sector, rows_start, nrows, states=None, via_cns=False):
    cl = sector.cluster
    cols, bond, cnt, diag = kpm.sector_matrix(sector, rows_start, nrows)
    cols = cols.cpu().numpy().view(np.uint32)
    bond, cnt, diag = bond.cpu().numpy(), cnt.cpu().numpy(), diag.cpu().numpy()
    rows = np.arange(rows_start, rows_start + nrows)
    if via_cns:
        N, k = cl.n_sites, sector.n_up
        for r in range(nrows):
            s = basis.cns_unrank(int(rows[r]), N, k)
            want, d = [], 0.0
            for b, (i, j, Jb) in enumerate(zip(cl.bond_i, cl.bond_j, cl.J)):
                if ((s >> int(i)) ^ (s >> int(j))) & 1:
                    want.append((int(basis.cns_rank([s ^ (1 << int(i)) ^ (1 << int(j))], N)[0]), b))
                    d -= 0.25 * Jb
                else:
                    d += 0.25 * Jb
            assert cnt[r] == len(want)
            assert [(int(c), int(b)) for c, b in zip(cols[r, :cnt[r]], bond[r, :cnt[r]])] == want
            assert abs(diag[r] - d) <= 4 * cl.n_bonds * np.spacing(max(abs(d), 1.0))
        return
    lists, dg = hamiltonian.sector_neighbors(cl, sector.n_up, rows, states)
    for r in range(nrows):
        assert cnt[r] == len(lists[r])
        assert [(int(c), int(b)) for c, b in zip(cols[r, :cnt[r]], bond[r, :cnt[r]])] == lists[r]
        assert abs(diag[r] - dg[r]) <= 4 * cl.n_bonds * np.spacing(max(abs(dg[r]), 1.0))


@pytest.mark.parametrize("cluster", [W.ring(12), W.j1j2_chain(14, 1.0, 0.5),
                                     W.random_regular_cluster(13, 3, 5, J_range=(0.5, 1.5)),
                                     W.ladder(12), W.sawtooth(12),
                                     W.Cluster(9, np.array([0, 3, 3, 8, 2]), np.array([5, 1, 1, 0, 7]),
                                               np.array([1.0, -0.5, 0.25, 2.0, 0.3]))])
def test_matrix_indexing_small(kpm, cluster):
    for sec in W.sectors(cluster):
        st = basis.sector_states(cluster.n_sites, sec.n_up)
        dim = st.size
        # full rows, with a ragged tail relative to the 256-row sub-tile
        _check_rows(kpm, sec, 0, dim, st)
        if dim > 300:
            _check_rows(kpm, sec, dim - 299, 299, st)


def test_matrix_indexing_n24_sampled(kpm):
    sec = W.sectors(W.ring(24), only_sz0=True)[0]
    st = basis.sector_states(24, 12)
    for start in (0, 123457, 2704156 - 513):
        _check_rows(kpm, sec, start, 513, st)


def test_matrix_indexing_n30_sampled(kpm):
    sec = W.sectors(W.random_regular_cluster(30, 4, 0), only_sz0=True)[0]
    for start in (0, 77777777, math.comb(30, 15) - 37):
        _check_rows(kpm, sec, start, 37, via_cns=True)


def test_matrix_values_against_hamiltonian(kpm):
    """Assembled from the export, H equals the oracle's sector matrix."""
    cl = W.random_regular_cluster(12, 3, 8, J_range=(0.5, 1.5))
    sec = W.Sector(cl, 7, 0)
    dim = math.comb(12, 7)
    cols, bond, cnt, diag = [x.cpu().numpy() for x in kpm.sector_matrix(sec, 0, dim)]
    H = np.diag(diag)
    for r in range(dim):
        for c, b in zip(cols[r, :cnt[r]].view(np.uint32), bond[r, :cnt[r]]):
            H[r, c] += 0.5 * cl.J[b]
    np.testing.assert_allclose(H, hamiltonian.sector_hamiltonian(cl, 7).toarray(), atol=1e-14)
