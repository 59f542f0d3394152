"""Pins of the spin-s sector oracle (oracle/spins.py), the basis of the
paper's spin-5/2 Fe10 molecule (Sec. III.B): counting rank = enumeration,
s = 1/2 = the spin-1/2 oracle, sector matrices = blocks of the Kronecker
product Hamiltonian, closed-form traces, the dimer spectrum and SU(2)
multiplets."""
import itertools
import math

import numpy as np
import pytest

import workloads as W
from oracle import hamiltonian, spins


@pytest.mark.parametrize("N,two_s", [(5, 1), (4, 2), (4, 3), (3, 5), (2, 7)])
def test_rank_formula_equals_enumeration(N, two_s):
    for n in range(two_s * N + 1):
        digs = spins.sector_digits(N, two_s, n)
        assert digs.shape[0] == spins.sector_dim(N, two_s, n)
        for k, d in enumerate(digs):
            assert spins.rank_formula(d, two_s) == k


def test_spin_half_is_the_spin_half_oracle():
    cl = W.random_regular_cluster(8, 3, 1, J_range=(0.5, 1.5))
    for n in range(4, 9):
        a = spins.sector_hamiltonian(cl, 1, n).toarray()
        b = hamiltonian.sector_hamiltonian(cl, n).toarray()
        np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("N,two_s", [(4, 2), (3, 3), (3, 5)])
def test_sectors_are_blocks_of_the_kronecker_hamiltonian(N, two_s):
    rng = np.random.default_rng(3)
    pairs = [(0, 1), (1, 2), (0, 2)] + ([(2, 3), (0, 3)] if N == 4 else [])
    cl = W.Cluster(N, np.array([p[0] for p in pairs]), np.array([p[1] for p in pairs]),
                   rng.uniform(-1.0, 1.5, len(pairs)))
    Hf = spins.full_hamiltonian_kron(cl, two_s)
    B = two_s + 1
    allvals = np.arange(B ** N)
    sums = sum((allvals // B ** i) % B for i in range(N))
    for n in range(two_s * N + 1):
        idx = allvals[sums == n]
        Hs = spins.sector_hamiltonian(cl, two_s, n).toarray()
        np.testing.assert_allclose(Hs, Hf[np.ix_(idx, idx)], atol=1e-12)
        # no matrix element leaves the sector (S^z conserved)
        out = np.ones(B ** N, bool); out[idx] = False
        assert np.abs(Hf[np.ix_(idx, allvals[out])]).max(initial=0.0) < 1e-12


@pytest.mark.parametrize("two_s", [2, 3, 5])
def test_traces_closed_form(two_s):
    """Tr H = 0 and Tr H^2 = B^N (s(s+1))^2/3 sum_b J_b^2 over the whole space."""
    s = two_s / 2
    cl = W.Cluster(4, np.array([0, 1, 2, 3, 0]), np.array([1, 2, 3, 0, 2]), np.array([1.0, 0.7, -0.4, 1.3, 0.5]))
    t1 = t2 = 0.0
    for n in range(two_s * cl.n_sites + 1):
        H = spins.sector_hamiltonian(cl, two_s, n)
        t1 += H.diagonal().sum()
        t2 += (H.multiply(H)).sum()
    B = two_s + 1
    assert abs(t1) < 1e-9
    assert t2 == pytest.approx(B ** 4 * (s * (s + 1)) ** 2 / 3 * np.sum(cl.J ** 2), rel=1e-12)


@pytest.mark.parametrize("two_s", [1, 2, 3, 5])
def test_dimer_spectrum(two_s):
    """S_1.S_2 = [S(S+1) - 2 s(s+1)]/2 with total spin S = 0..2s; the sector
    S^z = m holds one state of every S >= |m|."""
    s = two_s / 2
    J = 1.3
    cl = W.Cluster(2, np.array([0]), np.array([1]), np.array([J]))
    for n in range(two_s + 1, 2 * two_s + 1):
        m = n - two_s
        e = np.linalg.eigvalsh(spins.sector_hamiltonian(cl, two_s, n).toarray())
        want = sorted(J / 2 * (S * (S + 1) - 2 * s * (s + 1)) for S in range(int(round(m)), two_s + 1))
        np.testing.assert_allclose(e, want, atol=1e-12)


def test_su2_multiplets_fe10_like_ring():
    """Spectrum(n + 1) is contained in spectrum(n) for S^z >= 0 (ring N=5, s=1)."""
    cl = W.ring(5)
    two_s = 2
    prev = None
    for n in range(5, 11):
        e = np.sort(np.linalg.eigvalsh(spins.sector_hamiltonian(cl, two_s, n).toarray()))
        if prev is not None:
            for x in e:
                k = np.argmin(np.abs(prev - x))
                assert abs(prev[k] - x) < 1e-9
                prev = np.delete(prev, k)
        prev = e


@pytest.mark.parametrize("two_s,cl", [(2, W.ring(4)), (3, W.Cluster(3, np.array([0, 1, 0]), np.array([1, 2, 2]),
                                                                      np.array([1.0, 0.6, -0.8])))])
def test_sector_thermodynamics_with_mirrors_match_full_space(two_s, cl):
    """The S^z >= 0 sectors with weight 2 for S^z != 0 (two_s given to the
    thermodynamics) reproduce ln Z, E, C, chi and <S^z> in a field h of the
    whole B^N space, with H - h S^z_total from Kronecker products."""
    from oracle import thermo
    N = cl.n_sites
    secs = spins.sectors(cl, two_s)
    probs = [dict(cluster=0, n_sites=N, n_up=n, two_s=two_s) for n, _ in secs]
    spectra = [np.linalg.eigvalsh(spins.sector_hamiltonian(cl, two_s, n).toarray()) for n, _ in secs]
    M = 8
    mus = np.zeros((len(secs), M))
    ab = np.tile([1.0, 0.0], (len(secs), 1))
    T = np.array([0.2, 0.7, 1.5, 4.0])
    h = np.array([0.0, 0.5, -1.1, 2.0])
    out = thermo.thermo_hybrid(probs, mus, ab, spectra, T, h, "none", M)
    H = spins.full_hamiltonian_kron(cl, two_s)
    Sz = spins.spin_matrices(two_s)[2]
    B = two_s + 1
    Szt = sum(np.kron(np.kron(np.eye(B ** (N - 1 - p)), Sz), np.eye(B ** p)) for p in range(N)).real
    for t, (Tv, hv) in enumerate(zip(T, h)):
        e, U = np.linalg.eigh(H + hv * Szt)    # Zeeman term with the sign convention E + h m
        # <S^z> and <(S^z)^2> per eigenvector (degenerate eigenvectors may mix
        # S^z sectors, so the square is taken as an operator)
        mz = np.einsum("ij,ik,kj->j", U, Szt, U)
        mz2 = np.einsum("ij,ik,kj->j", U, Szt @ Szt, U)
        w = np.exp(-(e - e.min()) / Tv)
        Z = w.sum()
        E = (w * e).sum() / Z
        Mz = (w * mz).sum() / Z
        ref = dict(lnZ=np.log(Z) - e.min() / Tv, E=E, C=((w * (e - E) ** 2).sum() / Z) / Tv ** 2,
                   chi=((w * mz2).sum() / Z - Mz ** 2) / Tv, M=Mz)
        for k, v in ref.items():
            assert abs(out[k][0, t] - v) < 1e-9 * max(1.0, abs(v)), (k, t, out[k][0, t], v)


@pytest.mark.parametrize("N,two_s,n", [(4, 2, 4), (5, 3, 8), (3, 5, 7), (6, 1, 3), (4, 7, 14), (3, 2, 6)])
def test_rank_table_and_unrank_invert_enumeration(N, two_s, n):
    digs = spins.sector_digits(N, two_s, n)
    np.testing.assert_array_equal(spins.rank_many(digs, two_s, n), np.arange(len(digs)))
    for r in range(len(digs)):
        np.testing.assert_array_equal(spins.unrank_formula(r, N, two_s, n), digs[r])
    with pytest.raises(ValueError):
        spins.unrank_formula(len(digs), N, two_s, n)


@pytest.mark.parametrize("two_s,cl,n,kind", [
    (2, W.ring(5), 5, "rademacher"),
    (3, W.Cluster(4, np.array([0, 1, 2, 0]), np.array([1, 2, 3, 2]), np.array([1.0, -0.7, 0.4, 1.2])), 7,
     "gaussian"),
    (5, W.ring(3), 9, "complex_gaussian")])
def test_recursion_rows_match_dense_chebyshev(two_s, cl, n, kind):
    """Rows of T_m(H') v_0 from the cones equal the dense recursion on the
    enumerated sector (m = 0..4, every row)."""
    from oracle import hamiltonian, rng
    H = spins.sector_hamiltonian(cl, two_s, n).toarray()
    dim = H.shape[0]
    e = np.linalg.eigvalsh(H)
    a, b = hamiltonian.scale_from_bounds(e.min() - 0.1, e.max() + 0.1, 0.025)
    Ht = (H - b * np.eye(dim)) / a
    V0, _, R_eff = rng.random_columns(kind, 3, 2, n, 2, dim)
    prev, cur = None, V0
    for m in range(5):
        if m == 1:
            prev, cur = cur, Ht @ cur
        elif m > 1:
            prev, cur = cur, 2 * Ht @ cur - prev
        got = spins.recursion_rows(cl, two_s, n, a, b, kind, 3, 2, np.arange(dim), m, cluster_id=2)
        np.testing.assert_allclose(got, cur, rtol=0, atol=1e-12 * max(1.0, np.abs(cur).max()))


@pytest.mark.parametrize("N,two_s,n", [(5, 2, 4), (4, 5, 11), (6, 3, 9), (3, 7, 20)])
def test_depth_first_enumeration_equals_brute_force(N, two_s, n):
    np.testing.assert_array_equal(spins._walk_digits(N, two_s, n), spins.sector_digits(N, two_s, n))
