"""Oracle pins: Chebyshev moments, Eqs. (6)-(7)."""
import numpy as np
import pytest

import workloads as W
from oracle import hamiltonian, moments, rng


def _sector(cl, k):
    return W.Sector(cl, k, 0)


def _ab(H, eps=0.025):
    e = np.linalg.eigvalsh(H.toarray())
    return hamiltonian.scale_from_bounds(e.min(), e.max(), eps), e


def test_doubling_equals_direct_recursion():
    s = _sector(W.random_regular_cluster(12, 3, 2, J_range=(0.5, 1.5)), 6)
    H = hamiltonian.sector_hamiltonian(s.cluster, 6)
    (a, b), _ = _ab(H)
    for kind in ("rademacher", "complex_gaussian", "gaussian"):
        m1 = moments.sector_moments(s, a, b, 101, 4, kind, 3, H=H)
        m2 = moments.sector_moments(s, a, b, 101, 4, kind, 3, H=H, direct=True)
        assert np.abs(m1 - m2).max() <= 1e-12 * m1[0]


def test_complete_basis_equals_diagonalisation():
    """Sec. II: traces with a complete basis are the exact moments of Eq. (6)."""
    s = _sector(W.ring(10), 5)
    H = hamiltonian.sector_hamiltonian(s.cluster, 5)
    (a, b), e = _ab(H)
    mb = moments.sector_moments(s, a, b, 200, 0, "basis", 0, H=H)
    me = moments.exact_moments((e - b) / a, 200)
    assert np.abs(mb - me).max() <= 1e-11 * mb[0]
    assert mb[0] == pytest.approx(252)


def test_exact_moments_closed_form_dimer():
    """Dimer S^z=0: eigenvalues -3J/4, J/4, so mu_n = cos(n t1) + cos(n t2)."""
    d = W.dimer(1.0)
    a, b = hamiltonian.scale_from_bounds(-0.75, 0.25, 0.1)
    x = (np.array([-0.75, 0.25]) - b) / a
    n = np.arange(64)
    want = np.cos(n * np.arccos(x[0])) + np.cos(n * np.arccos(x[1]))
    got = moments.sector_moments(W.Sector(d, 1, 0), a, b, 64, 0, "basis", 0)
    np.testing.assert_allclose(got, want, atol=1e-13)
    got_ed = moments.sector_exact_moments(W.Sector(d, 1, 0), a, b, 64)
    np.testing.assert_allclose(got_ed, want, atol=1e-13)


def test_trace_of_first_moments_closed_form():
    """Exact mu_1 = (Tr_k H - b dim)/a, with Tr_k H in closed form."""
    import math
    cl = W.j1j2_chain(10, 1.0, 0.5)
    N, k = 10, 6
    s = _sector(cl, k)
    H = hamiltonian.sector_hamiltonian(cl, k)
    (a, b), _ = _ab(H)
    mb = moments.sector_moments(s, a, b, 4, 0, "basis", 0, H=H)
    c = math.comb
    trH = np.sum(cl.J) / 4 * (c(N - 2, k - 2) + c(N - 2, k) - 2 * c(N - 2, k - 1))
    dim = c(N, k)
    assert mb[1] == pytest.approx((trH - b * dim) / a, abs=1e-11)
    # mu_2 = 2 Tr(H'^2) - dim
    trH2 = (H.multiply(H)).sum()
    trHt2 = (trH2 - 2 * b * trH + b * b * dim) / a**2
    assert mb[2] == pytest.approx(2 * trHt2 - dim, abs=1e-10)


def test_rademacher_estimator_unbiased_with_known_variance():
    """<r|A|r> over Rademacher r: mean Tr A, variance 2(||A||_F^2 - sum A_ii^2)."""
    s = _sector(W.ring(8), 4)
    H = hamiltonian.sector_hamiltonian(s.cluster, 4)
    (a, b), e = _ab(H)
    n = 7
    Ht = hamiltonian.rescaled(H, a, b).toarray()
    # A = C_n(H') by the recursion on dense matrices
    T0, T1 = np.eye(Ht.shape[0]), Ht
    for _ in range(n - 1):
        T0, T1 = T1, 2 * Ht @ T1 - T0
    A = T1
    vals = []
    for seed in range(1500):
        r = rng.rademacher(seed, 0, 4, 0, Ht.shape[0])
        vals.append(r @ A @ r)
    vals = np.array(vals)
    var = 2 * (np.sum(A * A) - np.sum(np.diag(A) ** 2))
    assert abs(vals.mean() - np.trace(A)) < 5 * np.sqrt(var / vals.size)
    assert vals.var() == pytest.approx(var, rel=0.15)


def test_stochastic_error_scales_as_inverse_sqrt_R_dim():
    """Sec. II: the relative error of Eq. (7) falls like 1/sqrt(R dim)."""
    s = _sector(W.ring(12), 6)
    H = hamiltonian.sector_hamiltonian(s.cluster, 6)
    (a, b), e = _ab(H)
    exact = moments.exact_moments((e - b) / a, 32)
    err = {}
    for R in (2, 32):
        errs = [np.abs(moments.sector_moments(s, a, b, 32, R, "rademacher", sd, H=H) - exact)[1:].mean()
                for sd in range(6)]
        err[R] = np.mean(errs)
    ratio = err[2] / err[32]
    assert 2.0 < ratio < 8.0      # sqrt(16) = 4


def test_moment_magnitude_and_mu0():
    s = _sector(W.ring(12), 7)
    H = hamiltonian.sector_hamiltonian(s.cluster, 7)
    (a, b), _ = _ab(H)
    m = moments.sector_moments(s, a, b, 300, 5, "complex_gaussian", 0, H=H)
    assert m[0] == pytest.approx(792, rel=1e-14)
    assert np.all(np.abs(m) <= m[0] * (1 + 1e-12))


def test_narrow_bounds_make_moments_grow():
    s = _sector(W.ring(10), 5)
    H = hamiltonian.sector_hamiltonian(s.cluster, 5)
    e = np.linalg.eigvalsh(H.toarray())
    a, b = hamiltonian.scale_from_bounds(e.min(), e.max() - 0.5, 0.0)
    m = moments.sector_moments(s, a, b, 200, 2, "rademacher", 0, H=H)
    assert np.abs(m).max() > 1.5 * m[0]


def test_lanczos_bounds_enclose_spectrum():
    for cl in [W.ring(12), W.random_regular_cluster(12, 3, 4, J_range=(0.5, 1.5)), W.j1j2_chain(12)]:
        for k in range(6, 13):
            s = W.Sector(cl, k, 0)
            H = hamiltonian.sector_hamiltonian(cl, k)
            e = np.linalg.eigvalsh(H.toarray())
            lo, hi = moments.spectral_bounds(s, 50, 0.01, 0, H=H)
            assert lo <= e.min() and hi >= e.max()
            assert hi - lo <= 1.05 * max(e.max() - e.min(), 0) + 1.0 + 1e-12


def test_fp32_storage_close_to_fp64():
    s = _sector(W.ring(14), 7)
    H = hamiltonian.sector_hamiltonian(s.cluster, 7)
    (a, b), _ = _ab(H)
    m64 = moments.sector_moments(s, a, b, 512, 4, "rademacher", 0, H=H)
    m32 = moments.sector_moments(s, a, b, 512, 4, "rademacher", 0, H=H, store=np.float32)
    d = np.abs(m32 - m64).max() / m64[0]
    assert 1e-12 < d < 1e-6


def test_lanczos_bounds_enclose_symmetric_one_magnon_sectors():
    """Regression: in the n_up = N-1 sectors of the 64-cluster workload the top
    eigenvector is the uniform one-magnon state; a +-1 start vector with equal
    numbers of signs is orthogonal to it.  The Gaussian start must still find
    the exact extremes (steps >= dim: the Krylov space is the whole sector)."""
    import workloads as W
    from oracle import hamiltonian
    cls = W.batched_clusters()
    # cluster 24 (N = 18): its n_up = 17 start vector has nine +1 and nine -1
    for cid in (24, 0, 1, 2):
        cl = cls[cid]
        for n_up in (cl.n_sites - 1, cl.n_sites - 2):
            s = W.Sector(cl, n_up, cid)
            e = np.linalg.eigvalsh(hamiltonian.sector_hamiltonian(cl, n_up).toarray())
            lo, hi = moments.spectral_bounds(s, 50, 0.01, 0)
            assert lo <= e.min() and hi >= e.max(), (cid, n_up, lo, hi, e.min(), e.max())
