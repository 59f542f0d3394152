"""Pins of oracle.rows (single rows of v_n = C_n(H') v_0) against an
independent route: T_n(H') v_0 from the eigendecomposition of the dense sector
matrix, T_n(x) = cos(n arccos x) (the Chebyshev polynomials of Eq. (6))."""
import numpy as np
import pytest

import workloads as W
from oracle import hamiltonian, rng, rows


def _dense_tn(H, a, b, V0, n):
    x, U = np.linalg.eigh((H.toarray() - b * np.eye(H.shape[0])) / a)
    t = np.cos(n * np.arccos(np.clip(x, -1.0, 1.0)))
    return U @ (t[:, None] * (U.T @ V0))


@pytest.mark.parametrize("cl,n_up,kind,R", [
    (W.ring(10), 5, "rademacher", 3), (W.ring(10), 7, "complex_gaussian", 2),
    (W.random_regular_cluster(11, 3, 4, J_range=(0.5, 1.5)), 6, "gaussian", 2),
    (W.j1j2_chain(12, 1.0, 0.5), 6, "rademacher", 2), (W.ladder(10), 4, "complex_gaussian", 1)])
def test_rows_equal_dense_chebyshev(cl, n_up, kind, R):
    H = hamiltonian.sector_hamiltonian(cl, n_up)
    e = np.linalg.eigvalsh(H.toarray())
    a, b = hamiltonian.scale_from_bounds(e.min() - 0.1, e.max() + 0.1, 0.025)
    V0, _, _ = rng.random_columns(kind, 3, 2, n_up, R, H.shape[0])
    sample = np.random.default_rng(0).choice(H.shape[0], size=min(12, H.shape[0]), replace=False)
    for n in range(5):
        want = _dense_tn(H, a, b, V0, n)[sample]
        got = rows.recursion_rows(cl, n_up, a, b, kind, 3, R, sample, n, cluster_id=2)
        assert np.abs(got - want).max() <= 1e-11 * max(1.0, np.abs(want).max()), n


def test_start_rows_are_the_start_block():
    dim = 3003
    for kind in ("rademacher", "gaussian", "complex_gaussian"):
        V0, _, _ = rng.random_columns(kind, 7, 5, 9, 3, dim)
        idx = np.array([0, 1, 17, 2999, 3002])
        assert np.allclose(rows.start_rows(kind, 7, 5, 9, 3, idx, dim), V0[idx], rtol=1e-13, atol=0)


def test_float32_storage_rounds_every_vector():
    cl = W.ring(12)
    H = hamiltonian.sector_hamiltonian(cl, 6)
    a, b = hamiltonian.scale_from_bounds(-5.5, 3.1, 0.025)
    V0, _, _ = rng.random_columns("complex_gaussian", 1, 0, 6, 2, H.shape[0])
    Ht = hamiltonian.rescaled(H, a, b)
    prev = V0.astype(np.float32).astype(np.float64)
    cur = (Ht @ prev).astype(np.float32).astype(np.float64)
    for _ in range(2):
        prev, cur = cur, (2.0 * (Ht @ cur) - prev).astype(np.float32).astype(np.float64)
    sample = np.arange(0, H.shape[0], 37)
    got = rows.recursion_rows(cl, 6, a, b, "complex_gaussian", 1, 2, sample, 3, store=np.float32)
    assert np.abs(got - cur[sample]).max() <= 4e-7 * np.abs(cur).max()
