"""Pins of the FTLM oracle (oracle/ftlm.py): Gauss-quadrature exactness of the
Lanczos weights, the estimator assembly against exp(-beta H) from the dense
eigendecomposition, and exactness with the complete basis."""
import numpy as np
import pytest

import workloads as W
from oracle import ed, ftlm, hamiltonian, rng


def test_lanczos_quadrature_reproduces_power_moments():
    cl = W.j1j2_chain(12, 1.0, 0.5)
    H = hamiltonian.sector_hamiltonian(cl, 6)
    v = rng.random_columns("gaussian", 4, 0, 6, 1, H.shape[0])[0][:, 0]
    q = v / np.linalg.norm(v)
    L = 8
    a, b = ftlm.lanczos_coefficients(H, v, L)
    e, z2 = ftlm.ritz(a, b)
    x = q.copy()
    for k in range(2 * L):
        want = q @ x                                    # <q|H^k|q>
        got = np.sum(z2 * e ** k)
        assert abs(got - want) <= 1e-11 * (1 + np.abs(e).max()) ** k, k
        x = H @ x


@pytest.mark.parametrize("kind,R", [("rademacher", 3), ("complex_gaussian", 2), ("gaussian", 2)])
def test_full_krylov_equals_stochastic_trace_of_exp(kind, R):
    """With M_L = dim the Krylov expansion is exact: the FTLM estimate equals
    dim/R sum_r <r|exp(-beta H)|r>/<r|r> from the dense eigendecomposition."""
    cl = W.ring(8)
    s = W.Sector(cl, 4, 0)
    H = hamiltonian.sector_hamiltonian(cl, 4).toarray()
    dim = H.shape[0]
    lst = ftlm.sector_ritz(s, dim, R, kind, 5)
    V0, voc, R_eff = rng.random_columns(kind, 5, 0, 4, R, dim)
    ev, U = np.linalg.eigh(H)
    for beta in (0.3, 1.0, 3.0):
        f = U @ np.diag(np.exp(-beta * ev)) @ U.T
        num = np.zeros(R_eff)
        den = np.zeros(R_eff)
        np.add.at(num, voc, np.einsum("ic,ij,jc->c", V0, f, V0))
        np.add.at(den, voc, (V0 * V0).sum(0))
        want = dim / R_eff * np.sum(num / den)
        got = sum(np.sum(w * np.exp(-beta * e)) for e, w in lst)
        assert abs(got - want) <= 1e-10 * want, beta


def test_complete_basis_ftlm_equals_ed():
    cl = W.ring(8)
    secs = W.sectors(cl)
    probs = [dict(cluster=0, n_sites=8, n_up=s.n_up) for s in secs]
    lists = [ftlm.sector_ritz(s, s.dim, 0, "basis", 0) for s in secs]
    T = W.log_temperatures(25, 0.1, 10.0)
    out = ftlm.ftlm_thermo(probs, lists, T)
    ref = ed.thermo_from_spectra(ed.sector_spectra(secs), T)
    for k in ("lnZ", "E", "C", "chi"):
        assert np.abs(out[k][0] - ref[k]).max() <= 1e-8 * max(1.0, np.abs(ref[k]).max()), k
    assert np.abs(out["M"]).max() <= 1e-12


def test_complete_basis_ftlm_with_field_equals_dense_ed():
    cl = W.random_regular_cluster(7, 3, 1, J_range=(0.5, 1.5))
    secs = W.sectors(cl)
    probs = [dict(cluster=0, n_sites=7, n_up=s.n_up) for s in secs]
    lists = [ftlm.sector_ritz(s, s.dim, 0, "basis", 0) for s in secs]
    T = np.array([0.2, 0.5, 1.0, 3.0])
    h = np.array([0.7, -1.5, 2.0, 0.0])
    out = ftlm.ftlm_thermo(probs, lists, T, h)
    H0 = hamiltonian.full_hamiltonian_kron(cl)
    szt = np.array([bin(i).count("1") for i in range(1 << 7)]) - 3.5
    for t, (Tv, hv) in enumerate(zip(T, h)):
        e = np.linalg.eigvalsh(H0 + hv * np.diag(szt))
        w = np.exp(-(e - e.min()) / Tv)
        assert abs(out["lnZ"][0, t] - (np.log(w.sum()) - e.min() / Tv)) < 1e-9
        Em = (w * e).sum() / w.sum()
        assert abs(out["E"][0, t] - Em) < 1e-9
        assert abs(out["C"][0, t] - ((w * (e - Em) ** 2).sum() / w.sum()) / Tv**2) < 1e-8
