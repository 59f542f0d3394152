"""Oracle pins: derivatives with respect to the couplings J_b (bounds fixed)."""
import numpy as np
import pytest

import workloads as W
from oracle import adjoint, ed, hamiltonian, moments, thermo


def _bounds(sectors, eps=0.025):
    ab = []
    for s in sectors:
        e = np.linalg.eigvalsh(hamiltonian.sector_hamiltonian(s.cluster, s.n_up).toarray())
        lo, hi = e.min() - 0.05, e.max() + 0.05
        ab.append(hamiltonian.scale_from_bounds(lo, hi, eps))
    return np.array(ab)


def test_adjoint_matches_central_differences_j1j2_n8():
    cl = W.j1j2_chain(8, 1.0, 0.5)
    secs = W.sectors(cl, only_sz0=True) + [W.Sector(cl, 5, 0)]
    ab = _bounds(secs)
    T = np.array([0.2, 0.6, 1.5])
    wC = np.ones((1, 3))
    wX = np.array([[0.3, -0.2, 0.5]])
    args = (secs, ab, 40, 3, "rademacher", 0, T, wC, wX, "none", 40)
    g = adjoint.pipeline_grad(*args)
    fd = adjoint.pipeline_grad_fd(*args, h=1e-5)
    assert np.linalg.norm(g - fd) <= 1e-6 * np.linalg.norm(g)


def test_adjoint_with_jackson_and_complex_vectors():
    cl = W.random_regular_cluster(8, 3, 2, J_range=(0.5, 1.5))
    secs = W.sectors(cl)[:3]
    ab = _bounds(secs)
    T = np.array([0.5, 2.0])
    wC = np.array([[1.0, 0.5]])
    wX = np.array([[0.0, 1.0]])
    args = (secs, ab, 31, 2, "complex_gaussian", 4, T, wC, wX, "jackson", 40)
    g = adjoint.pipeline_grad(*args)
    fd = adjoint.pipeline_grad_fd(*args, h=1e-5)
    assert np.linalg.norm(g - fd) <= 1e-6 * np.linalg.norm(g)


def test_complete_basis_adjoint_equals_kpm_hellmann_feynman():
    """With exact traces, d mu_n/dJ_b = sum_i n U_{n-1}(x_i) <i|h_b|i> / a."""
    cl = W.j1j2_chain(8, 1.0, 0.5)
    s = W.Sector(cl, 4, 0)
    (a, b), = _bounds([s])
    M = 60
    hf = adjoint.kpm_hellmann_feynman(s, a, b, M)          # [n_bonds, M]
    lam = np.random.default_rng(1).normal(size=M)
    got = adjoint.sector_moments_vjp(s, a, b, M, 0, "basis", 0, lam)
    np.testing.assert_allclose(got, hf @ lam, rtol=1e-9, atol=1e-9 * np.abs(hf @ lam).max())


def test_ed_hellmann_feynman_matches_fd_and_euler_homogeneity():
    cl = W.random_regular_cluster(8, 3, 9, J_range=(0.5, 1.5))
    secs = W.sectors(cl)
    T = np.array([0.3, 0.8, 2.0])
    g = ed.hellmann_feynman_C(secs, T)
    h = 1e-5
    for bnd in (0, 5):
        Jp, Jm = cl.J.copy(), cl.J.copy()
        Jp[bnd] += h
        Jm[bnd] -= h
        Cp = ed.thermo_from_spectra(ed.sector_spectra([W.Sector(cl.with_J(Jp), s.n_up) for s in secs]), T)["C"]
        Cm = ed.thermo_from_spectra(ed.sector_spectra([W.Sector(cl.with_J(Jm), s.n_up) for s in secs]), T)["C"]
        np.testing.assert_allclose(g[bnd], (Cp - Cm) / (2 * h), rtol=1e-6)
    # C depends on beta J only: sum_b J_b dC/dJ_b = -T dC/dT
    spec = ed.sector_spectra(secs)
    dT = 1e-5
    dCdT = (ed.thermo_from_spectra(spec, T + dT)["C"] - ed.thermo_from_spectra(spec, T - dT)["C"]) / (2 * dT)
    np.testing.assert_allclose(cl.J @ g, -T * dCdT, rtol=1e-6)


def test_symmetric_bonds_have_equal_exact_gradients():
    """Ring: all bonds are equivalent, so exact-trace gradients coincide."""
    cl = W.ring(8)
    s = W.Sector(cl, 4, 0)
    (a, b), = _bounds([s])
    lam = np.random.default_rng(2).normal(size=30)
    got = adjoint.sector_moments_vjp(s, a, b, 30, 0, "basis", 0, lam)
    assert np.ptp(got) < 1e-10 * np.abs(got).max()
