"""GPU vs oracle: Jackson kernel, DOS weights and thermodynamics (Sec. II).

(i) kpm_thermo on identical moments: relative 1e-12 for ln Z and E,
    peak-normalised 1e-12 for C and chi, at every temperature;
(ii) end to end (GPU moments + GPU thermo vs oracle moments + oracle thermo on
    the same seeds): peak-normalised 1e-8 for T >= T_phys, the lowest grid
    temperature above which the float64 estimate has Z > 0 and C >= 0."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import ed, hamiltonian, moments, thermo

pytestmark = pytest.mark.gpu


def _probs(secs):
    return [dict(cluster=s.cluster_id, n_sites=s.cluster.n_sites, n_up=s.n_up) for s in secs]


def _exact_setup(secs, eps, M):
    mus, ab = [], []
    for s in secs:
        e = np.linalg.eigvalsh(hamiltonian.sector_hamiltonian(s.cluster, s.n_up).toarray())
        lo, hi = e.min(), e.max()
        if hi - lo < 1e-8:
            lo, hi = lo - 0.5, hi + 0.5
        a, b = hamiltonian.scale_from_bounds(lo, hi, eps)
        mus.append(moments.exact_moments((e - b) / a, M))
        ab.append((a, b))
    return np.array(mus), np.array(ab)


def _cmp(got, want, quantity, mask=None, tol=1e-12):
    g, w = got, want
    if mask is not None:
        g, w = g[:, mask], w[:, mask]
    if quantity in ("C", "chi"):
        err = np.abs(g - w).max() / np.abs(w).max()
    else:
        err = (np.abs(g - w) / np.maximum(np.abs(w), 1e-300)).max()
    assert err <= tol, (quantity, err)


@pytest.mark.parametrize("kernel", ["none", "jackson"])
def test_thermo_on_identical_moments_ring12(kpm, kernel):
    secs = W.sectors(W.ring(12))
    mus, ab = _exact_setup(secs, 0.025, 256)
    T = W.log_temperatures(200, 0.01, 10.0)
    out = kpm.thermo(torch.tensor(mus, device="cuda"), torch.tensor(ab, device="cuda"), secs, T, kernel)
    ref = thermo.thermo(_probs(secs), mus, ab, T, kernel)
    for q in ("lnZ", "E", "C", "chi"):
        _cmp(out[q].cpu().numpy(), ref[q], q)
    assert not out["z_nonpos"].any()


def test_thermo_multi_cluster_nodes_and_improper_dos(kpm):
    """Three clusters, Ntil != M, and moments whose DOS is improper (Z <= 0 at low T)."""
    secs = []
    for cid, cl in enumerate([W.ladder(8), W.random_regular_cluster(9, 3, 1, J_range=(0.5, 1.5)), W.ring(10)]):
        secs += W.sectors(cl, cluster_id=cid)
    mus, ab = _exact_setup(secs, 0.1, 60)
    mus[0, 1:] *= 1.3            # not a proper density any more
    T = W.log_temperatures(60, 0.005, 20.0)
    for Nt in (60, 97):
        out = kpm.thermo(torch.tensor(mus, device="cuda"), torch.tensor(ab, device="cuda"), secs, T,
                         "none", Nt)
        ref = thermo.thermo(_probs(secs), mus, ab, T, "none", Nt)
        zn = out["z_nonpos"].cpu().numpy().astype(bool)
        assert np.array_equal(zn, ref["z_nonpos"])
        ok = ~ref["z_nonpos"].any(axis=0)
        for q in ("E", "C", "chi"):
            _cmp(out[q].cpu().numpy(), ref[q], q, mask=ok, tol=1e-11)
        lz = out["lnZ"].cpu().numpy()
        assert np.all(np.isnan(lz[zn]))
        _cmp(lz, ref["lnZ"], "lnZ", mask=ok, tol=1e-12)


def test_thermo_vjp_matches_oracle(kpm):
    secs = W.sectors(W.j1j2_chain(10, 1.0, 0.5))
    mus, ab = _exact_setup(secs, 0.025, 80)
    T = W.log_temperatures(16, 0.05, 5.0)
    rng = np.random.default_rng(4)
    wC, wX = rng.normal(size=(1, 16)), rng.normal(size=(1, 16))
    for kernel in ("none", "jackson"):
        lam = kpm.thermo_vjp(torch.tensor(mus, device="cuda"), torch.tensor(ab, device="cuda"), secs, T,
                             wC, wX, kernel).cpu().numpy()
        ref = thermo.thermo_vjp(_probs(secs), mus, ab, T, wC, wX, kernel)
        assert np.abs(lam - ref).max() <= 1e-9 * np.abs(ref).max()


def test_end_to_end_ring12_config(kpm):
    """Ring N=12, all sectors, R=20 Rademacher from seed 0, M=256, eps=0.025,
    exact bounds, Jackson kernel, 200 log-spaced T in [0.01, 10]."""
    secs = W.sectors(W.ring(12))
    bl = []
    for s in secs:
        e = np.linalg.eigvalsh(hamiltonian.sector_hamiltonian(s.cluster, s.n_up).toarray())
        lo, hi = e.min(), e.max()
        bl.append((lo - 0.5, hi + 0.5) if hi - lo < 1e-8 else (lo, hi))
    T = W.log_temperatures(200, 0.01, 10.0)
    mu, ab = kpm.chebyshev_moments(secs, 256, 20, "rademacher", "fp64", 0.025, 0, bounds=bl)
    ref_mu = np.array([moments.sector_moments(s, *hamiltonian.scale_from_bounds(lo, hi, 0.025), 256, 20,
                                              "rademacher", 0) for s, (lo, hi) in zip(secs, bl)])
    for kernel in ("jackson", "none"):
        out = kpm.thermo(mu, ab, secs, T, kernel)
        ref = thermo.thermo(_probs(secs), ref_mu, ab.cpu().numpy(), T, kernel)
        C = ref["C"][0]
        bad = np.nonzero((C < 0) | ref["z_nonpos"][0])[0]
        t_phys = T[bad.max() + 1] if bad.size else T[0]
        band = T >= t_phys
        for q in ("lnZ", "E", "C", "chi"):
            _cmp(out[q].cpu().numpy(), ref[q], q, mask=band, tol=1e-8)
    # the stochastic estimate tracks exact diagonalisation at high T
    ex = ed.thermo_from_spectra(ed.sector_spectra(secs), T)
    hiT = T >= 0.5
    assert np.abs(out["C"].cpu().numpy()[0][hiT] - ex["C"][hiT]).max() < 0.05 * ex["C"].max()


@pytest.mark.parametrize("kernel", ["none", "jackson"])
def test_field_thermo_on_identical_moments(kpm, kernel):
    """kpm_thermo_field vs the oracle's thermo_field on identical moments: two
    clusters (even and odd N), 120 (T, h) points including h = 0 and h < 0."""
    secs = W.sectors(W.ring(10)) + W.sectors(W.random_regular_cluster(9, 3, 2, J_range=(0.5, 1.5)),
                                             cluster_id=1)
    mus, ab = _exact_setup(secs, 0.025, 200)
    T = np.tile(W.log_temperatures(40, 0.05, 8.0), 3)
    h = np.repeat([0.0, 1.7, -0.6], 40)
    out = kpm.thermo_field(torch.tensor(mus, device="cuda"), torch.tensor(ab, device="cuda"), secs, T, h, kernel)
    ref = thermo.thermo_field(_probs(secs), mus, ab, T, h, kernel)
    for q in ("lnZ", "E", "C", "chi"):
        _cmp(out[q].cpu().numpy(), ref[q], q)
    M = out["M"].cpu().numpy()
    assert np.abs(M - ref["M"]).max() <= 1e-12 * 5.0      # |<S^z>| <= N/2
    # zero field: the field kernel agrees with kpm_thermo to rounding
    z = kpm.thermo(torch.tensor(mus, device="cuda"), torch.tensor(ab, device="cuda"), secs, T[:40], kernel)
    for q in ("lnZ", "E", "C", "chi"):
        _cmp(out[q].cpu().numpy()[:, :40], z[q].cpu().numpy(), q)
    assert np.abs(M[:, :40]).max() <= 1e-12


def test_field_thermo_end_to_end_ring12(kpm):
    """GPU moments (float64, 20 Rademacher vectors) + GPU field thermodynamics
    against the oracle's moments + thermo_field on the same seeds and bounds."""
    secs = W.sectors(W.ring(12))
    bl = []
    for s in secs:
        e = np.linalg.eigvalsh(hamiltonian.sector_hamiltonian(s.cluster, s.n_up).toarray())
        bl.append((e.min() - 0.05, e.max() + 0.05))
    M = 256
    mu, ab = kpm.chebyshev_moments(secs, M, 20, "rademacher", "fp64", 0.025, 0, bounds=bl)
    T = np.tile(W.log_temperatures(30, 0.2, 10.0), 2)
    h = np.repeat([0.5, 2.0], 30)
    out = kpm.thermo_field(mu, ab, secs, T, h, "jackson")
    abh = ab.cpu().numpy()
    want_mu = np.array([moments.sector_moments(s, a, b, M, 20, "rademacher", 0) for s, (a, b) in zip(secs, abh)])
    ref = thermo.thermo_field(_probs(secs), want_mu, abh, T, h, "jackson")
    for q in ("lnZ", "E", "C", "chi"):
        _cmp(out[q].cpu().numpy(), ref[q], q, tol=1e-8)
    assert np.abs(out["M"].cpu().numpy() - ref["M"]).max() <= 1e-8 * 6.0
