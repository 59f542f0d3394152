"""GPU vs oracle: exact spectra of small sectors and the hybrid
thermodynamics that use them (Sec. II: small sectors are diagonalised
completely).

* kpm_sector_eigenvalues: every eigenvalue within 1e-10 * max(1, |E|max) of
  the oracle's dense diagonalisation, ascending, NaN past the spectrum and in
  the rows of sectors above max_dim;
* kpm_thermo_hybrid on identical inputs (the oracle's moments and spectra):
  1e-12 (relative for ln Z and E, peak-normalised for C and chi, over
  max(1, |M|) for the magnetisation);
* end to end (GPU spectra and moments vs the oracle's on the same seeds and
  bounds): 1e-9, and with every sector exact the result is dense ED."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import ed, hamiltonian, moments, thermo

pytestmark = pytest.mark.gpu


def _probs(secs):
    return [dict(cluster=s.cluster_id, n_sites=s.cluster.n_sites, n_up=s.n_up) for s in secs]


def _cmp(got, want, q, tol):
    if q == "M":      # <S^z> vanishes without a field: normalise by max(1, |M|)
        err = np.abs(got - want).max() / max(np.abs(want).max(), 1.0)
    elif q in ("C", "chi"):
        err = np.abs(got - want).max() / max(np.abs(want).max(), 1e-300)
    else:
        err = (np.abs(got - want) / np.maximum(np.abs(want), 1e-300)).max()
    assert err <= tol, (q, err)


@pytest.mark.parametrize("cl,max_dim", [
    (W.ring(12), 1000), (W.random_regular_cluster(11, 3, 2, J_range=(0.5, 1.5)), 500),
    (W.j1j2_chain(12, 1.0, 0.5), 924), (W.ladder(10), 300), (W.dimer(), 4)])
def test_spectra_match_dense_diagonalisation(kpm, cl, max_dim):
    secs = W.sectors(cl)
    ev = kpm.sector_eigenvalues(secs, max_dim).cpu().numpy()
    ref = ed.sector_spectra(secs)
    for p, (s, (e, _, _)) in enumerate(zip(secs, ref)):
        row = ev[p]
        if s.dim > max_dim:
            assert np.all(np.isnan(row)), p
            continue
        got = row[:s.dim]
        assert np.all(np.diff(got) >= 0), p
        scale = max(1.0, np.abs(e).max())
        assert np.abs(got - e).max() <= 1e-10 * scale, (p, s.n_up, np.abs(got - e).max())
        assert np.all(np.isnan(row[s.dim:])), p


def test_spectra_of_several_clusters_in_one_call(kpm):
    secs = []
    for cid, cl in enumerate([W.ring(8), W.random_regular_cluster(9, 3, 4, J_range=(0.5, 1.5)),
                              W.sawtooth(10)]):
        secs += W.sectors(cl, cluster_id=cid)
    ev = kpm.sector_eigenvalues(secs, 256).cpu().numpy()
    for p, (s, (e, _, _)) in enumerate(zip(secs, ed.sector_spectra(secs))):
        if s.dim <= 256:
            assert np.abs(ev[p, :s.dim] - e).max() <= 1e-10 * max(1.0, np.abs(e).max()), p


def _moment_setup(secs, M, eps=0.025):
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


@pytest.mark.parametrize("kernel,field", [("jackson", False), ("none", True)])
def test_hybrid_on_identical_inputs(kpm, kernel, field):
    secs = W.sectors(W.ladder(10), cluster_id=0) + W.sectors(W.ring(9), cluster_id=1)
    M = 128
    mus, ab = _moment_setup(secs, M)
    spec = ed.sector_spectra(secs)
    exact = np.array([s.dim <= 120 for s in secs], dtype=np.uint8)
    ld = 128
    evals = np.full((len(secs), ld), np.nan)
    for p, (e, _, _) in enumerate(spec):
        if exact[p]:
            evals[p, :e.size] = e
    T = W.log_temperatures(40, 0.02, 10.0)
    h = np.linspace(-0.5, 2.0, T.size) if field else None
    out = kpm.thermo_hybrid(torch.tensor(mus, device="cuda"), torch.tensor(ab, device="cuda"), secs,
                            torch.tensor(evals, device="cuda"), exact, T, h, kernel)
    ref = thermo.thermo_hybrid(_probs(secs), mus, ab, [spec[p][0] if exact[p] else None for p in range(len(secs))],
                               T, 0.0 if h is None else h, kernel)
    for q in ("lnZ", "E", "C", "chi", "M"):
        _cmp(out[q].cpu().numpy(), ref[q], q, 1e-12)
    assert not out["z_nonpos"].cpu().numpy().any()


def test_hybrid_end_to_end_stochastic_large_sectors(kpm):
    """GPU moments (Rademacher, same seeds and bounds as the oracle) for the
    large sectors, GPU spectra for the small ones, against the oracle's."""
    cl = W.random_regular_cluster(12, 3, 5, J_range=(0.5, 1.5))
    secs = W.sectors(cl)
    M, R = 96, 6
    mus_ex, ab = _moment_setup(secs, M)
    bl = [(b - a * (1 - 0.0125), b + a * (1 - 0.0125)) for a, b in ab]
    mu, abd = kpm.chebyshev_moments(secs, M, R, "rademacher", "fp64", 0.025, 3, bounds=bl)
    want_mu = np.array([moments.sector_moments(s, a, b, M, R, "rademacher", 3) for s, (a, b) in zip(secs, ab)])
    assert np.abs(mu.cpu().numpy() - want_mu).max() <= 1e-10 * want_mu[:, :1].max()
    exact = np.array([s.dim <= 220 for s in secs], dtype=np.uint8)
    ev = kpm.sector_eigenvalues(secs, 256)
    T = W.log_temperatures(30, 0.1, 10.0)
    out = kpm.thermo_hybrid(mu, abd, secs, ev, exact, T)
    spec = ed.sector_spectra(secs)
    ref = thermo.thermo_hybrid(_probs(secs), want_mu, np.array(ab),
                               [spec[p][0] if exact[p] else None for p in range(len(secs))], T, 0.0, "jackson")
    for q in ("lnZ", "E", "C", "chi"):
        _cmp(out[q].cpu().numpy(), ref[q], q, 1e-9)


def test_hybrid_all_exact_is_ed(kpm):
    cl = W.ring(12)
    secs = W.sectors(cl)
    ev = kpm.sector_eigenvalues(secs, 1000)
    mus, ab = _moment_setup(secs, 32)
    T = W.log_temperatures(50, 0.01, 10.0)
    out = kpm.thermo_hybrid(torch.tensor(mus, device="cuda"), torch.tensor(ab, device="cuda"), secs, ev,
                            np.ones(len(secs), dtype=np.uint8), T)
    ref = ed.thermo_from_spectra(ed.sector_spectra(secs), T)
    for q in ("lnZ", "E", "C", "chi"):
        _cmp(out[q].cpu().numpy()[0], ref[q], q, 1e-9)


def test_workspace_contract(kpm):
    import ctypes
    secs = W.sectors(W.ring(10))
    ps = kpm.ProblemSet(secs)
    lib = kpm.load()
    need = lib.kpm_sector_eigenvalues_workspace_size(ps.arr, len(ps), 300)
    ev = torch.empty((len(secs), 300), dtype=torch.float64, device="cuda")
    ws = torch.empty(need - 1, dtype=torch.uint8, device="cuda")
    assert lib.kpm_sector_eigenvalues(ps.arr, len(ps), 300, ctypes.c_void_p(ev.data_ptr()),
                                      ctypes.c_void_p(ws.data_ptr()), ws.numel(), None) == kpm.KPM_EWORKSPACE
    assert lib.kpm_sector_eigenvalues(ps.arr, len(ps), 300, ctypes.c_void_p(ev.data_ptr()), None, 0,
                                      None) == 0
