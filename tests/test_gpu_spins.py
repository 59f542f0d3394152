"""GPU vs oracle: spin-s Heisenberg sectors (the spin-5/2 Fe10 wheel of
Sec. III.B and other spin s > 1/2 clusters) through the spin-s step kernel.

* Chebyshev moments (Eqs. (6)-(7)) on identical seeds and bounds: float64
  vectors within 1e-10 of mu_0, float32 storage within 1e-6 of mu_0 against
  the oracle with the same float32 rounding, every column width the kernel
  is instantiated for;
* spin-1/2 sectors in a call that holds spin-s ones run through the same
  kernel and match the spin-1/2 oracle;
* Lanczos bounds, thermodynamics with the mirror weight and S^z = n - sN
  (with and without the Zeeman term), FTLM Ritz values and thermodynamics;
* the full Fe10 wheel (N = 10, s = 5/2, S^z = 0: 4,395,456 states; all 26
  S^z >= 0 sectors: 32,430,816 states): sampled rows of v_1..v_3 against the
  oracle's cone recursion, mu_0 = dim and |mu_n| <= mu_0 everywhere;
* exact spectra of small spin-s sectors (the five smallest Fe10 sectors
  among them) and the hybrid sums that mix them with moments;
* the gradient entry points refuse spin s."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import ftlm, hamiltonian, moments, spins, thermo

pytestmark = pytest.mark.gpu


def _H(sec):
    if isinstance(sec, W.SpinSector):
        return spins.sector_hamiltonian(sec.cluster, sec.two_s, sec.n)
    return hamiltonian.sector_hamiltonian(sec.cluster, sec.n_up)


def _bounds(H):
    e = np.linalg.eigvalsh(H.toarray())
    lo, hi = e.min(), e.max()
    if hi - lo < 1e-8:
        lo, hi = lo - 0.5, hi + 0.5
    return lo, hi


def _probs(secs):
    return [dict(cluster=s.cluster_id, n_sites=s.cluster.n_sites, n_up=s.n_up,
                 two_s=getattr(s, "two_s", 1)) for s in secs]


def _moments(kpm, secs, M, R, kind, precision, col_block=0, seed=0, eps=0.025):
    Hs = [_H(s) for s in secs]
    bl = [_bounds(H) for H in Hs]
    mu, ab = kpm.chebyshev_moments(secs, M, R, kind, precision, eps, seed, col_block, bounds=bl)
    st = kpm.last_run_stats()
    store = np.float32 if precision == "fp32" else np.float64
    want = []
    for s, (lo, hi), H in zip(secs, bl, Hs):
        a, b = hamiltonian.scale_from_bounds(lo, hi, eps)
        want.append(moments.sector_moments(s, a, b, M, R, kind, seed, store=store, H=H))
    return mu.cpu().numpy(), np.array(want), ab.cpu().numpy(), bl, st


def _close(got, want, tol):
    for p in range(want.shape[0]):
        err = np.abs(got[p] - want[p]).max() / abs(want[p, 0])
        assert err <= tol, (p, err)


CLUSTERS = {
    "s1_ring6": (2, W.ring(6)),
    "s3/2_ring5": (3, W.ring(5)),
    "s5/2_ring4": (5, W.ring(4)),
    "s1_random7": (2, W.random_regular_cluster(7, 2, 3, J_range=(-0.6, 1.4))),
    "s7/2_triangle": (7, W.Cluster(3, np.array([0, 1, 0]), np.array([1, 2, 2]), np.array([1.0, 0.6, -0.8]))),
}


@pytest.mark.parametrize("name", list(CLUSTERS))
def test_moments_fp64_all_sectors(kpm, name):
    two_s, cl = CLUSTERS[name]
    secs = W.spin_sectors(cl, two_s)
    got, want, ab, bl, st = _moments(kpm, secs, 128, 4, "rademacher", "fp64")
    assert st["kernel"] == 4, st
    _close(got, want, 1e-10)
    assert np.all(got[:, 0] == [s.dim for s in secs])      # fully polarised sector: dim 1


@pytest.mark.parametrize("col_block", [1, 2, 4, 8])
@pytest.mark.parametrize("precision", ["fp32", "fp64"])
def test_moments_column_widths(kpm, precision, col_block):
    secs = W.spin_sectors(W.ring(5), 3, cluster_id=0) + W.spin_sectors(W.ring(4), 5, cluster_id=1)
    got, want, _, _, st = _moments(kpm, secs, 64, 8, "gaussian", precision, col_block, seed=5)
    assert st["kernel"] == 4 and st["col_block"] == col_block, st
    _close(got, want, 1e-6 if precision == "fp32" else 1e-10)


def test_spin_half_sectors_through_the_spin_kernel(kpm):
    secs = W.sectors(W.ring(10), cluster_id=0) + W.spin_sectors(W.ring(5), 2, cluster_id=1)
    got, want, _, _, st = _moments(kpm, secs, 96, 3, "complex_gaussian", "fp64", seed=2)
    assert st["kernel"] == 4, st
    _close(got, want, 1e-10)


def test_lanczos_bounds(kpm):
    secs = W.spin_sectors(W.ring(5), 3)
    got = kpm.spectral_bounds(secs, 40, 0.01, 4)
    for p, s in enumerate(secs):
        want = moments.spectral_bounds(s, 40, 0.01, 4, H=_H(s))
        assert np.abs(got[p] - np.array(want)).max() <= 1e-9 * max(1.0, np.abs(want).max()), p


@pytest.mark.parametrize("field", [False, True])
def test_thermodynamics_end_to_end(kpm, field):
    secs = W.spin_sectors(W.ring(5), 2, cluster_id=0) + W.spin_sectors(W.ring(4), 5, cluster_id=1)
    M = 128
    got, want, ab, _, _ = _moments(kpm, secs, M, 6, "rademacher", "fp64", seed=9)
    T = W.log_temperatures(30, 0.1, 20.0)
    mu = torch.tensor(got, device="cuda")
    abt = torch.tensor(ab, device="cuda")
    if field:
        h = np.linspace(-0.5, 3.0, T.size)
        out = kpm.thermo_field(mu, abt, secs, T, h)
        ref = thermo.thermo_field(_probs(secs), want, ab, T, h, "jackson", M)
        qs = ("lnZ", "E", "C", "chi", "M")
    else:
        out = kpm.thermo(mu, abt, secs, T)
        ref = thermo.thermo(_probs(secs), want, ab, T, "jackson", M)
        qs = ("lnZ", "E", "C", "chi")
    for q in qs:
        g, w = out[q].cpu().numpy(), ref[q]
        assert np.abs(g - w).max() <= 1e-9 * max(1.0, np.abs(w).max()), (q, np.abs(g - w).max())


def test_ftlm_ritz_and_thermodynamics(kpm):
    secs = W.spin_sectors(W.ring(5), 2, cluster_id=0)
    M_L, R = 12, 2
    T = W.log_temperatures(20, 0.1, 10.0)
    h = np.linspace(0.0, 1.0, T.size)
    out = kpm.ftlm(secs, M_L, R, "rademacher", T=T, h=h, seed=4, ritz=True)
    lists = [ftlm.sector_ritz(s, M_L, R, "rademacher", 4, H=_H(s)) for s in secs]
    rz, wt = out["ritz"].cpu().numpy(), out["weight"].cpu().numpy()
    c = 0
    for s, lst in zip(secs, lists):
        for e_ref, w_ref in lst:
            n = e_ref.size
            order = np.argsort(rz[c, :n])
            assert np.abs(rz[c, :n][order] - e_ref).max() <= 1e-10 * max(1.0, np.abs(e_ref).max()), c
            assert np.abs(wt[c, :n][order] - w_ref).max() <= 1e-10 * s.dim / R, c
            c += 1
    ref = ftlm.ftlm_thermo(_probs(secs), lists, T, h)
    for q in ("lnZ", "E", "C", "chi", "M"):
        g, w = out[q].cpu().numpy(), ref[q]
        assert np.abs(g - w).max() <= 1e-9 * max(1.0, np.abs(w).max()), q


# ---------------------------------------------------------------- full size

FE10_BOUNDS = (-88.0, 63.0)    # -s(s+1) <= S_i.S_j <= s^2 per bond: E in [-87.5, 62.5]


@pytest.mark.parametrize("precision,kind,R,col_block,n", [
    ("fp32", "rademacher", 4, 4, 1), ("fp32", "rademacher", 4, 4, 3),
    ("fp64", "gaussian", 2, 2, 2)])
def test_fe10_sz0_sampled_rows(kpm, precision, kind, R, col_block, n):
    s = W.spin_sectors(W.fe10(), 5, only_sz0=True)[0]
    assert s.dim == 4395456
    V, ab = kpm.chebyshev_vectors(s, n, R, kind, precision, 0.025, 1, col_block, bounds=FE10_BOUNDS)
    sample = np.random.default_rng(n).choice(s.dim, size=12, replace=False)
    sample = np.concatenate([sample, [0, 1, s.dim - 1]])
    got = V[torch.as_tensor(sample, device="cuda")].double().cpu().numpy()
    a, b = hamiltonian.scale_from_bounds(*FE10_BOUNDS, 0.025)
    store = np.float32 if precision == "fp32" else np.float64
    want = spins.recursion_rows(s.cluster, 5, s.n, a, b, kind, 1, R, sample, n, store=store)
    tol = 1e-6 if precision == "fp32" else 1e-12
    assert np.abs(got - want).max() <= tol * np.abs(want).max()


def test_fe10_bench_configuration(kpm):
    """The benchmark's launch configuration (100 float32 columns, default
    blocks of 64 + 36): sampled rows of v_2 of the S^z = 0 sector against the
    oracle, and mu_0 = dim, |mu_n| <= mu_0 on all 26 sectors."""
    s = W.spin_sectors(W.fe10(), 5, only_sz0=True)[0]
    V, _ = kpm.chebyshev_vectors(s, 2, 100, "rademacher", "fp32", 0.025, 0, 0, bounds=FE10_BOUNDS)
    sample = np.concatenate([np.random.default_rng(7).choice(s.dim, size=10, replace=False), [0, s.dim - 1]])
    got = V[torch.as_tensor(sample, device="cuda")].double().cpu().numpy()
    del V
    a, b = hamiltonian.scale_from_bounds(*FE10_BOUNDS, 0.025)
    want = spins.recursion_rows(s.cluster, 5, s.n, a, b, "rademacher", 0, 100, sample, 2, store=np.float32)
    assert np.abs(got - want).max() <= 1e-6 * np.abs(want).max()
    secs = W.spin_sectors(W.fe10(), 5)
    mu, _ = kpm.chebyshev_moments(secs, 32, 100, "rademacher", "fp32", 0.025, 0, bounds=[FE10_BOUNDS] * len(secs))
    st = kpm.last_run_stats()
    assert st["kernel"] == 4 and st["col_block"] == 64, st
    mu = mu.cpu().numpy()
    for p, sec in enumerate(secs):
        assert abs(mu[p, 0] - sec.dim) <= 1e-9 * sec.dim, p
        assert np.all(np.abs(mu[p]) <= mu[p, 0] * (1 + 1e-6)), p


def test_fe10_all_sectors_properties(kpm):
    secs = W.spin_sectors(W.fe10(), 5)
    assert len(secs) == 26 and sum(s.dim for s in secs) == 32430816
    M = 64
    mu, _ = kpm.chebyshev_moments(secs, M, 4, "rademacher", "fp32", 0.025, 0, 4,
                                  bounds=[FE10_BOUNDS] * len(secs))
    assert kpm.last_run_stats()["kernel"] == 4
    mu = mu.cpu().numpy()
    for p, s in enumerate(secs):
        assert abs(mu[p, 0] - s.dim) <= 1e-9 * s.dim, p
        assert np.all(np.abs(mu[p]) <= mu[p, 0] * (1 + 1e-6)), p
    # the two smallest sectors against the oracle at the same bounds
    a, b = hamiltonian.scale_from_bounds(*FE10_BOUNDS, 0.025)
    for p in (len(secs) - 1, len(secs) - 3):
        want = moments.sector_moments(secs[p], a, b, M, 4, "rademacher", 0, store=np.float32, H=_H(secs[p]))
        assert np.abs(mu[p] - want).max() <= 1e-6 * want[0], p


def test_unsupported_entry_points_refuse_spin_s(kpm):
    secs = W.spin_sectors(W.ring(4), 2)
    with pytest.raises(kpm.KPMError):
        kpm.thermo_grad(secs, 16, 2, W.log_temperatures(4, 0.5, 2.0), np.ones(4), np.zeros(4))


@pytest.mark.parametrize("name", ["s1_ring6", "s5/2_ring4", "s1_random7", "s7/2_triangle"])
def test_exact_spectra_of_spin_sectors(kpm, name):
    two_s, cl = CLUSTERS[name]
    secs = W.spin_sectors(cl, two_s)
    ev = kpm.sector_eigenvalues(secs, 512).cpu().numpy()
    for p, s in enumerate(secs):
        if s.dim > 512:
            assert np.all(np.isnan(ev[p])), p
            continue
        e = np.linalg.eigvalsh(_H(s).toarray())
        assert np.abs(ev[p, :s.dim] - e).max() <= 1e-10 * max(1.0, np.abs(e).max()), p
        assert np.all(np.isnan(ev[p, s.dim:])), p


def test_fe10_small_sectors_exact(kpm):
    """The Fe10 sectors of dimension <= 1024 (S^z = 25..21: 1, 10, 55, 220, 715
    states) against the oracle's dense diagonalisation; the others NaN."""
    secs = W.spin_sectors(W.fe10(), 5)
    ev = kpm.sector_eigenvalues(secs, 1024).cpu().numpy()
    small = [p for p, s in enumerate(secs) if s.dim <= 1024]
    assert [secs[p].dim for p in small] == [715, 220, 55, 10, 1]
    for p in small:
        e = np.linalg.eigvalsh(_H(secs[p]).toarray())
        assert np.abs(ev[p, :secs[p].dim] - e).max() <= 1e-10 * max(1.0, np.abs(e).max()), p
    assert ev[-1, 0] == pytest.approx(62.5, abs=1e-10)     # the ferromagnetic state: N s^2 J
    assert all(np.all(np.isnan(ev[p])) for p in range(len(secs)) if p not in small)


def test_hybrid_thermodynamics_spin_sectors(kpm):
    """Spin-3/2 ring N=6: sectors with D <= 100 exact on the GPU, the others
    by GPU moments; against the oracle's hybrid sums on the same seeds."""
    secs = W.spin_sectors(W.ring(6), 3)
    M, R = 96, 5
    got, want, ab, _, _ = _moments(kpm, secs, M, R, "rademacher", "fp64", seed=6)
    exact = np.array([s.dim <= 100 for s in secs], dtype=np.uint8)
    assert 0 < exact.sum() < len(secs)
    ev = kpm.sector_eigenvalues(secs, 128)
    T = W.log_temperatures(30, 0.1, 20.0)
    h = np.linspace(0.0, 2.0, T.size)
    out = kpm.thermo_hybrid(torch.tensor(got, device="cuda"), torch.tensor(ab, device="cuda"), secs, ev, exact,
                            T, h)
    spectra = [np.linalg.eigvalsh(_H(s).toarray()) if exact[p] else None for p, s in enumerate(secs)]
    ref = thermo.thermo_hybrid(_probs(secs), want, ab, spectra, T, h, "jackson")
    for q in ("lnZ", "E", "C", "chi", "M"):
        g, w = out[q].cpu().numpy(), ref[q]
        assert np.abs(g - w).max() <= 1e-9 * max(1.0, np.abs(w).max()), (q, np.abs(g - w).max())
