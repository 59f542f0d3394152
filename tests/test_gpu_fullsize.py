"""Parity at the full sizes of the measured workloads, in the launch
configuration the benchmark times (default kernel choice, graph segments).

* Heisenberg ring N=24, S^z=0 (2,704,156 states), 10 complex Gaussian vectors
  = 20 float32 columns in one block: the first moments against the oracle's
  full sparse recursion with the same float32 storage; sampled rows of v_n.
* All 13 S^z >= 0 sectors of the ring in one call (float64): sampled sectors
  against the oracle, mu_0 and |mu_n| <= mu_0 everywhere.
* 64 random 3-regular clusters (N = 16..22, all sectors, ~42 M states),
  32 Rademacher vectors, float32, M = 1024: small sectors against the oracle
  at full M, mu_0 = dim and |mu_n| <= mu_0 for every sector.
* Random 4-regular graph N=30, S^z=0 (155,117,520 states), 4 Rademacher
  vectors, float32 and float64, M = 500: sampled rows of v_3 against the
  oracle's row-by-row recursion, mu_0 = dim, |mu_n| <= mu_0, and the two
  precisions' moments side by side.
* The largest words, N = 32 S^z = 0 (601,080,390 states) on a random
  3-regular graph, with the row kernel and the relabelled block-table kernel:
  sampled rows of v_2, mu_0 = dim and |mu_n| <= mu_0.

|mu_n| <= mu_0 holds for every estimate because ||T_n(H')|| <= 1 on the
rescaled spectrum and mu_0 = dim exactly for normalised vectors (Eq. (7))."""
import math

import numpy as np
import pytest
import torch

import workloads as W
from oracle import hamiltonian, moments, rows

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ring24_sz0():
    s = W.sectors(W.ring(24), only_sz0=True)[0]
    return s, hamiltonian.sector_hamiltonian(s.cluster, s.n_up)


def _props(mu, dims, tol0=1e-9):
    for p, d in enumerate(dims):
        assert abs(mu[p, 0] - d) <= tol0 * d, (p, mu[p, 0], d)
        assert np.all(np.abs(mu[p]) <= mu[p, 0] * (1 + 1e-6)), p


def test_ring24_sz0_bench_kernel_first_moments(kpm, ring24_sz0):
    s, H = ring24_sz0
    lo, hi = -11.0, 7.0                       # E_0 = -10.77, E_max = 6
    M = 10
    mu, ab = kpm.chebyshev_moments([s], M, 10, "complex_gaussian", "fp32", 0.025, 0, 20, bounds=[(lo, hi)])
    st = kpm.last_run_stats()
    assert st["col_block"] == 20 and st["kernel"] in (2, 3), st   # block or block-table kernel
    a, b = hamiltonian.scale_from_bounds(lo, hi, 0.025)
    want = moments.sector_moments(s, a, b, M, 10, "complex_gaussian", 0, store=np.float32, H=H)
    got = mu.cpu().numpy()[0]
    assert np.abs(got - want).max() <= 1e-6 * want[0], np.abs(got - want).max() / want[0]


@pytest.mark.parametrize("precision,kind,R,col_block,n", [
    ("fp32", "complex_gaussian", 10, 20, 0), ("fp32", "complex_gaussian", 10, 20, 1),
    ("fp32", "complex_gaussian", 10, 20, 3), ("fp64", "gaussian", 20, 1, 3)])
def test_ring24_sz0_sampled_rows(kpm, precision, kind, R, col_block, n):
    s = W.sectors(W.ring(24), only_sz0=True)[0]
    lo, hi = -11.0, 7.0
    V, ab = kpm.chebyshev_vectors(s, n, R, kind, precision, 0.025, 0, col_block, bounds=(lo, hi))
    sample = np.random.default_rng(n).choice(s.dim, size=24, replace=False)
    sample = np.concatenate([sample, [0, 1, s.dim - 1]])
    got = V[torch.as_tensor(sample, device="cuda")].double().cpu().numpy()
    a, b = hamiltonian.scale_from_bounds(lo, hi, 0.025)
    store = np.float32 if precision == "fp32" else np.float64
    want = rows.recursion_rows(s.cluster, s.n_up, a, b, kind, 0, R, sample, n, store=store)
    tol = 1e-6 if precision == "fp32" else 1e-12
    assert np.abs(got - want).max() <= tol * np.abs(want).max()


def test_ring24_all_sectors_one_call(kpm):
    ring = W.ring(24)
    secs = W.sectors(ring)
    lo, hi = -11.0, 7.0                       # encloses every sector (E_max = 6 in all)
    M = 12
    mu, _ = kpm.chebyshev_moments(secs, M, 10, "complex_gaussian", "fp64", 0.025, 0, 20,
                                  bounds=[(lo, hi)] * len(secs))
    mu = mu.cpu().numpy()
    _props(mu, [s.dim for s in secs])
    a, b = hamiltonian.scale_from_bounds(lo, hi, 0.025)
    for p, s in enumerate(secs):
        if s.n_up in (13, 19, 23, 24):         # dims 2,496,144 / 134,596 / 24 / 1
            want = moments.sector_moments(s, a, b, M, 10, "complex_gaussian", 0)
            assert np.abs(mu[p] - want).max() <= 1e-10 * want[0], s.n_up


def test_batched_64_clusters_full(kpm):
    wl = W.batched_workload()
    secs = wl.problems
    assert len({s.cluster_id for s in secs}) == 64
    # oracle-checked sectors get exact bounds on both sides; the rest use the
    # library's Lanczos bounds
    picked = [p for p, s in enumerate(secs) if 200 <= s.dim <= 2500][::9][:8]
    bounds = [None] * len(secs)
    for p in picked:
        e = np.linalg.eigvalsh(hamiltonian.sector_hamiltonian(secs[p].cluster, secs[p].n_up).toarray())
        bounds[p] = (e.min() - 0.05, e.max() + 0.05)
    mu, ab = kpm.chebyshev_moments(secs, wl.M, wl.R, wl.vec_kind, wl.precision, wl.eps, wl.seed,
                                   bounds=bounds)
    mu = mu.cpu().numpy()
    _props(mu, [s.dim for s in secs])
    assert sum(s.dim for s in secs) > 30_000_000
    for p in picked:
        s = secs[p]
        a, b = hamiltonian.scale_from_bounds(*bounds[p], wl.eps)
        want = moments.sector_moments(s, a, b, wl.M, wl.R, wl.vec_kind, wl.seed, store=np.float32)
        assert np.abs(mu[p] - want).max() <= 1e-5 * want[0], (p, s.dim)


def test_rr4_30_full_size(kpm):
    wl = W.rr4_30_workload()
    s = wl.problems[0]
    assert s.dim == 155_117_520 and len(s.cluster.J) == 60
    # rigorous bounds for J = 1: each bond lies in [-3/4, 1/4]
    lo, hi = -0.75 * 60, 0.25 * 60
    a, b = hamiltonian.scale_from_bounds(lo, hi, wl.eps)
    sample = np.concatenate([np.random.default_rng(30).choice(s.dim, size=8, replace=False), [0, s.dim - 1]])
    mus = {}
    for precision in ("fp32", "fp64"):
        V, _ = kpm.chebyshev_vectors(s, 3, wl.R, "rademacher", precision, wl.eps, 0, bounds=(lo, hi))
        got = V[torch.as_tensor(sample, device="cuda")].double().cpu().numpy()
        del V
        store = np.float32 if precision == "fp32" else np.float64
        want = rows.recursion_rows(s.cluster, s.n_up, a, b, "rademacher", 0, wl.R, sample, 3, store=store)
        tol = 1e-6 if precision == "fp32" else 1e-12
        assert np.abs(got - want).max() <= tol * np.abs(want).max(), precision
        torch.cuda.empty_cache()
        mu, _ = kpm.chebyshev_moments([s], wl.M, wl.R, "rademacher", precision, wl.eps, 0, bounds=[(lo, hi)])
        mus[precision] = mu.cpu().numpy()
        _props(mus[precision], [s.dim])
        torch.cuda.empty_cache()
    assert np.abs(mus["fp32"] - mus["fp64"]).max() <= 1e-4 * s.dim


@pytest.mark.parametrize("block", [None, "2"])
def test_n32_maximum_sites(kpm, monkeypatch, block):
    """The largest basis words (N = 32 sites, S^z = 0: 601,080,390 states) on a
    seeded random 3-regular graph, with the default kernel (row kernel for two
    columns) and with the block-table kernel, whose plan relabels the sites:
    sampled rows of v_2 against the oracle's row-by-row recursion (rows in the
    original order), mu_0 = dim and |mu_n| <= mu_0."""
    if block:
        monkeypatch.setenv("KPM_BLOCK", block)
    cl = W.random_regular_cluster(32, 3, 7)
    s = W.sectors(cl, only_sz0=True)[0]
    assert s.dim == 601080390
    lo, hi = -37.0, 13.0            # -3/4 <= s_i.s_j <= 1/4 per bond, 48 bonds
    V, _ = kpm.chebyshev_vectors(s, 2, 2, "rademacher", "fp32", 0.025, 3, 2, bounds=(lo, hi))
    sample = np.concatenate([np.random.default_rng(32).choice(s.dim, size=16, replace=False), [0, s.dim - 1]])
    got = V[torch.as_tensor(sample, device="cuda")].double().cpu().numpy()
    del V
    torch.cuda.empty_cache()
    a, b = hamiltonian.scale_from_bounds(lo, hi, 0.025)
    want = rows.recursion_rows(cl, s.n_up, a, b, "rademacher", 3, 2, sample, 2, store=np.float32)
    assert np.abs(got - want).max() <= 1e-6 * np.abs(want).max()
    mu, _ = kpm.chebyshev_moments([s], 8, 2, "rademacher", "fp32", 0.025, 3, 2, bounds=[(lo, hi)])
    st = kpm.last_run_stats()
    assert (st["kernel"], st["relabelled"]) == ((3, 1) if block else (1, 0)), st
    _props(mu.cpu().numpy(), [s.dim], tol0=1e-6)
