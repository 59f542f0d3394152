"""Parity at the full sizes of the measured workloads, in the launch
configuration the benchmark times (tuned kernel choice, graph segments).

* Heisenberg ring N=24, S^z=0 (2,704,156 states), 10 complex Gaussian vectors
  = 20 float32 columns: all M = 2000 moments against the oracle's
  full-length recursion (tests/golden/, written by make_fullsize_golden.py
  from the oracle alone) with the same float32 storage and in float64;
  sampled rows of v_n.
* All 13 sectors of the ring in float64 at M = 2000, every moment; the
  thermodynamics on the oracle's own moments at every T and end to end
  (Jackson kernel and g_n = 1, 200 T); the 50-step Lanczos bounds of every
  sector.
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
import os

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


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _golden(name):
    return np.loadtxt(os.path.join(GOLDEN, name))


def _golden_bounds():
    """{n_up: (E_lo, E_hi)}: the oracle's 50-step Lanczos bounds, 1 % margin."""
    return {int(r[0]): (float(r[1]), float(r[2])) for r in _golden("ring24_bounds.txt")}


@pytest.fixture(scope="module")
def ring24_all_fp64(kpm):
    """All 13 sectors of the 24-site ring, float64, M = 2000, the tuned launch
    shape (graph-replayed segments), the oracle's bounds."""
    secs = W.sectors(W.ring(24))
    gb = _golden_bounds()
    mu, ab = kpm.chebyshev_moments(secs, 2000, 10, "complex_gaussian", "fp64", 0.025, 0, 0,
                                   bounds=[gb[s.n_up] for s in secs], autotune=True)
    return secs, mu, ab, kpm.last_run_stats()


def test_ring24_sz0_bench_shape_all_moments(kpm):
    """The benchmark's workload and launch shape: S^z = 0 (2,704,156 states),
    10 complex Gaussian vectors, float32 storage, M = 2000 (1000 graph-replayed
    launches, block width and kernel chosen by the tuner): every mu_n against
    the oracle's float32-storage recursion (<= 1e-6 mu_0) and against its
    float64 recursion (<= 1e-5 mu_0)."""
    s = W.sectors(W.ring(24), only_sz0=True)[0]
    bl = _golden_bounds()[s.n_up]
    mu, ab = kpm.chebyshev_moments([s], 2000, 10, "complex_gaussian", "fp32", 0.025, 0, 0, bounds=[bl],
                                   autotune=True)
    st = kpm.last_run_stats()
    assert st["step_launches"] == 1000 and st["graph_segment"] > 0, st
    got = mu.cpu().numpy()[0]
    want32 = _golden("ring24_sz0_fp32_M2000.txt")
    want64 = _golden("ring24_all_fp64_M2000.txt")[:, 0]
    assert got.shape == want32.shape == (2000,)
    assert abs(want32[0] - s.dim) <= 1e-9 * s.dim
    err32 = np.abs(got - want32).max() / want32[0]
    err64 = np.abs(got - want64).max() / want64[0]
    print(f"kernel {st['kernel']} col_block {st['col_block']}: |dmu| / mu_0 = {err32:.2e} (float32 oracle), "
          f"{err64:.2e} (float64 oracle)")
    assert err32 <= 1e-6, err32
    assert err64 <= 1e-5, err64


def test_ring24_all_sectors_fp64_all_moments(ring24_all_fp64):
    """Every moment of every sector, float64 in the tuned shape, against the
    oracle's float64 recursion: <= 1e-10 mu_0."""
    secs, mu, ab, st = ring24_all_fp64
    want = _golden("ring24_all_fp64_M2000.txt").T          # [13][2000]
    got = mu.cpu().numpy()
    assert got.shape == want.shape
    for p, s in enumerate(secs):
        err = np.abs(got[p] - want[p]).max() / want[p, 0]
        assert abs(want[p, 0] - s.dim) <= 1e-9 * s.dim, p
        assert err <= 1e-10, (s.n_up, err)


def _thermo_errors(out, ref):
    """Per quantity and T: relative error for ln Z and E, peak-normalised for C
    and chi (the peak over the grid)."""
    errs = {}
    for col, name in ((1, "lnZ"), (2, "E"), (3, "C"), (4, "chi")):
        got = out[name].cpu().numpy()[0]
        want = ref[:, col]
        scale = np.abs(want) if name in ("lnZ", "E") else np.abs(want).max()
        errs[name] = np.abs(got - want) / scale
    return errs


@pytest.mark.parametrize("kernel", ["jackson", "none"])
def test_ring24_thermo_on_identical_moments(kpm, kernel):
    """The thermodynamics of Sec. II (kernel, DOS weights at the nodes, sector
    sums) on the oracle's own float64 moments and bounds, against the oracle's
    thermodynamics on the 200-point grid in [0.01, 10]: <= 5e-12 (relative for
    ln Z and E, peak-normalised for C and chi) on T >= 0.25, <= 1e-6 on
    T >= T_phys.  The oracle sums the 2000-term DOS weights and the Boltzmann
    sums exactly rounded, the library the weights by a compensated sum (near
    exact rounding) and the Boltzmann sums in a fixed float64 order, with its
    own node cosines; at low T the thermodynamics amplify the remaining
    last-bit differences of the weights of the lowest nodes (measured:
    <= 2.3e-12 on T >= 0.25; near T_phys up to 5e-8 with the Jackson kernel,
    4.6e-7 without)."""
    secs = W.sectors(W.ring(24))
    mu = torch.tensor(_golden("ring24_all_fp64_M2000.txt").T.copy(), device="cuda")
    gb = _golden_bounds()
    ab = torch.tensor([hamiltonian.scale_from_bounds(*gb[s.n_up], 0.025) for s in secs], dtype=torch.float64,
                      device="cuda")
    ref = _golden(f"ring24_thermo_{kernel}.txt")
    out = kpm.thermo(mu, ab, secs, torch.tensor(ref[:, 0], device="cuda"), kernel)
    T = ref[:, 0]
    bad = np.nonzero(~(np.isfinite(ref[:, 1]) & (ref[:, 3] >= 0)))[0]
    phys = np.arange(T.size) >= (bad.max() + 1 if bad.size else 0)   # T >= T_phys
    hi = T >= 0.25
    worst = {}
    for name, err in _thermo_errors(out, ref).items():
        over = np.nonzero(~(err <= 1e-12) & phys)[0]
        print(f"{kernel} {name}: identical moments: max error {err[phys].max():.2e} on T >= T_phys = "
              f"{T[phys][0]:.4f}, {err[hi].max():.2e} on T >= 0.25; <= 1e-12 for T >= "
              f"{T[over.max() + 1] if over.size else T[phys][0]:.4f}")
        worst[name] = (err[phys].max(), err[hi].max())
    assert max(w[1] for w in worst.values()) <= 5e-12, worst
    assert max(w[0] for w in worst.values()) <= 1e-6, worst


@pytest.mark.parametrize("kernel", ["jackson", "none"])
def test_ring24_thermo_end_to_end(kpm, ring24_all_fp64, kernel):
    """ln Z, E, C, chi of the whole ring from the GPU's own float64 moments
    against the oracle's end-to-end estimate on the same vectors: <= 1e-8
    (relative for ln Z and E, peak-normalised for C and chi) for T >= 0.2.
    Below that the two float64 runs (moments within ~1e-11 mu_0 of each other,
    summed in different orders) differ by that rounding times the
    thermodynamics' condition number in the moments, which exceeds 1e7 there
    (the float32-vs-float64 accuracy curves report it per T); the lowest T
    from which each quantity stays within 1e-8 is printed."""
    secs, mu, ab, _ = ring24_all_fp64
    ref = _golden(f"ring24_thermo_{kernel}.txt")
    T = ref[:, 0]
    out = kpm.thermo(mu, ab, secs, torch.tensor(T, device="cuda"), kernel)
    band = T >= 0.2
    for name, err in _thermo_errors(out, ref).items():
        bad = np.nonzero(~(err <= 1e-8))[0]
        lowest = T[bad.max() + 1] if bad.size and bad.max() + 1 < T.size else (T[0] if not bad.size else None)
        print(f"{kernel} {name}: within 1e-8 for T >= {lowest}")
        assert err[band].max() <= 1e-8, (kernel, name, err[band].max())


def test_ring24_lanczos_bounds(kpm):
    """The 50-step Lanczos bounds (1 % margin) of all 13 sectors against the
    oracle's: <= 1e-9 of the window width."""
    secs = W.sectors(W.ring(24))
    got = kpm.spectral_bounds(secs, 50, 0.01, 0)
    gb = _golden_bounds()
    for p, s in enumerate(secs):
        lo, hi = gb[s.n_up]
        assert np.abs(got[p] - np.array([lo, hi])).max() <= 1e-9 * (hi - lo), (s.n_up, got[p], lo, hi)


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
