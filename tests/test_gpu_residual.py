"""Float32 + 16-bit residual storage (KPM_FP32R_STORE, precision "fp32r") on
the slice kernel against the oracle's rule for the same storage
(`oracle.moments.f32_residual16`): the moments of Eq. (7) on the same
seeds and bounds.

Bars (|mu_gpu - mu_oracle| <= tol * mu_0): 1e-10 against the oracle with the
same storage on the small cases (float32 storage alone differs from float64
by ~1e-7 there, so a wrong residual would show), 1e-10 against float64
storage; at full size (24-site ring, S^z = 0, M = 2000) 1e-8 against the
oracle's float64 moments (the float32 form is 2.8e-7 off there)."""
import ctypes
import os

import numpy as np
import pytest
import torch

import workloads as W
from oracle import hamiltonian, moments

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


_CACHE = {}


def _bounds_h(sec):
    key = (id(sec.cluster), sec.n_up)
    if key in _CACHE:
        return _CACHE[key][1:]
    H = hamiltonian.sector_hamiltonian(sec.cluster, sec.n_up)
    if H.shape[0] <= 1000:
        e = np.linalg.eigvalsh(H.toarray())
        lo, hi = e.min(), e.max()
    else:
        lo, hi = moments.spectral_bounds(sec, 80, 0.02, 0, H=H)
    if hi - lo < 1e-8:
        lo, hi = lo - 0.5, hi + 0.5
    _CACHE[key] = (sec.cluster, (lo, hi), H)   # the cluster keeps its id valid
    return (lo, hi), H


def _check(kpm, secs, M, R, kind, col_block, seed, tol=1e-10):
    bl, Hs = zip(*[_bounds_h(s) for s in secs])
    mu, _ = kpm.chebyshev_moments(secs, M, R, kind, "fp32r", 0.025, seed, col_block, bounds=list(bl))
    st = kpm.last_run_stats()
    assert st["kernel"] == 5, st
    mu = mu.cpu().numpy()
    worst = worst64 = 0.0
    for p, (s, (lo, hi), H) in enumerate(zip(secs, bl, Hs)):
        a, b = hamiltonian.scale_from_bounds(lo, hi, 0.025)
        want = moments.sector_moments(s, a, b, M, R, kind, seed, store=moments.F32R, H=H)
        want64 = moments.sector_moments(s, a, b, M, R, kind, seed, H=H)
        worst = max(worst, np.abs(mu[p] - want).max() / abs(want[0]))
        worst64 = max(worst64, np.abs(mu[p] - want64).max() / abs(want64[0]))
    print(f"fp32r {kind} R={R} col_block={col_block}: vs oracle fp32r {worst:.2e}, vs float64 {worst64:.2e}")
    assert worst <= tol, worst
    assert worst64 <= tol, worst64
    return mu


@pytest.mark.parametrize("kind,R,col_block", [("rademacher", 5, 0), ("complex_gaussian", 3, 4),
                                              ("gaussian", 2, 2), ("rademacher", 8, 8),
                                              ("complex_gaussian", 4, 0)])
def test_ring12_all_sectors(kpm, kind, R, col_block):
    """Every S^z >= 0 sector of the 12-site ring (924 ... 1 states) in one
    call: rows of 2 and 4 float32 columns, one and two chunks per row."""
    _check(kpm, W.sectors(W.ring(12)), 128, R, kind, col_block, seed=3)


def test_batched_clusters(kpm):
    """Four clusters (ring, random 3-regular with random J, J1-J2 chain,
    ladder), all sectors, one call."""
    secs = []
    for cid, cl in enumerate([W.ring(8), W.random_regular_cluster(11, 3, 2, J_range=(0.5, 1.5)),
                              W.j1j2_chain(14, 1.0, 0.5), W.ladder(12)]):
        secs += W.sectors(cl, cluster_id=cid)
    _check(kpm, secs, 96, 6, "complex_gaussian", 0, seed=4)


def test_ring20_sz0_longer_recursion(kpm):
    """Ring N=20, S^z=0 (184,756 states), 4 Rademacher vectors, M = 400."""
    _check(kpm, W.sectors(W.ring(20), only_sz0=True), 400, 4, "rademacher", 0, seed=1)


def test_ring24_sz0_full_length_against_float64(kpm):
    """The benchmark's sector and vectors (10 complex Gaussian, seed 0, the
    oracle's Lanczos bounds), M = 2000, autotuned: every moment within 1e-8
    mu_0 of the oracle's float64 moments (tests/golden)."""
    s = W.sectors(W.ring(24), only_sz0=True)
    gb = {int(r[0]): (float(r[1]), float(r[2])) for r in np.loadtxt(os.path.join(GOLDEN, "ring24_bounds.txt"))}
    mu, _ = kpm.chebyshev_moments(s, 2000, 10, "complex_gaussian", "fp32r", 0.025, 0, 0,
                                  bounds=[gb[12]], autotune=True)
    assert kpm.last_run_stats()["kernel"] == 5
    mu = mu.cpu().numpy()[0]
    want = np.loadtxt(os.path.join(GOLDEN, "ring24_all_fp64_M2000.txt"))[:, 0]
    want32 = np.loadtxt(os.path.join(GOLDEN, "ring24_sz0_fp32_M2000.txt"))
    err = np.abs(mu - want).max() / want[0]
    err32 = np.abs(want32 - want).max() / want[0]
    print(f"N=24 S^z=0 M=2000: fp32r vs float64 {err:.2e} (float32 storage vs float64: {err32:.2e})")
    assert err <= 1e-8, err


def test_noalloc_takes_residual_storage(kpm):
    secs = W.sectors(W.ring(14))
    bl = [_bounds_h(s)[0] for s in secs]
    mu, _ = kpm.chebyshev_moments(secs, 80, 3, "complex_gaussian", "fp32r", 0.025, 2, 0, bounds=bl)
    mu2, _ = kpm.chebyshev_moments_noalloc(secs, 80, 3, "complex_gaussian", "fp32r", 0.025, 2, 0, bounds=bl)
    assert torch.equal(mu, mu2)


def test_other_entry_points_refuse_residual_storage(kpm):
    s = [x for x in W.sectors(W.ring(10)) if x.n_up == 5]
    bl = [_bounds_h(s[0])[0]]
    with pytest.raises(kpm.KPMError):
        kpm.chebyshev_vectors(s[0], 3, 2, "rademacher", "fp32r", bounds=bl[0])
    ps = kpm.ProblemSet(s, bl)
    q = kpm.make_params(M=16, R=2, precision="fp32r")
    lib = kpm.load()
    assert lib.chebyshev_moments_vjp_workspace_size(ps.arr, 1, ctypes.byref(q), 8) == 0
    # spin-1 sites have no slice plan
    sp = W.spin_sectors(W.ring(6), 2, only_sz0=True)
    with pytest.raises(kpm.KPMError):
        kpm.chebyshev_moments(sp, 16, 2, "rademacher", "fp32r", bounds=[(-8.0, 8.0)])
