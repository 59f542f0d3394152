"""GPU vs oracle: Chebyshev moments of Eqs. (6)-(7) on identical seeds and bounds.

Tolerances (|mu_gpu - mu_oracle| per moment, relative to mu_0 of the sector):
float64 vectors 1e-10; float32 storage 1e-5 against the oracle's float64."""
import math
import os

import numpy as np
import pytest

import workloads as W
from oracle import hamiltonian, moments

pytestmark = pytest.mark.gpu

TOL64 = 1e-10
TOL32 = 1e-5


def _exact_bounds(sec, pad=0.0):
    H = hamiltonian.sector_hamiltonian(sec.cluster, sec.n_up)
    if H.shape[0] <= 4000:
        e = np.linalg.eigvalsh(H.toarray())
        lo, hi = e.min(), e.max()
    else:
        lo, hi = moments.spectral_bounds(sec, 80, 0.02, 0, H=H)
    if hi - lo < 1e-8:
        lo, hi = lo - 0.5, hi + 0.5
    return (lo - pad, hi + pad), H


def _oracle(secs, bounds, Hs, M, R, kind, seed, eps, store=np.float64):
    out = []
    for s, (lo, hi), H in zip(secs, bounds, Hs):
        a, b = hamiltonian.scale_from_bounds(lo, hi, eps)
        out.append(moments.sector_moments(s, a, b, M, R, kind, seed, store=store, H=H))
    return np.array(out)


def _run(kpm, secs, M, R, kind, precision, eps=0.025, seed=0, col_block=0, pad=0.0):
    bl, Hs = zip(*[_exact_bounds(s, pad) for s in secs])
    mu, ab = kpm.chebyshev_moments(secs, M, R, kind, precision, eps, seed, col_block, bounds=list(bl))
    return mu.cpu().numpy(), ab.cpu().numpy(), list(bl), list(Hs)


def _assert_close(got, want, tol):
    for p in range(want.shape[0]):
        err = np.abs(got[p] - want[p]).max() / abs(want[p, 0])
        assert err <= tol, (p, err)


def test_ring12_all_sectors_fp64(kpm):
    """Ring N=12, all S^z >= 0 sectors, R=20 Rademacher, M=256, eps=0.025."""
    secs = W.sectors(W.ring(12))
    mu, ab, bl, Hs = _run(kpm, secs, 256, 20, "rademacher", "fp64")
    want = _oracle(secs, bl, Hs, 256, 20, "rademacher", 0, 0.025)
    _assert_close(mu, want, TOL64)
    for p, (lo, hi) in enumerate(bl):
        assert ab[p, 0] == (hi - lo) / (2 - 0.025) and ab[p, 1] == 0.5 * (hi + lo)
    assert np.all(mu[:, 0] == [math.comb(12, s.n_up) for s in secs])


def test_ring12_fp32_storage(kpm):
    secs = W.sectors(W.ring(12))
    mu, ab, bl, Hs = _run(kpm, secs, 256, 20, "rademacher", "fp32")
    want64 = _oracle(secs, bl, Hs, 256, 20, "rademacher", 0, 0.025)
    _assert_close(mu, want64, TOL32)
    want32 = _oracle(secs, bl, Hs, 256, 20, "rademacher", 0, 0.025, store=np.float32)
    _assert_close(mu, want32, 1e-6)


@pytest.mark.parametrize("kind,R,col_block,precision", [
    ("complex_gaussian", 5, 4, "fp64"), ("complex_gaussian", 5, 0, "fp32"),
    ("gaussian", 3, 1, "fp64"), ("rademacher", 7, 3, "fp32"), ("rademacher", 9, 2, "fp64"),
    ("rademacher", 33, 0, "fp32"), ("gaussian", 2, 5, "fp32")])
def test_vector_kinds_and_ragged_blocks(kpm, kind, R, col_block, precision):
    cl = W.random_regular_cluster(13, 3, 5, J_range=(0.5, 1.5))   # odd N: all sectors weight 2
    secs = W.sectors(cl)
    mu, ab, bl, Hs = _run(kpm, secs, 97, R, kind, precision, eps=0.1, seed=11, col_block=col_block)
    want = _oracle(secs, bl, Hs, 97, R, kind, 11, 0.1)
    _assert_close(mu, want, TOL64 if precision == "fp64" else TOL32)


def test_complete_basis_exact_traces(kpm):
    secs = W.sectors(W.ring(10))
    mu, ab, bl, Hs = _run(kpm, secs, 120, 0, "basis", "fp64", eps=0.025)
    for p, (s, (lo, hi), H) in enumerate(zip(secs, bl, Hs)):
        a, b = hamiltonian.scale_from_bounds(lo, hi, 0.025)
        ex = moments.exact_moments((np.linalg.eigvalsh(H.toarray()) - b) / a, 120)
        assert np.abs(mu[p] - ex).max() <= TOL64 * ex[0]


def test_batched_clusters_one_call(kpm):
    """Several clusters of uneven size, all their sectors, in one call."""
    secs = []
    for cid, cl in enumerate([W.ring(8), W.random_regular_cluster(11, 3, 2, J_range=(0.5, 1.5)),
                              W.j1j2_chain(14, 1.0, 0.5)]):
        secs += W.sectors(cl, cluster_id=cid)
    for precision, tol in (("fp64", TOL64), ("fp32", TOL32)):
        mu, ab, bl, Hs = _run(kpm, secs, 64, 8, "rademacher", precision, seed=3)
        want = _oracle(secs, bl, Hs, 64, 8, "rademacher", 3, 0.025)
        _assert_close(mu, want, tol)


def test_n20_sz0_many_tiles(kpm):
    sec = W.sectors(W.j1j2_chain(20, 1.0, 0.5), only_sz0=True)
    for precision, tol in (("fp64", TOL64), ("fp32", TOL32)):
        mu, ab, bl, Hs = _run(kpm, sec, 64, 4, "rademacher", precision)
        want = _oracle(sec, bl, Hs, 64, 4, "rademacher", 0, 0.025)
        _assert_close(mu, want, tol)


def test_graph_segments_match_direct_launches(kpm, monkeypatch):
    secs = W.sectors(W.ring(12))[:3]
    bl = [_exact_bounds(s)[0] for s in secs]
    mu_g, _ = kpm.chebyshev_moments(secs, 400, 6, "rademacher", "fp32", bounds=bl)
    st = kpm.last_run_stats()
    assert st["graph_segment"] >= 2 and st["step_launches"] == 200
    monkeypatch.setenv("KPM_GRAPH_SEGMENT", "0")
    mu_d, _ = kpm.chebyshev_moments(secs, 400, 6, "rademacher", "fp32", bounds=bl)
    assert kpm.last_run_stats()["graph_segment"] == 0
    assert np.array_equal(mu_g.cpu().numpy(), mu_d.cpu().numpy())


def test_bitwise_deterministic(kpm):
    secs = W.sectors(W.j1j2_chain(16, 1.0, 0.5))[:2]
    bl = [_exact_bounds(s)[0] for s in secs]
    a, _ = kpm.chebyshev_moments(secs, 150, 12, "complex_gaussian", "fp32", bounds=bl)
    b, _ = kpm.chebyshev_moments(secs, 150, 12, "complex_gaussian", "fp32", bounds=bl)
    assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())


def test_small_and_degenerate_sectors(kpm):
    cl = W.ring(6)
    secs = [W.Sector(cl, 6, 0), W.Sector(cl, 5, 0)]   # dims 1 and 6
    mu, ab, bl, Hs = _run(kpm, secs, 10, 3, "rademacher", "fp64")
    want = _oracle(secs, bl, Hs, 10, 3, "rademacher", 0, 0.025)
    _assert_close(mu, want, TOL64)
    mu2, _, _, _ = _run(kpm, [W.Sector(W.dimer(), 1, 0)], 2, 1, "rademacher", "fp64")
    assert mu2.shape == (1, 2) and mu2[0, 0] == 2.0


def test_narrow_bounds_raise_ebounds(kpm):
    s = W.sectors(W.ring(10), only_sz0=True)[0]
    e = np.linalg.eigvalsh(hamiltonian.sector_hamiltonian(s.cluster, 5).toarray())
    with pytest.raises(kpm.KPMError) as ei:
        kpm.chebyshev_moments([s], 200, 2, bounds=[(e.min(), e.max() - 0.5)], eps=0.0)
    assert ei.value.code == kpm.KPM_EBOUNDS


def test_lanczos_bounds_match_oracle(kpm):
    secs = W.sectors(W.ring(12)) + W.sectors(W.random_regular_cluster(14, 3, 1, J_range=(0.5, 1.5)),
                                             cluster_id=1)
    got = kpm.spectral_bounds(secs, 50, 0.01, 0)
    for s, (lo, hi) in zip(secs, got):
        wlo, whi = moments.spectral_bounds(s, 50, 0.01, 0)
        w = max(whi - wlo, 1.0)
        assert abs(lo - wlo) <= 1e-9 * w and abs(hi - whi) <= 1e-9 * w
        e = np.linalg.eigvalsh(hamiltonian.sector_hamiltonian(s.cluster, s.n_up).toarray())
        assert lo <= e.min() and hi >= e.max()


def test_nan_bounds_use_lanczos(kpm):
    secs = W.sectors(W.ring(10))
    mu, ab = kpm.chebyshev_moments(secs, 40, 4)
    lb = kpm.spectral_bounds(secs, 50, 0.01, 0)
    for p, (lo, hi) in enumerate(lb):
        assert ab[p, 0].item() == pytest.approx((hi - lo) / (2 - 0.025), rel=1e-14)
        assert ab[p, 1].item() == pytest.approx(0.5 * (hi + lo), rel=1e-14, abs=1e-14)


def test_workspace_contract(kpm):
    import torch
    secs = W.sectors(W.ring(8))
    ps = kpm.ProblemSet(secs, [_exact_bounds(s)[0] for s in secs])
    q = kpm.make_params(32, 4)
    n = kpm.moments_workspace_size(ps, q)
    ws = torch.empty(n, dtype=torch.uint8, device="cuda")
    a, _ = kpm.chebyshev_moments(None, 32, 4, workspace=ws, problems=ps)
    b, _ = kpm.chebyshev_moments(None, 32, 4, problems=ps)
    assert np.array_equal(a.cpu().numpy(), b.cpu().numpy())
    with pytest.raises(kpm.KPMError) as ei:
        kpm.chebyshev_moments(None, 32, 4, workspace=ws[: n // 2], problems=ps)
    assert ei.value.code == kpm.KPM_EWORKSPACE
