"""chebyshev_moments_noalloc (static per-GPU workspace, no device allocation)
against chebyshev_moments (library- or caller-allocated workspace) on the same
problems and parameters, through the C ABI.

Both run the planner's launch shape (autotune 0) with the same kernels, so the
moments of Eq. (7) and the (a, b) of Eq. (5) must agree to rounding; the bar
used is 1e-12 mu_0, far inside the 1e-6 relative tolerance of the float32
moment parity.  Three calls in a row on one GPU, each smaller than the one
before, so every later call runs on an array still holding the earlier call's
vectors, partial sums and tables.
"""
import ctypes

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def kpm():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2104_13218_amd import kpm as k
    k.load()
    return k


def _need(kpm, ps, q):
    return int(kpm.load().chebyshev_moments_workspace_size(ps.arr, len(ps), ctypes.byref(q)))


def _largest_R(kpm, secs, limit, **kw):
    """Largest R in a short ladder whose workspace still fits `limit` bytes."""
    ps = kpm.ProblemSet(secs)
    best = None
    for R in (4, 8, 12, 16, 24, 32, 40, 48):
        if _need(kpm, ps, kpm.make_params(R=R, **kw)) <= limit:
            best = R
    return best


def _compare(kpm, secs, bounds=None, **kw):
    ps = kpm.ProblemSet(secs, bounds)
    q = kpm.make_params(**kw)
    need = _need(kpm, ps, q)
    assert 0 < need <= kpm.NOALLOC_MAX_BYTES
    print(f"noalloc case: {len(secs)} problems, dims {[s.dim for s in secs][:4]}..., "
          f"workspace {need / 2**20:.2f} MiB, {kw}", flush=True)
    mu_ref, ab_ref = kpm.chebyshev_moments(secs, bounds=bounds, **kw)
    graph_ref = kpm.last_run_stats()["graph_segment"]
    mu, ab = kpm.chebyshev_moments_noalloc(secs, bounds=bounds, **{k: v for k, v in kw.items()
                                                                      if k != "autotune"})
    stats = kpm.last_run_stats()
    torch.cuda.synchronize()
    mu_ref, ab_ref, mu, ab = (t.cpu().numpy() for t in (mu_ref, ab_ref, mu, ab))
    assert stats["graph_segment"] == 0 and stats["recursion_ms"] == -1.0
    dims = np.array([s.dim for s in secs], float)
    np.testing.assert_array_equal(mu[:, 0] > 0, True)
    assert np.all(np.abs(ab - ab_ref) <= 1e-14 * np.abs(ab_ref).max())
    err = (np.abs(mu - mu_ref) / dims[:, None]).max()
    print(f"  max |mu_noalloc - mu| / mu_0 = {err:.3e} (graph segment of the allocating call: "
          f"{graph_ref})", flush=True)
    assert err <= 1e-12
    return need


def test_noalloc_matches_chebyshev_moments_three_calls_shrinking(kpm):
    # 1: S^z = 0 sector of the 20-site ring, float32 storage, R chosen so the
    #    workspace fills most of the array; M = 300 (150 steps: the allocating
    #    call captures graph segments, this one launches every step itself)
    ring20 = [s for s in W.sectors(W.ring(20)) if 2 * s.n_up == 20]
    R1 = _largest_R(kpm, ring20, kpm.NOALLOC_MAX_BYTES, M=300, vec_kind="gaussian", precision="fp32")
    assert R1 is not None
    n1 = _compare(kpm, ring20, M=300, R=R1, vec_kind="gaussian", precision="fp32", seed=5)
    assert n1 > kpm.NOALLOC_MAX_BYTES // 4
    # 2: every S^z >= 0 sector of the 18-site ring (10 problems), float64 complex
    #    Gaussian vectors, bounds by Lanczos inside the same array
    ring18 = W.sectors(W.ring(18))
    n2 = _compare(kpm, ring18, M=200, R=3, vec_kind="complex_gaussian", precision="fp64", seed=11)
    assert n2 < n1
    # 3: the S^z = 0 sector of the 12-site ring with given bounds, Rademacher
    ring12 = [s for s in W.sectors(W.ring(12)) if s.n_up == 6]
    n3 = _compare(kpm, ring12, bounds=[(-5.5, 3.1)], M=100, R=3, vec_kind="rademacher",
                  precision="fp64", seed=2)
    assert n3 < n2


def test_noalloc_rejects_oversize_and_autotune(kpm):
    lib = kpm.load()
    big = [s for s in W.sectors(W.ring(22)) if 2 * s.n_up == 22]
    ps = kpm.ProblemSet(big)
    q = kpm.make_params(M=64, R=10, vec_kind="complex_gaussian")
    assert _need(kpm, ps, q) > kpm.NOALLOC_MAX_BYTES
    mu = torch.full((1, 64), 7.0, dtype=torch.float64, device="cuda")
    rc = lib.chebyshev_moments_noalloc(ps.arr, 1, ctypes.byref(q), ctypes.c_void_p(mu.data_ptr()),
                                       None, None)
    assert rc == kpm.KPM_ETOOLARGE
    torch.cuda.synchronize()
    assert torch.all(mu == 7.0)                 # nothing written
    q_tuned = kpm.make_params(M=64, R=2, autotune=True)
    small = kpm.ProblemSet([s for s in W.sectors(W.ring(10)) if s.n_up == 5])
    assert lib.chebyshev_moments_noalloc(small.arr, 1, ctypes.byref(q_tuned),
                                         ctypes.c_void_p(mu.data_ptr()), None, None) == kpm.KPM_EINVAL
