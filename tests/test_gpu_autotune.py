"""Autotuned launch shapes: the tuned run agrees with the oracle like any
other plan, the choice is cached per problem shape, and the workspace query
covers every candidate."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import hamiltonian, moments

pytestmark = pytest.mark.gpu


def test_autotuned_matches_oracle_and_caches(kpm):
    kpm.autotune_reset()
    secs = W.sectors(W.j1j2_chain(16, 1.0, 0.5))
    bl = []
    for s in secs:
        e = np.linalg.eigvalsh(hamiltonian.sector_hamiltonian(s.cluster, s.n_up).toarray()) if s.dim <= 2000 \
            else np.array(moments.spectral_bounds(s, 80, 0.02, 0))
        bl.append((e.min() - 0.05, e.max() + 0.05))      # dim-1 sectors need a window
    for precision, tol in (("fp64", 1e-10), ("fp32", 1e-5)):
        mu, ab = kpm.chebyshev_moments(secs, 64, 10, "complex_gaussian", precision, 0.025, 5, bounds=bl,
                                       autotune=True)
        st1 = kpm.last_run_stats()
        mu2, _ = kpm.chebyshev_moments(secs, 64, 10, "complex_gaussian", precision, 0.025, 5, bounds=bl,
                                       autotune=True)
        st2 = kpm.last_run_stats()
        assert (st1["kernel"], st1["col_block"]) == (st2["kernel"], st2["col_block"])
        # same cached shape, deterministic; the first call planned after tuning with the map
        # (a, b) applied in make_plan, the second made its plan at the unit map while the
        # bounds resolved and applied the map afterwards: the same plan, bit for bit
        assert np.array_equal(mu.cpu().numpy(), mu2.cpu().numpy())
        mu = mu.cpu().numpy()
        for p, (s, (lo, hi)) in enumerate(zip(secs, bl)):
            a, b = hamiltonian.scale_from_bounds(lo, hi, 0.025)
            want = moments.sector_moments(s, a, b, 64, 10, "complex_gaussian", 5)
            assert np.abs(mu[p] - want).max() <= tol * want[0], (precision, p)
    kpm.autotune_reset()


def test_autotune_workspace_contract(kpm):
    secs = W.sectors(W.ring(18), only_sz0=True)
    bl = [(-8.5, 5.0)]
    ps = kpm.ProblemSet(secs, bl)
    q = kpm.make_params(40, 8, "rademacher", "fp32", autotune=True)
    q0 = kpm.make_params(40, 8, "rademacher", "fp32")
    n_tuned, n_plain = kpm.moments_workspace_size(ps, q), kpm.moments_workspace_size(ps, q0)
    assert n_tuned >= n_plain > 0
    ws = torch.empty(n_tuned, dtype=torch.uint8, device="cuda")
    mu, _ = kpm.chebyshev_moments(None, 40, 8, "rademacher", "fp32", workspace=ws, problems=ps, autotune=True)
    ref, _ = kpm.chebyshev_moments(secs, 40, 8, "rademacher", "fp32", bounds=bl)
    assert np.abs(mu.cpu().numpy() - ref.cpu().numpy()).max() <= 1e-6 * secs[0].dim
    small = torch.empty(n_plain // 2, dtype=torch.uint8, device="cuda")
    with pytest.raises(kpm.KPMError) as ei:
        kpm.chebyshev_moments(None, 40, 8, "rademacher", "fp32", workspace=small, problems=ps, autotune=True)
    assert ei.value.code == kpm.KPM_EWORKSPACE
