"""GPU adjoint (dL/dJ_b with the rescaling fixed) against the oracle's reverse
mode, against central finite differences, and, with exact traces, against the
Hellmann-Feynman form of the moments' derivative."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import adjoint, hamiltonian, moments

pytestmark = pytest.mark.gpu


def _bounds(secs, pad=0.05):
    out = []
    for s in secs:
        e = np.linalg.eigvalsh(hamiltonian.sector_hamiltonian(s.cluster, s.n_up).toarray())
        lo, hi = e.min() - pad, e.max() + pad
        out.append((lo, hi))
    return out


def _ab(bounds, eps):
    return np.array([hamiltonian.scale_from_bounds(lo, hi, eps) for lo, hi in bounds])


@pytest.mark.parametrize("kind,R,precision,col_block,ckpt", [
    ("rademacher", 3, "fp64", 0, 4), ("complex_gaussian", 2, "fp64", 2, 2),
    ("gaussian", 5, "fp64", 3, 64), ("rademacher", 6, "fp32", 4, 8)])
def test_moments_vjp_matches_oracle(kpm, kind, R, precision, col_block, ckpt):
    cl = W.j1j2_chain(10, 1.0, 0.5)
    secs = W.sectors(cl)[:3]
    bl = _bounds(secs)
    M = 41
    mu, ab = kpm.chebyshev_moments(secs, M, R, kind, precision, 0.025, 7, col_block, bounds=bl)
    lam = np.random.default_rng(3).normal(size=(len(secs), M))
    dJ = kpm.moments_vjp(secs, M, R, ab, torch.tensor(lam, device="cuda"), kind, precision, 0.025, 7,
                         col_block, ckpt_every=ckpt).cpu().numpy().reshape(len(secs), -1)
    abh = ab.cpu().numpy()
    store = np.float32 if precision == "fp32" else np.float64
    for p, s in enumerate(secs):
        want = adjoint.sector_moments_vjp(s, abh[p, 0], abh[p, 1], M, R, kind, 7, lam[p], store=store)
        tol = 1e-9 if precision == "fp64" else 1e-4
        assert np.abs(dJ[p] - want).max() <= tol * np.abs(want).max(), p


@pytest.mark.parametrize("kind,R,precision,ckpt", [
    ("rademacher", 3, "fp64", 4), ("gaussian", 5, "fp64", 64), ("complex_gaussian", 4, "fp32", 8)])
def test_checkpointed_forward_and_resumed_reverse(kpm, kind, R, precision, ckpt):
    """moments_ckpt gives chebyshev_moments' moments and (a, b); the reverse
    sweep resumed from its checkpoints gives moments_vjp's dL/dJ."""
    secs = W.sectors(W.j1j2_chain(12, 1.0, 0.5))[:3]
    bl = _bounds(secs)
    M = 60
    mu0, ab0 = kpm.chebyshev_moments(secs, M, R, kind, precision, 0.025, 5, bounds=bl)
    ps = kpm.ProblemSet(secs, bl)
    mu, ab, ws = kpm.moments_ckpt(None, M, R, kind, precision, 0.025, 5, 0, ckpt, problems=ps)
    assert torch.equal(ab, ab0)
    m0 = mu0.cpu().numpy()
    tol = 1e-10 if precision == "fp64" else 1e-5
    assert np.abs(mu.cpu().numpy() - m0).max() <= tol * np.abs(m0[:, 0]).max()
    lam = torch.tensor(np.random.default_rng(2).normal(size=(len(secs), M)), device="cuda")
    want = kpm.moments_vjp(secs, M, R, ab, lam, kind, precision, 0.025, 5, 0, ckpt_every=ckpt).cpu().numpy()
    got = kpm.moments_vjp_resume(ps, M, R, ab, lam, ws, kind, precision, 0.025, 5, 0, ckpt).cpu().numpy()
    assert np.abs(got - want).max() <= 1e-12 * np.abs(want).max()


def test_checkpoint_interval_does_not_change_result(kpm):
    secs = W.sectors(W.ring(12))[:2]
    bl = _bounds(secs)
    M = 90
    mu, ab = kpm.chebyshev_moments(secs, M, 4, bounds=bl)
    lam = torch.tensor(np.random.default_rng(1).normal(size=(2, M)), device="cuda")
    ref = kpm.moments_vjp(secs, M, 4, ab, lam, ckpt_every=1000).cpu().numpy()
    for c in (2, 6, 44):
        got = kpm.moments_vjp(secs, M, 4, ab, lam, ckpt_every=c).cpu().numpy()
        assert np.array_equal(got, ref), c


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_thermo_grad_whole_trajectory_equals_checkpointed(kpm, precision):
    """ckpt_every >= M/2 keeps every v_n of the forward pass (which also
    gives the moments) resident and recomputes nothing; L and dL/dJ are
    bit-identical to the checkpointed run's."""
    secs = W.sectors(W.j1j2_chain(12, 1.0, 0.5))[:3]
    bl = _bounds(secs)
    T = np.linspace(0.2, 3.0, 12)
    wC = np.full(len(T), 0.5)
    wX = np.full(len(T), 0.25)
    out = {}
    for c in (6, 200):
        L, dJ, _ = kpm.thermo_grad(secs, 120, 3, T, wC, wX, "rademacher", precision, kernel="jackson",
                                   ckpt_every=c, bounds=bl)
        out[c] = (L.cpu().numpy(), dJ.cpu().numpy())
    assert np.array_equal(out[6][0], out[200][0])
    assert np.array_equal(out[6][1], out[200][1])


def test_thermo_grad_matches_oracle_and_finite_differences(kpm):
    cl = W.j1j2_chain(8, 1.0, 0.5)
    secs = W.sectors(cl, only_sz0=True) + [W.Sector(cl, 5, 0)]
    bl = _bounds(secs)
    ab = _ab(bl, 0.025)
    T = np.array([0.2, 0.6, 1.5])
    wC = np.ones((1, 3))
    wX = np.array([[0.3, -0.2, 0.5]])
    L, dJ, abd = kpm.thermo_grad(secs, 40, 3, T, wC, wX, "rademacher", "fp64", 0.025, 0, kernel="none",
                                 n_nodes=40, ckpt_every=4, bounds=bl)
    g = dJ.cpu().numpy().reshape(len(secs), -1).sum(0)
    want = adjoint.pipeline_grad(secs, ab, 40, 3, "rademacher", 0, T, wC, wX, "none", 40)
    assert np.linalg.norm(g - want) <= 1e-9 * np.linalg.norm(want)
    Lw = adjoint.pipeline_loss(secs, ab, 40, 3, "rademacher", 0, T, wC, wX, "none", 40)
    assert abs(L.item() - Lw) <= 1e-10 * abs(Lw)
    fd = adjoint.pipeline_grad_fd(secs, ab, 40, 3, "rademacher", 0, T, wC, wX, "none", 40)
    assert np.linalg.norm(g - fd) <= 1e-5 * np.linalg.norm(g)


def test_gradient_vs_gpu_finite_differences_jackson(kpm):
    cl = W.random_regular_cluster(10, 3, 4, J_range=(0.5, 1.5))
    secs = W.sectors(cl)
    bl = _bounds(secs, 0.1)
    T = W.log_temperatures(8, 0.1, 4.0)
    wC = np.ones((1, 8))
    wX = np.linspace(-1, 1, 8)[None, :]
    L, dJ, _ = kpm.thermo_grad(secs, 64, 4, T, wC, wX, "complex_gaussian", "fp64", 0.05, 2, kernel="jackson",
                               ckpt_every=8, bounds=bl)
    g = dJ.cpu().numpy().reshape(len(secs), -1).sum(0)
    h = 1e-5
    for b in (0, 4, 11):
        vals = []
        for sgn in (1, -1):
            J = cl.J.copy()
            J[b] += sgn * h
            s2 = [W.Sector(cl.with_J(J), s.n_up, 0) for s in secs]
            Lh, _, _ = kpm.thermo_grad(s2, 64, 4, T, wC, wX, "complex_gaussian", "fp64", 0.05, 2,
                                       kernel="jackson", ckpt_every=8, bounds=bl)
            vals.append(Lh.item())
        fd = (vals[0] - vals[1]) / (2 * h)
        assert abs(g[b] - fd) <= 1e-5 * np.abs(g).max(), (b, g[b], fd)


def test_complete_basis_adjoint_is_hellmann_feynman_n12(kpm):
    cl = W.j1j2_chain(12, 1.0, 0.5)
    s = W.Sector(cl, 7, 0)
    bl = _bounds([s])
    M = 100
    mu, ab = kpm.chebyshev_moments([s], M, 0, "basis", "fp64", 0.025, bounds=bl)
    a, b = ab.cpu().numpy()[0]
    hf = adjoint.kpm_hellmann_feynman(s, a, b, M)            # [n_bonds, M]
    lam = np.random.default_rng(5).normal(size=M) / np.arange(1, M + 1)
    dJ = kpm.moments_vjp([s], M, 0, ab, torch.tensor(lam[None, :], device="cuda"), "basis", "fp64",
                         ckpt_every=16).cpu().numpy()
    want = hf @ lam
    assert np.abs(dJ - want).max() <= 1e-9 * np.abs(want).max()


def test_autograd_functions_compose(kpm):
    cl = W.j1j2_chain(8, 1.0, 0.5)
    n_ups = [4, 5, 6]
    secs = [W.Sector(cl, k, 0) for k in n_ups]
    bl = _bounds(secs)
    T = torch.tensor([0.3, 1.0, 2.0], dtype=torch.float64)
    J = torch.tensor(cl.J, dtype=torch.float64, requires_grad=True)
    mu, ab = kpm.KPMMoments.apply(J, cl, n_ups, 40, 3, "rademacher", "fp64", 0.025, 0, 0, bl, 8)
    C, chi = kpm.KPMThermo.apply(mu, ab, secs, T, "none", 0)
    L = C.sum() + 0.5 * chi.sum()
    L.backward()
    _, dJ, _ = kpm.thermo_grad(secs, 40, 3, T, np.ones((1, 3)), 0.5 * np.ones((1, 3)), bounds=bl,
                               ckpt_every=8)
    want = dJ.cpu().numpy().reshape(3, -1).sum(0)
    np.testing.assert_allclose(J.grad.numpy(), want, rtol=1e-10, atol=1e-12 * np.abs(want).max())


@pytest.mark.parametrize("t_lo,h,points", [(0.1, 1e-5, 2), (0.05, 4e-4, 4)])
def test_j1j2_n20_full_size_vs_finite_differences(kpm, t_lo, h, points):
    """J1-J2 chain N=20 (40 bonds), S^z=0 (dim 184,756), M=1000, R=16 Rademacher,
    loss sum_T C(T) over 64 log-spaced T in [t_lo, 5], checkpoints every 64
    steps; four bonds against finite differences.  On T in [0.1, 5] a central
    difference at h = 1e-5.  On T in [0.05, 5] C at T = 0.05 amplifies the
    moments' rounding so much that the quotient's error is ~1e-5 max|g| at any
    h in [2e-5, 4e-4] with no trend in h (roundoff, not truncation); that band
    uses the four-point stencil (error O(h^4)) at h = 4e-4, where the roundoff
    term is smallest."""
    wl = W.j1j2_grad_workload()
    secs = wl.problems
    cl = secs[0].cluster
    bl = [tuple(x) for x in kpm.spectral_bounds(secs)]
    T = W.log_temperatures(64, t_lo, 5.0)
    wC = np.ones((1, T.size))
    wX = np.zeros((1, T.size))
    L, dJ, _ = kpm.thermo_grad(secs, wl.M, wl.R, T, wC, wX, kernel="none", ckpt_every=64, bounds=bl)
    g = dJ.cpu().numpy()
    assert g.shape == (40,)

    def loss(b, dh):
        J = cl.J.copy()
        J[b] += dh
        Lh, _, _ = kpm.thermo_grad([W.Sector(cl.with_J(J), secs[0].n_up, 0)], wl.M, wl.R, T, wC, wX,
                                   kernel="none", ckpt_every=64, bounds=bl)
        return Lh.item()

    for b in (0, 7, 26, 33):
        if points == 2:
            fd = (loss(b, h) - loss(b, -h)) / (2 * h)
        else:
            fd = (8 * (loss(b, h) - loss(b, -h)) - (loss(b, 2 * h) - loss(b, -2 * h))) / (12 * h)
        # relative to the gradient's scale: bonds whose derivative is ~500x
        # smaller than the rest carry the same absolute quotient noise
        assert abs(g[b] - fd) <= 1e-5 * np.abs(g).max(), (b, g[b], fd)


def test_j1j2_n20_all_40_bonds_central_differences(kpm):
    """J1-J2 chain N=20 (40 couplings), S^z = 0, M = 1000, R = 16, loss
    sum_T C(T) over 64 log-spaced T in [0.1, 5], bounds fixed: the adjoint
    gradient against central differences on every bond (the forward of each
    difference is one chebyshev_moments call and kpm_thermo).
    * h = 1e-5 (two-point): ||g - fd||_2 / ||g||_2 <= 1e-5.  Per bond this
      quotient carries the loss's rounding divided by h, ~1e-5 max|g| here
      (reported, bounded at 2e-5 max|g|).
    * four-point stencil at h = 2e-4 (truncation O(h^4), rounding 20x
      smaller): every bond within 2e-6 max|g|, which places the h = 1e-5
      spread on the quotient, not on the adjoint."""
    wl = W.j1j2_grad_workload()
    secs = wl.problems
    cl, n_up = secs[0].cluster, secs[0].n_up
    bl = [tuple(x) for x in kpm.spectral_bounds(secs)]
    T = W.log_temperatures(64, 0.1, 5.0)
    wC, wX = np.ones((1, T.size)), np.zeros((1, T.size))
    L, dJ, _ = kpm.thermo_grad(secs, wl.M, wl.R, T, wC, wX, wl.vec_kind, "fp64", wl.eps, wl.seed,
                               kernel="none", ckpt_every=64, bounds=bl)
    g = dJ.cpu().numpy()
    Tt = torch.tensor(T, device="cuda")

    def loss(J):
        s = [W.Sector(cl.with_J(J), n_up, 0)]
        mu, ab = kpm.chebyshev_moments(s, wl.M, wl.R, wl.vec_kind, "fp64", wl.eps, wl.seed, bounds=bl)
        return float(kpm.thermo(mu, ab, s, Tt, "none")["C"].sum())

    assert abs(loss(cl.J.copy()) - L.item()) <= 1e-10 * abs(L.item())
    def shifted(b, dh):
        J = cl.J.copy()
        J[b] += dh
        return loss(J)

    h = 1e-5
    fd = np.array([(shifted(b, h) - shifted(b, -h)) / (2 * h) for b in range(cl.n_bonds)])
    rel = np.linalg.norm(g - fd) / np.linalg.norm(g)
    mx = np.abs(g - fd).max() / np.abs(g).max()
    h4 = 2e-4
    fd4 = np.array([(8 * (shifted(b, h4) - shifted(b, -h4)) - (shifted(b, 2 * h4) - shifted(b, -2 * h4)))
                    / (12 * h4) for b in range(cl.n_bonds)])
    rel4 = np.linalg.norm(g - fd4) / np.linalg.norm(g)
    mx4 = np.abs(g - fd4).max() / np.abs(g).max()
    print(f"N=20 J1-J2, 40 bonds, T in [0.1, 5]: h = 1e-5 central: ||g - fd|| / ||g|| = {rel:.2e}, "
          f"max |g_b - fd_b| / max |g| = {mx:.2e}; h = 2e-4 four-point: {rel4:.2e}, {mx4:.2e}")
    assert rel <= 1e-5, rel
    assert mx <= 2e-5, mx
    assert mx4 <= 2e-6, mx4


def test_exact_trace_gradient_vs_ed_hellmann_feynman_n12(kpm):
    """J1-J2 chain N = 12 (24 couplings), S^z = 0 (dim 924), exact traces
    (complete basis), M = 1000, loss sum_T C(T) over 64 log-spaced T in
    [0.05, 5]: the GPU adjoint against the Hellmann-Feynman derivative of the
    exactly diagonalised thermodynamics (dE_i/dJ_b = <i|h_b|i>).  Their
    difference is the Chebyshev truncation error of the method at this M,
    reported, and bounded by 1e-6 of the gradient's norm."""
    from oracle import ed
    cl = W.j1j2_chain(12, 1.0, 0.5)
    s = W.Sector(cl, 6, 0)
    bl = _bounds([s], pad=0.05)
    T = W.log_temperatures(64, 0.05, 5.0)
    wC, wX = np.ones((1, T.size)), np.zeros((1, T.size))
    L, dJ, _ = kpm.thermo_grad([s], 1000, 1, T, wC, wX, "basis", "fp64", 0.025, 0, kernel="none",
                               ckpt_every=64, bounds=bl)
    g = dJ.cpu().numpy()
    want = ed.hellmann_feynman_C([s], T).sum(axis=1)
    C_ed = ed.thermo_from_spectra(ed.sector_spectra([s]), T)["C"].sum()
    rel = np.linalg.norm(g - want) / np.linalg.norm(want)
    mx = np.abs(g - want).max() / np.abs(want).max()
    print(f"N=12 exact traces, M=1000: ||g - g_HF|| / ||g_HF|| = {rel:.2e}, max = {mx:.2e}; "
          f"|L - L_ED| / L_ED = {abs(L.item() - C_ed) / C_ed:.2e}")
    assert abs(L.item() - C_ed) <= 1e-6 * C_ed
    assert rel <= 1e-6, rel


def test_cluster_bond_grad_sums_sectors(kpm):
    """kpm_cluster_bond_grad: per-cluster sums of per-sector dL/dJ, two
    clusters with different bond lists, in problem order."""
    c0, c1 = W.j1j2_chain(8, 1.0, 0.5), W.ring(7)
    secs = W.sectors(c0, cluster_id=0) + W.sectors(c1, cluster_id=1)
    rng = np.random.default_rng(3)
    per = [rng.normal(size=s.cluster.n_bonds) for s in secs]
    got = kpm.cluster_bond_grad(secs, torch.tensor(np.concatenate(per), device="cuda")).cpu().numpy()
    n0 = len(W.sectors(c0))
    want = np.concatenate([np.sum(per[:n0], axis=0), np.sum(per[n0:], axis=0)])
    np.testing.assert_allclose(got, want, rtol=1e-14, atol=1e-14)
