"""Oracle pins: Jackson kernel, Gauss-Chebyshev quadrature and thermodynamics."""
import numpy as np
import pytest

import workloads as W
from oracle import ed, hamiltonian, moments, thermo


def _exact_problem_set(cl, eps=0.025, M=256):
    secs = W.sectors(cl)
    spec = ed.sector_spectra(secs)
    mus, ab, probs = [], [], []
    for s, (e, _, _) in zip(secs, spec):
        lo, hi = e.min(), e.max()
        if hi - lo < 1e-8:
            lo, hi = lo - 0.5, hi + 0.5
        a, b = hamiltonian.scale_from_bounds(lo, hi, eps)
        mus.append(moments.exact_moments((e - b) / a, M))
        ab.append((a, b))
        probs.append(dict(cluster=0, n_sites=cl.n_sites, n_up=s.n_up))
    return probs, np.array(mus), np.array(ab), spec


def test_jackson_closed_values():
    for M in (2, 10, 100, 1000):
        g = thermo.jackson(M)
        assert g[0] == pytest.approx(1.0, abs=1e-14)
        if M > 1:
            assert g[1] == pytest.approx(np.cos(np.pi / (M + 1)), abs=1e-14)
        assert np.all(np.diff(g) < 0) and g[-1] > 0
    # extending to n = M gives the inert top coefficient of the paper's sum
    M = 50
    n = M
    q = np.pi / (M + 1)
    top = ((M - n + 1) * np.cos(q * n) + np.sin(q * n) / np.tan(q)) / (M + 1)
    assert abs(top) < 1e-15


def test_jackson_keeps_delta_expansion_nonnegative():
    M = 64
    g = thermo.jackson(M)
    x = np.linspace(-0.999, 0.999, 2001)
    for x0 in (-0.9, -0.3, 0.0, 0.55, 0.97):
        mu = np.cos(np.arange(M) * np.arccos(x0))
        c = g * mu * np.where(np.arange(M) == 0, 1, 2)
        rho = np.polynomial.chebyshev.chebval(x, c)
        assert rho.min() > -1e-12
        c1 = mu * np.where(np.arange(M) == 0, 1, 2)
        assert np.polynomial.chebyshev.chebval(x, c1).min() < -1.0   # Gibbs without kernel


def test_quadrature_exact_for_low_degree():
    """Sec. II: the Gauss-Chebyshev rule is exact up to degree 2 Ntil - 1."""
    Nt = 16
    x = thermo.nodes(Nt)
    for deg in range(2 * Nt):
        c = np.zeros(deg + 1); c[-1] = 1
        q = np.pi / Nt * np.polynomial.chebyshev.chebval(x, c).sum()
        want = np.pi if deg == 0 else 0.0
        assert q == pytest.approx(want, abs=1e-12)


def test_exact_trace_kpm_matches_ed_ring12():
    """g_n = 1, Ntil = M, exact traces: the KPM heat capacity of the N=12 ring
    equals exact diagonalisation over T in [0.01, 10]."""
    cl = W.ring(12)
    probs, mus, ab, spec = _exact_problem_set(cl, 0.025, 256)
    T = W.log_temperatures(200, 0.01, 10.0)
    out = thermo.thermo(probs, mus, ab, T, "none", 256)
    ref = ed.thermo_from_spectra(spec, T)
    assert np.abs(out["C"][0] - ref["C"]).max() < 1e-8
    assert np.abs(out["chi"][0] - ref["chi"]).max() < 1e-10
    assert np.abs(out["E"][0] - ref["E"]).max() < 1e-9
    assert np.abs(out["lnZ"][0] - ref["lnZ"]).max() < 1e-9
    assert not out["z_nonpos"].any()


def test_dimer_closed_form_thermodynamics():
    J = 1.0
    d = W.dimer(J)
    probs, mus, ab, _ = _exact_problem_set(d, 0.0, 64)
    T = np.array([0.2, 0.5, 1.0, 3.0, 10.0])
    out = thermo.thermo(probs, mus, ab, T, "none", 64)
    beta = 1 / T
    Z = np.exp(0.75 * beta * J) + 3 * np.exp(-0.25 * beta * J)
    E = (-0.75 * J * np.exp(0.75 * beta * J) + 0.75 * J * np.exp(-0.25 * beta * J)) / Z
    E2 = (0.5625 * np.exp(0.75 * beta * J) + 3 * 0.0625 * np.exp(-0.25 * beta * J)) / Z
    C = beta**2 * (E2 - E**2)
    chi = beta * 2 * np.exp(-0.25 * beta * J) / Z
    np.testing.assert_allclose(out["lnZ"][0], np.log(Z), atol=1e-10)
    np.testing.assert_allclose(out["C"][0], C, atol=1e-10)
    np.testing.assert_allclose(out["chi"][0], chi, atol=1e-10)


def test_high_temperature_limits():
    """Z -> 2^N, chi T -> N/4, C T^2 -> Tr H^2 / 2^N = (3/16) sum J^2."""
    cl = W.random_regular_cluster(10, 3, 3, J_range=(0.5, 1.5))
    probs, mus, ab, _ = _exact_problem_set(cl, 0.025, 128)
    T = np.array([1e5])
    out = thermo.thermo(probs, mus, ab, T, "none", 128)
    assert out["lnZ"][0, 0] == pytest.approx(10 * np.log(2), abs=1e-4)
    assert out["chi"][0, 0] * 1e5 == pytest.approx(10 / 4, rel=1e-4)
    assert out["C"][0, 0] * 1e10 == pytest.approx(3 / 16 * np.sum(cl.J**2), rel=1e-4)


def test_jackson_exact_traces_give_positive_C_and_chi():
    cl = W.ring(10)
    probs, mus, ab, _ = _exact_problem_set(cl, 0.025, 100)
    T = W.log_temperatures(100, 1e-3, 10)
    out = thermo.thermo(probs, mus, ab, T, "jackson", 100)
    assert out["C"].min() >= -1e-9 and out["chi"].min() >= -1e-12


def test_thermo_vjp_matches_finite_differences():
    cl = W.ring(8)
    probs, mus, ab, _ = _exact_problem_set(cl, 0.025, 40)
    T = np.array([0.3, 1.0, 2.5])
    rng = np.random.default_rng(0)
    wC, wX = rng.normal(size=(1, 3)), rng.normal(size=(1, 3))
    for kern in ("none", "jackson"):
        lam = thermo.thermo_vjp(probs, mus, ab, T, wC, wX, kern, 48)
        L = lambda m: (lambda o: np.sum(wC * o["C"]) + np.sum(wX * o["chi"]))(
            thermo.thermo(probs, m, ab, T, kern, 48))
        for p in (0, 2):
            for n in (0, 1, 7, 39):
                h = 1e-4 * max(1.0, abs(mus[p, n]))
                mp, mm = mus.copy(), mus.copy()
                mp[p, n] += h
                mm[p, n] -= h
                fd = (L(mp) - L(mm)) / (2 * h)
                assert lam[p, n] == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_ghost_dip_behaviour_ladder14():
    """Qualitative statements of Sec. III.A (ladder, exact traces, Table I
    parameters N_deg = Ntil = 100, eps = 0, g_n = 1), at N = 14: a negative
    'ghost dip' of C in 1e-3 <= T <= 1e-2 while T >= 0.1 is exact; the Jackson
    kernel turns the dip into a peak and spoils T >= 0.1; eps > 0 deepens the
    dip; N_deg = 500 removes it."""
    cl = W.ladder(14)
    secs = W.sectors(cl)
    spec = ed.sector_spectra(secs)
    T = W.log_temperatures(300, 1e-3, 10)
    ref = ed.thermo_from_spectra(spec, T)["C"]

    def C(Nd, eps, kern):
        mus, ab, probs = [], [], []
        for s, (e, _, _) in zip(secs, spec):
            lo, hi = e.min(), e.max()
            if hi - lo < 1e-8:
                lo, hi = lo - 0.5, hi + 0.5
            a, b = hamiltonian.scale_from_bounds(lo, hi, eps)
            mus.append(moments.exact_moments((e - b) / a, Nd))
            ab.append((a, b))
            probs.append(dict(cluster=0, n_sites=14, n_up=s.n_up))
        return thermo.thermo(probs, np.array(mus), np.array(ab), T, kern, Nd)["C"][0]

    w = (T >= 1e-3) & (T <= 1e-2)
    hi = T >= 0.1
    c0 = C(100, 0.0, "none")
    assert c0[w].min() < -0.1
    assert np.abs(c0 - ref)[hi].max() < 1e-9
    cj = C(100, 0.0, "jackson")
    assert (cj - ref)[w].min() > 0 and (cj - ref)[w].max() > 0.1
    assert np.abs(cj - ref)[hi].max() > 1e-2
    assert C(100, 0.025, "none")[w].min() < 10 * c0[w].min()
    assert C(100, 0.1, "none")[w].min() < 10 * c0[w].min()
    assert np.abs(C(500, 0.0, "none") - ref)[w].max() < 1e-5


def _dense_field_thermo(cl, T, h):
    """Reference from the dense 2^N Hamiltonian with the Zeeman term
    h S^z_total added (Kronecker construction, no sector logic)."""
    H0 = hamiltonian.full_hamiltonian_kron(cl)
    N = cl.n_sites
    idx = np.arange(1 << N)
    sz_tot = np.array([bin(i).count("1") for i in idx]) - 0.5 * N      # bit 1 = up
    out = {k: np.zeros(len(T)) for k in ("lnZ", "E", "C", "chi", "M")}
    for t, (Tv, hv) in enumerate(zip(T, h)):
        e, U = np.linalg.eigh(H0 + hv * np.diag(sz_tot))
        m_ii = (U * (sz_tot[:, None] * U)).sum(axis=0)       # <i|S^z|i>
        m2_ii = (U * (sz_tot[:, None] ** 2 * U)).sum(axis=0)
        beta = 1.0 / Tv
        w = np.exp(-beta * (e - e.min()))
        Z = w.sum()
        Em = (w * e).sum() / Z
        out["lnZ"][t] = np.log(Z) - beta * e.min()
        out["E"][t] = Em
        out["C"][t] = beta**2 * ((w * (e - Em) ** 2).sum() / Z)
        Mm = (w * m_ii).sum() / Z
        out["M"][t] = Mm
        out["chi"][t] = beta * ((w * m2_ii).sum() / Z - Mm**2)
    return out


def test_field_thermo_zero_field_is_thermo():
    cl = W.ring(10)
    probs, mus, ab, _ = _exact_problem_set(cl, 0.025, 128)
    T = W.log_temperatures(30, 0.05, 10.0)
    a = thermo.thermo(probs, mus, ab, T, "jackson")
    b = thermo.thermo_field(probs, mus, ab, T, np.zeros_like(T), "jackson")
    for k in ("lnZ", "E", "C", "chi"):
        np.testing.assert_allclose(b[k], a[k], rtol=1e-13, atol=1e-14)
    assert np.all(np.abs(b["M"]) <= 1e-12)


@pytest.mark.parametrize("cl", [W.ring(8), W.random_regular_cluster(9, 3, 2, J_range=(0.5, 1.5))])
def test_field_thermo_exact_traces_match_dense_ed(cl):
    """Exact traces, g_n = 1, Ntil = M = 400: KPM with the Zeeman term equals the
    dense diagonalisation of H_0 + h S^z (odd N: every sector has a mirror)."""
    probs, mus, ab, _ = _exact_problem_set(cl, 0.025, 400)
    T = np.array([0.3, 0.3, 0.7, 1.5, 4.0, 0.5])
    h = np.array([0.4, 2.5, 1.0, -1.3, 3.0, 0.0])
    out = thermo.thermo_field(probs, mus, ab, T, h, "none", 400)
    ref = _dense_field_thermo(cl, T, h)
    for k, tol in (("lnZ", 1e-9), ("E", 1e-9), ("C", 1e-8), ("chi", 1e-9), ("M", 1e-9)):
        assert np.abs(out[k][0] - ref[k]).max() < tol, k


def test_field_thermo_saturation_and_susceptibility():
    """Large field at low T polarises the ring (<S^z> -> -N/2 for h > 0 with
    H = H_0 + h S^z); chi = -d<S^z>/dh."""
    cl = W.ring(8)
    probs, mus, ab, _ = _exact_problem_set(cl, 0.025, 400)
    out = thermo.thermo_field(probs, mus, ab, [0.05, 0.05], [6.0, -6.0], "none", 400)
    assert abs(out["M"][0, 0] + 4.0) < 1e-6 and abs(out["M"][0, 1] - 4.0) < 1e-6
    T = np.full(3, 0.8)
    for h0 in (0.0, 0.7, 2.2):
        d = 1e-4
        o = thermo.thermo_field(probs, mus, ab, T, np.array([h0 - d, h0, h0 + d]), "none", 400)
        dM = (o["M"][0, 2] - o["M"][0, 0]) / (2 * d)
        assert abs(o["chi"][0, 1] + dM) < 1e-6 * max(1.0, abs(dM)), h0


@pytest.mark.parametrize("cl", [W.ring(8), W.random_regular_cluster(9, 3, 2, J_range=(0.5, 1.5))])
def test_hybrid_all_exact_is_dense_ed(cl):
    """Every sector diagonalised: the hybrid sums are the exact thermodynamics
    of H_0 + h S^z from the dense diagonalisation of the whole space."""
    probs, mus, ab, spec = _exact_problem_set(cl, 0.025, 64)
    T = np.array([0.05, 0.3, 0.7, 1.5, 4.0, 0.5])
    h = np.array([0.0, 2.5, 1.0, -1.3, 3.0, 0.2])
    out = thermo.thermo_hybrid(probs, mus, ab, [e for e, _, _ in spec], T, h, "jackson")
    ref = _dense_field_thermo(cl, T, h)
    for k in ("lnZ", "E", "C", "chi", "M"):
        assert np.abs(out[k][0] - ref[k]).max() < 1e-10 * max(1.0, np.abs(ref[k]).max()), k


def test_hybrid_no_exact_sector_is_field_thermo():
    cl = W.ladder(10)
    probs, mus, ab, _ = _exact_problem_set(cl, 0.025, 96)
    T = W.log_temperatures(20, 0.05, 10.0)
    h = np.linspace(0.0, 1.0, T.size)
    a = thermo.thermo_field(probs, mus, ab, T, h, "jackson", 150)
    b = thermo.thermo_hybrid(probs, mus, ab, [None] * len(probs), T, h, "jackson", 150)
    for k in ("lnZ", "E", "C", "chi", "M"):
        np.testing.assert_allclose(b[k], a[k], rtol=1e-13, atol=1e-14)


def test_hybrid_mixed_exact_traces_match_dense_ed():
    """Large sectors from exact-trace moments (g_n = 1, Ntil = M = 400), the
    three smallest diagonalised: equal to dense ED within the quadrature error."""
    cl = W.ring(10)
    probs, mus, ab, spec = _exact_problem_set(cl, 0.025, 400)
    dims = [e.size for e, _, _ in spec]
    small = set(np.argsort(dims)[:3])
    spectra = [spec[p][0] if p in small else None for p in range(len(probs))]
    T = np.array([0.3, 0.7, 1.5, 4.0, 0.5])
    h = np.array([0.4, 1.0, -1.3, 3.0, 0.0])
    out = thermo.thermo_hybrid(probs, mus, ab, spectra, T, h, "none", 400)
    ref = _dense_field_thermo(cl, T, h)
    for k, tol in (("lnZ", 1e-9), ("E", 1e-9), ("C", 1e-8), ("chi", 1e-9), ("M", 1e-9)):
        assert np.abs(out[k][0] - ref[k]).max() < tol, k
