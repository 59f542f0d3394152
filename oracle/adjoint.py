"""Derivatives of the moments and the thermodynamics with respect to the
couplings J_b, with the rescaling (a, b) of Eq. (5) held fixed (oracle).

Reverse mode through the recursion of `moments`.  With alpha_n = <v_n,v_n>,
beta_n = <v_{n+1},v_n>, and abar_n, bbar_n the loss derivatives with respect to
them, the direct derivative of the loss with respect to v_n is
  gbar_n = 2 abar_n v_n + bbar_n v_{n+1} + bbar_{n-1} v_{n-1},
the adjoint vectors are
  w_K = gbar_K,  w_{K-1} = gbar_{K-1} + 2 H' w_K,
  w_n = gbar_n + 2 H' w_{n+1} - w_{n+2}   (n = K-2 .. 1),
and, since dH'/dJ_b = h_b / a with h_b = s_i . s_j,
  dL/dJ_b = (1/a) [ <w_1, h_b v_0> + 2 sum_{n=1}^{K-1} <w_{n+1}, h_b v_n> ].
The doubling identities give abar, bbar from lambda_n = dL/dmu_n.

References written independently of that derivation: central finite
differences of the whole pipeline, and Hellmann-Feynman forms from exact
diagonalisation (dx_i/dJ_b = <i|h_b|i>/a).
"""
from __future__ import annotations

import numpy as np

from . import hamiltonian, moments, rng, thermo


def doubling_vjp(lam_cols: np.ndarray, K: int):
    """abar [K+1, c], bbar [K, c] from lambda [M, c] through `moments.doubling`."""
    M = lam_cols.shape[0]
    abar = np.zeros((K + 1,) + lam_cols.shape[1:])
    bbar = np.zeros((K,) + lam_cols.shape[1:])
    for n in range(M):
        h = n // 2
        if n == 0:
            abar[0] += lam_cols[n]
        elif n == 1:
            bbar[0] += lam_cols[n]
        elif n % 2 == 0:
            abar[h] += 2.0 * lam_cols[n]
            abar[0] -= lam_cols[n]
        else:
            bbar[h] += 2.0 * lam_cols[n]
            bbar[0] -= lam_cols[n]
    return abar, bbar


def recursion_vjp(Ht, hbs, a: float, V: list, abar, bbar) -> np.ndarray:
    """dL/dJ_b given the stored vectors V[0..K] and abar, bbar (per column)."""
    K = len(V) - 1
    f = lambda x: np.asarray(x, dtype=np.float64)

    def gbar(n):
        g = 2.0 * abar[n] * f(V[n])
        if n < K:
            g = g + bbar[n] * f(V[n + 1])
        if n >= 1:
            g = g + bbar[n - 1] * f(V[n - 1])
        return g

    grad = np.zeros(len(hbs))
    w_next2 = None
    w_next = gbar(K)
    # contribution of step n -> n+1 for n = K-1 (uses w_K)
    ws = {K: w_next}
    for n in range(K - 1, 0, -1):
        w = gbar(n) + 2.0 * (Ht @ w_next)
        if w_next2 is not None:
            w = w - w_next2
        ws[n] = w
        w_next2, w_next = w_next, w
    for b, hb in enumerate(hbs):
        acc = np.sum(ws[1] * (hb @ f(V[0])))
        for n in range(1, K):
            acc += 2.0 * np.sum(ws[n + 1] * (hb @ f(V[n])))
        grad[b] = acc / a
    return grad


def sector_moments_vjp(sector, a: float, b: float, M: int, R: int, kind: str, seed: int,
                       lam: np.ndarray, store=np.float64) -> np.ndarray:
    """dL/dJ_b of one sector for lambda = dL/dmu (estimator of Eq. (7))."""
    H = hamiltonian.sector_hamiltonian(sector.cluster, sector.n_up)
    Ht = hamiltonian.rescaled(H, a, b)
    dim = H.shape[0]
    V0, vec_of_col, R_eff = rng.random_columns(kind, seed, sector.cluster_id, sector.n_up, R, dim)
    K = moments.n_steps(M)
    alpha, beta, V = moments.chebyshev_dots(Ht, V0, K, store=store, keep=True)
    norms = np.zeros(V0.shape[1])
    for r in np.unique(vec_of_col):
        cols = vec_of_col == r
        norms[cols] = alpha[0][cols].sum()
    lam_cols = lam[:, None] * (dim / R_eff) / norms[None, :]
    abar, bbar = doubling_vjp(lam_cols, K)
    hbs = [hamiltonian.bond_operator(sector.cluster, sector.n_up, bb)
           for bb in range(sector.cluster.n_bonds)]
    return recursion_vjp(Ht, hbs, a, V, abar, bbar)


def pipeline_loss(sectors, ab, M, R, kind, seed, T, wC, wchi, kernel, n_nodes, J=None):
    """L = sum wC C + wchi chi, with every sector's couplings replaced by J."""
    probs, mus = [], []
    for s, (a, b) in zip(sectors, ab):
        sec = s if J is None else type(s)(s.cluster.with_J(J), s.n_up, s.cluster_id)
        mus.append(moments.sector_moments(sec, a, b, M, R, kind, seed))
        probs.append(dict(cluster=s.cluster_id, n_sites=s.cluster.n_sites, n_up=s.n_up))
    out = thermo.thermo(probs, np.array(mus), np.asarray(ab), T, kernel, n_nodes)
    return float(np.sum(wC * out["C"]) + np.sum(wchi * out["chi"]))


def pipeline_grad(sectors, ab, M, R, kind, seed, T, wC, wchi, kernel, n_nodes):
    """Adjoint gradient of `pipeline_loss` with respect to the shared couplings."""
    probs = [dict(cluster=s.cluster_id, n_sites=s.cluster.n_sites, n_up=s.n_up) for s in sectors]
    mus = np.array([moments.sector_moments(s, a, b, M, R, kind, seed)
                    for s, (a, b) in zip(sectors, ab)])
    lam = thermo.thermo_vjp(probs, mus, np.asarray(ab), T, wC, wchi, kernel, n_nodes)
    g = np.zeros(sectors[0].cluster.n_bonds)
    for p, (s, (a, b)) in enumerate(zip(sectors, ab)):
        g += sector_moments_vjp(s, a, b, M, R, kind, seed, lam[p])
    return g


def pipeline_grad_fd(sectors, ab, M, R, kind, seed, T, wC, wchi, kernel, n_nodes, h=1e-5):
    """Central finite differences of `pipeline_loss` in each J_b."""
    J0 = sectors[0].cluster.J.copy()
    g = np.zeros(J0.size)
    for bnd in range(J0.size):
        Jp, Jm = J0.copy(), J0.copy()
        Jp[bnd] += h
        Jm[bnd] -= h
        g[bnd] = (pipeline_loss(sectors, ab, M, R, kind, seed, T, wC, wchi, kernel, n_nodes, Jp)
                  - pipeline_loss(sectors, ab, M, R, kind, seed, T, wC, wchi, kernel, n_nodes, Jm)) / (2 * h)
    return g


def kpm_hellmann_feynman(sector, a: float, b: float, M: int) -> np.ndarray:
    """d mu_n / dJ_b of the exact moments: sum_i n U_{n-1}(x_i) <i|h_b|i> / a
    (C_n' = n U_{n-1}).  Returns [n_bonds, M]."""
    H = hamiltonian.sector_hamiltonian(sector.cluster, sector.n_up).toarray()
    e, U = np.linalg.eigh(H)
    x = (e - b) / a
    # Chebyshev polynomials of the second kind U_m(x), m = 0..M-2
    Um = np.zeros((max(M - 1, 1), x.size))
    Um[0] = 1.0
    if M > 2:
        Um[1] = 2.0 * x
    for m in range(2, M - 1):
        Um[m] = 2.0 * x * Um[m - 1] - Um[m - 2]
    out = np.zeros((sector.cluster.n_bonds, M))
    for bb in range(sector.cluster.n_bonds):
        hb = hamiltonian.bond_operator(sector.cluster, sector.n_up, bb).toarray()
        hdiag = np.einsum("ji,jk,ki->i", U, hb, U)
        for n in range(1, M):
            out[bb, n] = n * np.dot(Um[n - 1], hdiag) / a
    return out
