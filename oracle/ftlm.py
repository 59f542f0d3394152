"""Finite-temperature Lanczos method (oracle), the comparison method of the
paper (Introduction and Sec. III.C; the paper cites Jaklic and Prelovsek for
its formulation).

For each start vector r of a sector (the same random vectors as Eq. (7)),
M_L steps of plain Lanczos (no reorthogonalisation) from q_0 = r/|r| give the
tridiagonal T with Ritz values eps_j and eigenvectors U; the Krylov expansion
of exp(-beta H) gives
    <r| f(H) |r> / <r|r>  ~  sum_j U_{0j}^2 f(eps_j),
exact for polynomials f of degree < 2 M_L, and the sector trace is estimated as
in Eq. (7): Tr_Gamma f(H) ~ dim/R sum_r <r|f(H)|r>/<r|r>.  A complex vector
r = a + i b contributes (|a|^2 <a|f|a>/|a|^2 + |b|^2 <b|f|b>/|b|^2)/(|a|^2+|b|^2)
since H is real.  The thermodynamic sums are those of `thermo.thermo_field`
with the Ritz values as nodes and dim/R U_{0j}^2 as weights (with the Zeeman
term h S^z, mirror sectors at -S^z).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg as sla

from . import hamiltonian, rng


def lanczos_coefficients(H, v0: np.ndarray, steps: int):
    """alpha_0..alpha_{L-1}, beta_0..beta_{L-2} of plain Lanczos from v0/|v0|;
    L <= steps, stopping early when the next off-diagonal falls below 1e-12."""
    steps = min(steps, H.shape[0])
    q = v0 / np.linalg.norm(v0)
    q_prev = np.zeros_like(q)
    a_list, b_list = [], []
    b_prev = 0.0
    for j in range(steps):
        w = H @ q - b_prev * q_prev
        a = float(np.dot(w, q))
        w = w - a * q
        a_list.append(a)
        bnext = float(np.linalg.norm(w))
        if j == steps - 1 or bnext < 1e-12:
            break
        b_list.append(bnext)
        q_prev, q, b_prev = q, w / bnext, bnext
    return np.array(a_list), np.array(b_list)


def ritz(alpha: np.ndarray, beta: np.ndarray):
    """Ritz values and squared first components of T's eigenvectors."""
    if alpha.size == 1:
        return alpha.copy(), np.ones(1)
    e, U = sla.eigh_tridiagonal(alpha, beta, lapack_driver="stev")
    return e, U[0, :] ** 2


def sector_ritz(sector, M_L: int, R: int, kind: str, seed: int, H=None):
    """Per real column of the start block: (Ritz values, weights) with the
    weights already multiplied by dim/R and the column's share of <r|r>."""
    if H is None:
        H = hamiltonian.sector_hamiltonian(sector.cluster, sector.n_up)
    dim = H.shape[0]
    V0, vec_of_col, R_eff = rng.random_columns(kind, seed, sector.cluster_id, sector.n_up, R, dim)
    n2 = (V0 * V0).sum(axis=0)
    tot = np.zeros(R_eff)
    np.add.at(tot, vec_of_col, n2)
    out = []
    for c in range(V0.shape[1]):
        a, b = lanczos_coefficients(H, V0[:, c], M_L)
        e, z2 = ritz(a, b)
        out.append((e, z2 * (dim / R_eff) * n2[c] / tot[vec_of_col[c]]))
    return out


def ftlm_thermo(problems, ritz_lists, T, h=0.0):
    """ln Z, E, C, chi, M = <S^z> per cluster and point (T[t], h[t]).
    problems: dicts with cluster, n_sites, n_up (two_s for spin-s sites);
    ritz_lists[p]: the
    (values, weights) pairs of sector p's columns."""
    T = np.asarray(T, dtype=np.float64)
    h = np.broadcast_to(np.asarray(h, dtype=np.float64), T.shape)
    cid = np.array([q["cluster"] for q in problems])
    sz = np.array([q["n_up"] - 0.5 * q.get("two_s", 1) * q["n_sites"] for q in problems])
    nc = int(cid.max()) + 1
    out = {k: np.zeros((nc, T.size)) for k in ("lnZ", "E", "C", "chi", "M")}
    for c in range(nc):
        sel = np.nonzero(cid == c)[0]
        for t, (Tv, hv) in enumerate(zip(T, h)):
            beta = 1.0 / Tv
            ws, Es, ms = [], [], []
            for p in sel:
                for m in ([sz[p]] if sz[p] == 0 else [sz[p], -sz[p]]):
                    for e, wt in ritz_lists[p]:
                        ws.append(wt)
                        Es.append(e + hv * m)
                        ms.append(np.full(e.size, m))
            wt, E, m = np.concatenate(ws), np.concatenate(Es), np.concatenate(ms)
            Eref = E.min()
            w = wt * np.exp(-beta * (E - Eref))
            S0 = math.fsum(w)
            Em = math.fsum(w * E) / S0
            m1 = math.fsum(w * m) / S0
            out["lnZ"][c, t] = math.log(S0) - beta * Eref
            out["E"][c, t] = Em
            out["C"][c, t] = beta**2 * math.fsum(w * (E - Em) ** 2) / S0
            out["chi"][c, t] = beta * math.fsum(w * (m - m1) ** 2) / S0
            out["M"][c, t] = m1
    return out
