"""Kernel damping, density-of-states weights and thermodynamics (oracle).

Jackson kernel, Eq. (8), with N_deg = M (the stray trailing factor in the
printed formula is dropped: with it the coefficients grow ~N_deg instead of
damping; without it the formula is the Jackson kernel of the cited review):
  g_n = [(M - n + 1) cos(pi n/(M+1)) + sin(pi n/(M+1)) cot(pi/(M+1))] / (M+1).

Gauss-Chebyshev quadrature (Sec. II, Eq. (9) and below) at the Ntil nodes
x_k = cos(pi (k - 1/2)/Ntil), k = 1..Ntil, with the DOS weights
  gamma_k = g_0 mu_0 + 2 sum_{n>=1} g_n mu_n cos(n pi (k - 1/2)/Ntil),
and per symmetry sector Gamma (the paper's sector sum)
  Z = (1/Ntil) sum_Gamma W_Gamma sum_k gamma_k^Gamma exp(-beta (a_Gamma x_k + b_Gamma)).
The exponent is read as exp(-beta E) (the sign printed in the definition of
f(x) contradicts Eq. (2)).  W_Gamma = 2 for S^z > 0 sectors (their S^z < 0
mirrors are degenerate, Sec. II), 1 for S^z = 0.  <E> and <E^2> use the same
nodes and weights with the integrand multiplied by E and E^2 (Eq. (2b));
chi uses the S^z-resolved sums of Eq. (3).  All weights are shifted by a common
E_ref (the lowest node energy of the cluster) so nothing overflows; C, E and
chi are shift-invariant and ln Z = ln(sum)-beta E_ref.  gamma_k and Z are never
clipped: a non-positive Z is reported by a flag (Sec. II remark on improper
densities).
"""
from __future__ import annotations

import math

import numpy as np


def jackson(M: int) -> np.ndarray:
    n = np.arange(M, dtype=np.float64)
    q = np.pi / (M + 1)
    return ((M - n + 1) * np.cos(q * n) + np.sin(q * n) / np.tan(q)) / (M + 1)


def kernel_coefficients(M: int, kernel: str) -> np.ndarray:
    if kernel in ("none", 0, None):
        return np.ones(M)
    if kernel in ("jackson", 1):
        return jackson(M)
    raise ValueError(kernel)


def nodes(n_nodes: int) -> np.ndarray:
    k = np.arange(1, n_nodes + 1, dtype=np.float64)
    return np.cos(np.pi * (k - 0.5) / n_nodes)


def cos_matrix(n_nodes: int, M: int) -> np.ndarray:
    """Cmat[k-1, n] = cos(n pi (k - 1/2)/Ntil), with the argument n (2k - 1)
    reduced modulo 4 Ntil in integers before scaling by pi / (2 Ntil) (the same
    angle; avoids rounding an argument that grows with n)."""
    k = np.arange(1, n_nodes + 1, dtype=np.int64)[:, None]
    n = np.arange(M, dtype=np.int64)[None, :]
    m = (n * (2 * k - 1)) % (4 * n_nodes)
    return np.cos(np.pi * m / (2 * n_nodes))


def dos_weights(mu: np.ndarray, g: np.ndarray, n_nodes: int) -> np.ndarray:
    """gamma_k for k = 1..Ntil: the direct sum over n, exactly rounded (math.fsum;
    the DCT-III is a faster route to the same numbers)."""
    M = mu.shape[-1]
    c = g * mu
    c = c * np.where(np.arange(M) == 0, 1.0, 2.0)
    terms = cos_matrix(n_nodes, M) * c[None, :]
    return np.array([math.fsum(row) for row in terms])


def _sector_table(problems):
    """cluster id, S^z and weight per problem; dense cluster ids.  For spin-s
    sites (key two_s = 2s, default 1) n_up is the sum of the site digits
    s + m_i, so S^z = n_up - s N; a sector with S^z != 0 stands for its
    degenerate mirror too (weight 2)."""
    cid = np.array([p["cluster"] for p in problems])
    tsn = np.array([p.get("two_s", 1) * p["n_sites"] for p in problems])
    sz = np.array([p["n_up"] - 0.5 * t for p, t in zip(problems, tsn)])
    W = np.array([1.0 if 2 * p["n_up"] == t else 2.0 for p, t in zip(problems, tsn)])
    return cid, sz, W


def thermo(problems, mu: np.ndarray, ab: np.ndarray, T: np.ndarray,
           kernel: str = "jackson", n_nodes: int = 0):
    """ln Z, E = <E>, C = beta^2 (<E^2> - <E>^2), chi = beta (<S_z^2> - <S_z>^2)
    per cluster and temperature (k_B = g mu_B = 1), and the Z <= 0 flag.

    problems: list of dicts with keys cluster, n_sites, n_up (and two_s for
    spin-s sites); mu [P, M];
    ab [P, 2] = (a, b) of each problem's rescaling."""
    mu = np.atleast_2d(mu)
    P, M = mu.shape
    Nt = n_nodes or M
    g = kernel_coefficients(M, kernel)
    x = nodes(Nt)
    cid, sz, W = _sector_table(problems)
    nc = int(cid.max()) + 1
    T = np.asarray(T, dtype=np.float64)
    out = {k: np.zeros((nc, T.size)) for k in ("lnZ", "E", "C", "chi")}
    out["z_nonpos"] = np.zeros((nc, T.size), dtype=bool)
    gam = np.stack([dos_weights(mu[p], g, Nt) for p in range(P)])
    Ek = ab[:, 0:1] * x[None, :] + ab[:, 1:2]                      # [P, Nt]
    for c in range(nc):
        sel = np.nonzero(cid == c)[0]
        Eref = Ek[sel].min()
        for t, Tv in enumerate(T):
            beta = 1.0 / Tv
            ws, Es, ms = [], [], []
            for p in sel:
                w = gam[p] * np.exp(-beta * (Ek[p] - Eref))
                # both signs of S^z (the mirror sector of S^z > 0 is degenerate)
                for m in ([sz[p]] if W[p] == 1.0 else [sz[p], -sz[p]]):
                    ws.append(w)
                    Es.append(Ek[p])
                    ms.append(np.full(Nt, m))
            w, E, m = np.concatenate(ws), np.concatenate(Es), np.concatenate(ms)
            S0 = math.fsum(w)                             # sums exactly rounded
            Em = math.fsum(w * E) / S0
            varE = math.fsum(w * (E - Em) ** 2) / S0      # <E^2> - <E>^2
            m1 = math.fsum(w * m) / S0
            varM = math.fsum(w * (m - m1) ** 2) / S0      # <S_z^2> - <S_z>^2
            out["z_nonpos"][c, t] = S0 <= 0.0
            out["lnZ"][c, t] = (np.log(S0 / Nt) if S0 > 0 else np.nan) - beta * Eref
            out["E"][c, t] = Em
            out["C"][c, t] = beta**2 * varE
            out["chi"][c, t] = beta * varM
    return out


def thermo_field(problems, mu: np.ndarray, ab: np.ndarray, T: np.ndarray, h: np.ndarray,
                 kernel: str = "jackson", n_nodes: int = 0):
    """Thermodynamics with the Zeeman term of the ladder Hamiltonian (Sec. III.A,
    Eq. (E-3-1-1)): H = H_0 + h S^z_total with h = g mu_B B, at the points
    (T[t], h[t]).  S^z commutes with H_0, so a sector S^z = m keeps the DOS of
    its zero-field moments and shifts every energy by h m; a sector S^z > 0
    stands for itself (m = +S^z) and its mirror (m = -S^z).
    Returns ln Z, E = <E>, C = beta^2 (<E^2> - <E>^2), chi = beta (<m^2> - <m>^2),
    M = <m> = <S^z_total> per cluster and point, and the Z <= 0 flag; the
    Boltzmann factors are shifted by the lowest node energy of the point."""
    mu = np.atleast_2d(mu)
    P, M = mu.shape
    Nt = n_nodes or M
    g = kernel_coefficients(M, kernel)
    x = nodes(Nt)
    cid, sz, W = _sector_table(problems)
    nc = int(cid.max()) + 1
    T = np.asarray(T, dtype=np.float64)
    h = np.broadcast_to(np.asarray(h, dtype=np.float64), T.shape)
    out = {k: np.zeros((nc, T.size)) for k in ("lnZ", "E", "C", "chi", "M")}
    out["z_nonpos"] = np.zeros((nc, T.size), dtype=bool)
    gam = np.stack([dos_weights(mu[p], g, Nt) for p in range(P)])
    Ek = ab[:, 0:1] * x[None, :] + ab[:, 1:2]                      # [P, Nt]
    for c in range(nc):
        sel = np.nonzero(cid == c)[0]
        for t, (Tv, hv) in enumerate(zip(T, h)):
            beta = 1.0 / Tv
            gs, Es, ms = [], [], []
            for p in sel:
                for m in ([sz[p]] if W[p] == 1.0 else [sz[p], -sz[p]]):
                    gs.append(gam[p])
                    Es.append(Ek[p] + hv * m)
                    ms.append(np.full(Nt, m))
            gw, E, m = np.concatenate(gs), np.concatenate(Es), np.concatenate(ms)
            Eref = E.min()
            w = gw * np.exp(-beta * (E - Eref))
            S0 = math.fsum(w)
            Em = math.fsum(w * E) / S0
            varE = math.fsum(w * (E - Em) ** 2) / S0
            m1 = math.fsum(w * m) / S0
            varM = math.fsum(w * (m - m1) ** 2) / S0
            out["z_nonpos"][c, t] = S0 <= 0.0
            out["lnZ"][c, t] = (np.log(S0 / Nt) if S0 > 0 else np.nan) - beta * Eref
            out["E"][c, t] = Em
            out["C"][c, t] = beta**2 * varE
            out["chi"][c, t] = beta * varM
            out["M"][c, t] = m1
    return out


def thermo_hybrid(problems, mu: np.ndarray, ab: np.ndarray, spectra, T: np.ndarray, h=0.0,
                  kernel: str = "jackson", n_nodes: int = 0):
    """Thermodynamics with the small sectors treated exactly (Sec. II: sectors
    whose dimension is small are diagonalised completely instead of being
    estimated stochastically).  spectra[p] is None for a sector taken from its
    moments (nodes x_k, weights gamma_k as in thermo_field) or the array of its
    eigenvalues; an eigenvalue carries weight Ntil, the scale on which the
    gamma_k of a dimension-D sector sum to Ntil * D (discrete orthogonality),
    so both kinds add into one Z.  Zeeman term, mirror sectors, shift and
    flags as in thermo_field."""
    mu = np.atleast_2d(mu)
    P, M = mu.shape
    Nt = n_nodes or M
    g = kernel_coefficients(M, kernel)
    x = nodes(Nt)
    cid, sz, W = _sector_table(problems)
    nc = int(cid.max()) + 1
    T = np.asarray(T, dtype=np.float64)
    h = np.broadcast_to(np.asarray(h, dtype=np.float64), T.shape)
    out = {k: np.zeros((nc, T.size)) for k in ("lnZ", "E", "C", "chi", "M")}
    out["z_nonpos"] = np.zeros((nc, T.size), dtype=bool)
    pts = []
    for p in range(P):
        if spectra[p] is None:
            pts.append((dos_weights(mu[p], g, Nt), ab[p, 0] * x + ab[p, 1]))
        else:
            e = np.asarray(spectra[p], dtype=np.float64)
            pts.append((np.full(e.size, float(Nt)), e))
    for c in range(nc):
        sel = np.nonzero(cid == c)[0]
        for t, (Tv, hv) in enumerate(zip(T, h)):
            beta = 1.0 / Tv
            gs, Es, ms = [], [], []
            for p in sel:
                wp, Ep = pts[p]
                for m in ([sz[p]] if W[p] == 1.0 else [sz[p], -sz[p]]):
                    gs.append(wp)
                    Es.append(Ep + hv * m)
                    ms.append(np.full(Ep.size, m))
            gw, E, m = np.concatenate(gs), np.concatenate(Es), np.concatenate(ms)
            Eref = E.min()
            w = gw * np.exp(-beta * (E - Eref))
            S0 = math.fsum(w)
            Em = math.fsum(w * E) / S0
            varE = math.fsum(w * (E - Em) ** 2) / S0
            m1 = math.fsum(w * m) / S0
            varM = math.fsum(w * (m - m1) ** 2) / S0
            out["z_nonpos"][c, t] = S0 <= 0.0
            out["lnZ"][c, t] = (np.log(S0 / Nt) if S0 > 0 else np.nan) - beta * Eref
            out["E"][c, t] = Em
            out["C"][c, t] = beta**2 * varE
            out["chi"][c, t] = beta * varM
            out["M"][c, t] = m1
    return out


def thermo_vjp(problems, mu: np.ndarray, ab: np.ndarray, T: np.ndarray,
               wC: np.ndarray, wchi: np.ndarray, kernel: str = "jackson", n_nodes: int = 0):
    """lambda[p, n] = dL/dmu_n^p for L = sum_{c,T} wC[c,T] C[c,T] + wchi[c,T] chi[c,T].

    The sums S_0 = sum w, S_1 = sum w E, S_2 = sum w E^2, S_M = sum w m^2 are
    linear in the moments; C = beta^2 (S_2/S_0 - S_1^2/S_0^2) and
    chi = beta S_M/S_0 are differentiated by hand (the mirror sectors make
    sum w m vanish identically)."""
    mu = np.atleast_2d(mu)
    P, M = mu.shape
    Nt = n_nodes or M
    g = kernel_coefficients(M, kernel)
    x = nodes(Nt)
    Cm = cos_matrix(Nt, M) * np.where(np.arange(M) == 0, 1.0, 2.0)[None, :] * g[None, :]
    cid, sz, W = _sector_table(problems)
    nc = int(cid.max()) + 1
    gam = np.stack([dos_weights(mu[p], g, Nt) for p in range(P)])
    Ek = ab[:, 0:1] * x[None, :] + ab[:, 1:2]
    lam = np.zeros((P, M))
    for c in range(nc):
        sel = np.nonzero(cid == c)[0]
        Eref = Ek[sel].min()
        for t, Tv in enumerate(np.asarray(T, dtype=np.float64)):
            beta = 1.0 / Tv
            e = {p: W[p] * np.exp(-beta * (Ek[p] - Eref)) for p in sel}
            S0 = sum(np.dot(gam[p], e[p]) for p in sel)
            S1 = sum(np.dot(gam[p], e[p] * Ek[p]) for p in sel)
            S2 = sum(np.dot(gam[p], e[p] * Ek[p] ** 2) for p in sel)
            SM = sum(sz[p] ** 2 * np.dot(gam[p], e[p]) for p in sel)
            dC0 = beta**2 * (-S2 / S0**2 + 2.0 * S1**2 / S0**3)
            dC1 = -2.0 * beta**2 * S1 / S0**2
            dC2 = beta**2 / S0
            dX0 = -beta * SM / S0**2
            dXM = beta / S0
            a0 = wC[c, t] * dC0 + wchi[c, t] * dX0
            a1 = wC[c, t] * dC1
            a2 = wC[c, t] * dC2
            aM = wchi[c, t] * dXM
            for p in sel:
                node_adj = e[p] * (a0 + a1 * Ek[p] + a2 * Ek[p] ** 2 + aM * sz[p] ** 2)
                lam[p] += node_adj @ Cm
    return lam
