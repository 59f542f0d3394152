"""Thermodynamics from exact diagonalisation (oracle).

Z = sum_n exp(-beta E_n) (Eq. (2)), C = beta^2 (<E^2> - <E>^2) (Eq. (2b)),
chi = beta (<S_z^2> - <S_z>^2) with the S^z-resolved sums of Eq. (3); S^z < 0
sectors enter through their degenerate S^z > 0 mirrors.  Energies are shifted
by the ground-state energy before exponentiation.
"""
from __future__ import annotations

import numpy as np

from . import hamiltonian


def sector_spectra(sectors):
    """[(eigenvalues, S^z, weight)] for each S^z >= 0 sector."""
    out = []
    for s in sectors:
        H = hamiltonian.sector_hamiltonian(s.cluster, s.n_up).toarray()
        out.append((np.linalg.eigvalsh(H), s.n_up - 0.5 * s.cluster.n_sites,
                    1 if 2 * s.n_up == s.cluster.n_sites else 2))
    return out


def thermo_from_spectra(spectra, T):
    T = np.asarray(T, dtype=np.float64)
    E0 = min(e.min() for e, _, _ in spectra)
    res = {k: np.zeros(T.size) for k in ("lnZ", "E", "C", "chi")}
    for t, Tv in enumerate(T):
        beta = 1.0 / Tv
        S0 = S1 = S2 = SM1 = SM2 = 0.0
        for e, m, w in spectra:
            bz = np.exp(-beta * (e - E0))
            for mm in ([m] if w == 1 else [m, -m]):
                S0 += bz.sum()
                S1 += np.dot(bz, e)
                S2 += np.dot(bz, e * e)
                SM1 += mm * bz.sum()
                SM2 += mm * mm * bz.sum()
        Em = S1 / S0
        varE = 0.0
        for e, m, w in spectra:
            bz = np.exp(-beta * (e - E0))
            varE += (1 if w == 1 else 2) * np.dot(bz, (e - Em) ** 2)
        res["lnZ"][t] = np.log(S0) - beta * E0
        res["E"][t] = Em
        res["C"][t] = beta**2 * varE / S0
        res["chi"][t] = beta * (SM2 / S0 - (SM1 / S0) ** 2)
    return res


def hellmann_feynman_C(sectors, T):
    """dC/dJ_b of the exact thermodynamics, from dE_i/dJ_b = <i|h_b|i>.
    Returns [n_bonds, n_T]."""
    cl = sectors[0].cluster
    T = np.asarray(T, dtype=np.float64)
    data = []
    for s in sectors:
        H = hamiltonian.sector_hamiltonian(cl, s.n_up).toarray()
        e, U = np.linalg.eigh(H)
        hd = np.stack([np.einsum("ji,jk,ki->i", U,
                                 hamiltonian.bond_operator(cl, s.n_up, b).toarray(), U)
                       for b in range(cl.n_bonds)])
        data.append((e, hd, 1 if 2 * s.n_up == cl.n_sites else 2))
    E0 = min(e.min() for e, _, _ in data)
    out = np.zeros((cl.n_bonds, T.size))
    for t, Tv in enumerate(T):
        beta = 1.0 / Tv
        Z = Z1 = Z2 = 0.0
        dZ = np.zeros(cl.n_bonds); dZ1 = np.zeros(cl.n_bonds); dZ2 = np.zeros(cl.n_bonds)
        for e, hd, w in data:
            bz = w * np.exp(-beta * (e - E0))
            Z += bz.sum(); Z1 += np.dot(bz, e); Z2 += np.dot(bz, e * e)
            # d/dJ of sum exp(-beta e) f(e) = sum exp(-beta e) (f'(e) - beta f(e)) de/dJ
            dZ += hd @ (bz * (-beta))
            dZ1 += hd @ (bz * (1.0 - beta * e))
            dZ2 += hd @ (bz * (2.0 * e - beta * e * e))
        # the common shift E0 depends on J too, but C is shift-invariant and the
        # shift cancels between numerator and denominator of every ratio
        Em = Z1 / Z
        dEm = dZ1 / Z - Z1 * dZ / Z**2
        dE2 = dZ2 / Z - Z2 * dZ / Z**2
        out[:, t] = beta**2 * (dE2 - 2.0 * Em * dEm)
    return out
