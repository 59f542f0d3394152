#!/usr/bin/env python3
"""Write the full-length expected values of the 24-site ring workloads.

Calls nothing but the CPU oracle (`oracle/`) and the seeded workload
generator (`workloads.py`).  Outputs, all plain text under tests/golden/:

  ring24_bounds.txt            per S^z >= 0 sector (n_up 12..24): the oracle's
                               50-step Lanczos extremes widened by 1 % of the
                               width on each side (the bounds of Eq. (5) as the
                               paper estimates them, Sec. III.A.2.b), seed 0
  ring24_sz0_fp32_M2000.txt    S^z = 0 sector, 10 complex Gaussian vectors,
                               eps = 0.025, M = 2000, float32 vector storage
                               with float64 products and dots (Eq. (7) through
                               the recursion and doubling identities)
  ring24_all_fp64_M2000.txt    every sector, same vectors, float64 storage
  ring24_thermo_<kernel>.txt   Z, E, C, chi of the whole ring (Sec. II sector
                               sum) from those float64 moments, Jackson kernel
                               and g_n = 1, 200 log-spaced T in [0.01, 10]

Each recursion column is independent, so the columns of a sector are run in
forked worker processes (one BLAS thread each) and joined before the oracle's
doubling identities and estimator; the result is the same as one call on all
columns.  About 10 minutes on 8 cores.

    python tests/golden/make_fullsize_golden.py [--workers 6]
"""
from __future__ import annotations

import argparse
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import hamiltonian, moments, rng, thermo  # noqa: E402

M = 2000
R = 10
KIND = "complex_gaussian"
EPS = 0.025
SEED = 0
T_GRID = (200, 0.01, 10.0)

_SHARED = {}


def _dots(args):
    cols, store = args
    from threadpoolctl import threadpool_limits
    with threadpool_limits(1):
        a, b = moments.chebyshev_dots(_SHARED["Ht"], _SHARED["V0"][:, cols], moments.n_steps(M),
                                      store=store)
    return cols, a, b


def sector_moments_parallel(sec, H, a, b, store, workers):
    """moments.sector_moments with the recursion's columns spread over processes."""
    Ht = hamiltonian.rescaled(H, a, b)
    dim = H.shape[0]
    V0, vec_of_col, R_eff = rng.random_columns(KIND, SEED, sec.cluster_id, sec.n_up, R, dim)
    ncol = V0.shape[1]
    K = moments.n_steps(M)
    alpha = np.zeros((K + 1, ncol))
    beta = np.zeros((K, ncol))
    groups = [list(g) for g in np.array_split(np.arange(ncol), min(workers, ncol)) if len(g)]
    _SHARED.update(Ht=Ht, V0=V0)
    with mp.get_context("fork").Pool(len(groups)) as pool:
        for cols, al, be in pool.imap_unordered(_dots, [(g, store) for g in groups]):
            alpha[:, cols] = al
            beta[:, cols] = be
    _SHARED.clear()
    mu_cols = moments.doubling(alpha, beta, M)
    return moments.estimator(mu_cols, alpha[0], vec_of_col, dim, R_eff)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workers", type=int, default=max(1, min(8, os.cpu_count() or 1)))
    args = ap.parse_args()
    t_start = time.time()
    secs = W.sectors(W.ring(24))
    bounds, mu64 = [], []
    mu32 = None
    for s in secs:
        t0 = time.time()
        H = hamiltonian.sector_hamiltonian(s.cluster, s.n_up)
        lo, hi = moments.spectral_bounds(s, 50, 0.01, SEED, H=H)
        a, b = hamiltonian.scale_from_bounds(lo, hi, EPS)
        bounds.append((s.n_up, lo, hi))
        mu64.append(sector_moments_parallel(s, H, a, b, np.float64, args.workers))
        if 2 * s.n_up == s.cluster.n_sites:
            mu32 = sector_moments_parallel(s, H, a, b, np.float32, args.workers)
        print(f"n_up={s.n_up} dim={s.dim} bounds=({lo:.12f}, {hi:.12f}) {time.time() - t0:.0f} s",
              flush=True)
    mu64 = np.array(mu64)
    ab = np.array([hamiltonian.scale_from_bounds(lo, hi, EPS) for _, lo, hi in bounds])
    head = (f"ring N=24 J=1, {R} complex Gaussian vectors, seed {SEED}, eps {EPS}, M {M}; "
            "written by tests/golden/make_fullsize_golden.py from the oracle")
    np.savetxt(os.path.join(HERE, "ring24_bounds.txt"), np.array(bounds), fmt=["%d", "%.17g", "%.17g"],
               header=head + "\ncolumns: n_up, E_lo, E_hi (50-step Lanczos, 1 % margin each side)")
    np.savetxt(os.path.join(HERE, "ring24_sz0_fp32_M2000.txt"), mu32, fmt="%.17g",
               header=head + "\nS^z = 0 sector, float32 vector storage: mu_n, n = 0..M-1")
    np.savetxt(os.path.join(HERE, "ring24_all_fp64_M2000.txt"), mu64.T, fmt="%.17g",
               header=head + "\nfloat64: column p = sector n_up = 12 + p, row n = mu_n")
    T = W.log_temperatures(*T_GRID)
    probs = [dict(cluster=0, n_sites=24, n_up=s.n_up) for s in secs]
    for kern in ("jackson", "none"):
        out = thermo.thermo(probs, mu64, ab, T, kern)
        cols = [T] + [np.asarray(out[k])[0] for k in ("lnZ", "E", "C", "chi")]
        np.savetxt(os.path.join(HERE, f"ring24_thermo_{kern}.txt"), np.array(cols).T, fmt="%.17g",
                   header=head + f"\nkernel {kern}, Ntilde = M; columns: T, lnZ, E, C, chi")
    print(f"done in {time.time() - t_start:.0f} s", flush=True)


if __name__ == "__main__":
    main()
