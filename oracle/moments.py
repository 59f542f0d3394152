"""Chebyshev moments mu_n = Tr C_n(H'), Eqs. (6)-(7) (oracle).

Exact:      mu_n = sum_i C_n(x_i) over the eigenvalues x_i of H' (Eq. (6); the
            paper's complete-basis traces, Sec. II).
Stochastic: mu_n ~ dim/R sum_r <r|C_n(H')|r> / <r|r>  (Eq. (7)).

The paper defers the recursion to Weisse et al. (Rev. Mod. Phys. 78, 275):
v_0 = r, v_1 = H' v_0, v_{n+1} = 2 H' v_n - v_{n-1}, so v_n = C_n(H') r.
Two routes to <r|v_n> are written out: directly (`moments_direct`) and via the
doubling identities C_2n = 2 C_n^2 - C_0, C_2n+1 = 2 C_n+1 C_n - C_1
(`doubling`), which need only M/2 products.  Moment count: M moments
mu_0..mu_{M-1}; the paper's N_deg is M (its top term mu_{N_deg} carries zero
weight under the Jackson kernel and vanishes at the N_deg quadrature nodes).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from . import basis, hamiltonian, rng


F32R = "f32r"   # storage name of the float32 + 16-bit residual form


def f32_residual16(x) -> np.ndarray:
    """The stored values of the float32 + 16-bit residual storage form.

    Not in the paper (it fixes no storage format): a reduced-storage form of
    this implementation, defined here as its reference.  Each element x is kept
    as hi = float32(x) (round to nearest even) and the integer
    q = rint((x - hi) * 2**(165 - e)) (half to even), where e is the biased
    exponent of hi, at least 1; the stored value is hi + q * 2**(e - 165).
    |x - hi| <= 2**(e - 151), so |q| <= 2**14 and the stored value is x to
    within 2**(e - 166) (relative 2**-39 for normal hi).  Returns float64."""
    x = np.asarray(x, dtype=np.float64)
    hi = x.astype(np.float32)
    e = np.maximum((hi.view(np.uint32) >> 23) & 0xFF, 1).astype(np.int64)
    unit = np.ldexp(np.ones_like(x), (e - 165).astype(np.int32))
    q = np.rint((x - hi.astype(np.float64)) / unit)
    return hi.astype(np.float64) + q * unit


def stored(x, store) -> np.ndarray:
    """x rounded as the storage form `store` keeps it: a numpy float type
    (float64, float32) or F32R."""
    if isinstance(store, str) and store == F32R:
        return f32_residual16(x)
    return np.asarray(x).astype(store)


def n_steps(M: int) -> int:
    """Matrix-vector products needed for mu_0..mu_{M-1} by doubling."""
    return max(1, M // 2)


def chebyshev_dots(Ht, V0: np.ndarray, K: int, store=np.float64, keep=False):
    """Run the recursion for K products.  Vectors are stored in `store`
    precision (float64, float32 or F32R for the reduced-storage forms);
    products and sums are float64.  Returns alpha[n] = <v_n, v_n> (n = 0..K)
    and beta[n] = <v_{n+1}, v_n> (n = 0..K-1), per column, from the stored
    values."""
    f64 = np.float64
    prev = stored(np.asarray(V0, dtype=f64), store)
    alpha = np.zeros((K + 1, V0.shape[1]))
    beta = np.zeros((K, V0.shape[1]))
    alpha[0] = np.einsum("ij,ij->j", prev.astype(f64), prev.astype(f64))
    cur = stored(Ht @ prev.astype(f64), store)
    saved = [prev, cur] if keep else None
    alpha[1] = np.einsum("ij,ij->j", cur.astype(f64), cur.astype(f64))
    beta[0] = np.einsum("ij,ij->j", cur.astype(f64), prev.astype(f64))
    for n in range(1, K):
        nxt = stored(2.0 * (Ht @ cur.astype(f64)) - prev.astype(f64), store)
        alpha[n + 1] = np.einsum("ij,ij->j", nxt.astype(f64), nxt.astype(f64))
        beta[n] = np.einsum("ij,ij->j", nxt.astype(f64), cur.astype(f64))
        prev, cur = cur, nxt
        if keep:
            saved.append(cur)
    return (alpha, beta, saved) if keep else (alpha, beta)


def doubling(alpha: np.ndarray, beta: np.ndarray, M: int) -> np.ndarray:
    """<r|C_n|r> for n < M from alpha, beta (per column)."""
    mu = np.zeros((M,) + alpha.shape[1:])
    for n in range(M):
        h = n // 2
        if n == 0:
            mu[n] = alpha[0]
        elif n == 1:
            mu[n] = beta[0]
        elif n % 2 == 0:
            mu[n] = 2.0 * alpha[h] - alpha[0]
        else:
            mu[n] = 2.0 * beta[h] - beta[0]
    return mu


def moments_direct(Ht, V0: np.ndarray, M: int) -> np.ndarray:
    """<v_0|v_n> for n < M by running the recursion M-1 times (per column)."""
    v0 = np.asarray(V0, dtype=np.float64)
    mu = np.zeros((M, v0.shape[1]))
    prev, cur = v0, Ht @ v0
    mu[0] = np.einsum("ij,ij->j", v0, v0)
    if M > 1:
        mu[1] = np.einsum("ij,ij->j", v0, cur)
    for n in range(2, M):
        prev, cur = cur, 2.0 * (Ht @ cur) - prev
        mu[n] = np.einsum("ij,ij->j", v0, cur)
    return mu


def estimator(mu_cols: np.ndarray, norms: np.ndarray, vec_of_col: np.ndarray,
              dim: int, R: int) -> np.ndarray:
    """Eq. (7): dim/R sum_r <r|C_n|r>/<r|r>.  A complex vector's two real
    columns are summed in numerator and denominator (H' is real)."""
    out = np.zeros(mu_cols.shape[0])
    for r in np.unique(vec_of_col):
        cols = vec_of_col == r
        out += mu_cols[:, cols].sum(axis=1) / norms[cols].sum()
    return out * (dim / R)


def exact_moments(eigs_scaled: np.ndarray, M: int) -> np.ndarray:
    """Eq. (6) by diagonalisation: sum_i C_n(x_i)."""
    x = np.asarray(eigs_scaled, dtype=np.float64)
    return np.polynomial.chebyshev.chebvander(x, M - 1).sum(axis=0)


def lanczos_extremes(H, v0: np.ndarray, steps: int):
    """Extreme Ritz values of plain Lanczos (no reorthogonalisation) started at
    v0; stops early when the next off-diagonal falls below 1e-12."""
    dim = H.shape[0]
    steps = min(steps, dim)
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
    th = sla.eigh_tridiagonal(np.array(a_list), np.array(b_list), eigvals_only=True)
    return float(th[0]), float(th[-1])


def spectral_bounds(sector, steps: int = 50, margin: float = 0.01, seed: int = 0, H=None):
    """E_min, E_max for Eq. (5) from Lanczos (the paper's ground-state estimate
    uses Lanczos, Sec. III.A.2.b), widened by `margin` of the width on each
    side; a (near-)degenerate window is widened to E -/+ 1/2."""
    if H is None:
        H = hamiltonian.sector_hamiltonian(sector.cluster, sector.n_up)
    # real Gaussian start (Box-Muller, stream r = 1023): a +-1 vector can be
    # exactly orthogonal to an extreme eigenvector (e.g. the uniform one-magnon
    # state of an N = 18, n_up = 17 sector when half the signs are +1), which
    # leaves that eigenvalue out of the Krylov space; a Gaussian one is
    # orthogonal with probability zero
    v0, _ = rng.box_muller(seed, sector.cluster_id, sector.n_up, rng.LANCZOS_STREAM, H.shape[0])
    lo, hi = lanczos_extremes(H, v0, steps)
    W = hi - lo
    if W < 1e-8 * max(1.0, abs(lo), abs(hi)):
        return lo - 0.5, hi + 0.5
    return lo - margin * W, hi + margin * W


def sector_moments(sector, a: float, b: float, M: int, R: int, kind: str, seed: int,
                   store=np.float64, H=None, direct=False):
    """Stochastic (or complete-basis) moments of one sector, Eq. (7), via the
    doubling identities (or directly)."""
    if H is None:
        H = hamiltonian.sector_hamiltonian(sector.cluster, sector.n_up)
    Ht = hamiltonian.rescaled(H, a, b)
    dim = H.shape[0]
    V0, vec_of_col, R_eff = rng.random_columns(kind, seed, sector.cluster_id, sector.n_up, R, dim)
    if direct:
        mu_cols = moments_direct(Ht, stored(V0, store).astype(np.float64), M)
        norms = mu_cols[0]
    else:
        alpha, beta = chebyshev_dots(Ht, V0, n_steps(M), store=store)
        mu_cols = doubling(alpha, beta, M)
        norms = alpha[0]
    return estimator(mu_cols, norms, vec_of_col, dim, R_eff)


def sector_exact_moments(sector, a: float, b: float, M: int, H=None) -> np.ndarray:
    if H is None:
        H = hamiltonian.sector_hamiltonian(sector.cluster, sector.n_up)
    x = (np.linalg.eigvalsh(H.toarray()) - b) / a
    return exact_moments(x, M)
