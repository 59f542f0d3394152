"""Random vectors for the trace estimator, Eq. (7) (oracle).

The paper draws Gaussian components r_nu (Sec. II, after Eq. (7)) but names
no generator.  Both sides of the parity tests implement, independently, the
counter-based form of SplitMix64 (Steele, Lea and Flood, OOPSLA 2014):

  u(ctr) = mix(seed + G * (ctr + 1)),   G = 0x9E3779B97F4A7C15,
  mix(z): z ^= z >> 30; z *= 0xBF58476D1CE4E5B9; z ^= z >> 27;
          z *= 0x94D049BB133111EB; z ^= z >> 31       (all mod 2^64),

i.e. the (ctr+1)-th output of the sequential generator started at `seed`.
ctr = (stream << 32) | idx with stream = (cluster << 16) | (n_up << 10) | r.

  Rademacher       column r, row nu: +1 if the top bit of u(idx=nu) is 0 else -1.
  real Gaussian    column r: Box-Muller, u1 = U(idx 2nu), u2 = U(idx 2nu+1),
                   value sqrt(-2 ln u1) cos(2 pi u2), U(u) = ((u >> 11) + 1/2) 2^-53.
  complex Gaussian vector r -> real columns 2r (Re, the cos branch) and 2r+1
                   (Im, the sin branch) of the same Box-Muller pair.
Gaussian vectors are rescaled in float64 to <r|r> = dim; the estimator is
invariant to that normalisation.  The complete-basis mode (Sec. II, exact
traces) uses the unit vectors e_nu.
"""
from __future__ import annotations

import numpy as np

G = 0x9E3779B97F4A7C15
LANCZOS_STREAM = 1023


def mix64(z: np.ndarray) -> np.ndarray:
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def counter_u64(seed: int, stream: int, idx) -> np.ndarray:
    idx = np.asarray(idx, dtype=np.uint64)
    ctr = (np.uint64(stream) << np.uint64(32)) | idx
    with np.errstate(over="ignore"):
        z = np.uint64(seed % 2**64) + np.uint64(G) * (ctr + np.uint64(1))
    return mix64(z)


def stream_id(cluster: int, n_up: int, r: int) -> int:
    assert 0 <= r < 1024 and 0 <= n_up < 64 and 0 <= cluster < 65536
    return (cluster << 16) | (n_up << 10) | r


def uniform01(u: np.ndarray) -> np.ndarray:
    return ((u >> np.uint64(11)).astype(np.float64) + 0.5) * 2.0**-53


def rademacher(seed, cluster, n_up, r, dim) -> np.ndarray:
    u = counter_u64(seed, stream_id(cluster, n_up, r), np.arange(dim, dtype=np.uint64))
    return np.where((u >> np.uint64(63)) == 0, 1.0, -1.0)


def box_muller(seed, cluster, n_up, r, dim):
    s = stream_id(cluster, n_up, r)
    nu = np.arange(dim, dtype=np.uint64)
    u1 = uniform01(counter_u64(seed, s, 2 * nu))
    u2 = uniform01(counter_u64(seed, s, 2 * nu + np.uint64(1)))
    rad = np.sqrt(-2.0 * np.log(u1))
    return rad * np.cos(2.0 * np.pi * u2), rad * np.sin(2.0 * np.pi * u2)


VEC_KINDS = ("rademacher", "complex_gaussian", "gaussian", "basis")


def random_columns(kind: str, seed: int, cluster: int, n_up: int, R: int, dim: int):
    """Start block V0 [dim, ncols] (float64) and the map column -> vector r.

    Returns (V0, vec_of_col, R_eff): R_eff is the number of vectors in Eq. (7)
    (R, or dim for the complete basis)."""
    if kind == "rademacher":
        V = np.stack([rademacher(seed, cluster, n_up, r, dim) for r in range(R)], axis=1)
        return V, np.arange(R), R
    if kind == "gaussian":
        cols = []
        for r in range(R):
            re, _ = box_muller(seed, cluster, n_up, r, dim)
            cols.append(re * np.sqrt(dim / np.dot(re, re)))
        return np.stack(cols, axis=1), np.arange(R), R
    if kind == "complex_gaussian":
        cols = []
        for r in range(R):
            re, im = box_muller(seed, cluster, n_up, r, dim)
            s = np.sqrt(dim / (np.dot(re, re) + np.dot(im, im)))
            cols += [re * s, im * s]
        return np.stack(cols, axis=1), np.repeat(np.arange(R), 2), R
    if kind == "basis":
        return np.eye(dim), np.arange(dim), dim
    raise ValueError(kind)
