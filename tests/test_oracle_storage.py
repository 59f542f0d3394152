"""The float32 + 16-bit residual storage form of the oracle
(`oracle.moments.f32_residual16`), pinned against an exact rational
construction of the same rule, its error bound, and its effect on the
Chebyshev moments (Eq. (7)): much closer to float64 storage than float32
storage is.  The format is this implementation's (the paper fixes none)."""
import math
import struct
from fractions import Fraction

import numpy as np

import workloads as W
from oracle import hamiltonian, moments


def _exact(x: float) -> float:
    """The rule with exact rationals: hi = float32(x) by IEEE conversion
    (struct), e its biased exponent (at least 1), q = x - hi in units of
    2^(e - 165) rounded half to even (Python's round), value hi + q unit."""
    hi = struct.unpack("<f", struct.pack("<f", x))[0]
    e = max((struct.unpack("<I", struct.pack("<f", hi))[0] >> 23) & 0xFF, 1)
    unit = Fraction(2) ** (e - 165)
    q = round((Fraction(x) - Fraction(hi)) / unit)
    assert abs(q) <= 2 ** 14
    out = Fraction(hi) + q * unit
    assert float(out) == out          # exactly a float64
    return float(out)


def _samples():
    rng = np.random.default_rng(11)
    x = [rng.normal(size=3000), rng.normal(size=500) * 1e-30, rng.normal(size=500) * 1e30,
         rng.uniform(-1, 1, size=500) * 2.0 ** -140,                    # float32 subnormal range
         np.ldexp(1.0, rng.integers(-60, 60, size=300)) * (1 - rng.uniform(0, 1e-7, size=300)),
         np.ldexp(1.0, rng.integers(-60, 60, size=300)) * (1 + rng.uniform(0, 1e-7, size=300)),
         np.array([0.0, -0.0, 1.0, -1.0, 1 + 2.0 ** -24, 1 + 3 * 2.0 ** -25, 1 + 2.0 ** -40])]
    return np.concatenate(x)


def test_rule_matches_exact_rational_construction():
    x = _samples()
    got = moments.f32_residual16(x)
    want = np.array([_exact(float(v)) for v in x])
    assert np.array_equal(got, want)


def test_error_bound_idempotence_and_float32_values():
    x = _samples()
    y = moments.f32_residual16(x)
    hi = x.astype(np.float32)
    e = np.maximum((hi.view(np.uint32) >> 23) & 0xFF, 1).astype(np.int64)
    assert np.all(np.abs(y - x) <= np.ldexp(1.0, (e - 166).astype(np.int32)))
    normal = np.abs(hi) >= np.float32(2.0 ** -126)
    rel = np.abs(y - x)[normal] / np.abs(x)[normal]
    assert rel.max() <= 2.0 ** -38
    assert np.array_equal(moments.f32_residual16(y), y)
    f = x.astype(np.float32).astype(np.float64)
    assert np.array_equal(moments.f32_residual16(f), f)
    # the residual recovers what float32 rounding drops: on the Gaussian
    # samples float32 alone is off by ~2^-25 relative, the stored value by < 2^-38
    g = slice(0, 3000)
    assert np.median(np.abs(f[g] - x[g]) / np.abs(x[g])) > 2.0 ** -27
    assert np.median(np.abs(y[g] - x[g]) / np.abs(x[g])) < 2.0 ** -39


def test_moments_with_residual_storage_track_float64():
    """Ring N=12, S^z=0 (924 states), 4 real Gaussian vectors, M=256: the
    residual form's moments are within 1e-11 mu_0 of float64 storage, and
    at least 1000 times closer than float32 storage."""
    s = [x for x in W.sectors(W.ring(12)) if x.n_up == 6][0]
    H = hamiltonian.sector_hamiltonian(s.cluster, s.n_up)
    e = np.linalg.eigvalsh(H.toarray())
    a, b = hamiltonian.scale_from_bounds(e.min() - 0.01, e.max() + 0.01, 0.025)
    args = (s, a, b, 256, 4, "gaussian", 3)
    m64 = moments.sector_moments(*args, H=H)
    m32 = moments.sector_moments(*args, H=H, store=np.float32)
    m32r = moments.sector_moments(*args, H=H, store=moments.F32R)
    e32 = np.abs(m32 - m64).max() / m64[0]
    e32r = np.abs(m32r - m64).max() / m64[0]
    assert e32r <= 1e-11, e32r
    assert e32r * 1000 <= e32, (e32r, e32)
    assert math.isclose(m32r[0], s.dim, rel_tol=1e-12)
