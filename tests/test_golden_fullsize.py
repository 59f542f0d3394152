"""Pins of the full-length expected values of the 24-site ring
(tests/golden/ring24_*.txt, written from the oracle by
make_fullsize_golden.py) against facts that do not come from the oracle's
recursion itself:

* Eq. (7) with normalised vectors: mu_0 = dim exactly; |mu_n| <= mu_0 since
  |T_n(x)| <= 1 on the rescaled spectrum.
* float32 storage with float64 arithmetic stays within 1e-5 mu_0 of float64.
* Bounds of Eq. (5): every sector holds the fully polarised-like top state
  with E_max = sum_b J_b / 4 = 6 (an exact eigenvalue of the ring in every
  S^z sector), so 6 lies inside [E_lo, E_hi] within the 1 % margin; the
  dimension-1 sector (all spins up, E = 6) gets the widened window 6 -/+ 1/2.
* High-temperature expansion of the thermodynamics (Sec. II sums):
  ln Z = N ln 2 + beta^2 Tr H^2 / (2 2^N) + O(beta^3) with
  Tr H^2 / 2^N = (3/16) sum_b J_b^2 = 4.5 for the ring, and the Curie law
  chi T -> N/4 with the nearest-neighbour correction chi T ~ (N/4) T/(T + J/2).
"""
import math
import os

import numpy as np

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
N = 24


def _load(name):
    return np.loadtxt(os.path.join(GOLDEN, name))


def test_moments_normalisation_and_bound():
    mu = _load("ring24_all_fp64_M2000.txt").T          # [13][2000]
    assert mu.shape == (13, 2000)
    for p, n_up in enumerate(range(12, 25)):
        dim = math.comb(N, n_up)
        assert abs(mu[p, 0] - dim) <= 1e-12 * dim
        assert np.all(np.abs(mu[p]) <= mu[p, 0] * (1 + 1e-12))


def test_float32_storage_close_to_float64():
    mu64 = _load("ring24_all_fp64_M2000.txt")[:, 0]
    mu32 = _load("ring24_sz0_fp32_M2000.txt")
    assert abs(mu32[0] - math.comb(N, 12)) <= 1e-9 * mu32[0]
    err = np.abs(mu32 - mu64).max() / mu64[0]
    assert 0 < err <= 1e-5, err


def test_bounds_enclose_the_known_top_eigenvalue():
    b = _load("ring24_bounds.txt")
    assert [int(x) for x in b[:, 0]] == list(range(12, 25))
    for n_up, lo, hi in b:
        assert lo < 6.0 <= hi, (n_up, lo, hi)
        if n_up < 24:
            width = (hi - lo) / 1.02
            assert hi - 6.0 <= 0.0101 * width + 1e-9, (n_up, hi)   # Lanczos converges to E_max
        else:
            assert (lo, hi) == (5.5, 6.5)
    # the S^z = 0 ground state of the 24-site ring, E_0 = -10.7715 (E_0/N = -0.4488,
    # Bethe ansatz), lies inside the window, which the 1 % margin keeps tight
    lo0 = b[0, 1]
    assert -10.95 < lo0 < -10.7715


def test_high_temperature_expansion():
    for kern in ("jackson", "none"):
        th = _load(f"ring24_thermo_{kern}.txt")
        T, lnZ, E, C, chi = th.T
        assert T.size == 200 and abs(T[0] - 0.01) < 1e-12 and abs(T[-1] - 10.0) < 1e-12
        beta = 1.0 / T[-1]
        lead = N * math.log(2.0) + beta ** 2 * 4.5 / 2.0
        assert abs(lnZ[-1] - lead) < 5e-4, (kern, lnZ[-1], lead)
        assert abs(E[-1] + 4.5 * beta) < 0.05, (kern, E[-1])            # <E> ~ -beta Tr H^2/2^N
        assert abs(chi[-1] * T[-1] - (N / 4) * T[-1] / (T[-1] + 0.5)) < 0.02, (kern, chi[-1])
