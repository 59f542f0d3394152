"""CPU oracle for the stochastic Chebyshev-moment (kernel polynomial) typicality
method of Schlueter, Gayk, Schmidt, Honecker and Schnack, "Accuracy of the
typicality approach using Chebyshev polynomials" (arXiv:2104.13218).

TEST INFRASTRUCTURE ONLY.  Plain, slow, obviously-correct NumPy/SciPy code in
float64 that the GPU library is checked against.  Only the test suite, the
smoke check and the benchmark's CPU-baseline leg may import it.  It shares no
code, table or helper with the HIP library (the library never imports it); the
only common module is `workloads`, which describes problems (bond lists,
sectors, temperature grids) and does none of the method's arithmetic.

Every function cites the passage of the paper it follows (section / equation).
Points where the paper is silent or ambiguous are resolved by explicit
readings, each restated in the docstring of the function that uses it.

Modules
  basis        S^z-sector enumeration, combinatorial-number-system rank
  hamiltonian  sector matrices of H = sum_b J_b s_i.s_j (CSR), Kronecker build
  rng          counter-based SplitMix64 random vectors
  rows         single rows of v_n = C_n(H') v_0 for sectors too large to hold
  ftlm         finite-temperature Lanczos (the comparison method)
  moments      three-term recursion, doubling identities, estimator Eq. (7),
               exact traces by diagonalisation, Lanczos bounds
  thermo       Jackson kernel Eq. (8), Gauss-Chebyshev quadrature, Z, E, C, chi
               and their derivatives with respect to the moments
  adjoint      reverse-mode derivative of the moments with respect to J_b,
               finite differences and Hellmann-Feynman references
  ed           thermodynamics from exact diagonalisation
"""
from . import basis, hamiltonian, rng, rows, moments, thermo, adjoint, ed, ftlm  # noqa: F401
