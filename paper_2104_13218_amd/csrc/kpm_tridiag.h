// Symmetric tridiagonal eigenproblem for the Lanczos quadrature of the
// finite-temperature Lanczos method: eigenvalues of T (diagonal d[0..n),
// off-diagonal e[i] between rows i and i+1, i < n-1) and the first component
// of every normalised eigenvector, by the implicit QL method with the shift
// from the trailing 2x2 block.  Only row 0 of the accumulated plane rotations
// is kept (it starts as the unit vector e_0), so the cost is O(n^2).
//
// Source of the method: the implicit QL algorithm of A. Bowdler, R. S. Martin,
// C. Reinsch and J. H. Wilkinson, "The QR and QL algorithms for symmetric
// matrices", Numer. Math. 11, 293-306 (1968), as distributed in EISPACK (tql1,
// tql2) and restated in Numerical Recipes (tqli).  The sweep, the Wilkinson-
// type shift, the deflation test |e_m| + (|d_m| + |d_m+1|) == |d_m| + |d_m+1|
// and the single-letter variable names follow that published form; the change
// here is that the eigenvector update is restricted to row 0.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace kpm {

// d[n], e[n] (e[n-1] is scratch), z[n] out: d -> eigenvalues (unordered),
// z -> first eigenvector components.  Returns false if an eigenvalue needed
// more than 60 sweeps.
__host__ __device__ inline bool tridiag_ql_first_row(double* d, double* e, double* z, int n) {
  for (int i = 0; i < n; ++i) z[i] = i == 0 ? 1.0 : 0.0;
  if (n <= 0) return true;
  e[n - 1] = 0.0;
  for (int l = 0; l < n; ++l) {
    int iter = 0;
    int m;
    do {
      // smallest m >= l whose off-diagonal is negligible next to its diagonal
      // pair (d[m + 1] carried to the next test in a register)
      double dm = d[l];
      for (m = l; m < n - 1; ++m) {
        const double dm1 = d[m + 1];
        const double dd = fabs(dm) + fabs(dm1);
        if (fabs(e[m]) + dd == dd) break;
        dm = dm1;
      }
      if (m != l) {
        if (++iter > 60) return false;
        double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
        double r = hypot(g, 1.0);
        g = d[m] - d[l] + e[l] / (g + copysign(r, g));
        double s = 1.0, c = 1.0, p = 0.0;
        // the sweep from i = m - 1 down to l: z[i + 1] and d[i + 1] of each
        // rotation are the values the previous one left, carried in registers
        // (zc, dn) so that the serial chain does not pass through memory
        double zc = z[m], dn = d[m];
        bool deflated = false;
        for (int i = m - 1; i >= l; --i) {
          const double ei = e[i], di = d[i], zi = z[i];
          double f = s * ei;
          const double b = c * ei;
          // f and g are of the order of the spectral width (Lanczos
          // coefficients), far from float64 overflow and underflow: the plain
          // norm and one reciprocal replace hypot and two divisions
          r = sqrt(fma(f, f, g * g));
          e[i + 1] = r;
          if (r == 0.0) {
            d[i + 1] = dn - p;
            z[i + 1] = zc;
            e[m] = 0.0;
            deflated = true;
            break;
          }
          const double inv = 1.0 / r;
          s = f * inv;
          c = g * inv;
          g = dn - p;
          r = (di - g) * s + 2.0 * c * b;
          p = s * r;
          d[i + 1] = g + p;
          g = c * r - b;
          z[i + 1] = s * zi + c * zc;
          zc = c * zi - s * zc;
          dn = di;
        }
        if (deflated) continue;
        z[l] = zc;
        d[l] -= p;
        e[l] = g;
        e[m] = 0.0;
      }
    } while (m != l);
  }
  return true;
}

}  // namespace kpm
