// Finite-temperature Lanczos method (the paper's comparison method): per
// start vector r, plain Lanczos gives a tridiagonal T; its Ritz values eps_j
// and squared first eigenvector components w_j give
//   <r| f(H) |r> / <r|r>  ~  sum_j w_j f(eps_j),
// and the sector trace is estimated as in Eq. (7), dim/R sum_r (...).  The
// Lanczos recursion itself runs through the same step kernels as the
// Chebyshev recursion; these kernels turn its coefficients into Ritz values
// and weights and sum the thermodynamics (with the optional Zeeman term h S^z,
// mirror sectors at -S^z, as in thermo_field_kernel).
#include <hip/hip_runtime.h>

#include "kpm_internal.h"
#include "kpm_tridiag.h"

namespace kpm {

namespace {

__device__ __forceinline__ double ftlm_wsum(double v, double* sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  return ((sh[0] + sh[1]) + sh[2]) + sh[3];
}

__device__ __forceinline__ double ftlm_wmin(double v, double* sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_down(v, off, 64));
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  return fmin(fmin(sh[0], sh[1]), fmin(sh[2], sh[3]));
}

}  // namespace

// One Lanczos column per workgroup, worked by its first lane: the
// tridiagonal is cut at the first negligible off-diagonal (beta < 1e-12) or
// at the sector dimension, then Ritz values and weights (squared first
// components times the column's weight in the estimator: dim/R, or its share
// of |r|^2 for the two real columns of a complex vector, or 1 for the
// complete basis).  The QL sweeps are a serial chain of dependent loads and
// stores, so d, e and z live in LDS when 3 S doubles fit (kRitzLds), else in
// the global result arrays.
constexpr int kRitzLds = 64 * 1024;

__global__ __launch_bounds__(64) void ftlm_ritz_kernel(const FtlmArgs a) {
  extern __shared__ double ritz_sh[];
  const int c = blockIdx.x;
  if (c >= a.total_cols || threadIdx.x != 0) return;
  const UnitDev U = a.units[a.job_unit[2 * c]];
  const ProbDev P = a.probs[U.prob];
  const int S = a.steps;
  double* dg = a.ritz + (int64_t)c * S;
  double* zg = a.weight + (int64_t)c * S;
  const int lc = c - U.col_off;          // column inside the block; padding past ncols
  if (lc >= U.ncols) {
    for (int j = 0; j < S; ++j) dg[j] = zg[j] = 0.0;
    a.len[c] = 0;
    return;
  }
  const bool in_lds = (size_t)3 * S * sizeof(double) <= (size_t)kRitzLds;
  double* d = in_lds ? ritz_sh : dg;
  double* e = in_lds ? ritz_sh + S : a.escr + (int64_t)c * S;
  double* z = in_lds ? ritz_sh + 2 * S : zg;
  const int L = (int)min((int64_t)S, P.dim);
  int n = 0;
  for (int j = 0; j < L; ++j) {
    d[n++] = a.dots[(int64_t)j * a.total_cols + c];
    const double bn = sqrt(fmax(a.b2[(int64_t)j * a.total_cols + c], 0.0));
    if (j == L - 1 || bn < 1e-12) break;
    e[j] = bn;
  }
  if (!tridiag_ql_first_row(d, e, z, n) && a.err) atomicOr(a.err, 8);
  double cw;
  if (a.vec_kind == 3) {
    cw = 1.0;
  } else if (a.vec_kind == 1) {
    const int partner = ((U.col0 + lc) & 1) ? c - 1 : c + 1;   // Re / Im of one vector
    cw = (double)P.dim / a.R * a.norms[c] / (a.norms[c] + a.norms[partner]);
  } else {
    cw = (double)P.dim / a.R;
  }
  for (int j = 0; j < n; ++j) {
    dg[j] = d[j];
    zg[j] = z[j] * z[j] * cw;
  }
  for (int j = n; j < S; ++j) {
    dg[j] = 0.0;
    zg[j] = 0.0;
  }
  a.len[c] = n;
}

hipError_t launch_ftlm_ritz(const FtlmArgs& a, hipStream_t st) {
  const size_t want = (size_t)3 * a.steps * sizeof(double);
  const size_t lds = want <= (size_t)kRitzLds ? want : 0;
  hipLaunchKernelGGL(ftlm_ritz_kernel, dim3(a.total_cols), dim3(64), lds, st, a);
  return hipGetLastError();
}

// Per (point, cluster): sums over the cluster's sectors, both signs of S^z,
// columns and Ritz values, shifted by the lowest energy of the point.
__global__ __launch_bounds__(kThreads) void ftlm_thermo_kernel(const FtlmArgs a) {
  __shared__ double sh[4];
  const int t = blockIdx.x, cl = blockIdx.y;
  const int S = a.steps;
  const int q0 = a.cl_start[cl], q1 = a.cl_start[cl + 1];
  const double beta = 1.0 / a.T[t];
  const double hf = a.h ? a.h[t] : 0.0;

  // pass 0: lowest energy; pass 1: sums; pass 2: centred variances
  double emin = INFINITY, s0 = 0.0, s1 = 0.0, s2 = 0.0, ve = 0.0, vm = 0.0;
  double eref = 0.0, S0 = 0.0, Ebar = 0.0, Mbar = 0.0;
  for (int pass = 0; pass < 3; ++pass) {
    for (int qq = q0; qq < q1; ++qq) {
      const int p = a.cl_list[qq];
      const ThermoProb tp = a.tp[p];
      // the problem's columns: its blocks are consecutive (padding has no Ritz values)
      const int c0 = a.units[a.prob_unit0[p]].col_off;
      const UnitDev Ul = a.units[a.prob_unit0[p + 1] - 1];
      const int c1 = Ul.col_off + Ul.ld;
      const int64_t items = (int64_t)(c1 - c0) * S;
      const int nm = tp.weight > 1 ? 2 : 1;
      for (int64_t i = threadIdx.x; i < items; i += kThreads) {
        const int c = c0 + (int)(i / S);
        const int j = (int)(i % S);
        if (j >= a.len[c]) continue;
        const double eps = a.ritz[(int64_t)c * S + j];
        const double wt = a.weight[(int64_t)c * S + j];
        for (int k = 0; k < nm; ++k) {
          const double m = k == 0 ? tp.sz : -tp.sz;
          const double E = eps + hf * m;
          if (pass == 0) {
            emin = fmin(emin, E);
          } else {
            const double w = wt * exp(-beta * (E - eref));
            if (pass == 1) {
              s0 += w;
              s1 = fma(w, E, s1);
              s2 = fma(w, m, s2);
            } else {
              const double de = E - Ebar, dm = m - Mbar;
              ve = fma(w, de * de, ve);
              vm = fma(w, dm * dm, vm);
            }
          }
        }
      }
    }
    if (pass == 0) {
      eref = ftlm_wmin(emin, sh);
    } else if (pass == 1) {
      S0 = ftlm_wsum(s0, sh);
      Ebar = ftlm_wsum(s1, sh) / S0;
      Mbar = ftlm_wsum(s2, sh) / S0;
    }
  }
  const double VarE = ftlm_wsum(ve, sh) / S0;
  const double VarM = ftlm_wsum(vm, sh) / S0;
  if (threadIdx.x == 0) {
    const int64_t o = (int64_t)cl * a.n_pts + t;
    a.lnZ[o] = (S0 > 0.0 ? log(S0) : NAN) - beta * eref;
    a.E[o] = Ebar;
    a.C[o] = beta * beta * VarE;
    a.chi[o] = beta * VarM;
    if (a.mag) a.mag[o] = Mbar;
  }
}

hipError_t launch_ftlm_thermo(const FtlmArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(ftlm_thermo_kernel, dim3(a.n_pts, a.n_clusters), dim3(kThreads), 0, st, a);
  return hipGetLastError();
}

}  // namespace kpm
