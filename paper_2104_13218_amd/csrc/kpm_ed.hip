// Exact spectra of small S^z sectors (Sec. II: a sector of small dimension is
// diagonalised completely instead of being estimated stochastically) and the
// thermodynamics that mix such spectra with the moments of the other sectors.
//
// The dense float64 matrix of H on each sector basis (rank order) is built in
// the workspace and reduced to a symmetric tridiagonal matrix by Householder
// reflections applied from both sides, one column per step for all sectors at
// once (three launches per step, the trailing block split over row tiles so
// that large sectors spread over the chip); the eigenvalues of the
// tridiagonal matrix then come from bisection on Sturm counts, one
// workgroup per sector and one eigenvalue per thread.
#include <hip/hip_runtime.h>

#include <cmath>

#include "kpm_device.h"
#include "kpm_internal.h"

namespace kpm {

namespace {

// Sum over the workgroup, returned to every thread (fixed order).
__device__ __forceinline__ double ed_sum(double v, double* sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  const double r = ((sh[0] + sh[1]) + sh[2]) + sh[3];
  __syncthreads();
  return r;
}

// Rows of H on a spin-s sector (digits d_i = s + m_i with sum n_up): diagonal
// sum_b J_b m_i m_j, S^+_i S^-_j and S^-_i S^+_j with amplitude
// J_b/2 sqrt(s(s+1) - m(m+1)) sqrt(s(s+1) - m'(m'-1)).  One row per thread.
__device__ void spin_rows(const EigProb& P, const EigArgs& a, const uint32_t* s_sites, const double* s_J,
                          double* A) {
  const int N = P.n_sites, two_s = P.two_s, B = two_s + 1, R1 = two_s * N + 1, D = P.dim;
  const double sv = 0.5 * two_s;
  const uint32_t* tab = a.tables + P.tab_off;
  for (int r = threadIdx.x; r < D; r += kThreads) {
    uint64_t dg = 0;
    uint32_t rem = (uint32_t)r;
    int left = P.n_up;
    for (int i = N - 1; i >= 0; --i) {
      int d = min(two_s, left);
      while (d > 0 && tab[(i * R1 + left) * B + d] > rem) --d;
      rem -= tab[(i * R1 + left) * B + d];
      dg |= (uint64_t)d << (4 * i);
      left -= d;
    }
    double diag = 0.0;
    for (int q = 0; q < P.n_bonds; ++q) {
      const int i = (int)(s_sites[q] & 0xFFu), j = (int)(s_sites[q] >> 8);
      const int di = (int)((dg >> (4 * i)) & 15u), dj = (int)((dg >> (4 * j)) & 15u);
      diag += s_J[q] * (di - sv) * (dj - sv);
      for (int w = 0; w < 2; ++w) {
        const int a1 = w == 0 ? i : j, a2 = w == 0 ? j : i;
        const int d1 = w == 0 ? di : dj, d2 = w == 0 ? dj : di;
        if (d1 >= two_s || d2 <= 0) continue;
        const double m1 = d1 - sv, m2 = d2 - sv;
        const double amp = 0.5 * s_J[q] * sqrt(sv * (sv + 1.0) - m1 * (m1 + 1.0)) *
                           sqrt(sv * (sv + 1.0) - m2 * (m2 - 1.0));
        const uint32_t c =
            spin_rank(dg + ((uint64_t)1 << (4 * a1)) - ((uint64_t)1 << (4 * a2)), N, P.n_up, R1, B, tab);
        if (c < (uint32_t)D) A[(int64_t)r * D + c] += amp;
        else if (a.err) atomicOr(a.err, 2);
      }
    }
    A[(int64_t)r * D + r] += diag;
  }
}

}  // namespace

// Dense H of every sector (one workgroup per sector, one row per thread).
__global__ __launch_bounds__(kThreads) void ed_build_kernel(const EigArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x;
  const EigProb P = a.probs[blockIdx.x];
  const int D = P.dim;
  uint32_t* sb = reinterpret_cast<uint32_t*>(smem);                       // [33 * 33]
  uint32_t* s_mask = sb + kBinomN * kBinomN;                               // [lds_bonds]
  double* s_J = reinterpret_cast<double*>(smem + a.o_bonds);              // [lds_bonds]
  for (int i = tid; i < kBinomN * kBinomN; i += kThreads) sb[i] = a.binom[i];
  for (int q = tid; q < P.n_bonds; q += kThreads) {
    s_mask[q] = a.bmask[P.bond_off + q];
    s_J[q] = a.J[P.bond_off + q];
  }
  double* A = a.mat + P.mat_off;
  for (int64_t i = tid; i < (int64_t)D * D; i += kThreads) A[i] = 0.0;
  __syncthreads();
  if (P.two_s > 1) {
    spin_rows(P, a, s_mask, s_J, A);
    return;
  }
  // s_i s_j = 1/4 for equal spins, -1/4 otherwise; unequal spins are
  // exchanged with amplitude J/2.
  for (int r = tid; r < D; r += kThreads) {
    const uint32_t s = unrank((uint32_t)r, P.n_sites, P.n_up, sb);
    double diag = 0.0;
    for (int q = 0; q < P.n_bonds; ++q) {
      const uint32_t m = s_mask[q];
      const uint32_t x = s & m;
      if (x == 0u || x == m) {
        diag += 0.25 * s_J[q];
      } else {
        diag -= 0.25 * s_J[q];
        const uint32_t c = word_rank(s ^ m, sb);
        if (c < (uint32_t)D) A[(int64_t)r * D + c] += 0.5 * s_J[q];
        else if (a.err) atomicOr(a.err, 2);
      }
    }
    A[(int64_t)r * D + r] += diag;
  }
}

// Householder step k, part 1 (one workgroup per active sector): the part of
// row k right of the diagonal, x, becomes alpha e_1 under I - 2 v v^T with
// v = (x - alpha e_1) / |x - alpha e_1|, alpha = -sign(x_0) |x|; d[k], e[k]
// are recorded.  A row that is already zero there keeps v = 0.
__global__ __launch_bounds__(kThreads) void ed_hh_vec_kernel(const EigArgs a, int k) {
  __shared__ double sh[4];
  const EigProb P = a.probs[blockIdx.x];
  const int D = P.dim, n2 = D - k - 1;
  if (k + 2 >= D) return;
  const double* x = a.mat + P.mat_off + (int64_t)k * D + (k + 1);
  double* v = a.hv + P.vec_off;
  double part = 0.0;
  for (int i = threadIdx.x; i < n2; i += kThreads) part = fma(x[i], x[i], part);
  const double sigma = ed_sum(part, sh);
  const double x0 = x[0];
  const double tail = sigma - x0 * x0;
  if (threadIdx.x == 0) a.hd[P.vec_off + k] = a.mat[P.mat_off + (int64_t)k * D + k];
  if (!(tail > 1e-300)) {
    if (threadIdx.x == 0) a.he[P.vec_off + k] = x0;
    for (int i = threadIdx.x; i < n2; i += kThreads) v[i] = 0.0;
    return;
  }
  const double alpha = -copysign(sqrt(sigma), x0);
  if (threadIdx.x == 0) a.he[P.vec_off + k] = alpha;
  const double v0 = x0 - alpha;
  const double inv = 1.0 / sqrt(tail + v0 * v0);
  for (int i = threadIdx.x; i < n2; i += kThreads) v[i] = (i == 0 ? v0 : x[i]) * inv;
}

// Part 2 (grid: active sectors x tiles of kEdRows rows): p = 2 A' v over the
// trailing block A' (rows and columns k+1..D-1); each wave takes rows of the
// tile, its lanes stride over the row.
__global__ __launch_bounds__(kThreads) void ed_hh_matvec_kernel(const EigArgs a, int k) {
  const EigProb P = a.probs[blockIdx.x];
  const int D = P.dim, n2 = D - k - 1;
  if (k + 2 >= D) return;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const double* v = a.hv + P.vec_off;
  double* pv = a.hp + P.vec_off;
  for (int rr = wv; rr < kEdRows; rr += kThreads / 64) {
    const int i = blockIdx.y * kEdRows + rr;
    if (i >= n2) break;
    const double* row = a.mat + P.mat_off + (int64_t)(k + 1 + i) * D + (k + 1);
    double acc = 0.0;
    for (int j = lane; j < n2; j += 64) acc = fma(row[j], v[j], acc);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
    if (lane == 0) pv[i] = 2.0 * acc;
  }
}

// Part 3 (same grid): K = v.p, w = p - K v, A' -= v w^T + w v^T on the tile's
// rows (every workgroup sums K in the same order).
__global__ __launch_bounds__(kThreads) void ed_hh_update_kernel(const EigArgs a, int k) {
  __shared__ double sh[4];
  const EigProb P = a.probs[blockIdx.x];
  const int D = P.dim, n2 = D - k - 1;
  if (k + 2 >= D) return;
  const double* v = a.hv + P.vec_off;
  const double* pv = a.hp + P.vec_off;
  double part = 0.0;
  for (int i = threadIdx.x; i < n2; i += kThreads) part = fma(v[i], pv[i], part);
  const double K = ed_sum(part, sh);
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int rr = wv; rr < kEdRows; rr += kThreads / 64) {
    const int i = blockIdx.y * kEdRows + rr;
    if (i >= n2) break;
    const double vi = v[i], wi = fma(-K, vi, pv[i]);
    double* row = a.mat + P.mat_off + (int64_t)(k + 1 + i) * D + (k + 1);
    for (int j = lane; j < n2; j += 64) {
      const double wj = fma(-K, v[j], pv[j]);
      row[j] = fma(-vi, wj, fma(-wi, v[j], row[j]));
    }
  }
}

// Number of eigenvalues below x of the symmetric tridiagonal matrix (d, e):
// the negative pivots of the LDL^T factorisation of T - x (Sturm sequence),
// a pivot of magnitude below pivmin taken as -pivmin.
// 1/q from the hardware estimate and two Newton steps, r <- r (2 - q r)
// (each squares the relative error; |q| >= pivmin keeps q normal): the
// quotient below then differs from a correctly rounded division by a few ulps,
// which moves no pivot's sign except at the rounding level that bounds the
// bisection anyway, at a fraction of the divide sequence's latency on this
// serial chain.
__device__ __forceinline__ double sturm_recip(double q) {
  double r = __builtin_amdgcn_rcp(q);
  r = fma(r, fma(-q, r, 1.0), r);
  return fma(r, fma(-q, r, 1.0), r);
}

__device__ __forceinline__ int sturm_count(const double* d, const double* e2, int n, double x, double pivmin) {
  int cnt = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  cnt += q < 0.0;
  for (int i = 1; i < n; ++i) {
    q = (d[i] - x) - e2[i - 1] * sturm_recip(q);
    if (fabs(q) < pivmin) q = -pivmin;
    cnt += q < 0.0;
  }
  return cnt;
}

// Last part, 1 (one workgroup per sector): the final 2 x 2 block, the
// squared off-diagonal, the Gershgorin interval and the pivot floor.
__global__ __launch_bounds__(kThreads) void ed_tri_kernel(const EigArgs a) {
  __shared__ double sh_lo[kThreads], sh_hi[kThreads], sh_e2[kThreads];
  const int tid = threadIdx.x;
  const EigProb P = a.probs[blockIdx.x];
  const int D = P.dim;
  double* d = a.hd + P.vec_off;
  double* e = a.he + P.vec_off;
  double* e2 = a.hp + P.vec_off;
  const double* A = a.mat + P.mat_off;
  if (tid == 0) {
    if (D >= 2) {
      d[D - 2] = A[(int64_t)(D - 2) * D + (D - 2)];
      d[D - 1] = A[(int64_t)(D - 1) * D + (D - 1)];
      e[D - 2] = A[(int64_t)(D - 1) * D + (D - 2)];
    } else {
      d[0] = A[0];
    }
    e[D - 1] = 0.0;
  }
  __syncthreads();
  double lo = INFINITY, hi = -INFINITY, m2 = 0.0;
  for (int i = tid; i < D; i += kThreads) {
    const double r = fabs(e[i]) + (i > 0 ? fabs(e[i - 1]) : 0.0);
    lo = fmin(lo, d[i] - r);
    hi = fmax(hi, d[i] + r);
    e2[i] = e[i] * e[i];
    m2 = fmax(m2, e2[i]);
  }
  sh_lo[tid] = lo;
  sh_hi[tid] = hi;
  sh_e2[tid] = m2;
  __syncthreads();
  for (int st = kThreads / 2; st > 0; st >>= 1) {
    if (tid < st) {
      sh_lo[tid] = fmin(sh_lo[tid], sh_lo[tid + st]);
      sh_hi[tid] = fmax(sh_hi[tid], sh_hi[tid + st]);
      sh_e2[tid] = fmax(sh_e2[tid], sh_e2[tid + st]);
    }
    __syncthreads();
  }
  if (tid == 0) {
    const double span = fmax(fabs(sh_lo[0]), fabs(sh_hi[0]));
    double* g = a.hv + P.vec_off;   // the Householder vectors are no longer needed
    g[0] = sh_lo[0] - 1e-14 * span - 1e-300;
    g[1] = sh_hi[0] + 1e-14 * span + 1e-300;
    g[2] = 1e-290 * fmax(1.0, sh_e2[0]);
    g[3] = span;
  }
}

// Last part, 2 (grid: sectors x tiles of 64 eigenvalue indices, one per
// thread): eigenvalue idx by bisection on the Sturm count from the Gershgorin
// interval, down to adjacent floating-point numbers or 1e-16 of the spectral
// radius; written in ascending order.
__global__ __launch_bounds__(64) void ed_bisect_kernel(const EigArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const EigProb P = a.probs[blockIdx.x];
  const int D = P.dim;
  if ((int)blockIdx.y * 64 >= D) return;
  double* d = reinterpret_cast<double*>(smem);
  double* e2 = d + a.max_dim;
  for (int i = threadIdx.x; i < D; i += 64) {
    d[i] = a.hd[P.vec_off + i];
    e2[i] = a.hp[P.vec_off + i];
  }
  const double* g = a.hv + P.vec_off;
  const double g_lo = g[0], g_hi = g[1], pivmin = g[2], span = g[3];
  __syncthreads();
  const int idx = blockIdx.y * 64 + threadIdx.x;
  if (idx >= D) return;
  double x0 = g_lo, x1 = g_hi;
  for (int it = 0; it < 256; ++it) {
    const double mid = 0.5 * (x0 + x1);
    // adjacent numbers, or a width at the rounding level of the matrix
    if (!(mid > x0 && mid < x1) || x1 - x0 <= 1e-16 * span) break;
    if (sturm_count(d, e2, D, mid, pivmin) > idx) x1 = mid;
    else x0 = mid;
  }
  a.evals[(int64_t)P.out_row * a.ld + idx] = 0.5 * (x0 + x1);
}

// The sectors are sorted by descending dimension, so the sectors still active
// at step k (D > k + 2) are a prefix.
hipError_t launch_sector_eig(const EigArgs& a, const int* dims, int n_sectors, size_t lds_build,
                             size_t lds_finish, hipStream_t st) {
  if (n_sectors == 0) return hipSuccess;
  hipLaunchKernelGGL(ed_build_kernel, dim3(n_sectors), dim3(kThreads), lds_build, st, a);
  int active = n_sectors;
  for (int k = 0; k + 2 < dims[0]; ++k) {
    while (active > 0 && dims[active - 1] <= k + 2) --active;
    const int n2 = dims[0] - k - 1;
    const dim3 grid(active, (n2 + kEdRows - 1) / kEdRows);
    hipLaunchKernelGGL(ed_hh_vec_kernel, dim3(active), dim3(kThreads), 0, st, a, k);
    hipLaunchKernelGGL(ed_hh_matvec_kernel, grid, dim3(kThreads), 0, st, a, k);
    hipLaunchKernelGGL(ed_hh_update_kernel, grid, dim3(kThreads), 0, st, a, k);
  }
  hipLaunchKernelGGL(ed_tri_kernel, dim3(n_sectors), dim3(kThreads), 0, st, a);
  hipLaunchKernelGGL(ed_bisect_kernel, dim3(n_sectors, (dims[0] + 63) / 64), dim3(64), lds_finish, st, a);
  return hipGetLastError();
}

// Thermodynamics at the points (T, h) of every cluster: a sector with an
// exact spectrum (ed_count > 0) contributes its eigenvalues with weight Nt
// each (the scale on which a dimension-D sector's gamma_k sum to Nt * D),
// the others their nodes and gamma_k as in thermo_field_kernel.  Mirror
// sectors, the shift by the lowest energy of the point and the centred
// second passes as there.
__global__ __launch_bounds__(kThreads) void thermo_hybrid_kernel(const ThermoArgs a) {
  __shared__ double sh[4];
  const int t = blockIdx.x, c = blockIdx.y;
  const int Nt = a.n_nodes;
  const int p0 = a.cl_start[c], p1 = a.cl_start[c + 1];
  const double beta = 1.0 / a.T[t];
  const double hf = a.h ? a.h[t] : 0.0;

  double emin = INFINITY, s0 = 0.0, s1 = 0.0, s2 = 0.0, ve = 0.0, vm = 0.0;
  double eref = 0.0, S0 = 0.0, Ebar = 0.0, Mbar = 0.0;
  for (int pass = 0; pass < 3; ++pass) {
    for (int qq = p0; qq < p1; ++qq) {
      const int p = a.cl_list[qq];
      const ThermoProb tp = a.tp[p];
      const int ned = a.ed_count[p];
      const int items = ned > 0 ? ned : Nt;
      const int nm = tp.weight > 1.0 ? 2 : 1;
      for (int i = threadIdx.x; i < items; i += kThreads) {
        double E, g;
        if (ned > 0) {
          E = a.evals[(int64_t)p * a.evals_ld + i];
          g = (double)Nt;
        } else {
          const double x = cos(M_PI * ((double)i + 0.5) / (double)Nt);
          E = a.ab[2 * p] * x + a.ab[2 * p + 1];
          g = a.gamma[(int64_t)p * Nt + i];
        }
        for (int j = 0; j < nm; ++j) {
          const double m = j == 0 ? tp.sz : -tp.sz;
          const double Et = E + hf * m;
          if (pass == 0) {
            emin = fmin(emin, Et);
          } else {
            const double wgt = g * exp(-beta * (Et - eref));
            if (pass == 1) {
              s0 += wgt;
              s1 = fma(wgt, Et, s1);
              s2 = fma(wgt, m, s2);
            } else {
              const double de = Et - Ebar, dm = m - Mbar;
              ve = fma(wgt, de * de, ve);
              vm = fma(wgt, dm * dm, vm);
            }
          }
        }
      }
    }
    if (pass == 0) {
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) emin = fmin(emin, __shfl_down(emin, off, 64));
      const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
      __syncthreads();
      if (lane == 0) sh[wv] = emin;
      __syncthreads();
      eref = fmin(fmin(sh[0], sh[1]), fmin(sh[2], sh[3]));
      __syncthreads();
    } else if (pass == 1) {
      S0 = ed_sum(s0, sh);
      Ebar = ed_sum(s1, sh) / S0;
      Mbar = ed_sum(s2, sh) / S0;
    }
  }
  const double VarE = ed_sum(ve, sh) / S0;
  const double VarM = ed_sum(vm, sh) / S0;
  if (threadIdx.x == 0) {
    const int64_t o = (int64_t)c * a.n_T + t;
    a.lnZ[o] = (S0 > 0.0 ? log(S0 / (double)Nt) : NAN) - beta * eref;
    a.E[o] = Ebar;
    a.C[o] = beta * beta * VarE;
    a.chi[o] = beta * VarM;
    if (a.mag) a.mag[o] = Mbar;
    if (a.znonpos) a.znonpos[o] = S0 > 0.0 ? 0 : 1;
  }
}

hipError_t launch_thermo_hybrid(const ThermoArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(thermo_hybrid_kernel, dim3(a.n_T, a.n_clusters), dim3(kThreads), 0, st, a);
  return hipGetLastError();
}

}  // namespace kpm
