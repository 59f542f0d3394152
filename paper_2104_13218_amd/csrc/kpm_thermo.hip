// Kernel damping, density-of-states weights and thermodynamics on the GPU
// (float64 throughout).
//
//  g_n      Jackson kernel, the paper's Eq. (8) with N_deg = M (the trailing
//           factor printed in Eq. (8) is a typesetting residue: with it the
//           coefficients would grow instead of damping).
//  gamma_k  weights of the Gauss-Chebyshev rule at x_k = cos(pi (k - 1/2)/Nt):
//           gamma_k = g_0 mu_0 + 2 sum_n g_n mu_n cos(n pi (k - 1/2)/Nt)
//           (Sec. II); the cosine argument is reduced exactly in integers,
//           n (2k - 1) mod 4 Nt, before scaling by pi / (2 Nt).
//  sums     per cluster and temperature, over its S^z sectors (weight 2 for
//           S^z > 0: the mirror sector, Sec. II) and the nodes, with Boltzmann
//           factors exp(-(E_k - E_ref)/T), E_k = a x_k + b, E_ref = the lowest
//           node energy of the cluster (no overflow; C, E, chi are shift
//           invariant, ln Z = ln(sum/Nt) - E_ref/T).  C is beta^2 times the
//           weighted variance of E taken about the mean (Eq. (2b)); chi is
//           beta <S_z^2> (Eq. (3); <S_z> vanishes by the mirror sectors).
// Each reduction is a fixed-order workgroup tree: results are reproducible.
#include <hip/hip_runtime.h>

#include <cmath>

#include "kpm_internal.h"

namespace kpm {

namespace {

__device__ __forceinline__ double wsum(double v, double* sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  const double r = ((sh[0] + sh[1]) + sh[2]) + sh[3];
  __syncthreads();
  return r;   // every thread gets the total
}

__device__ __forceinline__ double wmin(double v, double* sh) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fmin(v, __shfl_down(v, off, 64));
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) sh[w] = v;
  __syncthreads();
  const double r = fmin(fmin(sh[0], sh[1]), fmin(sh[2], sh[3]));
  __syncthreads();
  return r;
}

// cos(m pi / (2 Nt)) for the reduced argument m = n (2k - 1) mod 4 Nt.
__device__ __forceinline__ double reduced_cos(int64_t m, int64_t Nt) {
  return cos(M_PI * (double)m / (double)(2 * Nt));
}
// cos(n pi (k - 1/2) / Nt) for 1-based k, argument reduced exactly.
__device__ __forceinline__ double node_cos(int64_t n, int64_t k, int64_t Nt) {
  return reduced_cos((n * (2 * k - 1)) % (4 * Nt), Nt);
}

__device__ __forceinline__ double node_x(int64_t k, int64_t Nt) {
  return cos(M_PI * ((double)k - 0.5) / (double)Nt);
}

}  // namespace

__global__ __launch_bounds__(kThreads) void kernel_coef_kernel(int M, int kernel, double* g) {
  const int n = blockIdx.x * kThreads + threadIdx.x;
  if (n >= M) return;
  if (kernel == 0) {
    g[n] = 1.0;
    return;
  }
  const double q = M_PI / (double)(M + 1);
  g[n] = ((double)(M - n + 1) * cos(q * n) + sin(q * n) / tan(q)) / (double)(M + 1);
}

hipError_t launch_kernel_coef(int M, int kernel, double* g, hipStream_t st) {
  hipLaunchKernelGGL(kernel_coef_kernel, dim3((M + kThreads - 1) / kThreads), dim3(kThreads), 0, st,
                     M, kernel, g);
  return hipGetLastError();
}

// gamma[p][k-1], one wave per node.  Without damping the weights of the
// lowest nodes are small differences of large terms, so the sum is compensated
// (the Dot2 scheme of Ogita, Rump and Oishi, "Accurate sum and dot product",
// SIAM J. Sci. Comput. 26 (2005)): each product's rounding error from an fma,
// each addition's from TwoSum, carried in a second sum; lane l takes the terms
// n = l, l + 64, ... in order, then the lanes' (sum, error) pairs combine in a
// fixed butterfly (lane 0's order).  The reduced cosine argument
// m = n (2k - 1) mod 4 Nt advances by the reduced stride each term, exactly as
// the direct reduction gives it.
__device__ __forceinline__ void two_sum(double a, double b, double& s, double& e) {
#pragma clang fp contract(off)
  s = a + b;
  const double bb = s - a;
  e = (a - (s - bb)) + (b - bb);
}

__global__ __launch_bounds__(kThreads) void gamma_kernel(int M, int Nt, const double* g,
                                                         const double* mu, double* gamma) {
#pragma clang fp contract(off)
  const int p = blockIdx.y;
  const int lane = threadIdx.x & 63;
  const int k = blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6) + 1;
  if (k > Nt) return;   // k is the same across the wave
  const double* mp = mu + (int64_t)p * M;
  const int64_t period = 4 * (int64_t)Nt;
  const int64_t stride = (64 * (2 * (int64_t)k - 1)) % period;
  int64_t m = ((int64_t)lane * (2 * (int64_t)k - 1)) % period;
  double sum = 0.0, err = 0.0;
  for (int n = lane; n < M; n += 64) {
    const double cn = g[n] * mp[n] * (n == 0 ? 1.0 : 2.0);
    const double cv = reduced_cos(m, Nt);
    const double x = cn * cv;
    const double ex = fma(cn, cv, -x);
    double e;
    two_sum(sum, x, sum, e);
    err += e + ex;
    m += stride;
    if (m >= period) m -= period;
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const double s2 = __shfl_xor(sum, off, 64);
    const double e2 = __shfl_xor(err, off, 64);
    double e;
    two_sum(sum, s2, sum, e);
    err += e2 + e;
  }
  if (lane == 0) gamma[(int64_t)p * Nt + (k - 1)] = sum + err;
}

hipError_t launch_gamma(int n_probs, int M, int n_nodes, const double* g, const double* mu,
                        double* gamma, hipStream_t st) {
  constexpr int kNodesPerGroup = kThreads / 64;
  dim3 grid((n_nodes + kNodesPerGroup - 1) / kNodesPerGroup, n_probs);
  hipLaunchKernelGGL(gamma_kernel, grid, dim3(kThreads), 0, st, M, n_nodes, g, mu, gamma);
  return hipGetLastError();
}

// One workgroup per (temperature, cluster).
__global__ __launch_bounds__(kThreads) void thermo_kernel(const ThermoArgs a) {
  __shared__ double sh[4];
  const int t = blockIdx.x, c = blockIdx.y;
  const int Nt = a.n_nodes;
  const int p0 = a.cl_start[c], p1 = a.cl_start[c + 1];
  const int64_t items = (int64_t)(p1 - p0) * Nt;
  const double beta = 1.0 / a.T[t];

  double emin = INFINITY;
  for (int64_t i = threadIdx.x; i < items; i += kThreads) {
    const int p = a.cl_list[p0 + i / Nt];
    const int k = (int)(i % Nt) + 1;
    emin = fmin(emin, a.ab[2 * p] * node_x(k, Nt) + a.ab[2 * p + 1]);
  }
  const double eref = wmin(emin, sh);

  double s0 = 0.0, s1 = 0.0, sm = 0.0;
  for (int64_t i = threadIdx.x; i < items; i += kThreads) {
    const int p = a.cl_list[p0 + i / Nt];
    const int k = (int)(i % Nt) + 1;
    const double E = a.ab[2 * p] * node_x(k, Nt) + a.ab[2 * p + 1];
    const double w = a.tp[p].weight * a.gamma[(int64_t)p * Nt + (k - 1)] * exp(-beta * (E - eref));
    s0 += w;
    s1 = fma(w, E, s1);
    sm = fma(w, a.tp[p].sz * a.tp[p].sz, sm);
  }
  const double S0 = wsum(s0, sh);
  const double S1 = wsum(s1, sh);
  const double SM = wsum(sm, sh);
  const double Ebar = S1 / S0;

  double v = 0.0;
  for (int64_t i = threadIdx.x; i < items; i += kThreads) {
    const int p = a.cl_list[p0 + i / Nt];
    const int k = (int)(i % Nt) + 1;
    const double E = a.ab[2 * p] * node_x(k, Nt) + a.ab[2 * p + 1];
    const double w = a.tp[p].weight * a.gamma[(int64_t)p * Nt + (k - 1)] * exp(-beta * (E - eref));
    const double d = E - Ebar;
    v = fma(w, d * d, v);
  }
  const double Var = wsum(v, sh) / S0;

  if (threadIdx.x == 0) {
    const int64_t o = (int64_t)c * a.n_T + t;
    a.lnZ[o] = (S0 > 0.0 ? log(S0 / (double)Nt) : NAN) - beta * eref;
    a.E[o] = Ebar;
    a.C[o] = beta * beta * Var;
    a.chi[o] = beta * SM / S0;
    if (a.znonpos) a.znonpos[o] = S0 > 0.0 ? 0 : 1;
    if (a.stats) {
      double* st = a.stats + o * 6;
      st[0] = S0;
      st[1] = Ebar;
      st[2] = Var;
      st[3] = SM / S0;
      st[4] = eref;
      st[5] = beta;
    }
  }
}

hipError_t launch_thermo(const ThermoArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(thermo_kernel, dim3(a.n_T, a.n_clusters), dim3(kThreads), 0, st, a);
  return hipGetLastError();
}

// Thermodynamics with the Zeeman term h S^z (h = g mu_B B, per point): the
// sector S^z = m keeps its zero-field DOS and every energy moves by h m; a
// sector with S^z > 0 stands for m = +S^z and its mirror m = -S^z.  Sums as in
// thermo_kernel, shifted by the lowest node energy of the point; the energy
// and S^z variances are centred second passes.
__global__ __launch_bounds__(kThreads) void thermo_field_kernel(const ThermoArgs a) {
  __shared__ double sh[4];
  const int t = blockIdx.x, c = blockIdx.y;
  const int Nt = a.n_nodes;
  const int p0 = a.cl_start[c], p1 = a.cl_start[c + 1];
  const int64_t items = (int64_t)(p1 - p0) * Nt;
  const double beta = 1.0 / a.T[t];
  const double hf = a.h[t];

  double emin = INFINITY;
  for (int64_t i = threadIdx.x; i < items; i += kThreads) {
    const int p = a.cl_list[p0 + i / Nt];
    const int k = (int)(i % Nt) + 1;
    const double E = a.ab[2 * p] * node_x(k, Nt) + a.ab[2 * p + 1];
    const double sz = a.tp[p].sz;
    emin = fmin(emin, E + hf * sz);
    if (a.tp[p].weight > 1.0) emin = fmin(emin, E - hf * sz);
  }
  const double eref = wmin(emin, sh);

  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int64_t i = threadIdx.x; i < items; i += kThreads) {
    const int p = a.cl_list[p0 + i / Nt];
    const int k = (int)(i % Nt) + 1;
    const double E = a.ab[2 * p] * node_x(k, Nt) + a.ab[2 * p + 1];
    const double gk = a.gamma[(int64_t)p * Nt + (k - 1)];
    const double sz = a.tp[p].sz;
    const int nm = a.tp[p].weight > 1.0 ? 2 : 1;
    for (int j = 0; j < nm; ++j) {
      const double m = j == 0 ? sz : -sz;
      const double Et = E + hf * m;
      const double w = gk * exp(-beta * (Et - eref));
      s0 += w;
      s1 = fma(w, Et, s1);
      s2 = fma(w, m, s2);
    }
  }
  const double S0 = wsum(s0, sh);
  const double Ebar = wsum(s1, sh) / S0;
  const double Mbar = wsum(s2, sh) / S0;

  double ve = 0.0, vm = 0.0;
  for (int64_t i = threadIdx.x; i < items; i += kThreads) {
    const int p = a.cl_list[p0 + i / Nt];
    const int k = (int)(i % Nt) + 1;
    const double E = a.ab[2 * p] * node_x(k, Nt) + a.ab[2 * p + 1];
    const double gk = a.gamma[(int64_t)p * Nt + (k - 1)];
    const double sz = a.tp[p].sz;
    const int nm = a.tp[p].weight > 1.0 ? 2 : 1;
    for (int j = 0; j < nm; ++j) {
      const double m = j == 0 ? sz : -sz;
      const double Et = E + hf * m;
      const double w = gk * exp(-beta * (Et - eref));
      const double de = Et - Ebar, dm = m - Mbar;
      ve = fma(w, de * de, ve);
      vm = fma(w, dm * dm, vm);
    }
  }
  const double VarE = wsum(ve, sh) / S0;
  const double VarM = wsum(vm, sh) / S0;

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

hipError_t launch_thermo_field(const ThermoArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(thermo_field_kernel, dim3(a.n_T, a.n_clusters), dim3(kThreads), 0, st, a);
  return hipGetLastError();
}

// dL/dgamma at every node: for L = sum wC C + wchi chi,
//   dC/dgamma_k  = beta^2 W e_k ((E_k - Ebar)^2 - Var) / S0,
//   dchi/dgamma_k = beta W e_k (m^2 - <m^2>) / S0,   e_k = exp(-beta (E_k - E_ref)).
__global__ __launch_bounds__(kThreads) void node_adj_kernel(const ThermoVjpArgs a) {
  const int p = blockIdx.y;
  const int k = blockIdx.x * kThreads + threadIdx.x + 1;
  if (k > a.n_nodes) return;
  const ThermoProb P = a.tp[p];
  const double E = a.ab[2 * p] * node_x(k, a.n_nodes) + a.ab[2 * p + 1];
  const double m2 = P.sz * P.sz;
  double acc = 0.0;
  for (int t = 0; t < a.n_T; ++t) {
    const int64_t o = (int64_t)P.cluster * a.n_T + t;
    const double* st = a.stats + o * 6;
    const double S0 = st[0], Ebar = st[1], Var = st[2], m2bar = st[3], eref = st[4], beta = st[5];
    const double e = P.weight * exp(-beta * (E - eref)) / S0;
    const double d = E - Ebar;
    acc += a.wC[o] * beta * beta * e * (d * d - Var) + a.wchi[o] * beta * e * (m2 - m2bar);
  }
  a.node_adj[(int64_t)p * a.n_nodes + (k - 1)] = acc;
}

// lambda_n = g_n (2 - delta_n0) sum_k node_adj_k cos(n pi (k - 1/2)/Nt).
__global__ __launch_bounds__(kThreads) void lambda_kernel(const ThermoVjpArgs a) {
  __shared__ double ns[kThreads];
  const int p = blockIdx.y;
  const int n = blockIdx.x * kThreads + threadIdx.x;
  double acc = 0.0;
  for (int k0 = 1; k0 <= a.n_nodes; k0 += kThreads) {
    const int k = k0 + threadIdx.x;
    __syncthreads();
    ns[threadIdx.x] = k <= a.n_nodes ? a.node_adj[(int64_t)p * a.n_nodes + (k - 1)] : 0.0;
    __syncthreads();
    if (n < a.M) {
      const int lim = min(kThreads, a.n_nodes - k0 + 1);
      for (int j = 0; j < lim; ++j) acc = fma(ns[j], node_cos(n, k0 + j, a.n_nodes), acc);
    }
  }
  if (n < a.M) a.lambda[(int64_t)p * a.M + n] = a.g[n] * (n == 0 ? 1.0 : 2.0) * acc;
}

hipError_t launch_thermo_vjp(const ThermoVjpArgs& a, hipStream_t st) {
  dim3 g1((a.n_nodes + kThreads - 1) / kThreads, a.n_probs);
  hipLaunchKernelGGL(node_adj_kernel, g1, dim3(kThreads), 0, st, a);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  dim3 g2((a.M + kThreads - 1) / kThreads, a.n_probs);
  hipLaunchKernelGGL(lambda_kernel, g2, dim3(kThreads), 0, st, a);
  return hipGetLastError();
}

}  // namespace kpm
