// Reverse-mode derivative of the Chebyshev moments with respect to the bond
// couplings J_b, with the rescaling (a, b) of the paper's Eq. (5) held fixed.
//
// With alpha_n = <v_n, v_n>, beta_n = <v_{n+1}, v_n> (the doubling-identity
// dots) and abar_n, bbar_n the loss derivatives with respect to them, the
// adjoint vectors of v_{n+1} = 2 H' v_n - v_{n-1} (v_1 = H' v_0) obey
//   w_n = gbar_n + 2 H' w_{n+1} - w_{n+2},   w_{K+1} = w_{K+2} = 0,
//   gbar_n = 2 abar_n v_n + bbar_n v_{n+1} + bbar_{n-1} v_{n-1},
// and since dH'/dJ_b = h_b / a (h_b = s_i . s_j),
//   dL/dJ_b = (1/a) [ <w_1, h_b v_0> + 2 sum_{n=1}^{K-1} <w_{n+1}, h_b v_n> ].
// One launch per n computes w_n and adds that step's bond dots: the gathers of
// w_{n+1} that form H' w_{n+1} also give <w_{n+1}, h_b v_n>, because per row
//   (h_b w)_rho . v_rho = (+-1/4) w_rho . v_rho + (1/2)[bits differ] w_nb . v_rho.
// Bond dots are summed over a tile's rows through LDS in a fixed order and
// accumulated per tile across launches: the result is reproducible.
#include <hip/hip_runtime.h>

#include "kpm_device.h"
#include "kpm_internal.h"

namespace kpm {

// abar, bbar for every real column from lambda = dL/dmu, through the
// estimator (mu = dim/R sum_r <r|T_n|r>/<r|r>) and the doubling identities.
__global__ __launch_bounds__(kThreads) void doubling_vjp_kernel(const DoublingVjpArgs a) {
  const int col = blockIdx.x * kThreads + threadIdx.x;
  if (col >= a.total_cols) return;
  const UnitDev U = a.units[a.job_unit[2 * col]];
  const ProbDev P = a.probs[U.prob];
  const int c = col - U.col_off;
  const int K = a.K;
  const int64_t TC = a.total_cols;
  for (int n = 0; n <= K; ++n) a.abar[n * TC + col] = 0.0;
  for (int n = 0; n < K; ++n) a.bbar[n * TC + col] = 0.0;
  if (c >= U.ncols) return;
  double norm = a.alpha0[col];
  if (a.cols_per_vec == 2) {
    const int c0 = c & ~1;
    norm = a.alpha0[U.col_off + c0] + a.alpha0[U.col_off + c0 + 1];
  }
  const double Reff = a.R > 0 ? (double)a.R : (double)P.dim;
  const double scale = (double)P.dim / (Reff * norm);
  const double* lam = a.lambda + (int64_t)U.prob * a.M;
  double a0 = 0.0, b0 = 0.0;
  for (int n = 0; n < a.M; ++n) {
    const double l = lam[n] * scale;
    const int h = n >> 1;
    if (n == 0) {
      a0 += l;
    } else if (n == 1) {
      b0 += l;
    } else if ((n & 1) == 0) {
      a.abar[h * TC + col] += 2.0 * l;
      a0 -= l;
    } else {
      a.bbar[h * TC + col] += 2.0 * l;
      b0 -= l;
    }
  }
  a.abar[col] += a0;
  a.bbar[col] += b0;
}

hipError_t launch_doubling_vjp(const DoublingVjpArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(doubling_vjp_kernel, dim3((a.total_cols + kThreads - 1) / kThreads),
                     dim3(kThreads), 0, st, a);
  return hipGetLastError();
}

// One reverse step (or, with dots_only, the final <w_1, h_b v_0> pass).
// Q = LD / CPT consecutive threads share a basis state, each with CPT of its
// block's LD columns (row dots are summed across the Q lanes); a sub-tile has
// sub_rows states and the workgroup sub_rows * Q threads.
template <typename T, int LD>
__global__ __launch_bounds__(kThreads) void adjoint_kernel(const AdjArgs a) {
  constexpr int CPT = LD < kAdjCpt ? LD : kAdjCpt;
  constexpr int Q = LD / CPT;
  extern __shared__ __align__(16) unsigned char smem[];
  const int nthr = blockDim.x;
  int tile = blockIdx.x;
  if (a.xcd_remap) tile = (blockIdx.x & 7) * (a.grid_tiles >> 3) + (blockIdx.x >> 3);
  if (tile >= a.n_tiles) return;
  const UnitDev U = a.units[a.tile_unit[tile]];
  const ProbDev P = a.probs[U.prob];
  const int nb = P.n_bonds;
  const int SR = a.sub_rows;

  size_t o = 0;
  auto take = [&](size_t bytes) {
    unsigned char* p = smem + o;
    o = (o + bytes + 15) & ~size_t(15);
    return p;
  };
  uint32_t* s_binom = reinterpret_cast<uint32_t*>(take(kBinomN * kBinomN * 4));
  uint32_t* s_tab = reinterpret_cast<uint32_t*>(take((size_t)a.lds_tab * 4));
  uint32_t* s_mask = reinterpret_cast<uint32_t*>(take((size_t)a.lds_bonds * 4));
  double* s_off = reinterpret_cast<double*>(take((size_t)a.lds_bonds * 8));
  double* s_zz = reinterpret_cast<double*>(take((size_t)a.lds_bonds * 8));
  double* s_contrib = reinterpret_cast<double*>(take((size_t)SR * a.lds_bonds * 8));

  for (int i = threadIdx.x; i < kBinomN * kBinomN; i += nthr) s_binom[i] = a.binom[i];
  for (int i = threadIdx.x; i < P.tab_len; i += nthr) s_tab[i] = a.tables[P.tab_off + i];
  for (int i = threadIdx.x; i < nb; i += nthr) {
    s_mask[i] = a.bmask[P.bond_off + i];
    s_off[i] = a.boff[P.bond_off + i];
    s_zz[i] = a.bzz[P.bond_off + i];
  }
  __syncthreads();
  const RankTables RT = make_tables(s_tab, P);

  const int64_t S = a.slot_stride;
  const T* vb = reinterpret_cast<const T*>(a.vseg) + U.vec_off;
  T* wb = reinterpret_cast<T*>(a.wbuf) + U.vec_off;
  const T* Wx = wb + a.wx_slot * S;
  T* Wy = wb + a.wy_slot * S;
  const T* Vn = vb + a.v0_slot * S;
  const T* Vm1 = a.vm1_slot >= 0 ? vb + a.vm1_slot * S : nullptr;
  const T* Vp1 = a.vp1_slot >= 0 ? vb + a.vp1_slot * S : nullptr;
  const int co = U.col_off;

  double bacc = 0.0;   // thread b < nb: this tile's sum for bond b
  const int64_t tile_row0 = a.tile_row0[tile];
  const int tile_rows = a.tile_nrows[tile];
  const int t = threadIdx.x;
  const int rr = t / Q, cq = t - rr * Q;   // state of the sub-tile, column group
  const int c0 = cq * CPT;
  for (int st = 0; st * SR < tile_rows; ++st) {
    const int64_t row0 = tile_row0 + (int64_t)st * SR;
    const int nrows = min(SR, tile_rows - st * SR);
    if (rr < nrows) {
      const int64_t rho = row0 + rr;
      const uint32_t s = unrank((uint32_t)rho, P.n_sites, P.n_up, s_binom);
      double w[CPT], v[CPT], acc[CPT];
#pragma unroll
      for (int c = 0; c < CPT; ++c) {
        w[c] = (double)Wx[rho * LD + c0 + c];
        v[c] = (double)Vn[rho * LD + c0 + c];
      }
      // <w, v> of the state over all LD columns (the Q lanes of a state are
      // consecutive and take the same branches)
      double self = 0.0;
#pragma unroll
      for (int c = 0; c < CPT; ++c) self = fma(w[c], v[c], self);
#pragma unroll
      for (int off = 1; off < Q; off <<= 1) self += __shfl_xor(self, off, 64);
      double dg = P.shift;
      for (int b = 0; b < nb; ++b) {
        const uint32_t m = s_mask[b];
        const uint32_t x = s & m;
        const bool differ = !(x == 0u || x == m);
        dg += differ ? -s_zz[b] : s_zz[b];
        if (cq == 0) s_contrib[rr * nb + b] = differ ? -0.25 * self : 0.25 * self;
      }
#pragma unroll
      for (int c = 0; c < CPT; ++c) acc[c] = dg * w[c];
      for (int b = 0; b < nb; ++b) {
        const uint32_t m = s_mask[b];
        const uint32_t x = s & m;
        if (x == 0u || x == m) continue;
        uint32_t r = RT.rank(s ^ m);
        if (r >= (uint32_t)P.dim) {
          if (a.err) atomicOr(a.err, 2);
          r = (uint32_t)rho;
        }
        const T* g = Wx + (int64_t)r * LD + c0;
        const double cf = s_off[b];
        double pk = 0.0;
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
          const double gv = (double)g[c];
          acc[c] = fma(cf, gv, acc[c]);
          pk = fma(gv, v[c], pk);
        }
#pragma unroll
        for (int off = 1; off < Q; off <<= 1) pk += __shfl_xor(pk, off, 64);
        if (cq == 0) s_contrib[rr * nb + b] += 0.5 * pk;
      }
      if (!a.dots_only) {
#pragma unroll
        for (int c = 0; c < CPT; ++c) {
          const int col = c0 + c;
          double g = 2.0 * a.abar_n[co + col] * v[c];
          if (Vp1) g = fma(a.bbar_n[co + col], (double)Vp1[rho * LD + col], g);
          if (Vm1) g = fma(a.bbar_nm1[co + col], (double)Vm1[rho * LD + col], g);
          const double wn = g + 2.0 * acc[c] - (double)Wy[rho * LD + col];
          Wy[rho * LD + col] = (T)wn;
        }
      }
    }
    __syncthreads();
    for (int b = t; b < nb; b += nthr) {
      double sum = 0.0;
      for (int r = 0; r < nrows; ++r) sum += s_contrib[r * nb + b];
      if (b == t) bacc += sum;
    }
    __syncthreads();
  }
  if (threadIdx.x < nb) {
    double* dst = a.part_bd + U.bd_off + (int64_t)(tile - U.tile0) * nb + threadIdx.x;
    *dst = a.accumulate ? *dst + a.coef * bacc : a.coef * bacc;
  }
}

size_t adjoint_lds_bytes(const DevicePlan& p) {
  auto a16 = [](size_t x) { return (x + 15) & ~size_t(15); };
  size_t o = 0;
  o = a16(o + kBinomN * kBinomN * 4);
  o = a16(o + (size_t)p.lds_tab * 4);
  o = a16(o + (size_t)p.lds_bonds * 4);
  o = a16(o + (size_t)p.lds_bonds * 8);
  o = a16(o + (size_t)p.lds_bonds * 8);
  o = a16(o + (size_t)p.sub_rows * p.lds_bonds * 8);
  return o;
}

template <typename T, int LD>
static hipError_t launch_adj_t(const AdjArgs& a, size_t lds, int grid, int threads,
                               hipStream_t st) {
  hipLaunchKernelGGL((adjoint_kernel<T, LD>), dim3(grid), dim3(threads), lds, st, a);
  return hipGetLastError();
}

hipError_t launch_adjoint(const DevicePlan& p, AdjArgs a, int ld, hipStream_t st) {
  a.probs = p.probs;
  a.units = p.units;
  a.tile_unit = p.tile_unit;
  a.tile_row0 = p.tile_row0;
  a.tile_nrows = p.tile_nrows;
  a.tables = p.tables;
  a.bmask = p.bmask;
  a.boff = p.boff;
  a.bzz = p.bzz;
  a.binom = p.binom;
  a.n_tiles = p.n_tiles;
  a.grid_tiles = p.grid_tiles;
  a.sub_rows = p.sub_rows;
  a.sub_per_tile = p.sub_per_tile;
  a.lds_tab = p.lds_tab;
  a.lds_bonds = p.lds_bonds;
  a.xcd_remap = p.xcd_remap;
  a.slot_stride = p.slot_stride;
  a.err = p.err;
  // Q threads per state (adjoint_kernel); every bond needs a thread for the
  // per-tile reduction
  const int thr = p.sub_rows * adjoint_lanes(ld);
  if (p.lds_bonds > thr || thr > kThreads) return hipErrorInvalidValue;
  const size_t lds = adjoint_lds_bytes(p);
  const int grid = p.grid_tiles;
#define KPM_ADJ_CASE(L)                                                         \
  case L:                                                                       \
    return p.fp32 ? launch_adj_t<float, L>(a, lds, grid, thr, st)               \
                  : launch_adj_t<double, L>(a, lds, grid, thr, st);
  switch (ld) {
    KPM_ADJ_CASE(1)
    KPM_ADJ_CASE(2)
    KPM_ADJ_CASE(4)
    KPM_ADJ_CASE(8)
    KPM_ADJ_CASE(16)
    default: return hipErrorInvalidValue;
  }
#undef KPM_ADJ_CASE
}

// dL/dJ_b for every (problem, bond): sum over the problem's blocks and tiles
// in a fixed order, times 1/a.  One workgroup per (problem, bond).
__global__ __launch_bounds__(kThreads) void bond_reduce_kernel(const BondReduceArgs a) {
  __shared__ double sh[kThreads];
  const int job = blockIdx.x;
  // problem of this bond: last p with bond_off <= job
  int lo = 0, hi = a.n_probs - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (a.probs[mid].bond_off <= job) lo = mid;
    else hi = mid - 1;
  }
  const ProbDev P = a.probs[lo];
  const int b = job - P.bond_off;
  double acc = 0.0;
  for (int u = a.prob_unit0[lo]; u < a.prob_unit0[lo + 1]; ++u) {
    const UnitDev U = a.units[u];
    for (int t = threadIdx.x; t < U.ntiles; t += kThreads) acc += a.part_bd[U.bd_off + (int64_t)t * P.n_bonds + b];
  }
  sh[threadIdx.x] = acc;
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    __syncthreads();
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
  }
  if (threadIdx.x == 0) a.dJ[job] = sh[0] * P.inv_a;
}

hipError_t launch_bond_reduce(const BondReduceArgs& a, int total_bonds, hipStream_t st) {
  if (total_bonds <= 0) return hipSuccess;
  hipLaunchKernelGGL(bond_reduce_kernel, dim3(total_bonds), dim3(kThreads), 0, st, a);
  return hipGetLastError();
}

// Per-cluster sums of per-problem bond derivatives: workgroup row c = cluster,
// one thread per bond; problems added in their order.  info: per problem
// (cluster, offset of its bonds in dJ); cinfo: per cluster (output offset,
// bond count).
__global__ __launch_bounds__(kThreads) void cluster_grad_kernel(const int32_t* info, int n,
                                                               const int32_t* cinfo, const double* dJ,
                                                               double* out) {
  const int c = blockIdx.y;
  const int b = blockIdx.x * kThreads + threadIdx.x;
  if (b >= cinfo[2 * c + 1]) return;
  double s = 0.0;
  for (int q = 0; q < n; ++q)
    if (info[2 * q] == c) s += dJ[info[2 * q + 1] + b];
  out[cinfo[2 * c] + b] = s;
}

hipError_t launch_cluster_grad(const int32_t* info, int n, const int32_t* cinfo, int n_clusters,
                               int max_bonds, const double* dJ, double* out, hipStream_t st) {
  if (n_clusters <= 0 || max_bonds <= 0) return hipSuccess;
  hipLaunchKernelGGL(cluster_grad_kernel, dim3((max_bonds + kThreads - 1) / kThreads, n_clusters),
                     dim3(kThreads), 0, st, info, n, cinfo, dJ, out);
  return hipGetLastError();
}

// L = sum_{c,T} wC C + wchi chi (one workgroup, fixed-order tree).
__global__ __launch_bounds__(kThreads) void loss_kernel(const double* C, const double* chi,
                                                        const double* wC, const double* wchi,
                                                        int n, double* L) {
  __shared__ double sh[kThreads];
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += kThreads) acc += wC[i] * C[i] + wchi[i] * chi[i];
  sh[threadIdx.x] = acc;
  for (int s = kThreads / 2; s > 0; s >>= 1) {
    __syncthreads();
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
  }
  if (threadIdx.x == 0) *L = sh[0];
}

hipError_t launch_loss(const double* C, const double* chi, const double* wC, const double* wchi,
                       int n, double* L, hipStream_t st) {
  hipLaunchKernelGGL(loss_kernel, dim3(1), dim3(kThreads), 0, st, C, chi, wC, wchi, n, L);
  return hipGetLastError();
}

}  // namespace kpm
