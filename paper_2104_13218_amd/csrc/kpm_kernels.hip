// gfx950 kernels of the Chebyshev-moment library.
//
// Hot path: one launch per recursion step v_{n+1} = 2 H' v_n - v_{n-1}
// (v_1 = H' v_0) over every (problem, column block) of the run, with
// H' = (H - b)/a applied matrix-free in the S^z-sector bit basis (paper,
// Eqs. (4)-(6) and the sector decomposition of Sec. II).  Each workgroup owns
// a tile of consecutive basis states of one block:
//   phase 1  one thread per state: unrank the state, walk the bonds, and stage
//            in LDS the neighbour ranks (combinatorial-number-system rank via
//            three table lookups) and the diagonal element;
//   phase 2  threads own (state, 4- or 2-column chunk) pairs: coalesced 16-byte
//            loads of the state's own rows, 16-byte gathers of neighbour rows,
//            float64 accumulation, one streaming store of v_{n+1} over v_{n-1};
//   dots     <v_{n+1}, v_{n+1}> and <v_{n+1}, v_n> per column, accumulated in
//            float64 from the stored values and reduced in a fixed order
//            (workgroup tree, then per-tile partials that the *next* step's
//            launch sums), so results are bitwise reproducible.
// No MFMA: the operator is a sparse gather, bound by HBM traffic.
#include <hip/hip_runtime.h>

#include <cmath>

#include "kpm_device.h"
#include "kpm_internal.h"
#include "kpm_vec.h"

namespace kpm {

// LDS carve-up shared by the step kernel and the matrix export.
struct StepSmem {
  uint32_t* binom;
  uint32_t* tab;
  uint32_t* mask;
  double* off;
  double* zz;
  double* diag;
  int32_t* cnt;
  uint32_t* nbr;
  uint16_t* nbb;
  double* red;
};

__device__ __forceinline__ size_t al16(size_t x) { return (x + 15) & ~size_t(15); }

__device__ __forceinline__ StepSmem carve(unsigned char* smem, int lds_tab, int lds_bonds,
                                          int sub_rows, int lds_nb) {
  StepSmem S;
  size_t o = 0;
  S.binom = reinterpret_cast<uint32_t*>(smem + o); o = al16(o + kBinomN * kBinomN * 4);
  S.tab = reinterpret_cast<uint32_t*>(smem + o);   o = al16(o + size_t(lds_tab) * 4);
  S.mask = reinterpret_cast<uint32_t*>(smem + o);  o = al16(o + size_t(lds_bonds) * 4);
  S.off = reinterpret_cast<double*>(smem + o);     o = al16(o + size_t(lds_bonds) * 8);
  S.zz = reinterpret_cast<double*>(smem + o);      o = al16(o + size_t(lds_bonds) * 8);
  S.diag = reinterpret_cast<double*>(smem + o);    o = al16(o + size_t(sub_rows) * 8);
  S.cnt = reinterpret_cast<int32_t*>(smem + o);    o = al16(o + size_t(sub_rows) * 4);
  S.red = reinterpret_cast<double*>(smem + o);     // aliases the lists after phase 2
  S.nbr = reinterpret_cast<uint32_t*>(smem + o);   o = al16(o + size_t(lds_nb) * sub_rows * 4);
  S.nbb = reinterpret_cast<uint16_t*>(smem + o);
  return S;
}

// Phase 1 for one row: unrank, walk bonds, stage neighbour ranks and diag.
// A neighbour rank outside the sector (impossible for consistent tables) is
// replaced by the row itself and reported through *err, so no gather can
// leave the vector.
// With dense = true, entry b of the row belongs to bond b (kNoNeighbour when
// its bits are equal), so lanes of consecutive rows gather for the same bond.
constexpr uint32_t kNoNeighbour = 0xFFFFFFFFu;

__device__ __forceinline__ void stage_row(uint32_t rank, const ProbDev& P, const RankTables& RT,
                                          const StepSmem& S, int slot, int stride, int* err,
                                          bool dense = false) {
  const uint32_t s = unrank(rank, P.n_sites, P.n_up, S.binom);
  double d = P.shift;
  int cnt = 0;
  for (int b = 0; b < P.n_bonds; ++b) {
    const uint32_t m = S.mask[b];
    const uint32_t v = s & m;
    if (v == 0u || v == m) {
      d += S.zz[b];
      if (dense) S.nbr[b * stride + slot] = kNoNeighbour;
    } else if (dense) {
      d -= S.zz[b];
      uint32_t nr = RT.rank(s ^ m);
      if (nr >= (uint32_t)P.dim) {
        if (err) atomicOr(err, 2);
        nr = rank;
      }
      S.nbr[b * stride + slot] = nr;
    } else {
      d -= S.zz[b];
      uint32_t nr = RT.rank(s ^ m);
      if (nr >= (uint32_t)P.dim) {
        if (err) atomicOr(err, 2);
        nr = rank;
      }
      S.nbr[cnt * stride + slot] = nr;
      S.nbb[cnt * stride + slot] = (uint16_t)b;
      ++cnt;
    }
  }
  S.diag[slot] = d;
  S.cnt[slot] = dense ? P.n_bonds : cnt;
}

__device__ __forceinline__ void load_problem_lds(const StepSmem& S, const ProbDev& P,
                                                 const uint32_t* tables, const uint32_t* bmask,
                                                 const double* boff, const double* bzz,
                                                 const uint32_t* binom) {
  for (int i = threadIdx.x; i < kBinomN * kBinomN; i += kThreads) S.binom[i] = binom[i];
  for (int i = threadIdx.x; i < P.tab_len; i += kThreads) S.tab[i] = tables[P.tab_off + i];
  for (int i = threadIdx.x; i < P.n_bonds; i += kThreads) {
    S.mask[i] = bmask[P.bond_off + i];
    S.off[i] = boff[P.bond_off + i];
    S.zz[i] = bzz[P.bond_off + i];
  }
}

// ------------------------------------------------------------ step kernel

template <typename T, int CPL, int GB>
__global__ __launch_bounds__(kThreads) void step_kernel(const StepArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x;

  // Reduce the previous step's per-tile partial dots: alpha_s, beta_{s-1}.
  if (a.n_jobs > 0) {
    const int64_t s = (a.step_base ? *a.step_base : 0) + a.step_add;
    double* sh = reinterpret_cast<double*>(smem);
    for (int job = blockIdx.x; job < a.n_jobs; job += gridDim.x) {
      const UnitDev U = a.units[a.job_unit[job]];
      const int v = job - 2 * U.col_off;
      const double sum = sum_partials(a.part_in + U.part_off + (int64_t)v * U.ntiles, U.ntiles, sh);
      if (tid == 0) {
        if (v < U.ld) a.alpha[s * a.total_cols + U.col_off + v] = sum;
        else a.beta[(s - 1) * a.total_cols + U.col_off + (v - U.ld)] = sum;
      }
    }
    __syncthreads();
  }

  const int tile = a.xcd_remap ? xcd_tile(blockIdx.x, a.grid_tiles) : (int)blockIdx.x;
  if (tile >= a.n_tiles) return;
  const UnitDev U = a.units[a.tile_unit[tile]];
  const ProbDev P = a.probs[U.prob];
  const StepSmem S = carve(smem, a.lds_tab, a.lds_bonds, a.sub_rows, a.lds_nb);
  load_problem_lds(S, P, a.tables, a.bmask, a.boff, a.bzz, a.binom);
  __syncthreads();
  const RankTables RT = make_tables(S.tab, P);

  const int ld = U.ld;
  const int nch = ld / CPL;
  const int nrg = kThreads / nch;
  const int c = tid % nch;
  const int rg = tid / nch;
  T* base = reinterpret_cast<T*>(a.vec) + U.vec_off;
  const T* X = base + a.x_slot * a.slot_stride;
  const T* Yin = base + a.yin_slot * a.slot_stride;
  T* Y = base + a.yout_slot * a.slot_stride;

  double acc_a[CPL], acc_b[CPL];
#pragma unroll
  for (int i = 0; i < CPL; ++i) acc_a[i] = acc_b[i] = 0.0;

  const int64_t tile_row0 = a.tile_row0[tile];
  const int tile_rows = a.tile_nrows[tile];
  for (int st = 0; st * a.sub_rows < tile_rows; ++st) {
    const int64_t row0 = tile_row0 + (int64_t)st * a.sub_rows;
    const int nrows = min(a.sub_rows, tile_rows - st * a.sub_rows);
    for (int r = tid; r < nrows; r += kThreads)
      stage_row((uint32_t)(row0 + r), P, RT, S, r, a.sub_rows, a.err, a.dense);
    __syncthreads();
    if (rg < nrg) {
      for (int r = rg; r < nrows; r += nrg) {
        const int64_t rho = row0 + r;
        const VecT<T, CPL> xv = vload<T, CPL>(X + rho * ld + c * CPL);
        const double dg = S.diag[r];
        double acc[CPL];
#pragma unroll
        for (int i = 0; i < CPL; ++i) acc[i] = dg * (double)xv.v[i];
        const int cnt = S.cnt[r];
        T* ys = Y + rho * ld + c * CPL;
        VecT<T, CPL> yv;
        if (!a.first) yv = vload_nt<T, CPL>(Yin + rho * ld + c * CPL);
        // gathers issued GB at a time (absent entries read the row
        // itself with a zero coefficient), then accumulated in order
        for (int k0 = 0; k0 < cnt; k0 += GB) {
          VecT<T, CPL> nv[GB];
          double cf[GB];
#pragma unroll
          for (int j = 0; j < GB; ++j) {
            const int k = k0 + j;
            uint32_t nb = k < cnt ? S.nbr[k * a.sub_rows + r] : kNoNeighbour;
            bool on = nb != kNoNeighbour;
            if (a.dense) {
              cf[j] = on ? S.off[k] : 0.0;
            } else {
              cf[j] = on ? S.off[S.nbb[k * a.sub_rows + r]] : 0.0;
            }
            if (!on) nb = (uint32_t)rho;
            nv[j] = vload<T, CPL>(X + (int64_t)nb * ld + c * CPL);
          }
#pragma unroll
          for (int j = 0; j < GB; ++j) {
#pragma unroll
            for (int i = 0; i < CPL; ++i) acc[i] = fma(cf[j], (double)nv[j].v[i], acc[i]);
          }
        }
        VecT<T, CPL> ov;
        if (a.first) {
#pragma unroll
          for (int i = 0; i < CPL; ++i) ov.v[i] = (T)acc[i];
        } else {
#pragma unroll
          for (int i = 0; i < CPL; ++i) ov.v[i] = (T)(2.0 * acc[i] - (double)yv.v[i]);
        }
        vstore_nt<T, CPL>(ys, ov);
#pragma unroll
        for (int i = 0; i < CPL; ++i) {
          const double o = (double)ov.v[i];
          acc_a[i] = fma(o, o, acc_a[i]);
          acc_b[i] = fma(o, (double)xv.v[i], acc_b[i]);
        }
      }
    }
    __syncthreads();
  }

  // Workgroup reduction over row groups, per column (fixed tree).
  double* red = S.red;
  if (rg < nrg) {
#pragma unroll
    for (int i = 0; i < CPL; ++i) {
      red[(2 * i) * kThreads + tid] = acc_a[i];
      red[(2 * i + 1) * kThreads + tid] = acc_b[i];
    }
  }
  int p2 = 1;
  while (p2 < nrg) p2 <<= 1;
  for (int sstride = p2 >> 1; sstride > 0; sstride >>= 1) {
    __syncthreads();
    if (rg < sstride && rg + sstride < nrg) {
#pragma unroll
      for (int v = 0; v < 2 * CPL; ++v) red[v * kThreads + tid] += red[v * kThreads + tid + sstride * nch];
    }
  }
  __syncthreads();
  if (tid < nch) {
    const int tl = tile - U.tile0;
#pragma unroll
    for (int i = 0; i < CPL; ++i) {
      const int col = c * CPL + i;
      a.part_out[U.part_off + (int64_t)col * U.ntiles + tl] = red[(2 * i) * kThreads + tid];
      a.part_out[U.part_off + (int64_t)(ld + col) * U.ntiles + tl] = red[(2 * i + 1) * kThreads + tid];
    }
  }
}

// ------------------------------------------------------------ spin kernel
//
// Spin-s sites (the spin-5/2 Fe10 wheel of the paper, Sec. III.B): a state is
// the digit string d_i = s + m_i, its rank the count of sector states of
// smaller value sum_i d_i (2s+1)^i, read off the table P[i][r][d] site by
// site from the most significant one.  Once per call spin_lists_kernel
// unranks every row and stores its digit string and the ranks of its
// neighbours S^+_i S^-_j and S^-_i S^+_j (slot 2b + w) in the state table.
// Per step and sub-tile one thread per row reads them, sums the diagonal
// sum_b J_b m_i m_j / a - b/a and lists the acting neighbours with their
// amplitudes J_b/(2a) sqrt(s(s+1) - m(m+1)) sqrt(s(s+1) - m'(m'-1)) in LDS;
// the (row, column chunk) items then gather as in step_kernel.

struct SpinSmem {
  uint32_t* sites;   // per bond: i | j << 8
  double* off;       // per bond: J_b / (2a)
  double* zz;        // per bond: J_b / (4a)
  double* up;        // [2s + 1]: sqrt(s(s+1) - m(m+1)), m = d - s
  double* diag;
  int32_t* cnt;
  uint32_t* nbr;
  double* nbc;
  double* red;
};

__host__ __device__ inline size_t spin_lds_layout(int lds_bonds, int sub_rows, int lds_nb, int cpl,
                                                  size_t* offs) {
  size_t o = 0;
  auto put = [&](size_t b) {
    const size_t r = o;
    o = (o + b + 15) & ~size_t(15);
    return r;
  };
  offs[0] = 0;
  offs[1] = put(size_t(lds_bonds) * 4);
  offs[2] = put(size_t(lds_bonds) * 8);
  offs[3] = put(size_t(lds_bonds) * 8);
  offs[4] = put(16 * 8);
  offs[5] = put(size_t(sub_rows) * 8);
  offs[6] = put(size_t(sub_rows) * 4);
  offs[7] = o;   // reduction buffer aliases the lists after the last sub-tile
  offs[8] = put(size_t(lds_nb) * sub_rows * 4);
  offs[9] = put(size_t(lds_nb) * sub_rows * 8);
  const size_t red_end = offs[7] + size_t(2 * cpl) * kThreads * 8;
  return o > red_end ? o : red_end;
}

size_t spin_lds_bytes(const DevicePlan& p) {
  size_t offs[10];
  return spin_lds_layout(p.lds_bonds, p.sub_rows, p.lds_nb, p.cpl, offs);
}

template <typename T, int CPL, int GB>
__global__ __launch_bounds__(kThreads) void spin_kernel(const StepArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x;

  if (a.n_jobs > 0) {
    const int64_t s = (a.step_base ? *a.step_base : 0) + a.step_add;
    double* sh = reinterpret_cast<double*>(smem);
    for (int job = blockIdx.x; job < a.n_jobs; job += gridDim.x) {
      const UnitDev U = a.units[a.job_unit[job]];
      const int v = job - 2 * U.col_off;
      const double sum = sum_partials(a.part_in + U.part_off + (int64_t)v * U.ntiles, U.ntiles, sh);
      if (tid == 0) {
        if (v < U.ld) a.alpha[s * a.total_cols + U.col_off + v] = sum;
        else a.beta[(s - 1) * a.total_cols + U.col_off + (v - U.ld)] = sum;
      }
    }
    __syncthreads();
  }

  const int tile = a.xcd_remap ? xcd_tile(blockIdx.x, a.grid_tiles) : (int)blockIdx.x;
  if (tile >= a.n_tiles) return;
  const UnitDev U = a.units[a.tile_unit[tile]];
  const ProbDev P = a.probs[U.prob];
  size_t offs[10];
  spin_lds_layout(a.lds_bonds, a.sub_rows, a.lds_nb, CPL, offs);
  SpinSmem S;
  S.sites = reinterpret_cast<uint32_t*>(smem + offs[1]);
  S.off = reinterpret_cast<double*>(smem + offs[2]);
  S.zz = reinterpret_cast<double*>(smem + offs[3]);
  S.up = reinterpret_cast<double*>(smem + offs[4]);
  S.diag = reinterpret_cast<double*>(smem + offs[5]);
  S.cnt = reinterpret_cast<int32_t*>(smem + offs[6]);
  S.red = reinterpret_cast<double*>(smem + offs[7]);
  S.nbr = reinterpret_cast<uint32_t*>(smem + offs[8]);
  S.nbc = reinterpret_cast<double*>(smem + offs[9]);
  const int two_s = P.two_s, B = two_s + 1;
  const double sv = 0.5 * two_s;
  const uint64_t* sdig = reinterpret_cast<const uint64_t*>(a.states) + P.state_off;
  const uint32_t* snbr = a.states + 2 * a.spin_rows + P.state_off * a.lds_nb;
  for (int i = tid; i < P.n_bonds; i += kThreads) {
    S.sites[i] = a.bmask[P.bond_off + i];
    S.off[i] = a.boff[P.bond_off + i];
    S.zz[i] = a.bzz[P.bond_off + i];
  }
  if (tid < B) {
    const double m = tid - sv;
    S.up[tid] = sqrt(fmax(sv * (sv + 1.0) - m * (m + 1.0), 0.0));
  }
  __syncthreads();

  const int ld = U.ld;
  const int nch = ld / CPL;
  const int nrg = kThreads / nch;
  const int c = tid % nch;
  const int rg = tid / nch;
  T* base = reinterpret_cast<T*>(a.vec) + U.vec_off;
  const T* X = base + a.x_slot * a.slot_stride;
  const T* Yin = base + a.yin_slot * a.slot_stride;
  T* Y = base + a.yout_slot * a.slot_stride;
  double acc_a[CPL], acc_b[CPL];
#pragma unroll
  for (int i = 0; i < CPL; ++i) acc_a[i] = acc_b[i] = 0.0;

  const int64_t tile_row0 = a.tile_row0[tile];
  const int tile_rows = a.tile_nrows[tile];
  for (int st = 0; st * a.sub_rows < tile_rows; ++st) {
    const int64_t row0 = tile_row0 + (int64_t)st * a.sub_rows;
    const int nrows = min(a.sub_rows, tile_rows - st * a.sub_rows);
    for (int rr = tid; rr < nrows; rr += kThreads) {
      const int64_t rho = row0 + rr;
      const uint64_t dg = sdig[rho];
      double diag = P.shift;
      int cnt = 0;
      for (int b = 0; b < P.n_bonds; ++b) {
        const int i = (int)(S.sites[b] & 0xFFu), j = (int)(S.sites[b] >> 8);
        const int di = (int)((dg >> (4 * i)) & 15u), dj = (int)((dg >> (4 * j)) & 15u);
        diag = fma(4.0 * S.zz[b], (di - sv) * (dj - sv), diag);
        // S^+_i S^-_j, then S^-_i S^+_j
        for (int w = 0; w < 2; ++w) {
          const int d1 = w == 0 ? di : dj, d2 = w == 0 ? dj : di;
          if (d1 >= two_s || d2 <= 0) continue;
          const uint32_t nr = snbr[(int64_t)(2 * b + w) * P.dim + rho];
          if (nr >= (uint32_t)P.dim || cnt >= a.lds_nb) {
            if (a.err) atomicOr(a.err, 2);
            continue;
          }
          S.nbr[cnt * a.sub_rows + rr] = nr;
          S.nbc[cnt * a.sub_rows + rr] = S.off[b] * S.up[d1] * S.up[d2 - 1];
          ++cnt;
        }
      }
      S.diag[rr] = diag;
      S.cnt[rr] = cnt;
    }
    __syncthreads();
    if (rg < nrg) {
      for (int rr = rg; rr < nrows; rr += nrg) {
        const int64_t rho = row0 + rr;
        const VecT<T, CPL> xv = vload<T, CPL>(X + rho * ld + c * CPL);
        const double dgn = S.diag[rr];
        double acc[CPL];
#pragma unroll
        for (int i = 0; i < CPL; ++i) acc[i] = dgn * (double)xv.v[i];
        const int cnt = S.cnt[rr];
        for (int k0 = 0; k0 < cnt; k0 += GB) {
          VecT<T, CPL> nv[GB];
          double cf[GB];
#pragma unroll
          for (int j = 0; j < GB; ++j) {
            const int k = k0 + j;
            const bool on = k < cnt;
            const uint32_t nb = on ? S.nbr[k * a.sub_rows + rr] : (uint32_t)rho;
            cf[j] = on ? S.nbc[k * a.sub_rows + rr] : 0.0;
            nv[j] = vload<T, CPL>(X + (int64_t)nb * ld + c * CPL);
          }
#pragma unroll
          for (int j = 0; j < GB; ++j) {
#pragma unroll
            for (int i = 0; i < CPL; ++i) acc[i] = fma(cf[j], (double)nv[j].v[i], acc[i]);
          }
        }
        VecT<T, CPL> ov;
        if (a.first) {
#pragma unroll
          for (int i = 0; i < CPL; ++i) ov.v[i] = (T)acc[i];
        } else {
          const VecT<T, CPL> yv = vload_nt<T, CPL>(Yin + rho * ld + c * CPL);
#pragma unroll
          for (int i = 0; i < CPL; ++i) ov.v[i] = (T)(2.0 * acc[i] - (double)yv.v[i]);
        }
        vstore_nt<T, CPL>(Y + rho * ld + c * CPL, ov);
#pragma unroll
        for (int i = 0; i < CPL; ++i) {
          const double o = (double)ov.v[i];
          acc_a[i] = fma(o, o, acc_a[i]);
          acc_b[i] = fma(o, (double)xv.v[i], acc_b[i]);
        }
      }
    }
    __syncthreads();
  }

  double* red = S.red;
  if (rg < nrg) {
#pragma unroll
    for (int i = 0; i < CPL; ++i) {
      red[(2 * i) * kThreads + tid] = acc_a[i];
      red[(2 * i + 1) * kThreads + tid] = acc_b[i];
    }
  }
  int p2 = 1;
  while (p2 < nrg) p2 <<= 1;
  for (int sstride = p2 >> 1; sstride > 0; sstride >>= 1) {
    __syncthreads();
    if (rg < sstride && rg + sstride < nrg) {
#pragma unroll
      for (int v = 0; v < 2 * CPL; ++v) red[v * kThreads + tid] += red[v * kThreads + tid + sstride * nch];
    }
  }
  __syncthreads();
  if (tid < nch) {
    const int tl = tile - U.tile0;
#pragma unroll
    for (int i = 0; i < CPL; ++i) {
      const int col = c * CPL + i;
      a.part_out[U.part_off + (int64_t)col * U.ntiles + tl] = red[(2 * i) * kThreads + tid];
      a.part_out[U.part_off + (int64_t)(ld + col) * U.ntiles + tl] = red[(2 * i + 1) * kThreads + tid];
    }
  }
}

// Digit strings and neighbour ranks of every row of every spin-s problem
// (grid: x strides over rows, y = problem); the rank table in LDS.
__global__ __launch_bounds__(kThreads) void spin_lists_kernel(const ProbDev* probs,
                                                              const uint32_t* tables,
                                                              const uint32_t* bmask, uint32_t* states,
                                                              int64_t spin_rows, int nb, int* err) {
  extern __shared__ __align__(16) unsigned char smem[];
  uint32_t* tab = reinterpret_cast<uint32_t*>(smem);
  const ProbDev P = probs[blockIdx.y];
  for (int i = threadIdx.x; i < P.tab_len; i += kThreads) tab[i] = tables[P.tab_off + i];
  __syncthreads();
  const int N = P.n_sites, two_s = P.two_s, B = two_s + 1, R1 = two_s * N + 1;
  uint64_t* dig = reinterpret_cast<uint64_t*>(states) + P.state_off;
  uint32_t* nbr = states + 2 * spin_rows + P.state_off * nb;
  for (int64_t rho = (int64_t)blockIdx.x * kThreads + threadIdx.x; rho < P.dim;
       rho += (int64_t)gridDim.x * kThreads) {
    // unrank: at each site, the largest digit whose table entry does not
    // exceed what is left of the rank
    uint64_t dg = 0;
    uint32_t rem = (uint32_t)rho;
    int r = P.n_up;
    for (int i = N - 1; i >= 0; --i) {
      int d = min(two_s, r);
      while (d > 0 && tab[(i * R1 + r) * B + d] > rem) --d;
      rem -= tab[(i * R1 + r) * B + d];
      dg |= (uint64_t)d << (4 * i);
      r -= d;
    }
    if ((rem != 0u || r != 0) && err) atomicOr(err, 4);
    dig[rho] = dg;
    for (int b = 0; b < P.n_bonds; ++b) {
      const uint32_t sij = bmask[P.bond_off + b];
      const int i = (int)(sij & 0xFFu), j = (int)(sij >> 8);
      const int di = (int)((dg >> (4 * i)) & 15u), dj = (int)((dg >> (4 * j)) & 15u);
      for (int w = 0; w < 2; ++w) {
        const int a1 = w == 0 ? i : j, a2 = w == 0 ? j : i;
        const int d1 = w == 0 ? di : dj, d2 = w == 0 ? dj : di;
        uint32_t nr = (uint32_t)rho;
        if (d1 < two_s && d2 > 0)
          nr = spin_rank(dg + ((uint64_t)1 << (4 * a1)) - ((uint64_t)1 << (4 * a2)), N, P.n_up, R1, B, tab);
        nbr[(int64_t)(2 * b + w) * P.dim + rho] = nr;
      }
    }
  }
}

static hipError_t build_spin_lists(const DevicePlan& p, hipStream_t st) {
  const size_t lds = (size_t)p.lds_tab * 4;
  hipLaunchKernelGGL(spin_lists_kernel, dim3(1024, p.n_probs), dim3(kThreads), lds, st, p.probs, p.tables,
                     p.bmask, p.states, p.spin_rows, p.lds_nb, p.err);
  return hipGetLastError();
}

template <typename T, int CPL>
static hipError_t launch_spin_t(const StepArgs& a, size_t lds, int grid, hipStream_t st) {
  hipLaunchKernelGGL((spin_kernel<T, CPL, 4>), dim3(grid), dim3(kThreads), lds, st, a);
  return hipGetLastError();
}

static hipError_t launch_spin(const DevicePlan& p, const StepArgs& a, hipStream_t st) {
  const size_t lds = spin_lds_bytes(p);
  const int grid = p.grid_tiles;
  if (p.fp32) {
    switch (p.cpl) {
      case 1: return launch_spin_t<float, 1>(a, lds, grid, st);
      case 2: return launch_spin_t<float, 2>(a, lds, grid, st);
      case 4: return launch_spin_t<float, 4>(a, lds, grid, st);
      default: return hipErrorInvalidValue;
    }
  }
  switch (p.cpl) {
    case 1: return launch_spin_t<double, 1>(a, lds, grid, st);
    case 2: return launch_spin_t<double, 2>(a, lds, grid, st);
    default: return hipErrorInvalidValue;
  }
}

// ------------------------------------------------------------- row kernel
//
// One lane per basis state carrying all LD columns of its block.  The state's
// bits come from the sector's state table; diagonal, active bonds and
// neighbour ranks are computed in registers (bond order, as in step_kernel);
// NB neighbour rows are in flight at a time.  The output row is staged in LDS
// and the column dots are then summed exactly as step_kernel sums them, so
// both kernels give bitwise identical moments.

template <typename T, int LD>
struct RowChunk {
  static constexpr int CH = sizeof(T) == 4 ? (LD % 4 == 0 ? 4 : (LD % 2 == 0 ? 2 : 1))
                                           : (LD % 2 == 0 ? 2 : 1);
};

template <typename T, int LD>
__device__ __forceinline__ void load_row(const T* p, T (&r)[LD]) {
  constexpr int V = sizeof(T) == 4 ? (LD % 4 == 0 ? 4 : (LD % 2 == 0 ? 2 : 1)) : (LD % 2 == 0 ? 2 : 1);
#pragma unroll
  for (int c = 0; c < LD; c += V) {
    const VecT<T, V> v = vload<T, V>(p + c);
#pragma unroll
    for (int i = 0; i < V; ++i) r[c + i] = v.v[i];
  }
}

template <typename T, int LD, int CW, int NB>
__global__ __launch_bounds__(kThreads) void row_kernel(const StepArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x;
  if (a.n_jobs > 0) {
    const int64_t s = (a.step_base ? *a.step_base : 0) + a.step_add;
    double* sh = reinterpret_cast<double*>(smem);
    for (int job = blockIdx.x; job < a.n_jobs; job += gridDim.x) {
      const UnitDev U = a.units[a.job_unit[job]];
      const int v = job - 2 * U.col_off;
      const double sum = sum_partials(a.part_in + U.part_off + (int64_t)v * U.ntiles, U.ntiles, sh);
      if (tid == 0) {
        if (v < U.ld) a.alpha[s * a.total_cols + U.col_off + v] = sum;
        else a.beta[(s - 1) * a.total_cols + U.col_off + (v - U.ld)] = sum;
      }
    }
    __syncthreads();
  }
  const int tile = a.xcd_remap ? xcd_tile(blockIdx.x, a.grid_tiles) : (int)blockIdx.x;
  if (tile >= a.n_tiles) return;
  const UnitDev U = a.units[a.tile_unit[tile]];
  const ProbDev P = a.probs[U.prob];
  constexpr int CH = RowChunk<T, LD>::CH;

  size_t o = 0;
  auto take = [&](size_t bytes) {
    unsigned char* q = smem + o;
    o = (o + bytes + 15) & ~size_t(15);
    return q;
  };
  uint32_t* s_tab = reinterpret_cast<uint32_t*>(take((size_t)a.lds_tab * 4));
  uint32_t* s_mask = reinterpret_cast<uint32_t*>(take((size_t)a.lds_bonds * 4));
  double* s_off = reinterpret_cast<double*>(take((size_t)a.lds_bonds * 8));
  double* s_zz = reinterpret_cast<double*>(take((size_t)a.lds_bonds * 8));
  unsigned char* tail = smem + o;
  T* s_out = reinterpret_cast<T*>(tail);              // [kThreads][LD]
  double* s_red = reinterpret_cast<double*>(tail);    // reused after the last sub-tile

  for (int i = tid; i < P.tab_len; i += kThreads) s_tab[i] = a.tables[P.tab_off + i];
  for (int i = tid; i < P.n_bonds; i += kThreads) {
    s_mask[i] = a.bmask[P.bond_off + i];
    s_off[i] = a.boff[P.bond_off + i];
    s_zz[i] = a.bzz[P.bond_off + i];
  }
  __syncthreads();
  const RankTables RT = make_tables(s_tab, P);
  const int nb = P.n_bonds;

  T* base = reinterpret_cast<T*>(a.vec) + U.vec_off;
  const T* X = base + a.x_slot * a.slot_stride;
  const T* Yin = base + a.yin_slot * a.slot_stride;
  T* Y = base + a.yout_slot * a.slot_stride;
  const uint32_t* states = a.states + P.state_off;

  const int nch = LD / CH;
  const int nrg = kThreads / nch;
  const int c = tid % nch;
  const int rg = tid / nch;
  double acc_a[CH], acc_b[CH];
#pragma unroll
  for (int i = 0; i < CH; ++i) acc_a[i] = acc_b[i] = 0.0;

  const int64_t tile_row0 = a.tile_row0[tile];
  const int tile_rows = a.tile_nrows[tile];
  for (int st = 0; st * kThreads < tile_rows; ++st) {
    const int64_t row0 = tile_row0 + (int64_t)st * kThreads;
    const int nrows = min(kThreads, tile_rows - st * kThreads);
    if (tid < nrows) {
      const int64_t rho = row0 + tid;
      const uint32_t s = states[rho];
      double dg = P.shift;
      for (int b = 0; b < nb; ++b) {
        const uint32_t m = s_mask[b];
        const uint32_t v = s & m;
        dg += (v == 0u || v == m) ? s_zz[b] : -s_zz[b];
      }
      // (CW = LD: one window; a narrower window re-gathers every neighbour row
      // per window and measured slower)
      constexpr int V = sizeof(T) == 4 ? (CW % 4 == 0 ? 4 : (CW % 2 == 0 ? 2 : 1)) : (CW % 2 == 0 ? 2 : 1);
#pragma unroll 1
      for (int c0 = 0; c0 < LD; c0 += CW) {
        double acc[CW];
        {
          T xr[CW];
          load_row<T, CW>(X + rho * LD + c0, xr);
#pragma unroll
          for (int i = 0; i < CW; ++i) acc[i] = dg * (double)xr[i];
        }
        for (int b0 = 0; b0 < nb; b0 += 64) {
          const int lim = min(64, nb - b0);
          uint64_t act = 0;
          for (int j = 0; j < lim; ++j) {
            const uint32_t m = s_mask[b0 + j];
            const uint32_t v = s & m;
            if (!(v == 0u || v == m)) act |= 1ull << j;
          }
          while (act) {
            int bb[NB];
            uint32_t rr[NB];
            double cf[NB];
#pragma unroll
            for (int q = 0; q < NB; ++q) {
              if (act) {
                const int j = __ffsll((unsigned long long)act) - 1;
                act &= act - 1;
                bb[q] = b0 + j;
                uint32_t r = RT.rank(s ^ s_mask[b0 + j]);
                if (r >= (uint32_t)P.dim) {
                  if (a.err) atomicOr(a.err, 2);
                  r = (uint32_t)rho;
                }
                rr[q] = r;
                cf[q] = s_off[b0 + j];
              } else {
                bb[q] = -1;
                rr[q] = (uint32_t)rho;
                cf[q] = 0.0;
              }
            }
            T g[NB][CW];
#pragma unroll
            for (int q = 0; q < NB; ++q) load_row<T, CW>(X + (int64_t)rr[q] * LD + c0, g[q]);
#pragma unroll
            for (int q = 0; q < NB; ++q) {
              if (bb[q] >= 0) {
#pragma unroll
                for (int i = 0; i < CW; ++i) acc[i] = fma(cf[q], (double)g[q][i], acc[i]);
              }
            }
          }
        }
#pragma unroll
        for (int i0 = 0; i0 < CW; i0 += V) {
          VecT<T, V> ov;
          if (a.first) {
#pragma unroll
            for (int i = 0; i < V; ++i) ov.v[i] = (T)acc[i0 + i];
          } else {
            const VecT<T, V> yv = vload_nt<T, V>(Yin + rho * LD + c0 + i0);
#pragma unroll
            for (int i = 0; i < V; ++i) ov.v[i] = (T)(2.0 * acc[i0 + i] - (double)yv.v[i]);
          }
          vstore_nt<T, V>(Y + rho * LD + c0 + i0, ov);
          vstore<T, V>(s_out + tid * LD + c0 + i0, ov);
        }
      }
    }
    __syncthreads();
    if (rg < nrg) {
      for (int r = rg; r < nrows; r += nrg) {
        const VecT<T, CH> ov = vload<T, CH>(s_out + r * LD + c * CH);
        const VecT<T, CH> xv = vload<T, CH>(X + (row0 + r) * LD + c * CH);
#pragma unroll
        for (int i = 0; i < CH; ++i) {
          const double od = (double)ov.v[i];
          acc_a[i] = fma(od, od, acc_a[i]);
          acc_b[i] = fma(od, (double)xv.v[i], acc_b[i]);
        }
      }
    }
    __syncthreads();
  }

  if (rg < nrg) {
#pragma unroll
    for (int i = 0; i < CH; ++i) {
      s_red[(2 * i) * kThreads + tid] = acc_a[i];
      s_red[(2 * i + 1) * kThreads + tid] = acc_b[i];
    }
  }
  int p2 = 1;
  while (p2 < nrg) p2 <<= 1;
  for (int sstride = p2 >> 1; sstride > 0; sstride >>= 1) {
    __syncthreads();
    if (rg < sstride && rg + sstride < nrg) {
#pragma unroll
      for (int v = 0; v < 2 * CH; ++v) s_red[v * kThreads + tid] += s_red[v * kThreads + tid + sstride * nch];
    }
  }
  __syncthreads();
  if (tid < nch) {
    const int tl = tile - U.tile0;
#pragma unroll
    for (int i = 0; i < CH; ++i) {
      const int col = c * CH + i;
      a.part_out[U.part_off + (int64_t)col * U.ntiles + tl] = s_red[(2 * i) * kThreads + tid];
      a.part_out[U.part_off + (int64_t)(LD + col) * U.ntiles + tl] = s_red[(2 * i + 1) * kThreads + tid];
    }
  }
}

size_t row_lds_bytes(const DevicePlan& p) {
  auto a16 = [](size_t x) { return (x + 15) & ~size_t(15); };
  size_t o = 0;
  o = a16(o + (size_t)p.lds_tab * 4);
  o = a16(o + (size_t)p.lds_bonds * 4);
  o = a16(o + (size_t)p.lds_bonds * 8);
  o = a16(o + (size_t)p.lds_bonds * 8);
  const size_t elt = p.fp32 ? 4 : 8;
  const size_t outs = (size_t)kThreads * p.row_ld * elt;
  const size_t red = (size_t)2 * 4 * kThreads * 8;
  return a16(o + (outs > red ? outs : red));
}

template <typename T, int LD, int CW, int NB>
static hipError_t launch_row_t(const StepArgs& a, size_t lds, int grid, hipStream_t st) {
  hipLaunchKernelGGL((row_kernel<T, LD, CW, NB>), dim3(grid), dim3(kThreads), lds, st, a);
  return hipGetLastError();
}

static hipError_t launch_row(const DevicePlan& p, const StepArgs& a, hipStream_t st) {
  const size_t lds = row_lds_bytes(p);
  const int grid = p.grid_tiles;
#define KPM_ROW(L, NBB)                                                                   \
  if (p.row_ld == L && p.gather_batch == NBB)                                             \
    return p.fp32 ? launch_row_t<float, L, L, NBB>(a, lds, grid, st)                      \
                  : launch_row_t<double, L, L, NBB>(a, lds, grid, st);
#define KPM_ROW3(L) KPM_ROW(L, 2) KPM_ROW(L, 4) KPM_ROW(L, 8)
  KPM_ROW3(1)
  KPM_ROW3(2)
  KPM_ROW3(4)
  KPM_ROW3(8)
#undef KPM_ROW3
#undef KPM_ROW
  return hipErrorInvalidValue;
}

// ----------------------------------------------------------- block kernel
//
// States sharing their high bits h = s >> L form a block of consecutive ranks.
// A member's index inside its block is the colex rank of its low bits l among
// the L-bit words with popc(l) set bits, and the block starts at the rank of
// (h << L) | (2^popc(l) - 1).  Tiles hold whole blocks (host packing).
//   low-low bond    the neighbour lies in the same block: read from the tile's
//                   LDS copy of v_n;
//   high-high bond  block h maps onto block h ^ m with the same low bits, so a
//                   block's rows gather one contiguous run of rows;
//   mixed bond      rank through the tables and a scattered gather.
// Per element the sum runs diagonal, low-low, high-high, mixed (each in bond
// order); the column dots are summed as in step_kernel.

struct BlockLds {
  size_t tab, mask, off, zz, lrank, row_l, row_b0, row_blk, mx_cnt, diag, wcnt, blk_h, hh_n, hh_row,
      hh_q, xs, mx_rank, mx_q, total;
};

__host__ __device__ inline BlockLds block_lds_layout(int lds_tab, int lds_bonds, int lds_lr,
                                                     int blk_max, int lds_hh, int lds_mx,
                                                     int rows, int ld_max, int elt, int cpl) {
  BlockLds L{};
  size_t o = 0;
  auto put = [&](size_t b) {
    const size_t r = o;
    o = (o + b + 15) & ~size_t(15);
    return r;
  };
  L.tab = put(size_t(lds_tab) * 4);
  L.mask = put(size_t(lds_bonds) * 4);
  L.off = put(size_t(lds_bonds) * 8);
  L.zz = put(size_t(lds_bonds) * 8);
  L.lrank = put(size_t(lds_lr) * 2);
  L.row_l = put(size_t(rows) * 2);
  L.row_b0 = put(size_t(rows) * 2);
  L.row_blk = put(size_t(rows));
  L.mx_cnt = put(size_t(rows) * 2);
  L.diag = put(size_t(rows) * 8);
  L.wcnt = put(4 * 4);
  L.blk_h = put(size_t(blk_max) * 4);
  L.hh_n = put(size_t(blk_max) * 4);
  L.hh_row = put(size_t(blk_max) * lds_hh * 4);
  L.hh_q = put(size_t(blk_max) * lds_hh * 2);
  L.xs = put(size_t(rows) * ld_max * elt);
  L.mx_rank = put(size_t(lds_mx) * rows * 4);
  L.mx_q = put(size_t(lds_mx) * rows * 2);
  const size_t red = L.xs + size_t(2 * cpl) * kThreads * 8;
  L.total = o > red ? o : red;
  return L;
}

size_t block_lds_bytes(const DevicePlan& p) {
  return block_lds_layout(p.lds_tab, p.lds_bonds, p.lds_lr, p.blk_max, p.lds_hh, p.lds_mx,
                          p.blk_rows, p.ld_max, p.fp32 ? 4 : 8, p.cpl)
      .total;
}


// One workgroup walks the sub-tiles [tile_sub0[t], tile_sub0[t + 1]) of its
// tile; each sub-tile is a run of whole blocks of at most blk_rows states.
template <typename T, int CPL, int GB>
__global__ __launch_bounds__(kThreads) void block_kernel(const StepArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x;

  if (a.n_jobs > 0) {
    const int64_t s = (a.step_base ? *a.step_base : 0) + a.step_add;
    double* sh = reinterpret_cast<double*>(smem);
    for (int job = blockIdx.x; job < a.n_jobs; job += gridDim.x) {
      const UnitDev U = a.units[a.job_unit[job]];
      const int v = job - 2 * U.col_off;
      const double sum = sum_partials(a.part_in + U.part_off + (int64_t)v * U.ntiles, U.ntiles, sh);
      if (tid == 0) {
        if (v < U.ld) a.alpha[s * a.total_cols + U.col_off + v] = sum;
        else a.beta[(s - 1) * a.total_cols + U.col_off + (v - U.ld)] = sum;
      }
    }
    __syncthreads();
  }

  const int tile = a.xcd_remap ? xcd_tile(blockIdx.x, a.grid_tiles) : (int)blockIdx.x;
  if (tile >= a.n_tiles) return;
  const UnitDev U = a.units[a.tile_unit[tile]];
  const ProbDev P = a.probs[U.prob];
  const int RC = a.blk_rows;
  const BlockLds Lo = block_lds_layout(a.lds_tab, a.lds_bonds, a.lds_lr, a.blk_max, a.lds_hh,
                                       a.lds_mx, RC, a.ld_max, (int)sizeof(T), CPL);
  uint32_t* s_tab = reinterpret_cast<uint32_t*>(smem + Lo.tab);
  uint32_t* s_mask = reinterpret_cast<uint32_t*>(smem + Lo.mask);
  double* s_off = reinterpret_cast<double*>(smem + Lo.off);
  double* s_zz = reinterpret_cast<double*>(smem + Lo.zz);
  uint16_t* s_lrank = reinterpret_cast<uint16_t*>(smem + Lo.lrank);
  uint16_t* s_row_l = reinterpret_cast<uint16_t*>(smem + Lo.row_l);
  uint16_t* s_row_b0 = reinterpret_cast<uint16_t*>(smem + Lo.row_b0);
  uint8_t* s_row_blk = reinterpret_cast<uint8_t*>(smem + Lo.row_blk);
  uint16_t* s_mx_cnt = reinterpret_cast<uint16_t*>(smem + Lo.mx_cnt);
  double* s_diag = reinterpret_cast<double*>(smem + Lo.diag);
  int32_t* s_wcnt = reinterpret_cast<int32_t*>(smem + Lo.wcnt);
  uint32_t* s_blk_h = reinterpret_cast<uint32_t*>(smem + Lo.blk_h);
  int32_t* s_hh_n = reinterpret_cast<int32_t*>(smem + Lo.hh_n);
  uint32_t* s_hh_row = reinterpret_cast<uint32_t*>(smem + Lo.hh_row);
  uint16_t* s_hh_q = reinterpret_cast<uint16_t*>(smem + Lo.hh_q);
  T* xs = reinterpret_cast<T*>(smem + Lo.xs);
  uint32_t* s_mx_rank = reinterpret_cast<uint32_t*>(smem + Lo.mx_rank);
  uint16_t* s_mx_q = reinterpret_cast<uint16_t*>(smem + Lo.mx_q);

  const int nb = P.n_bonds, nll = P.n_ll, nhh = P.n_hh;
  const int Lb = P.blk_L;
  for (int i = tid; i < P.tab_len; i += kThreads) s_tab[i] = a.tables[P.tab_off + i];
  for (int q = tid; q < nb; q += kThreads) {
    const int b = P.bond_off + a.bperm[P.bond_off + q];
    s_mask[q] = a.bmask[b];
    s_off[q] = a.boff[b];
    s_zz[q] = a.bzz[b];
  }
  // colex rank of a low word among the words of its popcount (independent of L)
  for (int l = tid; l < (1 << Lb); l += kThreads) s_lrank[l] = a.lrank[l];
  __syncthreads();
  const RankTables RT = make_tables(s_tab, P);

  const int ld = U.ld;
  T* base = reinterpret_cast<T*>(a.vec) + U.vec_off;
  const T* X = base + a.x_slot * a.slot_stride;
  const T* Yin = base + a.yin_slot * a.slot_stride;
  T* Y = base + a.yout_slot * a.slot_stride;
  const uint32_t lmask = (1u << Lb) - 1u;
  const int nch = ld / CPL;
  const int nrg = kThreads / nch;
  const int c = tid % nch;
  const int rg = tid / nch;
  const int lane = tid & 63, wv = tid >> 6;
  double acc_a[CPL], acc_b[CPL];
#pragma unroll
  for (int i = 0; i < CPL; ++i) acc_a[i] = acc_b[i] = 0.0;

  int64_t row0 = a.tile_row0[tile];
  const int sub1 = a.tile_sub0[tile + 1];
  for (int sub = a.tile_sub0[tile]; sub < sub1; ++sub) {
    const int nrows = a.sub_nrows[sub];
    {
      // the sub-tile's rows of v_n are one contiguous run of nrows * ld elements
      const T* src = X + row0 * ld;
      const int nv = nrows * ld / CPL;
      for (int e = tid; e < nv; e += kThreads) vstore<T, CPL>(xs + e * CPL, vload<T, CPL>(src + e * CPL));
    }
    // Phase A: one thread per row.
    bool is_start = false;
    uint32_t h = 0;
    if (tid < nrows) {
      const int64_t rho = row0 + tid;
      const uint32_t s = a.states[P.state_off + rho];
      h = s >> Lb;
      const uint32_t l = s & lmask;
      const int i = s_lrank[l];
      is_start = i == 0;
      int b0 = tid - i;
      if (b0 < 0) {
        if (a.err) atomicOr(a.err, 4);
        b0 = 0;
      }
      s_row_l[tid] = (uint16_t)l;
      s_row_b0[tid] = (uint16_t)b0;
      double d = P.shift;
      for (int q = 0; q < nb; ++q) {
        const uint32_t m = s_mask[q];
        const uint32_t v = s & m;
        d += (v == 0u || v == m) ? s_zz[q] : -s_zz[q];
      }
      s_diag[tid] = d;
      int cnt = 0;
      for (int q = nll + nhh; q < nb; ++q) {
        const uint32_t m = s_mask[q];
        const uint32_t v = s & m;
        if (v == 0u || v == m) continue;
        uint32_t r = RT.rank(s ^ m);
        if (r >= (uint32_t)P.dim) {
          if (a.err) atomicOr(a.err, 2);
          r = (uint32_t)rho;
        }
        s_mx_rank[cnt * RC + tid] = r;
        s_mx_q[cnt * RC + tid] = (uint16_t)q;
        ++cnt;
      }
      s_mx_cnt[tid] = (uint16_t)cnt;
    }
    // block slot of each row: block starts at or before it, minus one
    const uint64_t bal = __ballot(is_start);
    if (lane == 0) s_wcnt[wv] = __popcll(bal);
    __syncthreads();
    int kslot = __popcll(bal & ((1ull << lane) - 1ull)) + (is_start ? 1 : 0) - 1;
    for (int w = 0; w < wv; ++w) kslot += s_wcnt[w];
    const int nblk = min(s_wcnt[0] + s_wcnt[1] + s_wcnt[2] + s_wcnt[3], a.blk_max);
    if (tid < nrows) {
      if (kslot < 0 || kslot >= a.blk_max) {
        if (a.err) atomicOr(a.err, 4);
        kslot = 0;
        is_start = false;
      }
      s_row_blk[tid] = (uint8_t)kslot;
      if (is_start) s_blk_h[kslot] = h;
    }
    __syncthreads();

    // Phase A2: for every (block, high-high bond) the first row of the target
    // run, then each block's acting bonds compacted in bond order.
    for (int t = tid; t < nblk * nhh; t += kThreads) {
      const int kb = t / nhh, q = t - kb * nhh;
      const uint32_t hb = s_blk_h[kb];
      const int cl = P.n_up - __popc(hb);
      uint32_t st = kNoRun;
      const uint32_t mh = s_mask[nll + q] >> Lb;
      const uint32_t x = hb & mh;
      if (cl < 0 || cl > Lb) {
        if (a.err) atomicOr(a.err, 4);
      } else if (!(x == 0u || x == mh)) {
        st = RT.rank(((hb ^ mh) << Lb) | ((1u << cl) - 1u));
        if ((int64_t)st + a.binom[Lb * kBinomN + cl] > P.dim) {
          if (a.err) atomicOr(a.err, 2);
          st = kNoRun;
        }
      }
      s_hh_row[kb * a.lds_hh + q] = st;
    }
    __syncthreads();
    for (int kb = tid; kb < nblk; kb += kThreads) {
      int n = 0;
      for (int q = 0; q < nhh; ++q) {
        const uint32_t st = s_hh_row[kb * a.lds_hh + q];
        if (st == kNoRun) continue;
        s_hh_row[kb * a.lds_hh + n] = st;
        s_hh_q[kb * a.lds_hh + n] = (uint16_t)(nll + q);
        ++n;
      }
      s_hh_n[kb] = n;
    }
    __syncthreads();

    // Phase C: (row, column chunk) items.
    if (rg < nrg) {
      for (int r = rg; r < nrows; r += nrg) {
        const int64_t rho = row0 + r;
        const VecT<T, CPL> xv = vload<T, CPL>(xs + r * ld + c * CPL);
        const double dg = s_diag[r];
        double acc[CPL];
#pragma unroll
        for (int i = 0; i < CPL; ++i) acc[i] = dg * (double)xv.v[i];
        VecT<T, CPL> yv;
        if (!a.first) yv = vload_nt<T, CPL>(Yin + rho * ld + c * CPL);
        const uint32_t l = s_row_l[r];
        const int b0 = s_row_b0[r];
        const int kb = s_row_blk[r];
        const int64_t ib = r - b0;
        const int nh = s_hh_n[kb];
        const uint32_t* hrow = s_hh_row + kb * a.lds_hh;
        const uint16_t* hq = s_hh_q + kb * a.lds_hh;
        // The first batch of high-high rows is in flight while the low-low
        // neighbours are read from LDS (absent entries read the row itself
        // with a zero coefficient; the summation order is unchanged).
        VecT<T, CPL> hv[GB];
        double hcf[GB];
#pragma unroll
        for (int j = 0; j < GB; ++j) {
          const bool on = j < nh;
          const int64_t row = on ? (int64_t)hrow[j] + ib : rho;
          hcf[j] = on ? s_off[hq[j]] : 0.0;
          hv[j] = vload<T, CPL>(X + row * ld + c * CPL);
        }
        for (int q0 = 0; q0 < nll; q0 += 4) {
          int jj[4];
          double cl[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int q = q0 + u;
            const uint32_t m = q < nll ? s_mask[q] : 0u;
            const uint32_t v = l & m;
            const bool on = !(v == 0u || v == m);
            int j = on ? b0 + s_lrank[l ^ m] : r;
            if (j >= nrows) {
              if (a.err) atomicOr(a.err, 4);
              j = r;
            }
            jj[u] = j;
            cl[u] = on ? s_off[q] : 0.0;
          }
          VecT<T, CPL> nl[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) nl[u] = vload<T, CPL>(xs + jj[u] * ld + c * CPL);
#pragma unroll
          for (int u = 0; u < 4; ++u) {
#pragma unroll
            for (int i = 0; i < CPL; ++i) acc[i] = fma(cl[u], (double)nl[u].v[i], acc[i]);
          }
        }
#pragma unroll
        for (int j = 0; j < GB; ++j) {
#pragma unroll
          for (int i = 0; i < CPL; ++i) acc[i] = fma(hcf[j], (double)hv[j].v[i], acc[i]);
        }
        for (int k0 = GB; k0 < nh; k0 += GB) {
          VecT<T, CPL> nv[GB];
          double cf[GB];
#pragma unroll
          for (int j = 0; j < GB; ++j) {
            const int k = k0 + j;
            const bool on = k < nh;
            const int64_t row = on ? (int64_t)hrow[k] + ib : rho;
            cf[j] = on ? s_off[hq[k]] : 0.0;
            nv[j] = vload<T, CPL>(X + row * ld + c * CPL);
          }
#pragma unroll
          for (int j = 0; j < GB; ++j) {
#pragma unroll
            for (int i = 0; i < CPL; ++i) acc[i] = fma(cf[j], (double)nv[j].v[i], acc[i]);
          }
        }
        const int cnt = s_mx_cnt[r];
        for (int k0 = 0; k0 < cnt; k0 += GB) {
          VecT<T, CPL> nv[GB];
          double cf[GB];
#pragma unroll
          for (int j = 0; j < GB; ++j) {
            const int k = k0 + j;
            const bool on = k < cnt;
            const int64_t row = on ? (int64_t)s_mx_rank[k * RC + r] : rho;
            cf[j] = on ? s_off[s_mx_q[k * RC + r]] : 0.0;
            nv[j] = vload<T, CPL>(X + row * ld + c * CPL);
          }
#pragma unroll
          for (int j = 0; j < GB; ++j) {
#pragma unroll
            for (int i = 0; i < CPL; ++i) acc[i] = fma(cf[j], (double)nv[j].v[i], acc[i]);
          }
        }
        VecT<T, CPL> ov;
        if (a.first) {
#pragma unroll
          for (int i = 0; i < CPL; ++i) ov.v[i] = (T)acc[i];
        } else {
#pragma unroll
          for (int i = 0; i < CPL; ++i) ov.v[i] = (T)(2.0 * acc[i] - (double)yv.v[i]);
        }
        vstore_nt<T, CPL>(Y + rho * ld + c * CPL, ov);
#pragma unroll
        for (int i = 0; i < CPL; ++i) {
          const double o = (double)ov.v[i];
          acc_a[i] = fma(o, o, acc_a[i]);
          acc_b[i] = fma(o, (double)xv.v[i], acc_b[i]);
        }
      }
    }
    row0 += nrows;
    __syncthreads();
  }

  // Workgroup reduction over row groups, per column (same tree as step_kernel).
  double* red = reinterpret_cast<double*>(smem + Lo.xs);
  if (rg < nrg) {
#pragma unroll
    for (int i = 0; i < CPL; ++i) {
      red[(2 * i) * kThreads + tid] = acc_a[i];
      red[(2 * i + 1) * kThreads + tid] = acc_b[i];
    }
  }
  int p2 = 1;
  while (p2 < nrg) p2 <<= 1;
  for (int sstride = p2 >> 1; sstride > 0; sstride >>= 1) {
    __syncthreads();
    if (rg < sstride && rg + sstride < nrg) {
#pragma unroll
      for (int v = 0; v < 2 * CPL; ++v) red[v * kThreads + tid] += red[v * kThreads + tid + sstride * nch];
    }
  }
  __syncthreads();
  if (tid < nch) {
    const int tl = tile - U.tile0;
#pragma unroll
    for (int i = 0; i < CPL; ++i) {
      const int col = c * CPL + i;
      a.part_out[U.part_off + (int64_t)col * U.ntiles + tl] = red[(2 * i) * kThreads + tid];
      a.part_out[U.part_off + (int64_t)(ld + col) * U.ntiles + tl] = red[(2 * i + 1) * kThreads + tid];
    }
  }
}

template <typename T, int CPL>
static hipError_t launch_block_t(const StepArgs& a, size_t lds, int grid, int gb, hipStream_t st) {
  if (gb == 8) hipLaunchKernelGGL((block_kernel<T, CPL, 8>), dim3(grid), dim3(kThreads), lds, st, a);
  else hipLaunchKernelGGL((block_kernel<T, CPL, 4>), dim3(grid), dim3(kThreads), lds, st, a);
  return hipGetLastError();
}

static hipError_t launch_block(const DevicePlan& p, const StepArgs& a, hipStream_t st) {
  const size_t lds = block_lds_bytes(p);
  const int grid = p.grid_tiles;
  if (p.fp32) {
    switch (p.cpl) {
      case 1: return launch_block_t<float, 1>(a, lds, grid, p.gather_batch, st);
      case 2: return launch_block_t<float, 2>(a, lds, grid, p.gather_batch, st);
      case 4: return launch_block_t<float, 4>(a, lds, grid, p.gather_batch, st);
      default: return hipErrorInvalidValue;
    }
  }
  switch (p.cpl) {
    case 1: return launch_block_t<double, 1>(a, lds, grid, p.gather_batch, st);
    case 2: return launch_block_t<double, 2>(a, lds, grid, p.gather_batch, st);
    default: return hipErrorInvalidValue;
  }
}

// ----------------------------------------------------- block-table kernel
//
// Same tiles of whole low-bit blocks as the block kernel, but everything a
// block needs besides its own rows is looked up in per-block tables written
// once per call (tab_meta_kernel): the first rank of the target block of every
// acting high-high bond (compacted, in bond order) and of every mixed bond.
// Member i of block h (popcount class k of its low word) has the low word
// lunr[koff[k] + i]; its neighbours are
//   low-low    block start + lrank(l ^ m)          (same block)
//   high-high  target start + i                    (same low word)
//   mixed      target start + lrank(l ^ m_low)     (target class k +- 1).
// No state words are streamed and no ranks are computed per step; the own
// block's rows are read through L1 by the low-low bonds.  Per element the sum
// runs diagonal, low-low, high-high, mixed (each in bond order).

struct TabLds {
  size_t mask, off, zz, lrank, lunr, koff, bstart, bh, boff, bcnt, bhs, bhq, bms, rblk, rl, ri,
      rdiag, rlln, rll, xs, total;
};

// xs_bytes: the sub-tile's rows of v_n in LDS (0 = read through L1).
__host__ __device__ inline TabLds tab_lds_layout(int lds_bonds, int lds_lr, int blk_max,
                                                 int lds_hh, int lds_mx, int lds_ll, int rows,
                                                 int cpl, size_t xs_bytes) {
  TabLds L{};
  size_t o = 0;
  auto put = [&](size_t b) {
    const size_t r = o;
    o = (o + b + 15) & ~size_t(15);
    return r;
  };
  L.mask = put(size_t(lds_bonds) * 4);
  L.off = put(size_t(lds_bonds) * 8);
  L.zz = put(size_t(lds_bonds) * 8);
  L.lrank = put(size_t(lds_lr) * 2);
  L.lunr = put(size_t(lds_lr) * 2);
  L.koff = put(size_t(kKoffLen) * 4);
  L.bstart = put(size_t(blk_max) * 4);
  L.bh = put(size_t(blk_max) * 4);
  L.boff = put(size_t(blk_max) * 4);
  L.bcnt = put(size_t(blk_max) * 4);
  // + 8 entries: a batch of gathers may read up to GB - 1 entries past a
  // block's list (those lanes are masked)
  L.bhs = put((size_t(blk_max) * lds_hh + 8) * 4);
  L.bhq = put((size_t(blk_max) * lds_hh + 8) * 2);
  L.bms = put(size_t(blk_max) * lds_mx * 4);
  L.rblk = put(size_t(rows));
  L.rl = put(size_t(rows) * 2);
  L.ri = put(size_t(rows) * 2);
  L.rdiag = put(size_t(rows) * 8);
  L.rlln = put(size_t(rows));
  L.rll = put((size_t(rows) * lds_ll + 4) * 2);
  L.xs = put(xs_bytes);
  const size_t red = size_t(2 * cpl) * kThreads * 8;   // final reduction overlays all of it
  L.total = o > red ? o : red;
  return L;
}

size_t tab_lds_bytes(const DevicePlan& p) {
  const size_t xs = p.tab_xl ? size_t(p.blk_rows) * p.ld_max * (p.fp32 ? 4 : 8) : 0;
  return tab_lds_layout(p.lds_bonds, p.lds_lr, p.blk_max, p.lds_hh, p.lds_mx, p.lds_ll, p.blk_rows,
                        p.cpl, xs)
      .total;
}

struct TabMeta {
  size_t hcnt, hstart, mstart, hq, hcoef, dhh, wtab, brec, total;
};

// wtab_bytes > 0 (slice kernel): also per-block coefficients and diagonal
// parts, and the word tables.
__host__ __device__ inline TabMeta tab_meta_layout(int64_t n_blk, int hh, int mx, size_t wtab_bytes) {
  TabMeta m{};
  size_t o = 0;
  auto put = [&](size_t b) {
    const size_t r = o;
    o = (o + b + 255) & ~size_t(255);
    return r;
  };
  // + 16 entries: the slice kernel reads whole batches past a block's count
  m.hcnt = put(size_t(n_blk) * 4);
  m.hstart = put((size_t(n_blk) * hh + 16) * 4);
  m.mstart = put((size_t(n_blk) * mx + 16) * 4);
  m.hq = put(size_t(n_blk) * hh * 2);
  if (wtab_bytes) {
    m.hcoef = put((size_t(n_blk) * hh + 16) * 8);
    m.dhh = put(size_t(n_blk) * 8);
    m.wtab = put(wtab_bytes);
    m.brec = put(size_t(n_blk) * sizeof(SliceBlk));
  }
  m.total = o;
  return m;
}

static size_t slice_wtab_bytes(const DevicePlan& p) {
  return p.slice_wb ? size_t(p.n_probs) * p.slice_words * p.slice_wb : 0;
}

static TabMeta plan_meta(const DevicePlan& p) {
  return tab_meta_layout(p.n_blk, p.meta_hh, p.meta_mx, slice_wtab_bytes(p));
}

size_t tab_meta_bytes(const DevicePlan& p) { return plan_meta(p).total; }

// Rank of the first state of block hp with k low bits set: the k lowest bits
// contribute C(j - 1, j) = 0, so only the high bits count.
__device__ __forceinline__ uint32_t block_first_rank(uint32_t hp, int L, int k, const uint32_t* binom) {
  uint32_t r = 0;
  int j = k;
  for (uint32_t x = hp; x; x &= x - 1u) {
    const int pos = L + __ffs(x) - 1;
    ++j;
    r += binom[pos * kBinomN + j];
  }
  return r;
}

// Per-block tables of the block-table kernel, one thread per block.
__global__ __launch_bounds__(kThreads) void tab_meta_kernel(const ProbDev* probs,
                                                            const uint32_t* bmask,
                                                            const uint16_t* bperm,
                                                            const uint32_t* binom,
                                                            const uint32_t* blk_h, int meta_hh,
                                                            int meta_mx, uint32_t* hcnt,
                                                            uint32_t* hstart, uint32_t* mstart,
                                                            uint16_t* hq, const double* boff,
                                                            const double* bzz, double* hcoef,
                                                            double* dhh, const uint32_t* blk_start,
                                                            const int32_t* koff, SliceBlk* brec,
                                                            int* err) {
  __shared__ uint32_t sb[kBinomN * kBinomN];
  for (int i = threadIdx.x; i < kBinomN * kBinomN; i += kThreads) sb[i] = binom[i];
  __syncthreads();
  const ProbDev P = probs[blockIdx.y];
  const int L = P.blk_L;
  const int q_hh = P.bond_off + P.n_ll, q_mx = q_hh + P.n_hh;
  for (int64_t t = (int64_t)blockIdx.x * kThreads + threadIdx.x; t < P.n_blk;
       t += (int64_t)gridDim.x * kThreads) {
    const int64_t g = P.blk_off + t;
    const uint32_t h = blk_h[g];
    const int k = P.n_up - __popc(h);
    int n = 0;
    for (int q = 0; q < P.n_hh; ++q) {
      const uint32_t mh = bmask[P.bond_off + bperm[q_hh + q]] >> L;
      const uint32_t x = h & mh;
      if (x == 0u || x == mh) continue;
      const uint32_t st = block_first_rank(h ^ mh, L, k, sb);
      if (k < 0 || k > L || (int64_t)st + sb[L * kBinomN + k] > P.dim) {
        if (err) atomicOr(err, 2);
        continue;
      }
      hstart[g * meta_hh + n] = st;
      hq[g * meta_hh + n] = (uint16_t)q;
      if (hcoef) hcoef[g * meta_hh + n] = boff[P.bond_off + bperm[q_hh + q]];
      ++n;
    }
    hcnt[g] = (uint32_t)n;
    if (dhh) {
      // the diagonal's high-high part: sum_b (+-) J_b/(4a) over bonds between high sites
      double d = P.shift;
      for (int q = 0; q < P.n_hh; ++q) {
        const int b = P.bond_off + bperm[q_hh + q];
        const uint32_t mh = bmask[b] >> L, x = h & mh;
        d += (x == 0u || x == mh) ? bzz[b] : -bzz[b];
      }
      dhh[g] = d;
      if (brec) {
        SliceBlk r{};
        r.h = h;
        r.start = blk_start[g];
        r.size = (k >= 0 && k <= L) ? sb[L * kBinomN + k] : 0u;
        r.kofs = (k >= 0 && k <= L) ? (uint32_t)koff[k] : 0u;
        r.nh = (uint32_t)n;
        r.dhh = d;
        brec[g] = r;
      }
    }
    for (int q = 0; q < P.n_mx; ++q) {
      const uint32_t mh = bmask[P.bond_off + bperm[q_mx + q]] >> L;   // one high bit
      const int kk = (h & mh) ? k + 1 : k - 1;
      uint32_t st = kNoRun;
      if (kk >= 0 && kk <= L) {
        st = block_first_rank(h ^ mh, L, kk, sb);
        if ((int64_t)st + sb[L * kBinomN + kk] > P.dim) {
          if (err) atomicOr(err, 2);
          st = kNoRun;
        }
      }
      mstart[g * meta_mx + q] = st;
    }
  }
}

hipError_t build_tab_meta(const DevicePlan& p, hipStream_t st) {
  const TabMeta m = plan_meta(p);
  // the tables live in the plan's state-table region of the workspace
  if (m.total > (size_t)p.n_states * 4) return hipErrorInvalidValue;
  unsigned char* base = reinterpret_cast<unsigned char*>(p.states);
  const bool slice = p.slice_wb > 0;
  hipLaunchKernelGGL(tab_meta_kernel, dim3(256, p.n_probs), dim3(kThreads), 0, st, p.probs,
                     p.bmask, p.bperm, p.binom, p.blk_h, p.meta_hh, p.meta_mx,
                     reinterpret_cast<uint32_t*>(base + m.hcnt),
                     reinterpret_cast<uint32_t*>(base + m.hstart),
                     reinterpret_cast<uint32_t*>(base + m.mstart),
                     reinterpret_cast<uint16_t*>(base + m.hq), p.boff, p.bzz,
                     slice ? reinterpret_cast<double*>(base + m.hcoef) : nullptr,
                     slice ? reinterpret_cast<double*>(base + m.dhh) : nullptr, p.blk_start, p.koff,
                     slice ? reinterpret_cast<SliceBlk*>(base + m.brec) : nullptr, p.err);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && slice) e = build_slice_words(p, reinterpret_cast<uint8_t*>(base + m.wtab), st);
  return e;
}

// One batch of NB mixed bonds (one low and one high site) of a (row, chunk)
// item: the bond acts when the two sites differ; the neighbour row is the
// target block's first rank plus the colex rank of the flipped low word.
template <typename T, int CPL, int NB>
__device__ __forceinline__ void tab_mx_batch(const T* X, const uint32_t* mm, const double* mo,
                                             const uint32_t* ms, const uint16_t* lrank, int k0,
                                             int nmx, uint32_t l, uint32_t h, uint32_t lmask, int Lb,
                                             uint32_t rho, uint32_t ldu, uint32_t cc, int* err,
                                             double* acc) {
  VecT<T, CPL> nv[NB];
  double cf[NB];
#pragma unroll
  for (int j = 0; j < NB; ++j) {
    const int q = k0 + j;
    bool on = false;
    uint32_t row = rho;
    if (q < nmx) {
      const uint32_t m = mm[q];
      const uint32_t ml = m & lmask, mh = m >> Lb;
      on = ((l & ml) != 0u) != ((h & mh) != 0u);
      const uint32_t st = ms[q];
      if (on && st == kNoRun) {
        if (err) atomicOr(err, 2);
        on = false;
      }
      if (on) row = st + lrank[l ^ ml];
    }
    cf[j] = on ? mo[q] : 0.0;
    nv[j] = vload<T, CPL>(X + (row * ldu + cc));
  }
#pragma unroll
  for (int j = 0; j < NB; ++j) {
#pragma unroll
    for (int i = 0; i < CPL; ++i) acc[i] = fma(cf[j], (double)nv[j].v[i], acc[i]);
  }
}

// XL: the sub-tile's rows of v_n are copied to LDS first and the own row and
// the low-low neighbours are read from there.
template <typename T, int CPL, int GB, bool XL>
__global__ __launch_bounds__(kThreads) void tab_kernel(const StepArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const int tid = threadIdx.x;

  if (a.n_jobs > 0) {
    const int64_t s = (a.step_base ? *a.step_base : 0) + a.step_add;
    double* sh = reinterpret_cast<double*>(smem);
    for (int job = blockIdx.x; job < a.n_jobs; job += gridDim.x) {
      const UnitDev U = a.units[a.job_unit[job]];
      const int v = job - 2 * U.col_off;
      const double sum = sum_partials(a.part_in + U.part_off + (int64_t)v * U.ntiles, U.ntiles, sh);
      if (tid == 0) {
        if (v < U.ld) a.alpha[s * a.total_cols + U.col_off + v] = sum;
        else a.beta[(s - 1) * a.total_cols + U.col_off + (v - U.ld)] = sum;
      }
    }
    __syncthreads();
  }

  const int tile = a.xcd_remap ? xcd_tile(blockIdx.x, a.grid_tiles) : (int)blockIdx.x;
  if (tile >= a.n_tiles) return;
  const UnitDev U = a.units[a.tile_unit[tile]];
  const ProbDev P = a.probs[U.prob];
  const TabLds Lo = tab_lds_layout(a.lds_bonds, a.lds_lr, a.blk_max, a.lds_hh, a.lds_mx, a.lds_ll,
                                   a.blk_rows, CPL,
                                   XL ? size_t(a.blk_rows) * a.ld_max * sizeof(T) : 0);
  uint32_t* s_mask = reinterpret_cast<uint32_t*>(smem + Lo.mask);
  double* s_off = reinterpret_cast<double*>(smem + Lo.off);
  double* s_zz = reinterpret_cast<double*>(smem + Lo.zz);
  uint16_t* s_lrank = reinterpret_cast<uint16_t*>(smem + Lo.lrank);
  uint16_t* s_lunr = reinterpret_cast<uint16_t*>(smem + Lo.lunr);
  int32_t* s_koff = reinterpret_cast<int32_t*>(smem + Lo.koff);
  uint32_t* s_bstart = reinterpret_cast<uint32_t*>(smem + Lo.bstart);
  uint32_t* s_bh = reinterpret_cast<uint32_t*>(smem + Lo.bh);
  int32_t* s_boff = reinterpret_cast<int32_t*>(smem + Lo.boff);
  int32_t* s_bcnt = reinterpret_cast<int32_t*>(smem + Lo.bcnt);
  uint32_t* s_bhs = reinterpret_cast<uint32_t*>(smem + Lo.bhs);
  uint16_t* s_bhq = reinterpret_cast<uint16_t*>(smem + Lo.bhq);
  uint32_t* s_bms = reinterpret_cast<uint32_t*>(smem + Lo.bms);
  uint8_t* s_rblk = reinterpret_cast<uint8_t*>(smem + Lo.rblk);
  uint16_t* s_rl = reinterpret_cast<uint16_t*>(smem + Lo.rl);
  uint16_t* s_ri = reinterpret_cast<uint16_t*>(smem + Lo.ri);
  double* s_rdiag = reinterpret_cast<double*>(smem + Lo.rdiag);
  uint8_t* s_rlln = reinterpret_cast<uint8_t*>(smem + Lo.rlln);
  uint16_t* s_rll = reinterpret_cast<uint16_t*>(smem + Lo.rll);
  T* xs = reinterpret_cast<T*>(smem + Lo.xs);

  const int nb = P.n_bonds, nll = P.n_ll, nhh = P.n_hh, nmx = P.n_mx;
  const int Lb = P.blk_L;
  for (int q = tid; q < nb; q += kThreads) {
    const int b = P.bond_off + a.bperm[P.bond_off + q];
    s_mask[q] = a.bmask[b];
    s_off[q] = a.boff[b];
    s_zz[q] = a.bzz[b];
  }
  for (int l = tid; l < a.lds_lr; l += kThreads) {
    s_lrank[l] = a.lrank[l];
    s_lunr[l] = a.lunr[l];
  }
  for (int k = tid; k < kKoffLen; k += kThreads) s_koff[k] = a.koff[k];

  const int ld = U.ld;
  T* base = reinterpret_cast<T*>(a.vec) + U.vec_off;
  const T* X = base + a.x_slot * a.slot_stride;
  const T* Yin = base + a.yin_slot * a.slot_stride;
  T* Y = base + a.yout_slot * a.slot_stride;
  const uint32_t lmask = (1u << Lb) - 1u;
  const int nch = ld / CPL;
  const int nrg = kThreads / nch;
  const int c = tid % nch;
  const int rg = tid / nch;
  double acc_a[CPL], acc_b[CPL];
#pragma unroll
  for (int i = 0; i < CPL; ++i) acc_a[i] = acc_b[i] = 0.0;

  int64_t row0 = a.tile_row0[tile];
  const int sub1 = a.tile_sub0[tile + 1];
  for (int sub = a.tile_sub0[tile]; sub < sub1; ++sub) {
    const int nrows = a.sub_nrows[sub];
    const int g0 = a.sub_blk0[sub];
    const int nblk = min(a.sub_nblk[sub], a.blk_max);
    for (int t = tid; t < nblk; t += kThreads) {
      const uint32_t st = a.blk_start[g0 + t];
      s_bstart[t] = st;
      s_bh[t] = a.blk_h[g0 + t];
      s_boff[t] = (int)((int64_t)st - row0);
      s_bcnt[t] = (int)min(a.meta_hcnt[g0 + t], (uint32_t)nhh);
    }
    for (int t = tid; t < nblk * nhh; t += kThreads) {
      const int kb = t / nhh, j = t - kb * nhh;
      const int64_t src = (int64_t)(g0 + kb) * a.meta_hh + j;
      s_bhs[kb * a.lds_hh + j] = a.meta_hstart[src];
      s_bhq[kb * a.lds_hh + j] = a.meta_hq[src];
    }
    for (int t = tid; t < nblk * nmx; t += kThreads) {
      const int kb = t / nmx, j = t - kb * nmx;
      s_bms[kb * a.lds_mx + j] = a.meta_mstart[(int64_t)(g0 + kb) * a.meta_mx + j];
    }
    if (XL) {
      // the sub-tile's rows of v_n are one contiguous run of nrows * ld elements
      const T* src = X + row0 * ld;
      const int nv = nrows * ld / CPL;
      for (int e = tid; e < nv; e += kThreads) vstore<T, CPL>(xs + e * CPL, vload<T, CPL>(src + e * CPL));
    }
    __syncthreads();
    // Phase A: one thread per row (its block, low word and diagonal element).
    if (tid < nrows) {
      int kb = 0;
      while (kb + 1 < nblk && s_boff[kb + 1] <= tid) ++kb;
      int i = tid - s_boff[kb];
      const uint32_t h = s_bh[kb];
      const int k = P.n_up - __popc(h);
      uint32_t l = 0;
      if (k < 0 || k > Lb || i < 0 || i >= s_koff[k + 1] - s_koff[k]) {
        if (a.err) atomicOr(a.err, 4);
        i = 0;
      } else {
        l = s_lunr[s_koff[k] + i];
      }
      const uint32_t sw = (h << Lb) | l;
      double d = P.shift;
#pragma unroll 2
      for (int q = 0; q < nb; ++q) {
        const uint32_t m = s_mask[q];
        const uint32_t v = sw & m;
        d += (v == 0u || v == m) ? s_zz[q] : -s_zz[q];
      }
      // acting low-low bonds: the neighbour is row boff + lrank(l ^ m) of this
      // sub-tile; (row, bond) packed in 16 bits
      int nl = 0;
      for (int q = 0; q < nll; ++q) {
        const uint32_t m = s_mask[q];
        const uint32_t v = l & m;
        if (v == 0u || v == m) continue;
        const int jr = s_boff[kb] + s_lrank[l ^ m];
        if (jr < 0 || jr >= nrows) {
          if (a.err) atomicOr(a.err, 4);
          continue;
        }
        s_rll[tid * a.lds_ll + nl] = (uint16_t)(jr | (q << 8));
        ++nl;
      }
      s_rlln[tid] = (uint8_t)nl;
      s_rblk[tid] = (uint8_t)kb;
      s_rl[tid] = (uint16_t)l;
      s_ri[tid] = (uint16_t)i;
      s_rdiag[tid] = d;
    }
    __syncthreads();

    // Phase C: (row, column chunk) items.  Diagonal, low-low (own sub-tile),
    // high-high and mixed rows, GB loads in flight per batch (mixed ones 2 at
    // a time when the problem has at most 2); the own row is read again only
    // at the end, so that few registers stay live across the gathers.
    // Element offsets inside the block's slot fit 32 bits (the planner
    // guarantees dim * ld < 2^32); a slot past a row's count reads the row
    // itself with a zero coefficient, so every lane of a batch issues its
    // loads without branching.
    if (rg < nrg) {
      const uint32_t ldu = (uint32_t)ld, cc = (uint32_t)(c * CPL);
      for (int r = rg; r < nrows; r += nrg) {
        const uint32_t rho = (uint32_t)(row0 + r);
        // float32 storage: v_{n-1} is requested first, so its latency overlaps
        // the gathers (4 more registers, still 4 waves per SIMD); float64
        // storage reads it at the end and keeps 5 waves per SIMD
        constexpr bool kEarlyY = sizeof(T) == 4;
        VecT<T, CPL> yv{};
        if (kEarlyY && !a.first) yv = vload_nt<T, CPL>(Yin + (rho * ldu + cc));
        double acc[CPL];
        {
          const VecT<T, CPL> xv = XL ? vload<T, CPL>(xs + r * ld + c * CPL)
                                     : vload<T, CPL>(X + (rho * ldu + cc));
          const double dg = s_rdiag[r];
#pragma unroll
          for (int i = 0; i < CPL; ++i) acc[i] = dg * (double)xv.v[i];
        }
        {
          // acting low-low neighbours, four at a time
          const int nl = s_rlln[r];
          const uint16_t* ll = s_rll + r * a.lds_ll;
          for (int k0 = 0; k0 < nl; k0 += 4) {
            VecT<T, CPL> nv[4];
            double cl[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const bool on = k0 + u < nl;
              const uint32_t e = ll[k0 + u];
              cl[u] = s_off[on ? (e >> 8) : 0u];
              cl[u] = on ? cl[u] : 0.0;
              const uint32_t jr = on ? (e & 0xFFu) : (uint32_t)r;
              nv[u] = XL ? vload<T, CPL>(xs + jr * ldu + cc)
                         : vload<T, CPL>(X + (((uint32_t)row0 + jr) * ldu + cc));
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
#pragma unroll
              for (int i = 0; i < CPL; ++i) acc[i] = fma(cl[u], (double)nv[u].v[i], acc[i]);
            }
          }
        }
        const int kb = s_rblk[r];
        const uint32_t ib = s_ri[r];
        const int nh = s_bcnt[kb];
        const uint32_t* hs = s_bhs + kb * a.lds_hh;
        const uint16_t* hq = s_bhq + kb * a.lds_hh;
        // high-high rows: target block start + index in block
        for (int k0 = 0; k0 < nh; k0 += GB) {
          VecT<T, CPL> nv[GB];
          double cf[GB];
#pragma unroll
          for (int j = 0; j < GB; ++j) {
            const int k = k0 + j;
            const bool on = k < nh;
            const uint32_t hsv = hs[k];
            const uint32_t hqv = hq[k];
            const uint32_t row = on ? hsv + ib : rho;
            cf[j] = s_off[nll + (on ? hqv : 0u)];
            cf[j] = on ? cf[j] : 0.0;
            nv[j] = vload<T, CPL>(X + (row * ldu + cc));
          }
#pragma unroll
          for (int j = 0; j < GB; ++j) {
#pragma unroll
            for (int i = 0; i < CPL; ++i) acc[i] = fma(cf[j], (double)nv[j].v[i], acc[i]);
          }
        }
        if (nmx > 0) {
          const uint32_t l = s_rl[r];
          const uint32_t h = s_bh[kb];
          const uint32_t* ms = s_bms + kb * a.lds_mx;
          const uint32_t* mm = s_mask + nll + nhh;
          const double* mo = s_off + nll + nhh;
          // the batch size follows the problem's mixed-bond count (uniform)
          if (nmx <= 2) {
            tab_mx_batch<T, CPL, 2>(X, mm, mo, ms, s_lrank, 0, nmx, l, h, lmask, Lb, rho, ldu, cc, a.err, acc);
          } else {
            for (int k0 = 0; k0 < nmx; k0 += GB)
              tab_mx_batch<T, CPL, GB>(X, mm, mo, ms, s_lrank, k0, nmx, l, h, lmask, Lb, rho, ldu, cc, a.err, acc);
          }
        }
        VecT<T, CPL> ov;
        if (a.first) {
#pragma unroll
          for (int i = 0; i < CPL; ++i) ov.v[i] = (T)acc[i];
        } else {
          if (!kEarlyY) yv = vload_nt<T, CPL>(Yin + (rho * ldu + cc));
#pragma unroll
          for (int i = 0; i < CPL; ++i) ov.v[i] = (T)(2.0 * acc[i] - (double)yv.v[i]);
        }
        vstore_nt<T, CPL>(Y + (rho * ldu + cc), ov);
        const VecT<T, CPL> xv = XL ? vload<T, CPL>(xs + r * ld + c * CPL)
                                   : vload<T, CPL>(X + (rho * ldu + cc));
#pragma unroll
        for (int i = 0; i < CPL; ++i) {
          const double o = (double)ov.v[i];
          acc_a[i] = fma(o, o, acc_a[i]);
          acc_b[i] = fma(o, (double)xv.v[i], acc_b[i]);
        }
      }
    }
    row0 += nrows;
    __syncthreads();
  }

  // Workgroup reduction over row groups, per column (same tree as step_kernel).
  double* red = reinterpret_cast<double*>(smem);
  if (rg < nrg) {
#pragma unroll
    for (int i = 0; i < CPL; ++i) {
      red[(2 * i) * kThreads + tid] = acc_a[i];
      red[(2 * i + 1) * kThreads + tid] = acc_b[i];
    }
  }
  int p2 = 1;
  while (p2 < nrg) p2 <<= 1;
  for (int sstride = p2 >> 1; sstride > 0; sstride >>= 1) {
    __syncthreads();
    if (rg < sstride && rg + sstride < nrg) {
#pragma unroll
      for (int v = 0; v < 2 * CPL; ++v) red[v * kThreads + tid] += red[v * kThreads + tid + sstride * nch];
    }
  }
  __syncthreads();
  if (tid < nch) {
    const int tl = tile - U.tile0;
#pragma unroll
    for (int i = 0; i < CPL; ++i) {
      const int col = c * CPL + i;
      a.part_out[U.part_off + (int64_t)col * U.ntiles + tl] = red[(2 * i) * kThreads + tid];
      a.part_out[U.part_off + (int64_t)(ld + col) * U.ntiles + tl] = red[(2 * i + 1) * kThreads + tid];
    }
  }
}

template <typename T, int CPL>
static hipError_t launch_tab_t(const StepArgs& a, size_t lds, int grid, int gb, bool xl,
                               hipStream_t st) {
  if (xl) {
    if (gb == 8) hipLaunchKernelGGL((tab_kernel<T, CPL, 8, true>), dim3(grid), dim3(kThreads), lds, st, a);
    else hipLaunchKernelGGL((tab_kernel<T, CPL, 4, true>), dim3(grid), dim3(kThreads), lds, st, a);
  } else {
    if (gb == 8) hipLaunchKernelGGL((tab_kernel<T, CPL, 8, false>), dim3(grid), dim3(kThreads), lds, st, a);
    else hipLaunchKernelGGL((tab_kernel<T, CPL, 4, false>), dim3(grid), dim3(kThreads), lds, st, a);
  }
  return hipGetLastError();
}

static hipError_t launch_tab(const DevicePlan& p, const StepArgs& a, hipStream_t st) {
  const size_t lds = tab_lds_bytes(p);
  const int grid = p.grid_tiles;
  if (p.fp32) {
    switch (p.cpl) {
      case 1: return launch_tab_t<float, 1>(a, lds, grid, p.gather_batch, p.tab_xl, st);
      case 2: return launch_tab_t<float, 2>(a, lds, grid, p.gather_batch, p.tab_xl, st);
      case 4: return launch_tab_t<float, 4>(a, lds, grid, p.gather_batch, p.tab_xl, st);
      default: return hipErrorInvalidValue;
    }
  }
  switch (p.cpl) {
    case 1: return launch_tab_t<double, 1>(a, lds, grid, p.gather_batch, p.tab_xl, st);
    case 2: return launch_tab_t<double, 2>(a, lds, grid, p.gather_batch, p.tab_xl, st);
    default: return hipErrorInvalidValue;
  }
}

size_t step_lds_bytes(const DevicePlan& p) {
  auto a16 = [](size_t x) { return (x + 15) & ~size_t(15); };
  size_t o = 0;
  o = a16(o + kBinomN * kBinomN * 4);
  o = a16(o + size_t(p.lds_tab) * 4);
  o = a16(o + size_t(p.lds_bonds) * 4);
  o = a16(o + size_t(p.lds_bonds) * 8);
  o = a16(o + size_t(p.lds_bonds) * 8);
  o = a16(o + size_t(p.sub_rows) * 8);
  o = a16(o + size_t(p.sub_rows) * 4);
  const size_t lists = a16(size_t(p.lds_nb) * p.sub_rows * 4) + size_t(p.lds_nb) * p.sub_rows * 2;
  const size_t red = size_t(2 * p.cpl) * kThreads * 8;
  return a16(o + (lists > red ? lists : red));
}

static StepArgs make_step_args(const DevicePlan& p) {
  StepArgs a{};
  a.probs = p.probs;
  a.units = p.units;
  a.tile_unit = p.tile_unit;
  a.tile_row0 = p.tile_row0;
  a.tile_nrows = p.tile_nrows;
  a.job_unit = p.job_unit;
  a.tables = p.tables;
  a.bmask = p.bmask;
  a.boff = p.boff;
  a.bzz = p.bzz;
  a.binom = p.binom;
  a.n_tiles = p.n_tiles;
  a.grid_tiles = p.grid_tiles;
  a.total_cols = p.total_cols;
  a.sub_rows = p.sub_rows;
  a.sub_per_tile = p.sub_per_tile;
  a.lds_nb = p.lds_nb;
  a.lds_tab = p.lds_tab;
  a.lds_bonds = p.lds_bonds;
  a.xcd_remap = p.xcd_remap;
  a.slot_stride = p.slot_stride;
  a.dense = p.dense;
  a.states = p.states;
  a.spin_rows = p.spin_rows;
  a.bperm = p.bperm;
  a.blk_max = p.blk_max;
  a.blk_rows = p.blk_rows;
  a.lds_lr = p.lds_lr;
  a.lds_hh = p.lds_hh;
  a.lds_mx = p.lds_mx;
  a.ld_max = p.ld_max;
  a.tile_sub0 = p.tile_sub0;
  a.sub_nrows = p.sub_nrows;
  a.lrank = p.lrank;
  if (p.block >= 2) {
    const TabMeta m = plan_meta(p);
    const unsigned char* mb = reinterpret_cast<const unsigned char*>(p.states);
    a.blk_h = p.blk_h;
    a.blk_start = p.blk_start;
    a.sub_blk0 = p.sub_blk0;
    a.sub_nblk = p.sub_nblk;
    a.lunr = p.lunr;
    a.koff = p.koff;
    a.meta_hcnt = reinterpret_cast<const uint32_t*>(mb + m.hcnt);
    a.meta_hstart = reinterpret_cast<const uint32_t*>(mb + m.hstart);
    a.meta_mstart = reinterpret_cast<const uint32_t*>(mb + m.mstart);
    a.meta_hq = reinterpret_cast<const uint16_t*>(mb + m.hq);
    a.meta_hh = p.meta_hh;
    a.meta_mx = p.meta_mx;
    a.lds_ll = p.lds_ll;
    if (p.slice_wb) {
      a.cmask = p.cmask;
      a.coff = p.coff;
      a.czz = p.czz;
      a.meta_hcoef = reinterpret_cast<const double*>(mb + m.hcoef);
      a.meta_dhh = reinterpret_cast<const double*>(mb + m.dhh);
      a.wtab = reinterpret_cast<const uint8_t*>(mb + m.wtab);
      a.slice_wb = p.slice_wb;
      a.slice_words = p.slice_words;
      a.blk_lds_rows = p.slice_nw > 1 ? p.slice_tile_rows : p.blk_lds_rows;
      a.wg_rec = p.wg_rec;
      a.blk_rec = reinterpret_cast<const SliceBlk*>(mb + m.brec);
    }
  }
  return a;
}

template <typename T, int CPL>
static hipError_t launch_step_t(const StepArgs& a, size_t lds, int grid, int gb, hipStream_t st) {
  if (gb == 8) hipLaunchKernelGGL((step_kernel<T, CPL, 8>), dim3(grid), dim3(kThreads), lds, st, a);
  else hipLaunchKernelGGL((step_kernel<T, CPL, 4>), dim3(grid), dim3(kThreads), lds, st, a);
  return hipGetLastError();
}

hipError_t launch_step_args(const DevicePlan& p, const StepArgs& a, hipStream_t st);

hipError_t launch_step(const DevicePlan& p, void* vec, double* part_out, const double* part_in,
                       int n_jobs, double* alpha, double* beta, const int64_t* step_base,
                       int step_add, int x_parity, int first, hipStream_t st) {
  StepArgs a = make_step_args(p);
  a.err = p.err;
  a.vec = vec;
  a.vec_lo = p.resid ? reinterpret_cast<int16_t*>(reinterpret_cast<float*>(vec) + p.vec_elems) : nullptr;
  a.part_out = part_out;
  a.part_in = part_in;
  a.n_jobs = n_jobs;
  a.alpha = alpha;
  a.beta = beta;
  a.step_base = step_base;
  a.step_add = step_add;
  a.x_slot = x_parity;
  a.yin_slot = a.yout_slot = 1 - x_parity;
  a.first = first;
  return launch_step_args(p, a, st);
}

hipError_t launch_step_scaled(const DevicePlan& p, void* vec, double* part_out, int x_parity,
                              const double* yscale, hipStream_t st) {
  if (p.block != 3 || p.fp32 || !yscale) return hipErrorInvalidValue;
  StepArgs a = make_step_args(p);
  a.err = p.err;
  a.vec = vec;
  a.part_out = part_out;
  a.x_slot = x_parity;
  a.yin_slot = a.yout_slot = 1 - x_parity;
  a.yscale = yscale;
  return launch_step_args(p, a, st);
}

hipError_t launch_step_slots(const DevicePlan& p, void* vec, double* part_out, int x_slot,
                             int yin_slot, int yout_slot, int first, hipStream_t st) {
  StepArgs a = make_step_args(p);
  a.err = p.err;
  a.vec = vec;
  a.vec_lo = p.resid ? reinterpret_cast<int16_t*>(reinterpret_cast<float*>(vec) + p.vec_elems) : nullptr;
  a.part_out = part_out;
  a.x_slot = x_slot;
  a.yin_slot = yin_slot;
  a.yout_slot = yout_slot;
  a.first = first;
  return launch_step_args(p, a, st);
}

hipError_t launch_step_slots_dots(const DevicePlan& p, void* vec, double* part_out, const double* part_in,
                                  int n_jobs, double* alpha, double* beta, int step_add, int x_slot,
                                  int yin_slot, int yout_slot, hipStream_t st) {
  StepArgs a = make_step_args(p);
  a.err = p.err;
  a.vec = vec;
  a.vec_lo = p.resid ? reinterpret_cast<int16_t*>(reinterpret_cast<float*>(vec) + p.vec_elems) : nullptr;
  a.part_out = part_out;
  a.part_in = part_in;
  a.n_jobs = n_jobs;
  a.alpha = alpha;
  a.beta = beta;
  a.step_add = step_add;
  a.x_slot = x_slot;
  a.yin_slot = yin_slot;
  a.yout_slot = yout_slot;
  a.first = 0;
  return launch_step_args(p, a, st);
}

hipError_t launch_step_args(const DevicePlan& p, const StepArgs& a, hipStream_t st) {
  if (p.resid && p.block != 3) return hipErrorInvalidValue;   // residual storage: slice kernel only
  if (p.spin) return launch_spin(p, a, st);
  if (p.block == 3) return launch_slice(p, a, st);
  if (p.block == 2) return launch_tab(p, a, st);
  if (p.block) return launch_block(p, a, st);
  if (p.row_ld > 0) return launch_row(p, a, st);
  const size_t lds = step_lds_bytes(p);
  const int grid = p.grid_tiles;
  if (p.fp32) {
    switch (p.cpl) {
      case 1: return launch_step_t<float, 1>(a, lds, grid, p.gather_batch, st);
      case 2: return launch_step_t<float, 2>(a, lds, grid, p.gather_batch, st);
      case 4: return launch_step_t<float, 4>(a, lds, grid, p.gather_batch, st);
      default: return hipErrorInvalidValue;
    }
  }
  switch (p.cpl) {
    case 1: return launch_step_t<double, 1>(a, lds, grid, p.gather_batch, st);
    case 2: return launch_step_t<double, 2>(a, lds, grid, p.gather_batch, st);
    case 4: return launch_step_t<double, 4>(a, lds, grid, p.gather_batch, st);
    default: return hipErrorInvalidValue;
  }
}

// --------------------------------------------------------- reduce kernel


__global__ __launch_bounds__(kThreads) void reduce_kernel(const ReduceArgs a) {
  __shared__ double sh[4];
  for (int job = blockIdx.x; job < a.n_jobs; job += gridDim.x) {
    const UnitDev U = a.units[a.job_unit[job]];
    const int v = job - 2 * U.col_off;
    double* dst = v < U.ld ? a.dst_a : a.dst_b;
    const double sum = sum_partials(a.part + U.part_off + (int64_t)v * U.ntiles, U.ntiles, sh);
    if (threadIdx.x == 0 && dst) dst[U.col_off + (v < U.ld ? v : v - U.ld)] = sum;
  }
}

hipError_t launch_reduce(const DevicePlan& p, const double* part, double* dst_a, double* dst_b,
                         hipStream_t st) {
  ReduceArgs a{p.units, p.job_unit, part, dst_a, dst_b, 2 * p.total_cols};
  const int grid = a.n_jobs < 4096 ? a.n_jobs : 4096;
  hipLaunchKernelGGL(reduce_kernel, dim3(grid), dim3(kThreads), 0, st, a);
  return hipGetLastError();
}

// ---------------------------------------------------- random start vectors

// Counter-based SplitMix64 (Steele, Lea, Flood 2014): output ctr+1 of the
// sequential generator started at `seed`.
__device__ __forceinline__ uint64_t splitmix(uint64_t seed, uint64_t ctr) {
  uint64_t z = seed + 0x9E3779B97F4A7C15ull * (ctr + 1ull);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
__device__ __forceinline__ double unit_open(uint64_t u) {
  return ((double)(u >> 11) + 0.5) * 0x1.0p-53;
}


// Unnormalised start value of column pc (of the problem) at row rho.
__device__ __forceinline__ double start_value(int kind, uint64_t seed, const ProbDev& P, int pc,
                                              int64_t rho) {
  if (kind == 3) return rho == (int64_t)pc ? 1.0 : 0.0;
  const int r = kind == 1 ? (pc >> 1) : pc;
  const uint64_t stream = ((uint64_t)P.cluster << 16) | ((uint64_t)P.n_up << 10) | (uint64_t)r;
  if (kind == 0) {
    const uint64_t u = splitmix(seed, (stream << 32) | (uint64_t)rho);
    return (u >> 63) ? -1.0 : 1.0;
  }
  const uint64_t i1 = (uint64_t)(2 * rho), i2 = (uint64_t)(2 * rho + 1);
  const double u1 = unit_open(splitmix(seed, (stream << 32) | i1));
  const double u2 = unit_open(splitmix(seed, (stream << 32) | i2));
  const double rad = sqrt(-2.0 * log(u1));
  const double ang = 2.0 * M_PI * u2;
  return (kind == 1 && (pc & 1)) ? rad * sin(ang) : rad * cos(ang);
}

template <typename T>
__global__ __launch_bounds__(kThreads) void init_kernel(const InitArgs a) {
  __shared__ double red[kThreads];
  const int tile = xcd_tile(blockIdx.x, a.grid_tiles);
  if (tile >= a.n_tiles) return;
  const UnitDev U = a.units[a.tile_unit[tile]];
  const ProbDev P = a.probs[U.prob];
  const int ld = U.ld;
  const int nrg = kThreads / ld;
  const int tid = threadIdx.x;
  const int c = tid % ld, rg = tid / ld;
  const int64_t row0 = a.tile_row0[tile];
  const int64_t row1 = row0 + a.tile_nrows[tile];
  T* A = reinterpret_cast<T*>(a.vec) + U.vec_off;
  double scale = 1.0;
  if (a.mode == 2 && c < U.ncols) scale = 1.0 / sqrt(a.norms[U.col_off + c]);   // unit-norm Lanczos start
  if (a.mode == 1 && (a.vec_kind == 1 || a.vec_kind == 2) && c < U.ncols) {
    double n2 = a.norms[U.col_off + c];
    if (a.vec_kind == 1) {
      const int c0 = c & ~1;
      n2 = a.norms[U.col_off + c0] + a.norms[U.col_off + c0 + 1];
    }
    scale = sqrt((double)P.dim / n2);
  }
  double acc = 0.0;
  if (rg < nrg) {
    for (int64_t rho = row0 + rg; rho < row1; rho += nrg) {
      double x = 0.0;
      // a relabelled row draws the value of its word's original rank
      const int64_t idx = P.relabel ? (int64_t)word_rank(relabel_word(unrank((uint32_t)rho, P.n_sites, P.n_up,
                                                                                a.binom),
                                                                         P.perm, P.n_sites, false),
                                                             a.binom)
                                    : rho;
      if (c < U.ncols) x = start_value(a.vec_kind, a.seed, P, U.col0 + c, idx);
      if (a.mode == 0) {
        acc = fma(x, x, acc);
      } else if (a.lo) {
        // float32 + residual storage (T = float): the dot is of the stored value
        float hi;
        int16_t q;
        res_encode(x * scale, hi, q);
        A[rho * ld + c] = (T)hi;
        a.lo[U.vec_off + rho * ld + c] = q;
        const double xs = res_decode(hi, q);
        acc = fma(xs, xs, acc);
      } else {
        const T xs = (T)(x * scale);
        A[rho * ld + c] = xs;
        acc = fma((double)xs, (double)xs, acc);
      }
    }
  }
  red[tid] = rg < nrg ? acc : 0.0;
  int p2 = 1;
  while (p2 < nrg) p2 <<= 1;
  for (int s = p2 >> 1; s > 0; s >>= 1) {
    __syncthreads();
    if (rg < s && rg + s < nrg) red[tid] += red[tid + s * ld];
  }
  __syncthreads();
  if (tid < ld) {
    const int tl = tile - U.tile0;
    a.part_out[U.part_off + (int64_t)tid * U.ntiles + tl] = red[tid];
    a.part_out[U.part_off + (int64_t)(ld + tid) * U.ntiles + tl] = 0.0;
  }
}

hipError_t launch_init(const DevicePlan& p, void* vec, int mode, int vec_kind, uint64_t seed,
                       const double* norms, double* part_out, hipStream_t st) {
  InitArgs a{};
  a.probs = p.probs;
  a.units = p.units;
  a.tile_unit = p.tile_unit;
  a.vec = vec;
  a.lo = p.resid ? reinterpret_cast<int16_t*>(reinterpret_cast<float*>(vec) + p.vec_elems) : nullptr;
  a.norms = norms;
  a.part_out = part_out;
  a.seed = seed;
  a.n_tiles = p.n_tiles;
  a.grid_tiles = p.grid_tiles;
  a.mode = mode;
  a.vec_kind = vec_kind;
  a.tile_row0 = p.tile_row0;
  a.tile_nrows = p.tile_nrows;
  a.binom = p.binom;
  if (p.fp32) hipLaunchKernelGGL(init_kernel<float>, dim3(p.grid_tiles), dim3(kThreads), 0, st, a);
  else hipLaunchKernelGGL(init_kernel<double>, dim3(p.grid_tiles), dim3(kThreads), 0, st, a);
  return hipGetLastError();
}

// ------------------------------------------------- doubling + estimator


__global__ __launch_bounds__(kThreads) void finalize_kernel(const FinalArgs a) {
  const int64_t gid = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (gid >= (int64_t)a.n_probs * a.M) return;
  const int p = (int)(gid / a.M);
  const int n = (int)(gid % a.M);
  const int TC = a.total_cols;
  const int h = n >> 1;
  double acc = 0.0;
  bool bad = false;
  for (int u = a.prob_unit0[p]; u < a.prob_unit0[p + 1]; ++u) {
    const UnitDev U = a.units[u];
    for (int c = 0; c < U.ncols; c += a.cols_per_vec) {
      double num = 0.0, den = 0.0;
      for (int cc = 0; cc < a.cols_per_vec; ++cc) {
        const int col = U.col_off + c + cc;
        const double a0 = a.alpha[col];
        const double b0 = a.beta[col];
        double m;
        if (n == 0) m = a0;
        else if (n == 1) m = b0;
        else if ((n & 1) == 0) m = 2.0 * a.alpha[(int64_t)h * TC + col] - a0;
        else m = 2.0 * a.beta[(int64_t)h * TC + col] - b0;
        num += m;
        den += a0;
      }
      if (fabs(num) > den * (1.0 + 1e-6)) bad = true;
      acc += num / den;
    }
  }
  const ProbDev P = a.probs[p];
  const double Reff = a.R > 0 ? (double)a.R : (double)P.dim;
  a.mu[gid] = acc * ((double)P.dim / Reff);
  if (bad) atomicOr(a.flag, 1);
}

hipError_t launch_finalize(const FinalArgs& a, hipStream_t st) {
  const int64_t n = (int64_t)a.n_probs * a.M;
  const int grid = (int)((n + kThreads - 1) / kThreads);
  hipLaunchKernelGGL(finalize_kernel, dim3(grid), dim3(kThreads), 0, st, a);
  return hipGetLastError();
}

// -------------------------------------------------------------- vector export

// out[row][col] (row-major, n_cols wide) from slot `slot` of the blocks
// unit0, unit0 + 1, ... of one problem (block k holds columns [k*rb, ...)).
template <typename T>
__global__ __launch_bounds__(kThreads) void export_kernel(const ExportArgs a) {
  const T* base = reinterpret_cast<const T*>(a.vec) + (int64_t)a.slot * a.slot_stride;
  T* out = reinterpret_cast<T*>(a.out);
  const int64_t total = a.dim * a.n_cols;
  for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * kThreads) {
    const int64_t row = e / a.n_cols;
    const int col = (int)(e - row * a.n_cols);
    const UnitDev U = a.units[a.unit0 + col / a.rb];
    int64_t src = row;
    if (a.prob && a.prob->relabel) {
      const ProbDev& P = *a.prob;
      src = word_rank(relabel_word(unrank((uint32_t)row, P.n_sites, P.n_up, a.binom), P.perm, P.n_sites, true),
                      a.binom);
    }
    out[e] = base[U.vec_off + src * U.ld + (col % a.rb)];
  }
}

hipError_t launch_export(const ExportArgs& a, int fp32, hipStream_t st) {
  const int64_t total = a.dim * a.n_cols;
  const int grid = (int)std::min<int64_t>((total + kThreads - 1) / kThreads, 1 << 16);
  if (fp32) hipLaunchKernelGGL(export_kernel<float>, dim3(grid), dim3(kThreads), 0, st, a);
  else hipLaunchKernelGGL(export_kernel<double>, dim3(grid), dim3(kThreads), 0, st, a);
  return hipGetLastError();
}

// -------------------------------------------------------------- small kernels

__global__ void set_i64_kernel(int64_t* dst, int64_t v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *dst = v;
}
hipError_t launch_set_i64(int64_t* dst, int64_t v, hipStream_t st) {
  hipLaunchKernelGGL(set_i64_kernel, dim3(1), dim3(64), 0, st, dst, v);
  return hipGetLastError();
}

__global__ __launch_bounds__(kThreads) void states_kernel(int N, int k, const uint32_t* binom,
                                                          uint32_t* out, int64_t dim) {
  __shared__ uint32_t sb[kBinomN * kBinomN];
  for (int i = threadIdx.x; i < kBinomN * kBinomN; i += kThreads) sb[i] = binom[i];
  __syncthreads();
  for (int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x; r < dim;
       r += (int64_t)gridDim.x * kThreads)
    out[r] = unrank((uint32_t)r, N, k, sb);
}
hipError_t fill_states(const DevicePlan& p, hipStream_t st);

hipError_t launch_states(int N, int k, const uint32_t* binom, uint32_t* out, int64_t dim,
                         hipStream_t st) {
  int64_t g = (dim + kThreads - 1) / kThreads;
  const int grid = (int)(g < 65536 ? (g > 0 ? g : 1) : 65536);
  hipLaunchKernelGGL(states_kernel, dim3(grid), dim3(kThreads), 0, st, N, k, binom, out, dim);
  return hipGetLastError();
}

// Matrix export: phase 1 of the step kernel, written to global memory.

__global__ __launch_bounds__(kThreads) void matrix_kernel(const MatrixArgs a) {
  extern __shared__ __align__(16) unsigned char smem[];
  const ProbDev P = a.probs[0];
  const StepSmem S = carve(smem, a.lds_tab, a.lds_bonds, a.sub_rows, a.lds_nb);
  load_problem_lds(S, P, a.tables, a.bmask, a.boff, a.bzz, a.binom);
  __syncthreads();
  const RankTables RT = make_tables(S.tab, P);
  const int64_t r0 = a.row0 + (int64_t)blockIdx.x * a.sub_rows;
  const int64_t end = a.row0 + a.nrows;
  const int t = threadIdx.x;
  if (t < a.sub_rows && r0 + t < end) {
    stage_row((uint32_t)(r0 + t), P, RT, S, t, a.sub_rows, nullptr);
    const int64_t out = r0 + t - a.row0;
    const int n = S.cnt[t];
    for (int k = 0; k < n; ++k) {
      a.cols[out * a.max_nb + k] = S.nbr[k * a.sub_rows + t];
      a.bond[out * a.max_nb + k] = S.nbb[k * a.sub_rows + t];
    }
    a.cnt[out] = n;
    a.diag[out] = S.diag[t];
  }
}

// ------------------------------------------------------------ Lanczos helpers
// Blocks have one float64 column; each block's buffers sit at
// base + vec_off (+ dim for the "high" buffer of a pair).

__device__ __forceinline__ double* lz_sel(double* base, int hi, const UnitDev& U, int64_t stride) {
  return base + U.vec_off + (hi ? stride : 0);
}

// FTLM, one sweep per step where it is safe: with alpha = <w, q_j> and
// <w, w> from the recursion step, beta^2 = <w, w> - alpha^2 loses at most
// eps <w, w> / beta^2 to cancellation; for a column with beta^2 > kLzFast
// <w, w> the sweep writes y <- (w - alpha q_j) / beta and x <- beta q_j at
// once.  Other columns get y <- w - alpha q_j and their exact |y|^2 partials,
// and lz_fix_kernel finishes them.  The cut keeps the
// normalisation error of q_{j+1} near 1e-15: a looser one (1e-3) leaves
// errors near 1e-13 that surface as a residual above the 1e-12 exhaustion
// cut of an invariant Krylov space (the one-magnon sector of a 10-site ring).
// The shortcut also takes <q_j, q_j> as 1: where it is 1 + d the true
// |w - alpha q_j|^2 exceeds <w, w> - alpha^2 by alpha^2 d, so q_{j+1} carries
// the error (alpha^2 / beta^2) d on.  The sweep is therefore taken only where
// alpha^2 < beta^2 / 2, which damps the error; with the first cut alone a
// spectrum far from 0 (the three-magnon sector of the 24-site ring, energies
// in [0.077, 6], alpha^2 / beta^2 near 4) grew it geometrically and the Ritz
// values left the spectrum.
constexpr double kLzFast = 0.1;
constexpr double kLzDamp = 0.5;

__device__ __forceinline__ bool lz_fast(double ww, double al) {
  const double b2 = ww - al * al;
  return b2 > kLzFast * ww && b2 > 1e-24 && al * al < kLzDamp * b2;
}

__global__ __launch_bounds__(kThreads) void lz_fused_kernel(const LzArgs a, const double* ww) {
  __shared__ double red[kThreads];
  const int tile = xcd_tile(blockIdx.x, a.grid_tiles);
  if (tile >= a.n_tiles) return;
  const UnitDev U = a.units[a.tile_unit[tile]];
  const int64_t row0 = a.tile_row0[tile];
  const int64_t row1 = row0 + a.tile_nrows[tile];
  const int ld = U.ld;
  const int nrg = kThreads / ld;
  const int tid = threadIdx.x;
  const int c = tid % ld, rg = tid / ld;
  double* y = lz_sel(a.w, a.w_hi, U, a.slot_stride);
  double* x = lz_sel(const_cast<double*>(a.q), a.q_hi, U, a.slot_stride);
  double acc = 0.0;
  if (rg < nrg) {
    const double al = a.coef[U.col_off + c], w2 = ww[U.col_off + c];
    if (lz_fast(w2, al)) {
      const double b = sqrt(w2 - al * al), inv = 1.0 / b;
      if (a.ybeta) {
        // q_j stays; the next step scales it by b
        if (tile == U.tile0 && rg == 0) a.ybeta[U.col_off + c] = b;
        for (int64_t r = row0 + rg; r < row1; r += nrg) {
          const int64_t i = r * ld + c;
          y[i] = (y[i] - al * x[i]) * inv;
        }
      } else {
        for (int64_t r = row0 + rg; r < row1; r += nrg) {
          const int64_t i = r * ld + c;
          const double xv = x[i];
          y[i] = (y[i] - al * xv) * inv;
          x[i] = b * xv;
        }
      }
    } else {
      for (int64_t r = row0 + rg; r < row1; r += nrg) {
        const int64_t i = r * ld + c;
        const double wv = y[i] - al * x[i];
        y[i] = wv;
        acc = fma(wv, wv, acc);
      }
    }
  }
  red[tid] = rg < nrg ? acc : 0.0;
  int p2 = 1;
  while (p2 < nrg) p2 <<= 1;
  for (int s = p2 >> 1; s > 0; s >>= 1) {
    __syncthreads();
    if (rg < s && rg + s < nrg) red[tid] += red[tid + s * ld];
  }
  __syncthreads();
  if (tid < ld) {
    const int tl = tile - U.tile0;
    a.part_out[U.part_off + (int64_t)tid * U.ntiles + tl] = red[tid];
    a.part_out[U.part_off + (int64_t)(ld + tid) * U.ntiles + tl] = 0.0;
  }
}

// Records beta_{j+1}^2 of every column (first tile of each block) and
// finishes the columns lz_fused_kernel left, whose exact |w - alpha q_j|^2
// fixed[] holds: with beta^2 > 1e-24, y <- y / beta (= q_{j+1}) and
// x <- beta q_j (the term the next step subtracts); a column whose Krylov
// space is exhausted keeps q_j (y <- x) and drops the term (x <- 0).  The
// caller then swaps the two slots' roles.
__global__ __launch_bounds__(kThreads) void lz_fix_kernel(const LzArgs a, const double* ww,
                                                          const double* fixed, double* beta2) {
  const int tile = xcd_tile(blockIdx.x, a.grid_tiles);
  if (tile >= a.n_tiles) return;
  const UnitDev U = a.units[a.tile_unit[tile]];
  const int ld = U.ld;
  const int nrg = kThreads / ld;
  const int c = threadIdx.x % ld, rg = threadIdx.x / ld;
  if (rg >= nrg) return;
  const double al = a.coef[U.col_off + c], w2 = ww[U.col_off + c];
  const bool fast = lz_fast(w2, al);
  const double b2 = fast ? w2 - al * al : fixed[U.col_off + c];
  if (tile == U.tile0 && rg == 0) beta2[U.col_off + c] = b2;
  if (fast) return;
  double* y = lz_sel(a.w, a.w_hi, U, a.slot_stride);
  double* x = lz_sel(const_cast<double*>(a.q), a.q_hi, U, a.slot_stride);
  const int64_t row0 = a.tile_row0[tile];
  const int64_t row1 = row0 + a.tile_nrows[tile];
  const bool live = b2 > 1e-24;
  const double b = live ? sqrt(b2) : 0.0;
  const double inv = live ? 1.0 / b : 0.0;
  if (a.ybeta) {
    // q_j stays; the next step scales it by b (0: the term is dropped)
    if (tile == U.tile0 && rg == 0) a.ybeta[U.col_off + c] = b;
    for (int64_t r = row0 + rg; r < row1; r += nrg) {
      const int64_t i = r * ld + c;
      y[i] = live ? y[i] * inv : x[i];
    }
    return;
  }
  for (int64_t r = row0 + rg; r < row1; r += nrg) {
    const int64_t i = r * ld + c;
    const double xv = x[i];
    y[i] = live ? y[i] * inv : xv;
    x[i] = b * xv;
  }
}

hipError_t launch_lz_fused(const DevicePlan& p, double* vec, int y_hi, const double* alpha, const double* ww,
                           double* part_out, double* ybeta, hipStream_t st) {
  LzArgs a{};
  a.probs = p.probs;
  a.units = p.units;
  a.tile_unit = p.tile_unit;
  a.n_tiles = p.n_tiles;
  a.grid_tiles = p.grid_tiles;
  a.tile_row0 = p.tile_row0;
  a.tile_nrows = p.tile_nrows;
  a.slot_stride = p.slot_stride;
  a.w = vec;
  a.w_hi = y_hi;
  a.q = vec;
  a.q_hi = 1 - y_hi;
  a.coef = alpha;
  a.part_out = part_out;
  a.ybeta = ybeta;
  hipLaunchKernelGGL(lz_fused_kernel, dim3(p.grid_tiles), dim3(kThreads), 0, st, a, ww);
  return hipGetLastError();
}

hipError_t launch_lz_fix(const DevicePlan& p, double* vec, int y_hi, const double* alpha, const double* ww,
                         const double* fixed, double* beta2, double* ybeta, hipStream_t st) {
  LzArgs a{};
  a.probs = p.probs;
  a.units = p.units;
  a.tile_unit = p.tile_unit;
  a.n_tiles = p.n_tiles;
  a.grid_tiles = p.grid_tiles;
  a.tile_row0 = p.tile_row0;
  a.tile_nrows = p.tile_nrows;
  a.slot_stride = p.slot_stride;
  a.w = vec;
  a.w_hi = y_hi;
  a.q = vec;
  a.q_hi = 1 - y_hi;
  a.coef = alpha;
  a.ybeta = ybeta;
  hipLaunchKernelGGL(lz_fix_kernel, dim3(p.grid_tiles), dim3(kThreads), 0, st, a, ww, fixed, beta2);
  return hipGetLastError();
}

hipError_t launch_matrix(const MatrixArgs& a, size_t lds, int grid, hipStream_t st) {
  hipLaunchKernelGGL(matrix_kernel, dim3(grid), dim3(kThreads), lds, st, a);
  return hipGetLastError();
}
// Basis words of every sector, one unranking launch per sector.
__global__ __launch_bounds__(kThreads) void fill_states_kernel(const ProbDev* probs, int n_probs,
                                                              const uint32_t* binom,
                                                              uint32_t* states) {
  __shared__ uint32_t sb[kBinomN * kBinomN];
  for (int i = threadIdx.x; i < kBinomN * kBinomN; i += kThreads) sb[i] = binom[i];
  __syncthreads();
  const int p = blockIdx.y;
  const ProbDev P = probs[p];
  for (int64_t r = (int64_t)blockIdx.x * kThreads + threadIdx.x; r < P.dim;
       r += (int64_t)gridDim.x * kThreads)
    states[P.state_off + r] = unrank((uint32_t)r, P.n_sites, P.n_up, sb);
}

hipError_t fill_states(const DevicePlan& p, hipStream_t st) {
  if (!p.states || p.n_probs == 0) return hipSuccess;
  if (p.spin) return build_spin_lists(p, st);
  if (p.block >= 2) return build_tab_meta(p, st);
  hipLaunchKernelGGL(fill_states_kernel, dim3(2048, p.n_probs), dim3(kThreads), 0, st, p.probs,
                     p.n_probs, p.binom, p.states);
  return hipGetLastError();
}

}  // namespace kpm
