// C ABI of the Chebyshev-moment library (include/kpm.h): argument checks,
// planning of (problem, column block, tile) work, workspace layout, Lanczos
// bounds, the graph-segmented recursion driver and the thermodynamics calls.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <future>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <system_error>
#include <vector>

#include "kpm.h"
#include "kpm_internal.h"

using namespace kpm;

namespace {

thread_local kpm_run_stats g_stats{};

#define KPM_HIP(expr)                                  \
  do {                                                 \
    hipError_t e_ = (expr);                            \
    if (e_ != hipSuccess) return KPM_EDEVICE;          \
  } while (0)

// ------------------------------------------------------------------ host math

uint64_t binom64(int n, int k) {
  if (k < 0 || n < 0 || k > n) return 0;
  if (k > n - k) k = n - k;
  uint64_t r = 1;
  for (int i = 1; i <= k; ++i) r = r * (uint64_t)(n - k + i) / (uint64_t)i;
  return r;
}

// Spin-s sectors: 2s of a problem (1 for spin 1/2) and the counts
// cnt[i][r] of digit strings of length i (digits 0..2s) with sum r.
int two_s_of(const kpm_problem& p) { return p.two_s <= 1 ? 1 : p.two_s; }

std::vector<uint64_t> spin_counts(int N, int ts) {
  const int R1 = ts * N + 1;
  std::vector<uint64_t> cnt((size_t)(N + 1) * R1, 0);
  cnt[0] = 1;
  for (int i = 1; i <= N; ++i)
    for (int r = 0; r < R1; ++r) {
      uint64_t v = 0;
      for (int d = 0; d <= ts && d <= r; ++d) v += cnt[(size_t)(i - 1) * R1 + (r - d)];
      cnt[(size_t)i * R1 + r] = v;
    }
  return cnt;
}

// Sector dimension of a problem (C(N, n_up) for spin 1/2).
uint64_t prob_dim(const kpm_problem& p) {
  const int ts = two_s_of(p);
  if (ts == 1) return binom64(p.n_sites, p.n_up);
  if (p.n_up < 0 || p.n_up > ts * p.n_sites) return 0;
  return spin_counts(p.n_sites, ts)[(size_t)p.n_sites * (ts * p.n_sites + 1) + p.n_up];
}

// Rank table of a spin-s sector: P[i][r][d] = sum_{v < d} cnt[i][r - v].
void build_spin_table(int N, int ts, std::vector<uint32_t>& out) {
  const int R1 = ts * N + 1, B = ts + 1;
  const std::vector<uint64_t> cnt = spin_counts(N, ts);
  for (int i = 0; i < N; ++i)
    for (int r = 0; r < R1; ++r) {
      uint64_t acc = 0;
      for (int d = 0; d < B; ++d) {
        out.push_back((uint32_t)acc);
        if (r - d >= 0) acc += cnt[(size_t)i * R1 + (r - d)];
      }
    }
}

bool any_spin(const kpm_problem* p, int n) {
  for (int i = 0; p && i < n; ++i)
    if (two_s_of(p[i]) > 1) return true;
  return false;
}

std::vector<uint32_t> binom_table() {
  std::vector<uint32_t> t(kBinomN * kBinomN, 0);
  for (int n = 0; n < kBinomN; ++n)
    for (int j = 0; j < kBinomN; ++j) t[n * kBinomN + j] = (uint32_t)binom64(n, j);
  return t;
}

struct Split {
  int B0, B1, B2;
  size_t len() const { return (size_t(1) << B0) + (size_t(1) << B1) * (B0 + 1) + (size_t(1) << B2); }
};

// Three-way split of the N bits minimising the rank-table size.
Split choose_split(int N) {
  Split best{N, 0, 0};
  size_t best_len = SIZE_MAX;
  for (int B0 = 1; B0 <= N; ++B0)
    for (int B1 = 0; B0 + B1 <= N; ++B1) {
      const int B2 = N - B0 - B1;
      if (B0 + B1 > 31) continue;
      Split s{B0, B1, B2};
      if (s.len() < best_len) {
        best_len = s.len();
        best = s;
      }
    }
  return best;
}

// Rank tables of sector (N, k): rank(s) = T0[x0] + T1[x1][popc(x0)] + T2[x2]
// where each table sums C(position, index) over the set bits it covers.
void build_tables(int N, int k, Split sp, std::vector<uint32_t>& out) {
  (void)N;
  const size_t o0 = out.size();
  out.resize(o0 + sp.len(), 0u);
  uint32_t* T0 = out.data() + o0;
  uint32_t* T1 = T0 + (size_t(1) << sp.B0);
  uint32_t* T2 = T1 + (size_t(1) << sp.B1) * (sp.B0 + 1);
  for (uint32_t x = 0; x < (1u << sp.B0); ++x) {
    uint64_t r = 0;
    int j = 0;
    for (int q = 0; q < sp.B0; ++q)
      if (x >> q & 1) r += binom64(q, ++j);
    T0[x] = (uint32_t)r;
  }
  for (uint32_t x = 0; x < (1u << sp.B1); ++x)
    for (int c = 0; c <= sp.B0; ++c) {
      uint64_t r = 0;
      int j = c;
      for (int q = 0; q < sp.B1; ++q)
        if (x >> q & 1) r += binom64(sp.B0 + q, ++j);
      T1[(size_t)x * (sp.B0 + 1) + c] = (uint32_t)r;
    }
  for (uint32_t x = 0; x < (1u << sp.B2); ++x) {
    int j = k - __builtin_popcount(x);
    uint64_t r = 0;
    if (j >= 0)
      for (int q = 0; q < sp.B2; ++q)
        if (x >> q & 1) r += binom64(sp.B0 + sp.B1 + q, ++j);
    T2[x] = (uint32_t)r;
  }
}

// ------------------------------------------------------------------ validation

int check_problem(const kpm_problem& p) {
  if (p.two_s < 0 || p.two_s > 7 || p.reserved != 0) return KPM_EINVAL;
  const int ts = two_s_of(p);
  if (ts == 1) {
    if (p.n_sites < 1 || p.n_sites > 32) return KPM_EINVAL;
    if (2 * p.n_up < p.n_sites || p.n_up > p.n_sites) return KPM_EINVAL;
  } else {
    // digits in 4 bits of a 64-bit word; the digit sum is the RNG stream's 6-bit sector field
    if (p.n_sites < 1 || p.n_sites > 16 || ts * p.n_sites > 63) return KPM_EINVAL;
    if (2 * p.n_up < ts * p.n_sites || p.n_up > ts * p.n_sites) return KPM_EINVAL;
    if (prob_dim(p) >= (uint64_t(1) << 32)) return KPM_EINVAL;
  }
  if (p.n_bonds < 0 || p.n_bonds > kMaxBonds) return KPM_EINVAL;
  if (p.cluster < 0 || p.cluster > 65535) return KPM_EINVAL;
  if (p.n_bonds > 0 && (!p.bond_i || !p.bond_j || !p.J)) return KPM_EINVAL;
  for (int b = 0; b < p.n_bonds; ++b) {
    const int i = p.bond_i[b], j = p.bond_j[b];
    if (i < 0 || j < 0 || i >= p.n_sites || j >= p.n_sites || i == j) return KPM_EINVAL;
    if (!std::isfinite(p.J[b])) return KPM_EINVAL;
  }
  const bool lo_nan = std::isnan(p.e_lo), hi_nan = std::isnan(p.e_hi);
  if (!lo_nan && !hi_nan) {
    if (!std::isfinite(p.e_lo) || !std::isfinite(p.e_hi) || !(p.e_hi > p.e_lo)) return KPM_EINVAL;
  }
  return KPM_OK;
}

int check_params(const kpm_params& q) {
  if (!(q.eps >= 0.0 && q.eps < 1.0)) return KPM_EINVAL;
  if (q.M < 2 || q.M > (1 << 22)) return KPM_EINVAL;
  if (q.vec_kind < 0 || q.vec_kind > 3) return KPM_EINVAL;
  if (q.vec_kind != KPM_VEC_BASIS && (q.R < 1 || q.R > 1024)) return KPM_EINVAL;
  if (q.precision != KPM_FP64 && q.precision != KPM_FP32_STORE) return KPM_EINVAL;
  if (q.col_block < 0 || q.col_block > kMaxLd) return KPM_EINVAL;
  if (q.lanczos_steps < 0 || q.lanczos_steps > 100000) return KPM_EINVAL;
  if (!(q.bound_margin >= 0.0) || !std::isfinite(q.bound_margin)) return KPM_EINVAL;
  if (q.autotune != 0 && q.autotune != 1) return KPM_EINVAL;
  return KPM_OK;
}

// chebyshev_moments (and its allocation-free form) also take the float32 +
// residual storage; every other entry point refuses it through check_params.
int check_params_moments(const kpm_params& q) {
  if (q.precision != KPM_FP32R_STORE) return check_params(q);
  kpm_params r = q;
  r.precision = KPM_FP32_STORE;
  return check_params(r);
}

int check_problems(const kpm_problem* p, int n) {
  if (!p || n < 1) return KPM_EINVAL;
  for (int i = 0; i < n; ++i) {
    const int r = check_problem(p[i]);
    if (r != KPM_OK) return r;
  }
  return KPM_OK;
}

size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

// ------------------------------------------------------------------ planning

// Launch shape chosen by the autotuner (0 / -1 = the planner's heuristic);
// KPM_* environment variables, when set, override both.
struct Tune {
  int kernel = -1;        // -1 heuristic, 0 column-chunk, 1 row, 2 block, 3 block-table, 5 slice
  int col_block = 0;      // real columns per block
  int block_L = 0;        // low bits of a block (block kernel)
  int spt = 0;            // sub-tiles per workgroup (block kernel) / tiles' sub-tiles
  int gather_batch = 0;   // neighbour rows in flight per lane
  int lds_x = -1;         // block-table kernel: 1 rows of v_n staged in LDS, 0 not, -1 heuristic
  int rows = 0;           // slice kernel: rows per sub-tile (0 = heuristic)
  int waves = 0;          // slice kernel: waves per workgroup (0 = heuristic)
};

struct RunShape {
  Tune tune;
  int precision = KPM_FP64;
  int vec_kind = KPM_VEC_RADEMACHER;
  int R = 1;
  int col_block = 0;
  bool adjoint = false;   // block widths padded to the adjoint kernel's (1..16, power of 2)
  bool allow_row = true;  // the row kernel may run the recursion
  bool split_vectors = false;  // complex vectors may be split across blocks (one column each)
  bool allow_relabel = true;   // block kernels may relabel sites (rows then in relabelled order)
};

constexpr int kAdjMaxLd = 16;

// Columns per vector: a complex vector is two real columns (Re, Im).
int cols_per_vec(int vec_kind) { return vec_kind == KPM_VEC_COMPLEX_GAUSSIAN ? 2 : 1; }

int64_t total_columns(const kpm_problem& p, const RunShape& s) {
  if (s.vec_kind == KPM_VEC_BASIS) return (int64_t)prob_dim(p);
  return (int64_t)s.R * cols_per_vec(s.vec_kind);
}

struct Planned {
  std::vector<ProbDev> probs;
  std::vector<UnitDev> units;
  std::vector<int32_t> tile_unit, job_unit, prob_unit0, tile_nrows;
  std::vector<int64_t> tile_row0;
  std::vector<uint32_t> tables, bmask, binom;
  std::vector<double> boff, bzz;
  std::vector<uint16_t> bperm, lrank;
  std::vector<int32_t> tile_sub0, sub_nrows;
  // block-table kernel: blocks of every problem, sub-tile -> blocks, low-word tables
  std::vector<uint32_t> blk_h, blk_start;
  std::vector<int32_t> sub_blk0, sub_nblk, koff;
  std::vector<uint16_t> lunr;
  std::vector<uint32_t> cmask;        // bonds in class order (slice kernel)
  std::vector<double> coff, czz;
  std::vector<SliceWg> wg_rec;        // slice kernel: workgroup records
  DevicePlan plan;
  double bytes_per_step = 0;     // algorithmic (3 * storage * dim * real columns)
  double state_cols = 0;         // sum of dim * real columns
  // byte offsets of the packed plan arrays
  size_t o_probs, o_units, o_tile, o_job, o_pu0, o_tab, o_mask, o_off, o_zz, o_binom, o_trow0,
      o_tnrows, o_bperm, o_tsub0, o_subn, o_lrank, o_bh, o_bst, o_sb0, o_snb, o_lunr, o_koff, o_cmask,
      o_coff, o_czz, o_wgt, bytes;
};

int env_int(const char* name, int dflt) {
  const char* v = std::getenv(name);
  return v ? std::atoi(v) : dflt;
}

// Column block: all of a problem's columns up to 32 (float32 storage) or 16
// (float64), rounded to whole vectors; an explicit col_block wins.
int pick_col_block(const kpm_problem* p, int n, const RunShape& s) {
  const int cpv = cols_per_vec(s.vec_kind);
  int64_t maxc = 1;
  for (int i = 0; i < n; ++i) maxc = std::max<int64_t>(maxc, total_columns(p[i], s));
  // spin-s plans: the widest block (the per-row lists are read once per block
  // and step; measured fastest for the Fe10 wheel)
  const int dflt = any_spin(p, n) ? kMaxLd : (s.precision == KPM_FP32_STORE ? 32 : 16);
  int rb = s.col_block > 0 ? s.col_block : (s.tune.col_block > 0 ? s.tune.col_block : dflt);
  rb = (int)std::min<int64_t>(rb, maxc);
  if (!s.split_vectors) rb = (rb + cpv - 1) / cpv * cpv;
  return std::min(rb, kMaxLd);
}

// Site relabelling for the block kernels: a set S of L sites to become the low
// bits, chosen to cut few bonds (a bond with one end in S is a "mixed" bond,
// gathered row by row through the rank tables; bonds inside S stay in the
// block, bonds outside it move whole blocks).  Local search (best single swap
// between S and its complement until none lowers the cut) from the first L
// sites of a breadth-first walk from every site; the first L sites are kept
// unless a set with a strictly smaller cut is found.  S in ascending order
// gets labels 0..L-1.
//
// The high sites are then ordered for locality: states are ranked in
// ascending order of their words, so the highest labels vary slowest and a
// bond touching one of the top t sites moves a state far in rank (out of the
// range a cache holds at once).  The cost of an order is the number of bonds
// touching the top t sites, summed over t; the breadth-first order from S
// (sites bonded to S get the lowest high bits; the given order when S is the
// first L sites) is replaced by a greedy one that fills the top labels
// downwards, each time with the site having the most bonds into the sites
// already placed (ties: fewest bonds elsewhere, then lowest index), started
// from every high site, when that lowers the cost strictly.  perm[i] is the
// new label of site i; returns false when it is the identity.
bool choose_relabel(const kpm_problem& p, int L, std::vector<uint8_t>& perm) {
  const int N = p.n_sites;
  if (L <= 0 || L >= N || env_int("KPM_RELABEL", 1) == 0) return false;
  std::vector<std::vector<int>> adj(N);
  for (int k = 0; k < p.n_bonds; ++k) {
    adj[p.bond_i[k]].push_back(p.bond_j[k]);
    adj[p.bond_j[k]].push_back(p.bond_i[k]);
  }
  for (auto& a : adj) std::sort(a.begin(), a.end());
  auto cut_of = [&](const std::vector<char>& in) {
    int c = 0;
    for (int k = 0; k < p.n_bonds; ++k) c += in[p.bond_i[k]] != in[p.bond_j[k]];
    return c;
  };
  std::vector<char> best(N, 0);
  for (int i = 0; i < L; ++i) best[i] = 1;
  const int cut0 = cut_of(best);
  int best_cut = cut0;
  for (int seed = 0; seed < N; ++seed) {
    std::vector<char> in(N, 0);
    std::vector<int> order{seed};
    std::vector<char> seen(N, 0);
    seen[seed] = 1;
    for (size_t h = 0; h < order.size() && (int)order.size() < N; ++h)
      for (int v : adj[order[h]])
        if (!seen[v]) {
          seen[v] = 1;
          order.push_back(v);
        }
    for (int v = 0; v < N && (int)order.size() < N; ++v)
      if (!seen[v]) order.push_back(v);
    for (int t = 0; t < L; ++t) in[order[t]] = 1;
    int cut = cut_of(in);
    for (;;) {
      // gain of moving v across: bonds to the other side minus bonds to its own
      std::vector<int> g(N, 0);
      for (int v = 0; v < N; ++v)
        for (int u : adj[v]) g[v] += in[u] != in[v] ? 1 : -1;
      int bg = 0, ba = -1, bb = -1;
      for (int a = 0; a < N; ++a) {
        if (!in[a]) continue;
        for (int b = 0; b < N; ++b) {
          if (in[b]) continue;
          int shared = 0;
          for (int u : adj[a]) shared += u == b;
          const int gain = g[a] + g[b] - 2 * shared;
          if (gain > bg) {
            bg = gain;
            ba = a;
            bb = b;
          }
        }
      }
      if (ba < 0) break;
      in[ba] = 0;
      in[bb] = 1;
      cut -= bg;
    }
    if (cut < best_cut) {
      best_cut = cut;
      best = in;
    }
  }
  const bool moved = best_cut < cut0;
  std::vector<int> lab(N, -1);
  int next = 0;
  for (int v = 0; v < N; ++v)
    if (best[v]) lab[v] = next++;
  // high order A: breadth-first from S, or the given order when S is kept
  std::vector<int> high_a;
  if (moved) {
    std::vector<char> placed(best.begin(), best.end());
    std::vector<int> queue;
    for (int v = 0; v < N; ++v)
      if (best[v]) queue.push_back(v);
    for (size_t h = 0; h < queue.size(); ++h)
      for (int u : adj[queue[h]])
        if (!placed[u]) {
          placed[u] = 1;
          high_a.push_back(u);
          queue.push_back(u);
        }
    for (int v = 0; v < N; ++v)
      if (!placed[v]) high_a.push_back(v);
  } else {
    for (int v = 0; v < N; ++v)
      if (!best[v]) high_a.push_back(v);
  }
  // cost of a high order (lowest label first): bonds touching the top t sites, summed over t
  const int H = N - L;
  auto order_cost = [&](const std::vector<int>& high) {
    std::vector<int> rank(N, -1);   // position from the top: 0 = highest label
    for (int i = 0; i < H; ++i) rank[high[i]] = H - 1 - i;
    long c = 0;
    for (int k = 0; k < p.n_bonds; ++k) {
      int top = H;   // the bond touches the top t sites for every t > min rank
      if (rank[p.bond_i[k]] >= 0) top = std::min(top, rank[p.bond_i[k]]);
      if (rank[p.bond_j[k]] >= 0) top = std::min(top, rank[p.bond_j[k]]);
      if (top < H) c += H - 1 - top;   // t = top + 1 .. H - 1
    }
    return c;
  };
  std::vector<int> high = high_a;
  long best_cost = order_cost(high_a);
  for (int start : high_a) {
    std::vector<int> top{start};   // highest label first
    std::vector<char> placed(N, 0);
    placed[start] = 1;
    while ((int)top.size() < H) {
      int pick = -1, pin = -1, pout = 0;
      for (int v : high_a) {
        if (placed[v]) continue;
        int in_top = 0, out = 0;
        for (int u : adj[v]) (placed[u] ? in_top : out) += 1;
        if (in_top > pin || (in_top == pin && (out < pout || (out == pout && v < pick)))) {
          pick = v;
          pin = in_top;
          pout = out;
        }
      }
      placed[pick] = 1;
      top.push_back(pick);
    }
    std::vector<int> cand(top.rbegin(), top.rend());
    const long c = order_cost(cand);
    if (c < best_cost) {
      best_cost = c;
      high = cand;
    }
  }
  for (int v : high) lab[v] = next++;
  bool ident = true;
  for (int v = 0; v < N; ++v) ident = ident && lab[v] == v;
  if (ident) return false;
  perm.assign(32, 0);
  for (int v = 0; v < N; ++v) perm[v] = (uint8_t)lab[v];
  return true;
}

// Tiles of whole blocks for the block kernel: the blocks of sector (N, k)
// with L low bits, in rank order (ascending high bits h), packed greedily into
// tiles of at most `rows` states and `blk_max` blocks.
// With `blocks` the blocks themselves are listed too (high word, first rank)
// and each sub-tile's first block index and block count.
struct BlockList {
  std::vector<uint32_t> h, start;
  std::vector<int32_t> sub_b0, sub_nb;
};

void block_tiles(int N, int k, int L, int rows, int blk_max, std::vector<int64_t>& row0,
                 std::vector<int32_t>& nrows, BlockList* blocks = nullptr) {
  const uint64_t nh = 1ull << (N - L);
  int64_t start = 0, cur0 = 0;
  int cur_rows = 0, cur_blk = 0, cur_b0 = 0, nblk = 0;
  auto close = [&]() {
    row0.push_back(cur0);
    nrows.push_back(cur_rows);
    if (blocks) {
      blocks->sub_b0.push_back(cur_b0);
      blocks->sub_nb.push_back(cur_blk);
    }
  };
  for (uint64_t h = 0; h < nh; ++h) {
    const int c = k - __builtin_popcountll(h);
    if (c < 0 || c > L) continue;
    const int size = (int)binom64(L, c);
    if (cur_blk > 0 && (cur_rows + size > rows || cur_blk == blk_max)) {
      close();
      cur0 = start;
      cur_rows = 0;
      cur_blk = 0;
      cur_b0 = nblk;
    }
    if (blocks) {
      blocks->h.push_back((uint32_t)h);
      blocks->start.push_back((uint32_t)start);
    }
    cur_rows += size;
    ++cur_blk;
    ++nblk;
    start += size;
  }
  if (cur_blk > 0) close();
}

// a, b per problem must already be known (scale != nullptr) for the bond
// values; sizes do not depend on them.
// The spectral map H' = (H - b)/a (Sec. II) enters a plan only through each
// problem's diagonal shift -b/a and 1/a and the bond coefficients J/(2a),
// J/(4a), in input order and in class order.  A plan made at a = 1, b = 0
// takes its map here; make_plan applies the map the same way.
void apply_scale(const kpm_problem* p, int n, const double* a_arr, const double* b_arr, Planned& P) {
  for (int i = 0; i < n; ++i) {
    const double a = a_arr[i], b = b_arr[i];
    ProbDev& d = P.probs[i];
    d.shift = -b / a;
    d.inv_a = 1.0 / a;
    for (int k = 0; k < p[i].n_bonds; ++k) {
      P.boff[d.bond_off + k] = p[i].J[k] / (2.0 * a);
      P.bzz[d.bond_off + k] = p[i].J[k] / (4.0 * a);
    }
  }
  size_t c = 0;
  for (int i = 0; i < n; ++i)
    for (int q = 0; q < p[i].n_bonds; ++q, ++c) {
      const int b = P.probs[i].bond_off + P.bperm[P.probs[i].bond_off + q];
      P.coff[c] = P.boff[b];
      P.czz[c] = P.bzz[b];
    }
}

int make_plan(const kpm_problem* p, int n, const RunShape& s, const double* a_arr,
              const double* b_arr, Planned& P) {
  const int resid = s.precision == KPM_FP32R_STORE;
  const int fp32 = s.precision == KPM_FP32_STORE || resid;
  int rb = pick_col_block(p, n, s);
  int adj_ld = 0;
  if (s.adjoint) {
    rb = std::min(rb, kAdjMaxLd);
    adj_ld = 1;
    while (adj_ld < rb) adj_ld <<= 1;
  }
  // slice kernel (KPM_BLOCK=3 or tuned): rows of one or two 16-byte chunks, so
  // blocks of at most 8 float32 / 4 float64 columns, every unit padded to the
  // same width
  // float32 + residual storage runs on the slice kernel only (rows of 2 or 4
  // float32 columns and their residuals)
  if (resid && s.adjoint) return KPM_EINVAL;
  const bool slice_req =
      resid || (!s.adjoint && env_int("KPM_BLOCK", s.tune.kernel == 5 ? 3 : -1) == 3);
  if (slice_req) rb = std::min(rb, fp32 ? 8 : 4);
  int cpl = 1;
  if (fp32) cpl = rb >= (slice_req ? 3 : 4) ? 4 : (rb >= 2 ? 2 : 1);
  else cpl = rb >= 2 ? 2 : 1;
  if (const int f = env_int("KPM_CPL", 0)) cpl = f;
  if (resid) cpl = rb >= 3 ? 4 : 2;
  if (adj_ld) cpl = std::min(cpl, adj_ld);
  const int elt = fp32 ? 4 : 8;
  // One lane per state (row kernel) when the block width has an instantiation.
  int row_ld = 0;
  const int kern = s.tune.kernel;
  if (!s.adjoint && s.allow_row && env_int("KPM_ROW_KERNEL", kern < 0 || kern == 1 ? 1 : 0))
    for (int L : {1, 2, 4, 8})
      if (L >= rb) {
        row_ld = L;
        break;
      }

  P.binom = binom_table();
  // any spin s > 1/2: the spin kernel runs every problem of the plan
  const bool spin = any_spin(p, n);
  int max_bonds = 1, max_tab = 1;
  int64_t max_dim = 1, n_states = 0;
  size_t bond_total = 0;
  for (int i = 0; i < n; ++i) {
    ProbDev d{};
    d.dim = (int64_t)prob_dim(p[i]);
    d.n_sites = p[i].n_sites;
    d.n_up = p[i].n_up;
    d.n_bonds = p[i].n_bonds;
    d.bond_off = (int32_t)bond_total;
    d.two_s = two_s_of(p[i]);
    d.tab_off = (int32_t)P.tables.size();
    if (spin) {
      build_spin_table(p[i].n_sites, d.two_s, P.tables);
      d.tab_len = (int32_t)(P.tables.size() - d.tab_off);
    } else {
      const Split sp = choose_split(p[i].n_sites);
      d.B0 = sp.B0;
      d.B1 = sp.B1;
      d.B2 = sp.B2;
      d.tab_len = (int32_t)sp.len();
      build_tables(p[i].n_sites, p[i].n_up, sp, P.tables);
    }
    d.cluster = p[i].cluster;
    // unit map (a = 1, b = 0) here; apply_scale below sets the given one
    d.shift = 0.0;
    d.inv_a = 1.0;
    d.state_off = n_states;
    n_states += d.dim;
    for (int k = 0; k < p[i].n_bonds; ++k) {
      if (spin) P.bmask.push_back((uint32_t)p[i].bond_i[k] | ((uint32_t)p[i].bond_j[k] << 8));
      else P.bmask.push_back((1u << p[i].bond_i[k]) | (1u << p[i].bond_j[k]));
      P.boff.push_back(p[i].J[k] / 2.0);
      P.bzz.push_back(p[i].J[k] / 4.0);
    }
    bond_total += p[i].n_bonds;
    max_bonds = std::max(max_bonds, p[i].n_bonds);
    max_tab = std::max(max_tab, d.tab_len);
    max_dim = std::max(max_dim, d.dim);
    P.probs.push_back(d);
  }
  if (P.bmask.empty()) {
    P.bmask.push_back(0);
    P.boff.push_back(0);
    P.bzz.push_back(0);
  }

  DevicePlan& D = P.plan;
  D.fp32 = fp32;
  D.cpl = cpl;
  D.lds_tab = max_tab;
  D.lds_bonds = max_bonds;
  D.lds_nb = max_bonds;
  D.sub_rows = 256;
  // Prefer <= 32 KB of LDS per workgroup (occupancy) while keeping >= 64 rows
  // per sub-tile; never exceed 64 KB.
  const size_t lds_soft = (size_t)env_int("KPM_LDS_CAP", 32 * 1024);
  const size_t lds_hard = 64 * 1024;
  if (spin) {
    // spin kernel: every problem, no row/block kernels; two neighbours per bond
    if (s.adjoint) return KPM_EINVAL;
    D.spin = 1;
    D.lds_nb = 2 * max_bonds;
    while (spin_lds_bytes(D) > lds_soft && D.sub_rows > 32) D.sub_rows >>= 1;
    if (spin_lds_bytes(D) > lds_hard) return KPM_EINVAL;
    row_ld = 0;
  }
  while (!spin && step_lds_bytes(D) > lds_soft && D.sub_rows > 64) D.sub_rows >>= 1;
  while (!spin && step_lds_bytes(D) > lds_hard && D.sub_rows > 32) D.sub_rows >>= 1;
  if (s.adjoint) {
    // adjoint_kernel runs adjoint_lanes(ld) threads per state, <= kThreads per workgroup
    while (D.sub_rows * adjoint_lanes(adj_ld) > kThreads) D.sub_rows >>= 1;
    while (adjoint_lds_bytes(D) > lds_hard && D.sub_rows > 32) D.sub_rows >>= 1;
  }
  if (!spin && step_lds_bytes(D) > lds_hard) return KPM_EINVAL;
  if (s.adjoint && (adjoint_lds_bytes(D) > lds_hard || max_bonds > D.sub_rows * adjoint_lanes(adj_ld)))
    return KPM_EINVAL;
  D.row_ld = row_ld;
  if (row_ld && row_lds_bytes(D) > lds_hard) D.row_ld = row_ld = 0;
  if (row_ld) D.sub_rows = kThreads;
  D.n_states = spin ? n_states * (2 + D.lds_nb) : n_states;   // spin: digits + neighbour ranks
  D.spin_rows = spin ? n_states : 0;

  // Block kernel (tiles of whole low-bit blocks) when its LDS fits: bonds in
  // class order low-low, high-high, mixed.
  P.bperm.assign(std::max<size_t>(bond_total, 1), 0);
  for (int i = 0; i < n; ++i)
    for (int k = 0; k < p[i].n_bonds; ++k) P.bperm[P.probs[i].bond_off + k] = (uint16_t)k;
  D.block = 0;
  std::vector<std::vector<int64_t>> btile_row0(n);
  std::vector<std::vector<int32_t>> btile_nrows(n);
  std::vector<BlockList> blists(n);
  std::vector<std::vector<uint8_t>> relabels(n);
  // Default: the block-table kernel for blocks too wide for the row kernel
  // (the measured case where it is the fastest kernel); KPM_BLOCK=0/1/2 and
  // the autotuner override.
  const int block_env = resid ? 3
                              : env_int("KPM_BLOCK", kern < 0 ? -1
                                                              : (kern == 2 ? 1 : (kern == 3 ? 2 : (kern == 5 ? 3 : 0))));
  const bool block_default = rb > 8;
  // the block-table kernel addresses a block's slot with 32-bit element offsets
  int64_t max_elems = 0;
  for (int i = 0; i < n; ++i)
    max_elems = std::max<int64_t>(max_elems, (int64_t)prob_dim(p[i]) *
                                                 ((rb + cpl - 1) / cpl * cpl));
  // the slice kernel uses the block-table kernel's tiles and tables (64-bit offsets)
  const bool slice = block_env == 3;
  const bool tab =
      slice || ((block_env == 2 || (block_env < 0 && block_default)) && max_elems < (int64_t(1) << 32));
  if (!spin && !s.adjoint && s.allow_row && (block_env == 1 || tab || (block_env < 0 && block_default))) {
    D.ld_max = adj_ld ? adj_ld : (rb + cpl - 1) / cpl * cpl;
    // slice kernel: one lane per block of a sub-tile in its table pass (<= 64)
    D.blk_max = slice ? std::max(1, std::min(64, env_int("KPM_BLOCK_MAX", 64)))
                      : std::max(1, std::min(255, env_int("KPM_BLOCK_MAX", 16)));
    const size_t cap = (size_t)env_int("KPM_BLOCK_LDS", 64 * 1024);
    // rows of v_n staged in LDS: measured faster for float32 storage only
    D.tab_xl = tab && !slice ? env_int("KPM_TAB_XL", s.tune.lds_x >= 0 ? s.tune.lds_x : fp32) != 0 : 0;
    // slice kernel: sub-tiles of up to 1024 rows whose LDS copy of v_n stays
    // near 16 KB (the per-sub-tile barrier is paid once per sub-tile)
    const int rows0 = std::min(kThreads, std::max(32, env_int("KPM_BLOCK_ROWS", kThreads)));
    for (int rows = rows0; rows >= 32 && !D.block; rows >>= 1) {
      int Lm = std::max(1, std::min(env_int("KPM_BLOCK_L", s.tune.block_L > 0 ? s.tune.block_L : 9), 16));
      // slice kernel: blocks of at most 254 members (u8 LDS row numbers)
      if (slice) Lm = std::min(Lm, 10);
      while (Lm > 1 && binom64(Lm, Lm / 2) > (uint64_t)rows) --Lm;
      int lr = 1, hh = 1, mx = 1, ll = 1;
      for (int i = 0; i < n; ++i) {
        ProbDev& d = P.probs[i];
        const int L = std::min(p[i].n_sites, Lm);
        const uint32_t low = (L >= 32) ? 0xFFFFFFFFu : ((1u << L) - 1u);
        std::vector<uint8_t>& pm = relabels[i];
        pm.clear();
        // the sectors of one cluster share its bond arrays: one search per cluster
        const size_t nbb = (size_t)p[i].n_bonds * sizeof(int32_t);
        const int j = i > 0 && p[i - 1].n_bonds == p[i].n_bonds && p[i - 1].n_sites == p[i].n_sites &&
                              (nbb == 0 || (std::memcmp(p[i - 1].bond_i, p[i].bond_i, nbb) == 0 &&
                                            std::memcmp(p[i - 1].bond_j, p[i].bond_j, nbb) == 0))
                          ? i - 1
                          : -1;
        if (j >= 0) pm = relabels[j];
        else if (s.allow_relabel) choose_relabel(p[i], L, pm);
        auto lab = [&](int site) { return pm.empty() ? site : (int)pm[site]; };
        std::vector<uint16_t> cls[3];
        for (int k = 0; k < p[i].n_bonds; ++k) {
          const uint32_t m = (1u << lab(p[i].bond_i[k])) | (1u << lab(p[i].bond_j[k]));
          const int c = (m & ~low) == 0 ? 0 : ((m & low) == 0 ? 1 : 2);
          cls[c].push_back((uint16_t)k);
        }
        d.blk_L = L;
        d.n_ll = (int32_t)cls[0].size();
        d.n_hh = (int32_t)cls[1].size();
        d.n_mx = (int32_t)cls[2].size();
        int q = d.bond_off;
        for (auto& v : cls)
          for (uint16_t b : v) P.bperm[q++] = b;
        lr = std::max(lr, 1 << L);
        hh = std::max(hh, d.n_hh);
        mx = std::max(mx, d.n_mx);
        ll = std::max(ll, d.n_ll);
      }
      D.blk_rows = rows;
      D.lds_lr = lr;
      D.lds_hh = hh;
      D.lds_mx = mx;
      D.lds_ll = ll;
      // the block-table kernel packs (row, low-low bond) into 16 bits
      if (slice) {
        // word rows must hold each problem's mixed and low-low bonds, and a
        // slot must fit 32-bit buffer offsets
        int wb = 32, brows = 1;
        bool ok = (int64_t)max_elems * elt < (int64_t(1) << 32);
        // every unit is padded to the same width, 1 or 2 chunks of cpl columns
        const int nchu = D.ld_max / cpl;
        ok = ok && !adj_ld && (nchu == 1 || (nchu == 2 && cpl == (fp32 ? 4 : 2)));
        for (int i = 0; i < n && ok; ++i) {
          const int w = slice_word_bytes(P.probs[i].n_mx, P.probs[i].n_ll);
          ok = w > 0;
          wb = std::max(wb, w);
          brows = std::max(brows, (int)binom64(P.probs[i].blk_L, P.probs[i].blk_L / 2));
        }
        D.slice_wb = wb;
        D.slice_words = lr;
        D.blk_lds_rows = brows;
        if (ok && brows <= 254 && slice_lds_bytes(D) <= cap) {
          D.block = 3;
        } else {
          D.slice_wb = D.slice_words = D.blk_lds_rows = 0;
          break;
        }
      } else if ((tab ? tab_lds_bytes(D) : block_lds_bytes(D)) <= cap && (!tab || ll <= 255)) {
        D.block = tab ? 2 : 1;
      }
    }
  }
  int bspt = 1;
  if (resid && (D.block != 3 || spin)) return KPM_EINVAL;   // no slice plan for these problems
  D.resid = resid;
  if (D.block) D.row_ld = row_ld = 0;
  // relabelled sites: the kernels see the bonds (and so every word) in the new labels
  for (int i = 0; D.block && i < n; ++i) {
    if (relabels[i].empty()) continue;
    ProbDev& d = P.probs[i];
    d.relabel = 1;
    for (int t = 0; t < 32; ++t) d.perm[t] = relabels[i][t];
    for (int k = 0; k < p[i].n_bonds; ++k)
      P.bmask[d.bond_off + k] = (1u << relabels[i][p[i].bond_i[k]]) | (1u << relabels[i][p[i].bond_j[k]]);
  }
  // Neighbour rows in flight per lane: row kernel 2/4/8, others 4/8.
  D.gather_batch = (row_ld == 4 || row_ld == 8) ? 2 : 4;
  if (s.tune.gather_batch > 0) D.gather_batch = s.tune.gather_batch;
  if (const int f = env_int("KPM_GATHER_BATCH", 0)) D.gather_batch = f;
  if (D.gather_batch != 2 && D.gather_batch != 4 && D.gather_batch != 8) D.gather_batch = 4;
  if (!row_ld && D.gather_batch < 4) D.gather_batch = 4;
  // slice kernel: high-high rows in flight per lane per batch (4 or 8; default 8)
  if (D.block == 3) {
    D.gather_batch = s.tune.gather_batch > 0 ? s.tune.gather_batch : 8;
    if (const int f = env_int("KPM_GATHER_BATCH", 0)) D.gather_batch = f;
    if (D.gather_batch != 4) D.gather_batch = 8;
  }
  if (D.block) {
    D.row_ld = row_ld = 0;
    size_t max_sub = 1;
    int maxL = 1;
    for (int i = 0; i < n; ++i) {
      BlockList* bl = nullptr;
      if (D.block >= 2) {
        bl = &blists[i];
        P.probs[i].blk_off = (int32_t)P.blk_h.size();
      }
      block_tiles(p[i].n_sites, p[i].n_up, P.probs[i].blk_L, D.blk_rows, D.blk_max, btile_row0[i],
                  btile_nrows[i], bl);
      if (bl) {
        if (P.blk_h.size() + bl->h.size() > (size_t)INT32_MAX) return KPM_EINVAL;
        P.probs[i].n_blk = (int32_t)bl->h.size();
        P.blk_h.insert(P.blk_h.end(), bl->h.begin(), bl->h.end());
        P.blk_start.insert(P.blk_start.end(), bl->start.begin(), bl->start.end());
      }
      max_sub = std::max(max_sub, btile_row0[i].size());
      maxL = std::max(maxL, P.probs[i].blk_L);
    }
    // colex rank of every low word among the words of its popcount
    P.lrank.assign(size_t(1) << maxL, 0);
    for (uint32_t l = 0; l < (1u << maxL); ++l) {
      uint64_t r = 0;
      int j = 0;
      for (int q = 0; q < maxL; ++q)
        if ((l >> q) & 1u) r += binom64(q, ++j);
      P.lrank[l] = (uint16_t)r;
    }
    if (D.block >= 2) {
      // low words by popcount class, each class in colex order (its first
      // C(L, k) entries are the L-bit words for any L <= maxL)
      P.koff.assign(kKoffLen, 0);
      for (int k = 0; k + 1 < kKoffLen; ++k)
        P.koff[k + 1] = P.koff[k] + (k <= maxL ? (int32_t)binom64(maxL, k) : 0);
      P.lunr.assign(size_t(1) << maxL, 0);
      for (uint32_t l = 0; l < (1u << maxL); ++l)
        P.lunr[P.koff[__builtin_popcount(l)] + P.lrank[l]] = (uint16_t)l;
      D.meta_hh = D.lds_hh;
      D.meta_mx = D.lds_mx;
      D.n_blk = (int32_t)P.blk_h.size();
    }
    // Sub-tiles per workgroup: amortise the per-workgroup LDS fill (tables,
    // bonds, ranks) over the streamed rows, keeping >= 2048 workgroups on the
    // largest problem.
    const double fixed = (double)max_tab * 4 + (double)max_bonds * 20 + (double)(size_t(2) << maxL);
    const double per_sub = 3.0 * D.blk_rows * D.ld_max * elt;
    int spt = (int)std::ceil(8.0 * fixed / per_sub);
    spt = (int)std::max<size_t>(1, std::min<size_t>((size_t)spt, std::max<size_t>(1, max_sub / 2048)));
    // slice kernel: about 1000 rows per one-wave workgroup (no per-tile LDS fill)
    if (D.block == 3) spt = 4;
    if (s.tune.spt > 0) spt = s.tune.spt;
    if (const int f = env_int("KPM_SUB_PER_TILE", 0)) spt = f;
    bspt = std::max(1, std::min(spt, 64));
  }

  // Rows per workgroup tile: enough rows to amortise the per-tile LDS fill,
  // but keep >= 2048 tiles on the largest block when its size permits.
  const size_t fixed = (row_ld ? 0 : kBinomN * kBinomN * 4) + (size_t)max_tab * 4 + (size_t)max_bonds * 20;
  const int ldmax = row_ld ? row_ld : (rb + cpl - 1) / cpl * cpl;
  const double per_row = 3.0 * ldmax * elt;
  int spt = (int)std::ceil(16.0 * fixed / (per_row * D.sub_rows));
  const int64_t par = max_dim / (2048LL * D.sub_rows);
  spt = (int)std::max<int64_t>(1, std::min<int64_t>(spt, std::max<int64_t>(1, par)));
  spt = std::min(spt, 64);
  if (s.tune.spt > 0) spt = s.tune.spt;
  if (const int f = env_int("KPM_SUB_PER_TILE", 0)) spt = f;
  D.sub_per_tile = spt;
  // slice kernel: every XCD on the same column block at a time (measured 4 %
  // faster on the 24-site ring than contiguous tile ranges per XCD)
  D.xcd_remap = env_int("KPM_XCD_REMAP", D.block == 3 ? 2 : 1);
  D.dense = env_int("KPM_DENSE_LISTS", 0);
  const int64_t tile_rows = (int64_t)D.sub_rows * spt;

  int64_t vec_elems = 0, part_len = 0, bd_len = 0;
  int32_t tiles = 0, col_off = 0;
  for (int i = 0; i < n; ++i) {
    P.prob_unit0.push_back((int32_t)P.units.size());
    const int64_t nc = total_columns(p[i], s);
    const int64_t dim = P.probs[i].dim;
    for (int64_t c0 = 0; c0 < nc; c0 += rb) {
      UnitDev u{};
      u.prob = i;
      u.ncols = (int32_t)std::min<int64_t>(rb, nc - c0);
      u.ld = adj_ld ? adj_ld : (row_ld ? row_ld : (u.ncols + cpl - 1) / cpl * cpl);
      if (D.block == 3) u.ld = D.ld_max;   // the slice kernel's width is a template constant
      u.col0 = (int32_t)c0;
      u.vec_off = vec_elems;
      vec_elems += (int64_t)align_up((size_t)(dim * u.ld), 64);
      u.ntiles = D.block ? (int32_t)((btile_row0[i].size() + bspt - 1) / bspt)
                         : (int32_t)((dim + tile_rows - 1) / tile_rows);
      u.tile0 = tiles;
      u.part_off = part_len;
      part_len += (int64_t)2 * u.ld * u.ntiles;
      u.bd_off = bd_len;
      bd_len += (int64_t)u.ntiles * std::max(1, p[i].n_bonds);
      u.col_off = col_off;
      for (int t = 0; t < u.ntiles; ++t) {
        P.tile_unit.push_back((int32_t)P.units.size());
        if (D.block) {
          const size_t s0 = (size_t)t * bspt;
          const size_t s1 = std::min(s0 + bspt, btile_row0[i].size());
          int32_t rows = 0;
          P.tile_sub0.push_back((int32_t)P.sub_nrows.size());
          for (size_t k = s0; k < s1; ++k) {
            P.sub_nrows.push_back(btile_nrows[i][k]);
            rows += btile_nrows[i][k];
            if (D.block >= 2) {
              P.sub_blk0.push_back(P.probs[i].blk_off + blists[i].sub_b0[k]);
              P.sub_nblk.push_back(blists[i].sub_nb[k]);
            }
          }
          P.tile_row0.push_back(btile_row0[i][s0]);
          P.tile_nrows.push_back(rows);
        } else {
          P.tile_row0.push_back((int64_t)t * tile_rows);
          P.tile_nrows.push_back((int32_t)std::min<int64_t>(tile_rows, dim - (int64_t)t * tile_rows));
        }
      }
      for (int j = 0; j < 2 * u.ld; ++j) P.job_unit.push_back((int32_t)P.units.size());
      tiles += u.ntiles;
      col_off += u.ld;
      P.bytes_per_step += 3.0 * (resid ? 6 : elt) * (double)dim * u.ncols;
      P.state_cols += (double)dim * u.ncols;
      P.units.push_back(u);
    }
  }
  P.prob_unit0.push_back((int32_t)P.units.size());
  // the row and block kernels also stream the 4-byte state word of every row;
  // the block-table kernel reads its per-block tables instead
  // the per-block table layout depends on the problem count (word tables)
  D.n_probs = n;
  if (D.block >= 2) {
    for (const auto& u : P.units) {
      const ProbDev& d = P.probs[u.prob];
      if (D.block == 3)   // slice kernel: per block its record, targets, coefficients; per unit the word table
        P.bytes_per_step += (double)d.n_blk * (sizeof(SliceBlk) + 12.0 * d.n_hh + 4.0 * d.n_mx) +
                            (double)(1u << d.blk_L) * D.slice_wb;
      else
        P.bytes_per_step += (double)d.n_blk * (12.0 + 6.0 * d.n_hh + 4.0 * d.n_mx);
    }
    D.n_states = (int64_t)((tab_meta_bytes(D) + 3) / 4);
  } else if (D.row_ld || D.block) {
    for (const auto& u : P.units) P.bytes_per_step += 4.0 * (double)P.probs[u.prob].dim;
  } else if (D.spin) {
    // the spin kernel reads each row's digit string and its neighbour-rank slots
    for (const auto& u : P.units) {
      const ProbDev& d = P.probs[u.prob];
      P.bytes_per_step += (8.0 + 8.0 * d.n_bonds) * (double)d.dim;
    }
  }
  // bonds in class order (the slice kernel reads them with scalar loads)
  for (int i = 0; i < n; ++i)
    for (int q = 0; q < p[i].n_bonds; ++q) {
      const int b = P.probs[i].bond_off + P.bperm[P.probs[i].bond_off + q];
      P.cmask.push_back(P.bmask[b]);
      P.coff.push_back(P.boff[b]);
      P.czz.push_back(P.bzz[b]);
    }
  // zeros past the last bond: the slice kernel reads a few entries past a
  // problem's class ranges and uses them with zero weight
  for (int t = 0; t < 16; ++t) {
    P.cmask.push_back(0);
    P.coff.push_back(0);
    P.czz.push_back(0);
  }
  P.tile_sub0.push_back((int32_t)P.sub_nrows.size());
  if (P.sub_nrows.empty()) P.sub_nrows.push_back(0);
  if (P.lrank.empty()) P.lrank.push_back(0);
  D.n_probs = n;
  D.n_units = (int32_t)P.units.size();
  D.n_tiles = tiles;
  D.grid_tiles = (tiles + 7) / 8 * 8;
  // Slice kernel: one record per workgroup (its tile, column block, problem
  // and block range).  KPM_XCD_REMAP=2 (default): each column block's tiles
  // in 8 contiguous chunks, chunk x to XCD x (workgroup b runs on XCD b mod
  // 8), column blocks one after the other, so that all XCDs sweep the same
  // column block at a time; 1: contiguous tile ranges per XCD; 0: in order.
  P.wg_rec.clear();
  D.slice_grid = 0;
  if (D.block == 3) {
    auto rec = [&](int t) {
      SliceWg w{};
      w.tile = -1;
      if (t >= 0 && t < tiles) {
        const UnitDev& u = P.units[P.tile_unit[t]];
        const int s0 = P.tile_sub0[t], s1 = P.tile_sub0[t + 1];
        w.tile = t;
        w.unit = P.tile_unit[t];
        w.prob = u.prob;
        w.g0 = P.sub_blk0[s0];
        w.ng = P.sub_blk0[s1 - 1] + P.sub_nblk[s1 - 1] - w.g0;
      }
      return w;
    };
    if (D.xcd_remap == 2) {
      for (const UnitDev& u : P.units) {
        const int c = (u.ntiles + 7) / 8;
        for (int j = 0; j < c; ++j)
          for (int x = 0; x < 8; ++x) P.wg_rec.push_back(rec(x * c + j < u.ntiles ? u.tile0 + x * c + j : -1));
      }
    } else {
      const int per = D.grid_tiles / 8;
      for (int b = 0; b < D.grid_tiles; ++b)
        P.wg_rec.push_back(rec(D.xcd_remap ? (b & 7) * per + (b >> 3) : b));
    }
    if (P.wg_rec.empty() || P.wg_rec.size() > (size_t)INT32_MAX) return KPM_EINVAL;
    D.slice_grid = (int32_t)P.wg_rec.size();
    // waves per workgroup: 2 (default) or 4 share a tile (rows of 16 or 32
    // bytes staged by direct loads, or float32 + residual rows decoded
    // through registers; the tile's rows within the LDS limit), else 1.  On the 24-site ring (20 float32 columns in blocks of 4) two
    // waves per tile took 290-297 us per step against 307-311 us for one.
    D.slice_tile_rows = 0;
    for (int32_t r : P.tile_nrows) D.slice_tile_rows = std::max(D.slice_tile_rows, r);
    int nw = s.tune.waves > 0 ? s.tune.waves : 2;
    if (const int f = env_int("KPM_SLICE_WAVES", 0)) nw = f;
    if (nw != 2 && nw != 4) nw = 1;
    const size_t rowb = (size_t)D.ld_max * (fp32 ? 4 : 8);
    D.slice_nw = nw;
    if (nw > 1 && ((!resid && rowb % 16 != 0) || slice_lds_bytes(D) > (size_t)env_int("KPM_BLOCK_LDS", 64 * 1024)))
      D.slice_nw = 1;
  }
  D.total_cols = col_off;
  D.part_len = std::max<int64_t>(part_len, 1);
  D.slot_stride = vec_elems;
  D.vec_elems = 2 * vec_elems;
  D.bd_len = std::max<int64_t>(bd_len, 1);

  size_t o = 0;
  auto put = [&](size_t bytes) {
    const size_t r = o;
    o = align_up(o + bytes);
    return r;
  };
  P.o_probs = put(P.probs.size() * sizeof(ProbDev));
  P.o_units = put(P.units.size() * sizeof(UnitDev));
  P.o_tile = put(P.tile_unit.size() * 4);
  P.o_job = put(P.job_unit.size() * 4);
  P.o_pu0 = put(P.prob_unit0.size() * 4);
  P.o_tab = put(P.tables.size() * 4);
  P.o_mask = put(P.bmask.size() * 4);
  P.o_off = put(P.boff.size() * 8);
  P.o_zz = put(P.bzz.size() * 8);
  P.o_binom = put(P.binom.size() * 4);
  P.o_trow0 = put(P.tile_row0.size() * 8);
  P.o_tnrows = put(P.tile_nrows.size() * 4);
  P.o_bperm = put(P.bperm.size() * 2);
  P.o_tsub0 = put(P.tile_sub0.size() * 4);
  P.o_subn = put(P.sub_nrows.size() * 4);
  P.o_lrank = put(P.lrank.size() * 2);
  P.o_bh = put(P.blk_h.size() * 4);
  P.o_bst = put(P.blk_start.size() * 4);
  P.o_sb0 = put(P.sub_blk0.size() * 4);
  P.o_snb = put(P.sub_nblk.size() * 4);
  P.o_lunr = put(P.lunr.size() * 2);
  P.o_koff = put(P.koff.size() * 4);
  P.o_cmask = put(P.cmask.size() * 4);
  P.o_coff = put(P.coff.size() * 8);
  P.o_czz = put(P.czz.size() * 8);
  P.o_wgt = put(P.wg_rec.size() * sizeof(SliceWg));
  P.bytes = o;
  if (a_arr && b_arr) apply_scale(p, n, a_arr, b_arr, P);
  return KPM_OK;
}

// Copy the plan arrays to `dst` (device) and point the DevicePlan at them.
int upload_plan(Planned& P, unsigned char* dst, std::vector<unsigned char>& staging,
                hipStream_t st) {
  staging.assign(P.bytes, 0);
  auto cp = [&](size_t off, const void* src, size_t bytes) {
    if (bytes) std::memcpy(staging.data() + off, src, bytes);
  };
  cp(P.o_probs, P.probs.data(), P.probs.size() * sizeof(ProbDev));
  cp(P.o_units, P.units.data(), P.units.size() * sizeof(UnitDev));
  cp(P.o_tile, P.tile_unit.data(), P.tile_unit.size() * 4);
  cp(P.o_job, P.job_unit.data(), P.job_unit.size() * 4);
  cp(P.o_pu0, P.prob_unit0.data(), P.prob_unit0.size() * 4);
  cp(P.o_tab, P.tables.data(), P.tables.size() * 4);
  cp(P.o_mask, P.bmask.data(), P.bmask.size() * 4);
  cp(P.o_off, P.boff.data(), P.boff.size() * 8);
  cp(P.o_zz, P.bzz.data(), P.bzz.size() * 8);
  cp(P.o_binom, P.binom.data(), P.binom.size() * 4);
  cp(P.o_trow0, P.tile_row0.data(), P.tile_row0.size() * 8);
  cp(P.o_tnrows, P.tile_nrows.data(), P.tile_nrows.size() * 4);
  cp(P.o_bperm, P.bperm.data(), P.bperm.size() * 2);
  cp(P.o_tsub0, P.tile_sub0.data(), P.tile_sub0.size() * 4);
  cp(P.o_subn, P.sub_nrows.data(), P.sub_nrows.size() * 4);
  cp(P.o_lrank, P.lrank.data(), P.lrank.size() * 2);
  cp(P.o_bh, P.blk_h.data(), P.blk_h.size() * 4);
  cp(P.o_bst, P.blk_start.data(), P.blk_start.size() * 4);
  cp(P.o_sb0, P.sub_blk0.data(), P.sub_blk0.size() * 4);
  cp(P.o_snb, P.sub_nblk.data(), P.sub_nblk.size() * 4);
  cp(P.o_lunr, P.lunr.data(), P.lunr.size() * 2);
  cp(P.o_koff, P.koff.data(), P.koff.size() * 4);
  cp(P.o_cmask, P.cmask.data(), P.cmask.size() * 4);
  cp(P.o_coff, P.coff.data(), P.coff.size() * 8);
  cp(P.o_czz, P.czz.data(), P.czz.size() * 8);
  cp(P.o_wgt, P.wg_rec.data(), P.wg_rec.size() * sizeof(SliceWg));
  KPM_HIP(hipMemcpyAsync(dst, staging.data(), P.bytes, hipMemcpyHostToDevice, st));
  DevicePlan& D = P.plan;
  D.probs = reinterpret_cast<ProbDev*>(dst + P.o_probs);
  D.units = reinterpret_cast<UnitDev*>(dst + P.o_units);
  D.tile_unit = reinterpret_cast<int32_t*>(dst + P.o_tile);
  D.job_unit = reinterpret_cast<int32_t*>(dst + P.o_job);
  D.prob_unit0 = reinterpret_cast<int32_t*>(dst + P.o_pu0);
  D.tables = reinterpret_cast<uint32_t*>(dst + P.o_tab);
  D.bmask = reinterpret_cast<uint32_t*>(dst + P.o_mask);
  D.boff = reinterpret_cast<double*>(dst + P.o_off);
  D.bzz = reinterpret_cast<double*>(dst + P.o_zz);
  D.binom = reinterpret_cast<uint32_t*>(dst + P.o_binom);
  D.tile_row0 = reinterpret_cast<int64_t*>(dst + P.o_trow0);
  D.tile_nrows = reinterpret_cast<int32_t*>(dst + P.o_tnrows);
  D.bperm = reinterpret_cast<uint16_t*>(dst + P.o_bperm);
  D.tile_sub0 = reinterpret_cast<int32_t*>(dst + P.o_tsub0);
  D.sub_nrows = reinterpret_cast<int32_t*>(dst + P.o_subn);
  D.lrank = reinterpret_cast<uint16_t*>(dst + P.o_lrank);
  D.blk_h = reinterpret_cast<uint32_t*>(dst + P.o_bh);
  D.blk_start = reinterpret_cast<uint32_t*>(dst + P.o_bst);
  D.sub_blk0 = reinterpret_cast<int32_t*>(dst + P.o_sb0);
  D.sub_nblk = reinterpret_cast<int32_t*>(dst + P.o_snb);
  D.lunr = reinterpret_cast<uint16_t*>(dst + P.o_lunr);
  D.koff = reinterpret_cast<int32_t*>(dst + P.o_koff);
  D.cmask = reinterpret_cast<uint32_t*>(dst + P.o_cmask);
  D.coff = reinterpret_cast<double*>(dst + P.o_coff);
  D.czz = reinterpret_cast<double*>(dst + P.o_czz);
  D.wg_rec = P.wg_rec.empty() ? nullptr : reinterpret_cast<SliceWg*>(dst + P.o_wgt);
  return KPM_OK;
}

// Synchronises the stream when an entry point returns, so that host staging
// buffers of asynchronous copies outlive the copies on every return path.
struct StreamSync {
  hipStream_t st;
  ~StreamSync() { (void)hipStreamSynchronize(st); }
};

// Device memory owned by the library for one call.
struct DevBuf {
  void* p = nullptr;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
  int alloc(size_t bytes) {
    if (hipMalloc(&p, bytes ? bytes : 256) != hipSuccess) {
      p = nullptr;
      return KPM_ENOMEM;
    }
    return KPM_OK;
  }
};

// ------------------------------------------------------------- Lanczos bounds

struct LzLayout {
  size_t plan, vec, part, dots, b2, norm, ww, fixed, ybeta, err, states, total;
};

LzLayout lanczos_layout(const Planned& P, int steps) {
  LzLayout L{};
  size_t o = 0;
  auto put = [&](size_t bytes) {
    const size_t r = o;
    o = align_up(o + bytes);
    return r;
  };
  L.plan = put(P.bytes);
  L.vec = put((size_t)P.plan.vec_elems * 8);
  L.part = put((size_t)P.plan.part_len * 8);
  L.dots = put((size_t)steps * P.plan.total_cols * 8);
  L.b2 = put((size_t)steps * P.plan.total_cols * 8);
  L.norm = put((size_t)P.plan.total_cols * 8);
  L.ww = put((size_t)P.plan.total_cols * 8);
  L.fixed = put((size_t)P.plan.total_cols * 8);
  L.ybeta = put((size_t)P.plan.total_cols * 8);
  L.err = put(256);
  L.states = put((size_t)P.plan.n_states * 4);
  L.total = o;
  return L;
}

// Lanczos bounds: one float64 column per problem, on the slice kernel for
// spin-1/2 problems (the planner falls back to the other kernels where it
// does not apply)
RunShape lanczos_shape(const kpm_problem* p, int n) {
  RunShape s;
  s.precision = KPM_FP64;
  s.vec_kind = KPM_VEC_RADEMACHER;
  s.R = 1;
  s.col_block = 1;
  if (!any_spin(p, n)) {
    s.tune.kernel = 5;
    s.tune.block_L = 10;
    s.tune.spt = 2;
    s.tune.gather_batch = 4;
  }
  return s;
}

size_t lanczos_bytes(const kpm_problem* p, int n, int steps) {
  Planned P;
  if (make_plan(p, n, lanczos_shape(p, n), nullptr, nullptr, P) != KPM_OK) return 0;
  return lanczos_layout(P, steps).total;
}

// Extreme eigenvalues of the symmetric tridiagonal (diag a, off b) by
// bisection on Sturm counts.
double tri_count_below(const std::vector<double>& a, const std::vector<double>& b, double x) {
  int cnt = 0;
  double q = 1.0;
  for (size_t i = 0; i < a.size(); ++i) {
    const double bb = i ? b[i - 1] * b[i - 1] : 0.0;
    q = a[i] - x - (i ? bb / q : 0.0);
    if (q == 0.0) q = -1e-300;
    if (q < 0) ++cnt;
  }
  return cnt;
}

void tri_extremes(const std::vector<double>& a, const std::vector<double>& b, double& lo,
                  double& hi) {
  double gl = INFINITY, gu = -INFINITY;
  for (size_t i = 0; i < a.size(); ++i) {
    const double r = (i ? std::fabs(b[i - 1]) : 0.0) + (i < b.size() ? std::fabs(b[i]) : 0.0);
    gl = std::min(gl, a[i] - r);
    gu = std::max(gu, a[i] + r);
  }
  const int n = (int)a.size();
  auto kth = [&](int k) {   // k-th smallest (0-based)
    double l = gl, u = gu;
    for (int it = 0; it < 200; ++it) {
      const double m = 0.5 * (l + u);
      if (m <= l || m >= u) break;
      if (tri_count_below(a, b, m) > k) u = m;
      else l = m;
    }
    return 0.5 * (l + u);
  };
  lo = kth(0);
  hi = kth(n - 1);
}

// Lanczos recursion, every column its own (the spectral bounds of Eqs. (4)-(5)
// below and the FTLM that Sec. III.C compares against), on
// a plan of H' = H/2 whose two slots hold the unit start columns (slot 0) and
// zeros (slot 1).  Slot x holds q_j, slot y beta_j q_{j-1} (0 at j = 0).  One
// recursion step gives w_j = 2 H' q_j - y = H q_j - beta_j q_{j-1},
// alpha_j = <w_j, q_j> and <w_j, w_j>; then w_j -= alpha_j q_j with
// beta_{j+1}^2 = |w_j|^2, q_{j+1} = w_j / beta_{j+1} in slot y and
// beta_{j+1} q_j in slot x (one sweep where <w,w> - alpha^2 is safe, else an
// exact second pass), and the slots' roles swap.  On a float64 slice plan
// slot x keeps q_j instead and the next step scales it by beta_{j+1} (ybeta),
// the same product rounded the same way, so that the turn writes one vector
// instead of two.  alpha_j goes to dots[j], beta_{j+1}^2 to b2[j] (rows of
// total_cols); ww and fixed hold <w, w> and the exact |w - alpha q|^2 of the
// columns finished slowly; ybeta is total_cols doubles.
int lanczos_turns(const DevicePlan& D, double* vec, double* part, double* dots, double* b2, double* ww,
                  double* fixed, double* ybeta_buf, int steps, hipStream_t st) {
  const int TC = D.total_cols;
  double* ybeta = D.block == 3 && !D.fp32 ? ybeta_buf : nullptr;
  if (ybeta) KPM_HIP(hipMemsetAsync(ybeta, 0, (size_t)TC * 8, st));
  int px = 0;
  for (int j = 0; j < steps; ++j) {
    if (ybeta) KPM_HIP(launch_step_scaled(D, vec, part, px, ybeta, st));
    else KPM_HIP(launch_step(D, vec, part, nullptr, 0, nullptr, nullptr, nullptr, 0, px, 0, st));
    KPM_HIP(launch_reduce(D, part, ww, dots + (size_t)j * TC, st));
    KPM_HIP(launch_lz_fused(D, vec, 1 - px, dots + (size_t)j * TC, ww, part, ybeta, st));
    KPM_HIP(launch_reduce(D, part, fixed, nullptr, st));
    KPM_HIP(launch_lz_fix(D, vec, 1 - px, dots + (size_t)j * TC, ww, fixed, b2 + (size_t)j * TC, ybeta, st));
    px = 1 - px;
  }
  return KPM_OK;
}

// Batched Lanczos over every problem (one float64 column each), the recursion
// of lanczos_turns on H' = H/2.
int run_lanczos(const kpm_problem* p, int n, int steps, double margin, uint64_t seed,
                double* e_lo_hi, unsigned char* work, hipStream_t st) {
  Planned P;
  const std::vector<double> two(n, 2.0), zero_b(n, 0.0);
  int r = make_plan(p, n, lanczos_shape(p, n), two.data(), zero_b.data(), P);
  if (r != KPM_OK) return r;
  for (auto& u : P.units) u.col0 = 1023;   // RNG stream r = 1023 for the start vector
  int64_t max_dim = 1;
  for (auto& d : P.probs) max_dim = std::max(max_dim, d.dim);
  const int nsteps = (int)std::max<int64_t>(1, std::min<int64_t>(steps, max_dim));
  const LzLayout L = lanczos_layout(P, nsteps);
  std::vector<unsigned char> staging;
  r = upload_plan(P, work + L.plan, staging, st);
  if (r != KPM_OK) return r;
  DevicePlan& D = P.plan;
  D.err = reinterpret_cast<int*>(work + L.err);
  D.states = reinterpret_cast<uint32_t*>(work + L.states);
  KPM_HIP(hipMemsetAsync(D.err, 0, sizeof(int), st));
  if (D.row_ld || D.block || D.spin) KPM_HIP(fill_states(D, st));
  double* vec = reinterpret_cast<double*>(work + L.vec);
  double* part = reinterpret_cast<double*>(work + L.part);
  double* dots = reinterpret_cast<double*>(work + L.dots);
  double* b2 = reinterpret_cast<double*>(work + L.b2);
  const int TC = D.total_cols;
  KPM_HIP(hipMemsetAsync(vec, 0, (size_t)D.vec_elems * 8, st));
  // unit-norm real Gaussian start vector (RNG stream r = 1023)
  double* norm = reinterpret_cast<double*>(work + L.norm);
  KPM_HIP(launch_init(D, vec, 0, KPM_VEC_GAUSSIAN, seed, nullptr, part, st));
  KPM_HIP(launch_reduce(D, part, norm, nullptr, st));
  KPM_HIP(launch_init(D, vec, 2, KPM_VEC_GAUSSIAN, seed, norm, part, st));
  r = lanczos_turns(D, vec, part, dots, b2, reinterpret_cast<double*>(work + L.ww),
                    reinterpret_cast<double*>(work + L.fixed), reinterpret_cast<double*>(work + L.ybeta), nsteps, st);
  if (r != KPM_OK) return r;
  std::vector<double> h_dots((size_t)nsteps * TC), h_b2((size_t)nsteps * TC);
  int h_err = 0;
  KPM_HIP(hipMemcpyAsync(h_dots.data(), dots, h_dots.size() * 8, hipMemcpyDeviceToHost, st));
  KPM_HIP(hipMemcpyAsync(h_b2.data(), b2, h_b2.size() * 8, hipMemcpyDeviceToHost, st));
  KPM_HIP(hipMemcpyAsync(&h_err, D.err, sizeof(int), hipMemcpyDeviceToHost, st));
  KPM_HIP(hipStreamSynchronize(st));
  if (h_err) return KPM_EDEVICE;
  for (int i = 0; i < n; ++i) {
    const int col = P.units[P.prob_unit0[i]].col_off;
    const int steps_i = (int)std::min<int64_t>(steps, P.probs[i].dim);
    std::vector<double> av, bv;
    for (int j = 0; j < steps_i; ++j) {
      av.push_back(h_dots[(size_t)j * TC + col]);
      const double bn = std::sqrt(std::max(h_b2[(size_t)j * TC + col], 0.0));
      if (j == steps_i - 1 || bn < 1e-12) break;
      bv.push_back(bn);
    }
    double lo, hi;
    tri_extremes(av, bv, lo, hi);
    const double W = hi - lo;
    if (W < 1e-8 * std::max({1.0, std::fabs(lo), std::fabs(hi)})) {
      e_lo_hi[2 * i] = lo - 0.5;
      e_lo_hi[2 * i + 1] = hi + 0.5;
    } else {
      e_lo_hi[2 * i] = lo - margin * W;
      e_lo_hi[2 * i + 1] = hi + margin * W;
    }
  }
  return KPM_OK;
}

// ------------------------------------------------------------ moments driver

struct MomLayout {
  size_t plan, vec, part0, part1, alpha, beta, norms, flag, base, states, lz, total;
};

MomLayout moments_layout(const Planned& P, int K, size_t lz_bytes) {
  MomLayout L{};
  size_t o = 0;
  auto put = [&](size_t bytes) {
    const size_t r = o;
    o = align_up(o + bytes);
    return r;
  };
  // float32 + residual storage: the float32 part, then the int16 residuals
  const size_t elt = P.plan.resid ? 6 : (P.plan.fp32 ? 4 : 8);
  const size_t TC = (size_t)P.plan.total_cols;
  L.plan = put(P.bytes);
  L.lz = o;   // Lanczos runs first and may reuse everything below
  L.vec = put((size_t)P.plan.vec_elems * elt);
  L.part0 = put((size_t)P.plan.part_len * 8);
  L.part1 = put((size_t)P.plan.part_len * 8);
  L.alpha = put((size_t)(K + 1) * TC * 8);
  L.beta = put((size_t)K * TC * 8);
  L.norms = put(TC * 8);
  L.flag = put(256);
  L.base = put(256);
  L.states = put((size_t)P.plan.n_states * 4);
  L.total = std::max(o, align_up(L.lz + lz_bytes));
  return L;
}

RunShape shape_of(const kpm_params& q, const Tune* t = nullptr) {
  RunShape s;
  if (t) s.tune = *t;
  s.precision = q.precision;
  s.vec_kind = q.vec_kind;
  s.R = q.R;
  s.col_block = q.col_block;
  return s;
}

int n_steps(int M) { return std::max(1, M / 2); }

int lanczos_steps_of(const kpm_params& q) { return q.lanczos_steps > 0 ? q.lanczos_steps : 50; }

// ------------------------------------------------------------ autotuning
//
// Per device and problem shape (sector sizes, bond counts, precision, vector
// kind and count) the launch shape of the recursion -- block width, step
// kernel, low-bit block width, sub-tiles per workgroup, gathers in flight --
// is chosen by timing a few steps of every candidate the first time the shape
// is seen, and cached for the process.

std::vector<Tune> tune_candidates(const kpm_problem* p, int n, const kpm_params& q) {
  const bool resid = q.precision == KPM_FP32R_STORE;
  const bool fp32 = q.precision == KPM_FP32_STORE || resid;
  const RunShape s0 = shape_of(q);
  int64_t maxc = 1;
  for (int i = 0; i < n; ++i) maxc = std::max<int64_t>(maxc, total_columns(p[i], s0));
  const int cpv = cols_per_vec(q.vec_kind);
  std::vector<int> widths;
  if (q.col_block > 0) {
    widths.push_back(q.col_block);
  } else {
    for (int w : {1, 2, 4, 8, 16, 32, kMaxLd}) {
      int ww = (int)std::min<int64_t>(w, maxc);
      ww = (ww + cpv - 1) / cpv * cpv;
      if (fp32 && ww < 4 && maxc >= 4) continue;
      if (std::find(widths.begin(), widths.end(), ww) == widths.end()) widths.push_back(ww);
    }
  }
  std::vector<Tune> c;
  c.push_back(Tune{});                       // the planner's heuristic
  for (int w : widths) {
    Tune t;
    t.col_block = w;
    if (resid) {   // the slice kernel is the only one with this storage
      if (w <= 8)
        for (int spt : {2, 1, 3})
          for (int gh : {4, 8})
            for (int nw : {2, 1}) {
              Tune b = t;
              b.kernel = 5;
              b.block_L = 10;
              b.spt = spt;
              b.gather_batch = gh;
              b.waves = nw;
              c.push_back(b);
            }
      continue;
    }
    if (w <= 8) {
      t.kernel = 1;
      c.push_back(t);
      t.gather_batch = (w >= 4) ? 4 : 2;
      c.push_back(t);
      t.gather_batch = 0;
    }
    t.kernel = 0;
    c.push_back(t);
    if (w >= 4)
      for (int L : {9, 10})
        for (int spt : {0, 3}) {
          Tune b = t;
          b.kernel = 2;
          b.block_L = L;
          b.spt = spt;
          c.push_back(b);
        }
    for (int xl : {0, 1})
      for (int spt : {2, 4}) {
        Tune b = t;
        b.kernel = 3;
        b.block_L = 9;
        b.spt = spt;
        b.lds_x = xl;
        c.push_back(b);
      }
    // slice kernel (blocks of at most two 16-byte chunks per row): 10 low
    // bits, 1-3 sub-tiles per workgroup, 4 or 8 high-high rows in flight,
    // 2, 4 or 1 waves per tile (the planner falls back to 1 where rows are
    // not 16-byte multiples); the shape measured best on the 24-site ring
    // first
    if (w <= (fp32 ? 8 : 4))
      for (int spt : {2, 1, 3})
        for (int gh : {4, 8})
          for (int nw : {2, 4, 1}) {
            Tune b = t;
            b.kernel = 5;
            b.block_L = 10;
            b.spt = spt;
            b.gather_batch = gh;
            b.waves = nw;
            c.push_back(b);
          }
  }
  return c;
}

// Seconds per step of one candidate: plan, Rademacher start, three warm-up
// and `meas` timed steps (values are irrelevant to the timing; the steps
// reduce no dots).
double time_candidate(const kpm_problem* p, int n, const kpm_params& q, const Tune& t,
                      const double* a, const double* b, unsigned char* work, size_t bytes,
                      hipStream_t st, hipEvent_t e0, hipEvent_t e1, int meas = 6) {
  Planned P;
  if (make_plan(p, n, shape_of(q, &t), a, b, P) != KPM_OK) return INFINITY;
  const MomLayout L = moments_layout(P, 8, 0);
  if (L.total > bytes) return INFINITY;
  std::vector<unsigned char> staging;
  if (upload_plan(P, work + L.plan, staging, st) != KPM_OK) return INFINITY;
  DevicePlan& D = P.plan;
  D.err = reinterpret_cast<int*>(work + L.flag);
  D.states = reinterpret_cast<uint32_t*>(work + L.states);
  void* vec = work + L.vec;
  double* part[2] = {reinterpret_cast<double*>(work + L.part0),
                     reinterpret_cast<double*>(work + L.part1)};
  bool ok = hipMemsetAsync(D.err, 0, sizeof(int), st) == hipSuccess;
  if (ok && (D.row_ld || D.block || D.spin)) ok = fill_states(D, st) == hipSuccess;
  if (ok) ok = launch_init(D, vec, 1, KPM_VEC_RADEMACHER, q.seed, nullptr, part[0], st) == hipSuccess;
  const int warm = 3;
  for (int k = 0; ok && k < warm + meas; ++k) {
    if (k == warm) ok = hipEventRecord(e0, st) == hipSuccess;
    if (ok)
      ok = launch_step(D, vec, part[k & 1], nullptr, 0, nullptr, nullptr, nullptr, k, k & 1,
                       k == 0 ? 1 : 0, st) == hipSuccess;
  }
  if (ok) ok = hipEventRecord(e1, st) == hipSuccess;
  if (ok) ok = hipEventSynchronize(e1) == hipSuccess;
  float ms = 0.f;
  if (ok) ok = hipEventElapsedTime(&ms, e0, e1) == hipSuccess;
  (void)hipStreamSynchronize(st);   // staging outlives its copy
  return ok ? (double)ms / meas : INFINITY;
}

std::mutex g_tune_mu;
std::map<std::string, Tune> g_tune_cache;

std::string tune_key(int dev, const kpm_problem* p, int n, const kpm_params& q) {
  std::string k = std::to_string(dev) + "|" + std::to_string(q.precision) + "," +
                  std::to_string(q.vec_kind) + "," + std::to_string(q.R) + "," +
                  std::to_string(q.col_block) + "|";
  for (int i = 0; i < n; ++i) {
    // the bond graph and the site spin fix the launch shape (couplings do not)
    uint64_t hsh = 1469598103934665603ull;   // FNV-1a over the bond list
    for (int b = 0; b < p[i].n_bonds; ++b) {
      const uint32_t e = (uint32_t)p[i].bond_i[b] | ((uint32_t)p[i].bond_j[b] << 16);
      for (int t = 0; t < 4; ++t) hsh = (hsh ^ ((e >> (8 * t)) & 0xFFu)) * 1099511628211ull;
    }
    k += std::to_string(p[i].n_sites) + "." + std::to_string(p[i].n_up) + "." + std::to_string(p[i].n_bonds) +
         "." + std::to_string(two_s_of(p[i])) + "." + std::to_string(hsh) + ";";
  }
  return k;
}

// The cached or freshly measured launch shape for these problems.  `work`
// (bytes) is scratch for the trial runs.
// The launch shape measured earlier for these problems and parameters, if any.
bool cached_tune(const kpm_problem* p, int n, const kpm_params& q, Tune& out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  const std::string key = tune_key(dev, p, n, q);
  std::lock_guard<std::mutex> lock(g_tune_mu);
  auto it = g_tune_cache.find(key);
  if (it == g_tune_cache.end()) return false;
  out = it->second;
  return true;
}

int get_tune(const kpm_problem* p, int n, const kpm_params& q, const double* a, const double* b,
             unsigned char* work, size_t bytes, hipStream_t st, Tune& out) {
  int dev = 0;
  KPM_HIP(hipGetDevice(&dev));
  const std::string key = tune_key(dev, p, n, q);
  std::lock_guard<std::mutex> lock(g_tune_mu);
  auto it = g_tune_cache.find(key);
  if (it != g_tune_cache.end()) {
    out = it->second;
    return KPM_OK;
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  KPM_HIP(hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return KPM_EDEVICE;
  }
  // Every candidate over 6 steps, then those within 5 % of the fastest again
  // over 30 steps, in list order: a later one replaces the pick only when
  // more than 3 % faster, so shapes within the timing noise of each other
  // (and of one device to the next) resolve to the earlier one.
  const std::vector<Tune> cands = tune_candidates(p, n, q);
  std::vector<double> sec(cands.size());
  double first = INFINITY;
  for (size_t i = 0; i < cands.size(); ++i) {
    sec[i] = time_candidate(p, n, q, cands[i], a, b, work, bytes, st, e0, e1);
    first = std::min(first, sec[i]);
  }
  double best = INFINITY;
  Tune pick{};
  for (size_t i = 0; i < cands.size(); ++i) {
    if (!(sec[i] <= first * 1.05)) continue;
    const double s30 = time_candidate(p, n, q, cands[i], a, b, work, bytes, st, e0, e1, 30);
    if (s30 < best * (1.0 - 0.03)) {
      best = s30;
      pick = cands[i];
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  g_tune_cache[key] = pick;
  out = pick;
  return KPM_OK;
}

size_t moments_workspace(const kpm_problem* p, int n, const kpm_params& q) {
  std::vector<kpm_problem> need;
  for (int i = 0; i < n; ++i)
    if (std::isnan(p[i].e_lo) || std::isnan(p[i].e_hi)) need.push_back(p[i]);
  const size_t lz = need.empty() ? 0 : lanczos_bytes(need.data(), (int)need.size(), lanczos_steps_of(q));
  Planned P;
  if (make_plan(p, n, shape_of(q), nullptr, nullptr, P) != KPM_OK) return 0;
  size_t total = moments_layout(P, n_steps(q.M), lz).total;
  if (q.autotune) {
    // Before the first trial runs the workspace must hold every candidate's
    // plan; once a shape is cached for these problems only its plan is run
    // (planning all ~30 candidates took over a second per call on the 64
    // random clusters).
    std::vector<Tune> cands;
    int dev = 0;
    if (hipGetDevice(&dev) == hipSuccess) {
      std::lock_guard<std::mutex> lock(g_tune_mu);
      auto it = g_tune_cache.find(tune_key(dev, p, n, q));
      if (it != g_tune_cache.end()) cands.push_back(it->second);
    }
    if (cands.empty()) cands = tune_candidates(p, n, q);
    for (const Tune& t : cands) {
      Planned Pc;
      if (make_plan(p, n, shape_of(q, &t), nullptr, nullptr, Pc) == KPM_OK)
        total = std::max(total, moments_layout(Pc, n_steps(q.M), lz).total);
    }
  }
  return total;
}


int graph_segment() {
  int S = env_int("KPM_GRAPH_SEGMENT", 64);
  if (S < 0) S = 0;
  return S & ~1;
}

// Init, K recursion steps (graph-captured segments), final reduction,
// doubling identities and estimator.  `direct`: every step is launched on
// `st` itself, with no captured graph, helper stream or timing events (the
// allocation-free entry point; recursion_ms is then -1).
int run_moments(Planned& P, const MomLayout& L, unsigned char* work, const kpm_params& q,
                double* d_mu, hipStream_t st, bool direct) {
  DevicePlan& D = P.plan;
  const int K = n_steps(q.M);
  const int TC = D.total_cols;
  void* vec = work + L.vec;
  double* part[2] = {reinterpret_cast<double*>(work + L.part0),
                     reinterpret_cast<double*>(work + L.part1)};
  double* alpha = reinterpret_cast<double*>(work + L.alpha);
  double* beta = reinterpret_cast<double*>(work + L.beta);
  double* norms = reinterpret_cast<double*>(work + L.norms);
  int* flag = reinterpret_cast<int*>(work + L.flag);
  int64_t* base = reinterpret_cast<int64_t*>(work + L.base);
  P.plan.err = flag;
  P.plan.states = reinterpret_cast<uint32_t*>(work + L.states);
  KPM_HIP(hipMemsetAsync(flag, 0, sizeof(int), st));
  if (D.row_ld || D.block || D.spin) KPM_HIP(fill_states(D, st));

  if (q.vec_kind == KPM_VEC_GAUSSIAN || q.vec_kind == KPM_VEC_COMPLEX_GAUSSIAN) {
    KPM_HIP(launch_init(D, vec, 0, q.vec_kind, q.seed, nullptr, part[0], st));
    KPM_HIP(launch_reduce(D, part[0], norms, nullptr, st));
  }
  KPM_HIP(launch_init(D, vec, 1, q.vec_kind, q.seed, norms, part[0], st));
  KPM_HIP(launch_reduce(D, part[0], alpha, nullptr, st));
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  if (!direct) {
    KPM_HIP(hipEventCreate(&ev0));
    if (hipEventCreate(&ev1) != hipSuccess) {
      (void)hipEventDestroy(ev0);
      return KPM_EDEVICE;
    }
  }
  struct EvGuard {
    hipEvent_t a, b;
    ~EvGuard() {
      if (a) (void)hipEventDestroy(a);
      if (b) (void)hipEventDestroy(b);
    }
  } evg{ev0, ev1};
  if (ev0) KPM_HIP(hipEventRecord(ev0, st));
  KPM_HIP(launch_step(D, vec, part[0], nullptr, 0, alpha, beta, nullptr, 0, 0, 1, st));
  int s = 1;
  const int S = direct ? 0 : graph_segment();
  int used_segment = 0;
  if (S >= 2 && K - 1 >= S) {
    hipStream_t cap;
    KPM_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipError_t e = hipStreamBeginCapture(cap, hipStreamCaptureModeRelaxed);
    for (int j = 0; j < S && e == hipSuccess; ++j)
      e = launch_step(D, vec, part[(1 + j) & 1], part[j & 1], 2 * TC, alpha, beta, base, j,
                      (1 + j) & 1, 0, cap);
    hipError_t e2 = hipStreamEndCapture(cap, &graph);
    if (e == hipSuccess) e = e2;
    if (e == hipSuccess) e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    while (e == hipSuccess && s + S <= K) {
      e = launch_set_i64(base, s, st);
      if (e == hipSuccess) e = hipGraphLaunch(exec, st);
      s += S;
    }
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    (void)hipStreamDestroy(cap);
    if (e != hipSuccess) return KPM_EDEVICE;
    used_segment = S;
  }
  for (; s < K; ++s)
    KPM_HIP(launch_step(D, vec, part[s & 1], part[(s - 1) & 1], 2 * TC, alpha, beta, nullptr, s,
                        s & 1, 0, st));
  if (ev1) KPM_HIP(hipEventRecord(ev1, st));
  KPM_HIP(launch_reduce(D, part[(K - 1) & 1], alpha + (size_t)K * TC, beta + (size_t)(K - 1) * TC, st));
  FinalArgs fa{};
  fa.probs = D.probs;
  fa.units = D.units;
  fa.prob_unit0 = D.prob_unit0;
  fa.alpha = alpha;
  fa.beta = beta;
  fa.mu = d_mu;
  fa.flag = flag;
  fa.n_probs = D.n_probs;
  fa.M = q.M;
  fa.total_cols = TC;
  fa.cols_per_vec = cols_per_vec(q.vec_kind);
  fa.R = q.vec_kind == KPM_VEC_BASIS ? 0 : q.R;
  KPM_HIP(launch_finalize(fa, st));
  int h_flag = 0;
  KPM_HIP(hipMemcpyAsync(&h_flag, flag, sizeof(int), hipMemcpyDeviceToHost, st));
  KPM_HIP(hipStreamSynchronize(st));

  g_stats.step_launches = K;
  g_stats.bytes_per_launch = P.bytes_per_step;
  g_stats.state_col_steps = P.state_cols * K;
  g_stats.col_block = 0;
  for (auto& u : P.units) g_stats.col_block = std::max(g_stats.col_block, u.ncols);
  g_stats.rows_per_tile = D.sub_rows * D.sub_per_tile;
  if (D.block && !P.tile_nrows.empty()) {
    double rows = 0;
    for (int32_t r : P.tile_nrows) rows += r;
    g_stats.rows_per_tile = (int32_t)std::lround(rows / (double)P.tile_nrows.size());
  }
  g_stats.kernel = D.spin ? 4 : (D.block == 3 ? 5 : (D.block == 2 ? 3 : (D.block ? 2 : (D.row_ld ? 1 : 0))));
  g_stats.graph_segment = used_segment;
  g_stats.waves = D.block == 3 ? D.slice_nw : 1;
  g_stats.relabelled = 0;
  for (const auto& d : P.probs) g_stats.relabelled += d.relabel;
  float ms = 0.f;
  g_stats.recursion_ms = ev0 && hipEventElapsedTime(&ms, ev0, ev1) == hipSuccess ? (double)ms : -1.0;
  if (h_flag & 2) return KPM_EDEVICE;
  return (h_flag & 1) ? KPM_EBOUNDS : KPM_OK;
}

// Init and n recursion steps of one problem (the steps chebyshev_moments
// launches, without the dots' reduction), then v_n to d_out.
int run_vectors(Planned& P, const MomLayout& L, unsigned char* work, const kpm_params& q, int nv,
                void* d_out, hipStream_t st) {
  DevicePlan& D = P.plan;
  void* vec = work + L.vec;
  double* part[2] = {reinterpret_cast<double*>(work + L.part0),
                     reinterpret_cast<double*>(work + L.part1)};
  double* norms = reinterpret_cast<double*>(work + L.norms);
  int* flag = reinterpret_cast<int*>(work + L.flag);
  P.plan.err = flag;
  P.plan.states = reinterpret_cast<uint32_t*>(work + L.states);
  KPM_HIP(hipMemsetAsync(flag, 0, sizeof(int), st));
  if (D.row_ld || D.block || D.spin) KPM_HIP(fill_states(D, st));
  if (q.vec_kind == KPM_VEC_GAUSSIAN || q.vec_kind == KPM_VEC_COMPLEX_GAUSSIAN) {
    KPM_HIP(launch_init(D, vec, 0, q.vec_kind, q.seed, nullptr, part[0], st));
    KPM_HIP(launch_reduce(D, part[0], norms, nullptr, st));
  }
  KPM_HIP(launch_init(D, vec, 1, q.vec_kind, q.seed, norms, part[0], st));
  for (int s = 0; s < nv; ++s)
    KPM_HIP(launch_step(D, vec, part[s & 1], nullptr, 0, nullptr, nullptr, nullptr, s, s & 1,
                        s == 0 ? 1 : 0, st));
  ExportArgs ea{};
  ea.units = D.units;
  ea.vec = vec;
  ea.slot_stride = D.slot_stride;
  ea.slot = nv & 1;
  ea.unit0 = 0;
  ea.rb = P.units[0].ncols;
  ea.n_cols = 0;
  for (auto& u : P.units) ea.n_cols += u.ncols;
  ea.dim = P.probs[0].dim;
  ea.out = d_out;
  ea.prob = D.probs;
  ea.binom = D.binom;
  KPM_HIP(launch_export(ea, D.fp32, st));
  int h_flag = 0;
  KPM_HIP(hipMemcpyAsync(&h_flag, flag, sizeof(int), hipMemcpyDeviceToHost, st));
  KPM_HIP(hipStreamSynchronize(st));
  return (h_flag & 6) ? KPM_EDEVICE : KPM_OK;
}

// Resolve bounds (Lanczos where NaN) and the (a, b) of Eq. (5).
int resolve_scale(const kpm_problem* p, int n, const kpm_params& q, unsigned char* lz_work,
                  hipStream_t st, std::vector<double>& a, std::vector<double>& b) {
  std::vector<kpm_problem> need;
  std::vector<int> idx;
  for (int i = 0; i < n; ++i)
    if (std::isnan(p[i].e_lo) || std::isnan(p[i].e_hi)) {
      need.push_back(p[i]);
      idx.push_back(i);
    }
  std::vector<double> lohi(2 * n);
  for (int i = 0; i < n; ++i) {
    lohi[2 * i] = p[i].e_lo;
    lohi[2 * i + 1] = p[i].e_hi;
  }
  if (!need.empty()) {
    std::vector<double> got(2 * need.size());
    const int r = run_lanczos(need.data(), (int)need.size(), lanczos_steps_of(q), q.bound_margin,
                              q.seed, got.data(), lz_work, st);
    if (r != KPM_OK) return r;
    for (size_t j = 0; j < idx.size(); ++j) {
      lohi[2 * idx[j]] = got[2 * j];
      lohi[2 * idx[j] + 1] = got[2 * j + 1];
    }
  }
  a.resize(n);
  b.resize(n);
  for (int i = 0; i < n; ++i) {
    a[i] = (lohi[2 * i + 1] - lohi[2 * i]) / (2.0 - q.eps);
    b[i] = 0.5 * (lohi[2 * i + 1] + lohi[2 * i]);
    if (!(a[i] > 0.0) || !std::isfinite(a[i]) || !std::isfinite(b[i])) return KPM_EINVAL;
  }
  return KPM_OK;
}

// ------------------------------------------------------------- adjoint driver

struct VjpLayout {
  size_t plan, seg, w, ckpt, part, norms, alpha0, abar, bbar, bd, flag, planf, statesf, partf, partf2,
      falpha, fbeta, total;
  int nck, C, K;
};

// Plan of the forward and recompute steps of the adjoint: the fastest forward
// kernel (block-table or row kernel) on the same vector layout as the adjoint
// plan P (same blocks, widths and offsets; sites not relabelled).  Returns
// false when the layouts differ: the adjoint plan's own kernel then runs them.
bool forward_plan_for(const kpm_problem* p, int n, const kpm_params& q, const Planned& P,
                      const double* a, const double* b, Planned& F) {
  if (env_int("KPM_ADJ_FWD", 1) == 0 || P.units.empty()) return false;
  RunShape s = shape_of(q);
  s.allow_relabel = false;
  s.col_block = P.units[0].ncols;
  if (make_plan(p, n, s, a, b, F) != KPM_OK) return false;
  if (F.units.size() != P.units.size() || F.plan.slot_stride != P.plan.slot_stride || F.plan.fp32 != P.plan.fp32)
    return false;
  for (size_t i = 0; i < P.units.size(); ++i) {
    const UnitDev &u = P.units[i], &f = F.units[i];
    if (u.ld != f.ld || u.vec_off != f.vec_off || u.prob != f.prob || u.ncols != f.ncols || u.col0 != f.col0)
      return false;
  }
  return F.plan.block || F.plan.row_ld;
}

VjpLayout vjp_layout(const Planned& P, const Planned* F, int M, int ckpt_every) {
  VjpLayout L{};
  const int K = n_steps(M);
  const int C = std::max(2, ckpt_every & ~1);
  L.K = K;
  L.C = C;
  L.nck = (K - 1) / C + 1;
  const size_t elt = P.plan.fp32 ? 4 : 8;
  const size_t slot = (size_t)P.plan.slot_stride * elt;
  const size_t TC = (size_t)P.plan.total_cols;
  size_t o = 0;
  auto put = [&](size_t bytes) {
    const size_t r = o;
    o = align_up(o + bytes);
    return r;
  };
  L.plan = put(P.bytes);
  L.seg = put((size_t)(std::min(C, K) + 2) * slot);
  L.w = put(2 * slot);
  L.ckpt = put((size_t)L.nck * 2 * slot);
  L.part = put((size_t)P.plan.part_len * 8);
  L.norms = put(TC * 8);
  L.alpha0 = put(TC * 8);
  L.abar = put((size_t)(K + 1) * TC * 8);
  L.bbar = put((size_t)(K + 1) * TC * 8);
  L.bd = put((size_t)P.plan.bd_len * 8);
  L.flag = put(256);
  // the forward steps' dots (when the forward pass also gives the moments)
  const Planned& Q = F ? *F : P;
  if (F) {
    L.planf = put(F->bytes);
    L.statesf = put((size_t)F->plan.n_states * 4);
    L.partf = put((size_t)F->plan.part_len * 8);
  }
  L.partf2 = put((size_t)Q.plan.part_len * 8);
  L.falpha = put((size_t)(K + 1) * Q.plan.total_cols * 8);
  L.fbeta = put((size_t)K * Q.plan.total_cols * 8);
  L.total = o;
  return L;
}

RunShape adj_shape(const kpm_params& q) {
  RunShape s = shape_of(q);
  s.adjoint = true;
  return s;
}

size_t vjp_workspace(const kpm_problem* p, int n, const kpm_params& q, int ckpt_every) {
  Planned P, F;
  if (make_plan(p, n, adj_shape(q), nullptr, nullptr, P) != KPM_OK) return 0;
  const bool fwd = forward_plan_for(p, n, q, P, nullptr, nullptr, F);
  return vjp_layout(P, fwd ? &F : nullptr, q.M, ckpt_every).total;
}

// Forward recursion with checkpoints, then the reverse sweep segment by
// segment (recomputing each segment's v_n from its checkpoint).
// With d_mu, the forward pass also reduces its dots into the moments
// (doubling identities and estimator of Eq. (7)) and `between` runs after it,
// before d_dmu is read: the loss gradient may then be formed from those
// moments.  Returns KPM_EBOUNDS when |mu_n| > mu_0 there.  `phases` selects
// the forward pass (kVjpForward: v_0, the steps and their checkpoints), the
// reverse sweep (kVjpReverse, which reads what a forward pass with the same
// arguments left in `work`), or both.
constexpr int kVjpForward = 1, kVjpReverse = 2;
int run_vjp(const kpm_problem* p, int n, const kpm_params& q, const double* h_ab,
            const double* d_dmu, int ckpt_every, double* d_dJ, unsigned char* work,
            hipStream_t st, double* d_mu = nullptr, const std::function<int()>& between = {},
            int phases = kVjpForward | kVjpReverse) {
  std::vector<double> a(n), b(n);
  for (int i = 0; i < n; ++i) {
    a[i] = h_ab[2 * i];
    b[i] = h_ab[2 * i + 1];
    if (!(a[i] > 0.0) || !std::isfinite(a[i]) || !std::isfinite(b[i])) return KPM_EINVAL;
  }
  Planned P, F;
  int r = make_plan(p, n, adj_shape(q), a.data(), b.data(), P);
  if (r != KPM_OK) return r;
  const bool fwd = forward_plan_for(p, n, q, P, a.data(), b.data(), F);
  const VjpLayout L = vjp_layout(P, fwd ? &F : nullptr, q.M, ckpt_every);
  std::vector<unsigned char> staging, staging_f;
  r = upload_plan(P, work + L.plan, staging, st);
  if (r != KPM_OK) return r;
  DevicePlan& D = P.plan;
  int* flag = reinterpret_cast<int*>(work + L.flag);
  D.err = flag;
  KPM_HIP(hipMemsetAsync(flag, 0, sizeof(int), st));
  // forward and recompute steps: F's kernel on the same vectors (partial dots discarded)
  DevicePlan* Dfw = &D;
  double* part_fw = reinterpret_cast<double*>(work + L.part);
  if (fwd) {
    r = upload_plan(F, work + L.planf, staging_f, st);
    if (r != KPM_OK) return r;
    F.plan.err = flag;
    F.plan.states = reinterpret_cast<uint32_t*>(work + L.statesf);
    if (F.plan.row_ld || F.plan.block) KPM_HIP(fill_states(F.plan, st));
    Dfw = &F.plan;
    part_fw = reinterpret_cast<double*>(work + L.partf);
  }
  const int K = L.K, C = L.C;
  // C >= K: the segment buffer holds the whole trajectory v_0 .. v_K (slot j
  // holds v_j), written by the forward pass, so the reverse sweep recomputes
  // nothing (memory K + 2 vectors instead of 2 K / C + C + 2)
  const bool full = C >= K;
  const size_t elt = D.fp32 ? 4 : 8;
  const size_t slot_bytes = (size_t)D.slot_stride * elt;
  unsigned char* seg = work + L.seg;
  unsigned char* wbuf = work + L.w;
  unsigned char* ckpt = work + L.ckpt;
  double* part = reinterpret_cast<double*>(work + L.part);
  double* norms = reinterpret_cast<double*>(work + L.norms);
  double* alpha0 = reinterpret_cast<double*>(work + L.alpha0);
  double* abar = reinterpret_cast<double*>(work + L.abar);
  double* bbar = reinterpret_cast<double*>(work + L.bbar);
  double* bd = reinterpret_cast<double*>(work + L.bd);
  const int TC = D.total_cols;
  int ld = 1;
  for (auto& u : P.units) ld = std::max(ld, u.ld);

  // forward: v_0 (and its norms), steps with a checkpoint of (v_j, v_{j+1}) at j = 0, C, 2C, ...
  if (phases & kVjpForward) {
  if (q.vec_kind == KPM_VEC_GAUSSIAN || q.vec_kind == KPM_VEC_COMPLEX_GAUSSIAN) {
    KPM_HIP(launch_init(D, seg, 0, q.vec_kind, q.seed, nullptr, part, st));
    KPM_HIP(launch_reduce(D, part, norms, nullptr, st));
  }
  KPM_HIP(launch_init(D, seg, 1, q.vec_kind, q.seed, norms, part, st));
  KPM_HIP(launch_reduce(D, part, alpha0, nullptr, st));
  if (!d_mu) {
    KPM_HIP(launch_step_slots(*Dfw, seg, part_fw, 0, 1, 1, 1, st));
    for (int j = 0; j < K; ++j) {
      if (j > 0) {
        if (full) KPM_HIP(launch_step_slots(*Dfw, seg, part_fw, j, j - 1, j + 1, 0, st));
        else KPM_HIP(launch_step_slots(*Dfw, seg, part_fw, j & 1, (j + 1) & 1, (j + 1) & 1, 0, st));
      }
      if (!full && j % C == 0)
        KPM_HIP(hipMemcpyAsync(ckpt + (size_t)(j / C) * 2 * slot_bytes, seg, 2 * slot_bytes,
                               hipMemcpyDeviceToDevice, st));
    }
  } else {
    // the same steps with their dots reduced one launch later (as for the
    // moments alone), then the moments
    const int TF = Dfw->total_cols;
    double* pf[2] = {part_fw, reinterpret_cast<double*>(work + L.partf2)};
    double* fal = reinterpret_cast<double*>(work + L.falpha);
    double* fbe = reinterpret_cast<double*>(work + L.fbeta);
    KPM_HIP(hipMemcpyAsync(fal, alpha0, (size_t)TF * 8, hipMemcpyDeviceToDevice, st));   // <v_0, v_0>
    KPM_HIP(launch_step(*Dfw, seg, pf[0], nullptr, 0, fal, fbe, nullptr, 0, 0, 1, st));
    for (int j = 0; j < K; ++j) {
      if (j > 0) {
        if (full) {
          // v_{j+1} into slot j + 1, the dots as in the two-slot ring
          KPM_HIP(launch_step_slots_dots(*Dfw, seg, pf[j & 1], pf[(j - 1) & 1], 2 * TF, fal, fbe, j, j, j - 1,
                                         j + 1, st));
        } else {
          KPM_HIP(launch_step(*Dfw, seg, pf[j & 1], pf[(j - 1) & 1], 2 * TF, fal, fbe, nullptr, j, j & 1, 0, st));
        }
      }
      if (!full && j % C == 0)
        KPM_HIP(hipMemcpyAsync(ckpt + (size_t)(j / C) * 2 * slot_bytes, seg, 2 * slot_bytes,
                               hipMemcpyDeviceToDevice, st));
    }
    KPM_HIP(launch_reduce(*Dfw, pf[(K - 1) & 1], fal + (size_t)K * TF, fbe + (size_t)(K - 1) * TF, st));
    FinalArgs fa{};
    fa.probs = Dfw->probs;
    fa.units = Dfw->units;
    fa.prob_unit0 = Dfw->prob_unit0;
    fa.alpha = fal;
    fa.beta = fbe;
    fa.mu = d_mu;
    fa.flag = flag;
    fa.n_probs = Dfw->n_probs;
    fa.M = q.M;
    fa.total_cols = TF;
    fa.cols_per_vec = cols_per_vec(q.vec_kind);
    fa.R = q.vec_kind == KPM_VEC_BASIS ? 0 : q.R;
    KPM_HIP(launch_finalize(fa, st));
    int h_flag = 0;
    KPM_HIP(hipMemcpyAsync(&h_flag, flag, sizeof(int), hipMemcpyDeviceToHost, st));
    KPM_HIP(hipStreamSynchronize(st));
    if (h_flag & 2) return KPM_EDEVICE;
    if (h_flag & 1) return KPM_EBOUNDS;
    if (between) {
      const int rb = between();
      if (rb != KPM_OK) return rb;
    }
  }
  }
  if (!(phases & kVjpReverse)) {
    int h_flag = 0;
    KPM_HIP(hipMemcpyAsync(&h_flag, flag, sizeof(int), hipMemcpyDeviceToHost, st));
    KPM_HIP(hipStreamSynchronize(st));
    return h_flag ? KPM_EDEVICE : KPM_OK;
  }
  // Each checkpoint m holds v_{mC} in slot (mC)&1 = 0 (C is even) and v_{mC+1} in slot 1.
  DoublingVjpArgs dv{};
  dv.probs = D.probs;
  dv.units = D.units;
  dv.job_unit = D.job_unit;
  dv.lambda = d_dmu;
  dv.alpha0 = alpha0;
  dv.abar = abar;
  dv.bbar = bbar;
  dv.total_cols = TC;
  dv.M = q.M;
  dv.K = K;
  dv.cols_per_vec = cols_per_vec(q.vec_kind);
  dv.R = q.vec_kind == KPM_VEC_BASIS ? 0 : q.R;
  KPM_HIP(hipMemsetAsync(bbar + (size_t)K * TC, 0, (size_t)TC * 8, st));
  KPM_HIP(launch_doubling_vjp(dv, st));
  KPM_HIP(hipMemsetAsync(wbuf, 0, 2 * slot_bytes, st));

  bool first = true;
  for (int m = L.nck - 1; m >= 0; --m) {
    const int j0 = m * C;
    const int j1 = std::min(j0 + C, K);
    if (!full) {
      KPM_HIP(hipMemcpyAsync(seg, ckpt + (size_t)m * 2 * slot_bytes, 2 * slot_bytes,
                             hipMemcpyDeviceToDevice, st));
      const int top = std::min(j1 + 1, K);   // highest v index needed
      for (int t = 1; j0 + t + 1 <= top; ++t)
        KPM_HIP(launch_step_slots(*Dfw, seg, part_fw, t, t - 1, t + 1, 0, st));
    }
    for (int nn = j1; nn >= j0 + 1; --nn) {
      AdjArgs aa{};
      aa.vseg = seg;
      aa.wbuf = wbuf;
      aa.vm1_slot = nn - 1 - j0;
      aa.v0_slot = nn - j0;
      aa.vp1_slot = nn + 1 <= K ? nn + 1 - j0 : -1;
      aa.wx_slot = (nn + 1) & 1;
      aa.wy_slot = nn & 1;
      aa.abar_n = abar + (size_t)nn * TC;
      aa.bbar_n = bbar + (size_t)nn * TC;
      aa.bbar_nm1 = bbar + (size_t)(nn - 1) * TC;
      aa.part_bd = bd;
      aa.coef = 2.0;
      aa.accumulate = first ? 0 : 1;
      aa.dots_only = 0;
      KPM_HIP(launch_adjoint(D, aa, ld, st));
      first = false;
    }
  }
  // <w_1, h_b v_0> with weight 1 (segment 0 is resident: slot 0 holds v_0)
  AdjArgs fin{};
  fin.vseg = seg;
  fin.wbuf = wbuf;
  fin.vm1_slot = -1;
  fin.v0_slot = 0;
  fin.vp1_slot = -1;
  fin.wx_slot = 1;
  fin.wy_slot = 0;
  fin.abar_n = abar;
  fin.bbar_n = bbar;
  fin.bbar_nm1 = bbar;
  fin.part_bd = bd;
  fin.coef = 1.0;
  fin.accumulate = 1;
  fin.dots_only = 1;
  KPM_HIP(launch_adjoint(D, fin, ld, st));
  BondReduceArgs br{};
  br.probs = D.probs;
  br.units = D.units;
  br.prob_unit0 = D.prob_unit0;
  br.part_bd = bd;
  br.dJ = d_dJ;
  br.n_probs = n;
  int total_bonds = 0;
  for (int i = 0; i < n; ++i) total_bonds += p[i].n_bonds;
  KPM_HIP(launch_bond_reduce(br, total_bonds, st));
  int h_flag = 0;
  KPM_HIP(hipMemcpyAsync(&h_flag, flag, sizeof(int), hipMemcpyDeviceToHost, st));
  KPM_HIP(hipStreamSynchronize(st));
  return h_flag ? KPM_EDEVICE : KPM_OK;
}

// Thermodynamic metadata: per-problem table and problems grouped by cluster.
int thermo_meta(const kpm_problem* p, int n, std::vector<ThermoProb>& tp,
                std::vector<int32_t>& start, std::vector<int32_t>& list, int& n_clusters) {
  if (!p || n < 1) return KPM_EINVAL;
  n_clusters = 0;
  for (int i = 0; i < n; ++i) {
    const int ts = two_s_of(p[i]);
    if (p[i].two_s < 0 || p[i].two_s > 7 || p[i].n_sites < 1 || p[i].n_sites > 64 ||
        2 * p[i].n_up < ts * p[i].n_sites || p[i].n_up > ts * p[i].n_sites || p[i].cluster < 0 ||
        p[i].cluster > 65535)
      return KPM_EINVAL;
    n_clusters = std::max(n_clusters, p[i].cluster + 1);
  }
  tp.resize(n);
  start.assign(n_clusters + 1, 0);
  for (int i = 0; i < n; ++i) {
    tp[i].cluster = p[i].cluster;
    const int ts = two_s_of(p[i]);
    tp[i].weight = 2 * p[i].n_up == ts * p[i].n_sites ? 1 : 2;
    tp[i].sz = p[i].n_up - 0.5 * ts * p[i].n_sites;
    start[p[i].cluster + 1]++;
  }
  for (int c = 0; c < n_clusters; ++c) {
    if (start[c + 1] == 0) return KPM_EINVAL;   // cluster ids must be dense
    start[c + 1] += start[c];
  }
  list.assign(n, 0);
  std::vector<int32_t> fill(start.begin(), start.end() - 1);
  for (int i = 0; i < n; ++i) list[fill[p[i].cluster]++] = i;
  return KPM_OK;
}

struct ThermoDev {
  DevBuf buf;
  double* g = nullptr;
  double* gamma = nullptr;
  double* stats = nullptr;
  double* adj = nullptr;
  ThermoProb* tp = nullptr;
  int32_t* start = nullptr;
  int32_t* list = nullptr;
};

int thermo_forward(const double* d_mu, const double* d_ab, const kpm_problem* p, int n, int M,
                   int kernel, int n_nodes, const double* d_T, int n_T, double* lnZ, double* E,
                   double* C, double* chi, uint8_t* znonpos, hipStream_t st, ThermoDev& TD,
                   std::vector<ThermoProb>& tp, int& n_clusters, bool keep_adj,
                   const double* d_h = nullptr, double* d_mag = nullptr) {
  if (!d_mu || !d_ab || !d_T || M < 1 || n_T < 1 || n_nodes < 0 || (kernel != 0 && kernel != 1))
    return KPM_EINVAL;
  std::vector<int32_t> start, list;
  int r = thermo_meta(p, n, tp, start, list, n_clusters);
  if (r != KPM_OK) return r;
  const int Nt = n_nodes ? n_nodes : M;
  size_t o = 0;
  auto put = [&](size_t bytes) {
    const size_t rr = o;
    o = align_up(o + bytes);
    return rr;
  };
  const size_t og = put((size_t)M * 8), ogam = put((size_t)n * Nt * 8),
               ost = put((size_t)n_clusters * n_T * 6 * 8),
               oadj = put(keep_adj ? (size_t)n * Nt * 8 : 8), otp = put(tp.size() * sizeof(ThermoProb)),
               ostart = put(start.size() * 4), olist = put(list.size() * 4);
  r = TD.buf.alloc(o);
  if (r != KPM_OK) return r;
  unsigned char* w = static_cast<unsigned char*>(TD.buf.p);
  TD.g = reinterpret_cast<double*>(w + og);
  TD.gamma = reinterpret_cast<double*>(w + ogam);
  TD.stats = reinterpret_cast<double*>(w + ost);
  TD.adj = reinterpret_cast<double*>(w + oadj);
  TD.tp = reinterpret_cast<ThermoProb*>(w + otp);
  TD.start = reinterpret_cast<int32_t*>(w + ostart);
  TD.list = reinterpret_cast<int32_t*>(w + olist);
  KPM_HIP(hipMemcpyAsync(TD.tp, tp.data(), tp.size() * sizeof(ThermoProb), hipMemcpyHostToDevice, st));
  KPM_HIP(hipMemcpyAsync(TD.start, start.data(), start.size() * 4, hipMemcpyHostToDevice, st));
  KPM_HIP(hipMemcpyAsync(TD.list, list.data(), list.size() * 4, hipMemcpyHostToDevice, st));
  KPM_HIP(launch_kernel_coef(M, kernel, TD.g, st));
  KPM_HIP(launch_gamma(n, M, Nt, TD.g, d_mu, TD.gamma, st));
  ThermoArgs ta{};
  ta.tp = TD.tp;
  ta.cl_start = TD.start;
  ta.cl_list = TD.list;
  ta.gamma = TD.gamma;
  ta.ab = d_ab;
  ta.T = d_T;
  ta.lnZ = lnZ;
  ta.E = E;
  ta.C = C;
  ta.chi = chi;
  ta.znonpos = znonpos;
  ta.stats = TD.stats;
  ta.n_nodes = Nt;
  ta.n_T = n_T;
  ta.n_clusters = n_clusters;
  ta.h = d_h;
  ta.mag = d_mag;
  if (d_h) KPM_HIP(launch_thermo_field(ta, st));
  else KPM_HIP(launch_thermo(ta, st));
  // the host staging vectors die with the caller's frame: finish the copies now
  KPM_HIP(hipStreamSynchronize(st));
  return KPM_OK;
}

// ---------------------------------------------- finite-temperature Lanczos

struct FtlmLayout {
  size_t plan, vec, part, dots, b2, norm, ww, fixed, ybeta, err, states, ritz, escr, weight, len, total;
};

// Every real column runs its own Lanczos recursion; columns are batched in
// blocks like the Chebyshev recursion (q->col_block, 0 = the planner's width;
// width 1 splits a complex vector's Re and Im into separate blocks).
// FTLM runs float64 vectors.  Without a requested block width, spin-1/2
// problems take the slice kernel on blocks of 4 columns, 2 sub-tiles per
// tile, 4 high-high rows in flight (ring N=24, 20 columns, 200 steps: 195 ms
// per call, 201 ms on blocks of 2, 301 ms with the planner's block-table
// default); the planner falls back where no slice plan exists.
RunShape ftlm_shape(const kpm_params& q, const kpm_problem* p, int n) {
  RunShape s = shape_of(q);
  s.precision = KPM_FP64;
  s.split_vectors = q.col_block == 1;
  if (q.col_block == 0 && !any_spin(p, n)) {
    s.col_block = 4;
    s.tune.kernel = 5;
    s.tune.block_L = 10;
    s.tune.spt = 2;
    s.tune.gather_batch = 4;
  }
  return s;
}

int ftlm_steps(const Planned& P, int M) {
  int64_t max_dim = 1;
  for (auto& d : P.probs) max_dim = std::max(max_dim, d.dim);
  return (int)std::max<int64_t>(1, std::min<int64_t>(M, max_dim));
}

FtlmLayout ftlm_layout(const Planned& P, int steps) {
  FtlmLayout L{};
  size_t o = 0;
  auto put = [&](size_t bytes) {
    const size_t r = o;
    o = align_up(o + bytes);
    return r;
  };
  const size_t TC = (size_t)P.plan.total_cols;
  L.plan = put(P.bytes);
  L.vec = put((size_t)P.plan.vec_elems * 8);
  L.part = put((size_t)P.plan.part_len * 8);
  L.dots = put((size_t)steps * TC * 8);
  L.b2 = put((size_t)steps * TC * 8);
  L.norm = put(TC * 8);
  L.ww = put(TC * 8);
  L.fixed = put(TC * 8);
  L.ybeta = put(TC * 8);
  L.err = put(256);
  L.states = put((size_t)P.plan.n_states * 4);
  L.ritz = put(TC * steps * 8);
  L.escr = put(TC * steps * 8);
  L.weight = put(TC * steps * 8);
  L.len = put(TC * 4);
  L.total = o;
  return L;
}

// ------------------------------------------------ exact spectra (small sectors)

constexpr int kEdMaxDim = 1024;

struct EdPlan {
  std::vector<EigProb> probs;
  std::vector<uint32_t> bmask;
  std::vector<double> J;
  std::vector<uint32_t> tables;
  size_t o_probs = 0, o_mask = 0, o_J = 0, o_binom = 0, o_tab = 0, o_err = 0, o_mat = 0, o_vecs = 0, total = 0;
  int64_t vec_len = 0;   // doubles of each work vector set (sum of the dims)
  int max_bonds = 1;
};

int ed_plan(const kpm_problem* p, int n, int max_dim, EdPlan& E) {
  int r = check_problems(p, n);
  if (r != KPM_OK) return r;
  if (max_dim < 1 || max_dim > kEdMaxDim) return KPM_EINVAL;
  int64_t mat = 0;
  for (int i = 0; i < n; ++i) {
    const uint64_t dim = prob_dim(p[i]);
    if (dim > (uint64_t)max_dim) continue;
    EigProb e{};
    e.n_sites = p[i].n_sites;
    e.n_up = p[i].n_up;
    e.dim = (int32_t)dim;
    e.n_bonds = p[i].n_bonds;
    e.bond_off = (int32_t)E.bmask.size();
    e.out_row = i;
    e.two_s = two_s_of(p[i]);
    e.tab_off = (int32_t)E.tables.size();
    if (e.two_s > 1) build_spin_table(p[i].n_sites, e.two_s, E.tables);
    for (int k = 0; k < p[i].n_bonds; ++k) {
      if (e.two_s > 1) E.bmask.push_back((uint32_t)p[i].bond_i[k] | ((uint32_t)p[i].bond_j[k] << 8));
      else E.bmask.push_back((1u << p[i].bond_i[k]) | (1u << p[i].bond_j[k]));
      E.J.push_back(p[i].J[k]);
    }
    E.max_bonds = std::max(E.max_bonds, p[i].n_bonds);
    E.probs.push_back(e);
  }
  // descending dimension: the sectors still reducing at any step are a prefix
  std::stable_sort(E.probs.begin(), E.probs.end(),
                   [](const EigProb& x, const EigProb& y) { return x.dim > y.dim; });
  for (auto& e : E.probs) {
    e.mat_off = mat;
    e.vec_off = E.vec_len;
    mat += (int64_t)e.dim * (int64_t)e.dim;
    E.vec_len += std::max(e.dim, 4);   // >= 4: the bisection parameters reuse hv
  }
  size_t o = 0;
  auto put = [&](size_t bytes) {
    const size_t rr = o;
    o = align_up(o + bytes);
    return rr;
  };
  E.o_probs = put(std::max<size_t>(E.probs.size(), 1) * sizeof(EigProb));
  E.o_mask = put(std::max<size_t>(E.bmask.size(), 1) * 4);
  E.o_J = put(std::max<size_t>(E.J.size(), 1) * 8);
  E.o_binom = put((size_t)kBinomN * kBinomN * 4);
  E.o_tab = put(std::max<size_t>(E.tables.size(), 1) * 4);
  E.o_err = put(256);
  E.o_mat = put((size_t)std::max<int64_t>(mat, 1) * 8);
  E.o_vecs = put((size_t)std::max<int64_t>(E.vec_len, 1) * 4 * 8);
  E.total = o;
  return KPM_OK;
}

// chebyshev_moments on `need` bytes of device workspace at `work` (checked by
// the caller); `direct` as in run_moments.  Arguments are validated already.
int moments_on_workspace(const kpm_problem* p, int n, const kpm_params* q, double* d_mu,
                         double* d_ab, unsigned char* work, size_t need, hipStream_t st,
                         bool direct) {
  // When the launch shape is known already (no tuning, or measured before),
  // the host builds the plan at the unit map while the GPU runs the Lanczos
  // bounds, then applies the map.  The Lanczos region starts the workspace:
  // every layout of these problems holds at least its bytes, and it is done
  // (its tridiagonal read back) before anything else is uploaded.
  Tune tn{};
  bool known = !q->autotune || cached_tune(p, n, *q, tn);
  Planned P;
  std::future<int> planned;
  if (known) {
    try {
      planned = std::async(std::launch::async,
                           [&]() { return make_plan(p, n, shape_of(*q, &tn), nullptr, nullptr, P); });
    } catch (const std::system_error&) {
      known = false;   // no thread to be had: plan after the bounds
    }
  }
  std::vector<double> a, b;
  int r = resolve_scale(p, n, *q, work, st, a, b);
  const int rp = known ? planned.get() : KPM_OK;
  if (r != KPM_OK) return r;
  if (known) {
    if (rp != KPM_OK) return rp;
    apply_scale(p, n, a.data(), b.data(), P);
  } else {
    if (q->autotune) {
      r = get_tune(p, n, *q, a.data(), b.data(), work, need, st, tn);
      if (r != KPM_OK) return r;
    }
    r = make_plan(p, n, shape_of(*q, &tn), a.data(), b.data(), P);
    if (r != KPM_OK) return r;
  }
  const MomLayout L = moments_layout(P, n_steps(q->M), 0);
  if (L.total > need) return KPM_EWORKSPACE;
  std::vector<unsigned char> staging;
  r = upload_plan(P, work + L.plan, staging, st);
  if (r != KPM_OK) return r;
  std::vector<double> ab(2 * n);
  for (int i = 0; i < n; ++i) {
    ab[2 * i] = a[i];
    ab[2 * i + 1] = b[i];
  }
  if (d_ab) KPM_HIP(hipMemcpyAsync(d_ab, ab.data(), ab.size() * 8, hipMemcpyHostToDevice, st));
  return run_moments(P, L, work, *q, d_mu, st, direct);
}

}  // namespace

// Workspace of chebyshev_moments_noalloc: one array per GPU, loaded with the
// library's code object and held until the process ends.  In host code
// `scratch` names only a host-side stand-in; kernels get the device address
// that scratch_address() looks up.
static __device__ __align__(256) unsigned char scratch[KPM_NOALLOC_MAX_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu[kMaxDevices];              // held for a whole call on that GPU
unsigned char* g_scratch_ptr[kMaxDevices] = {};    // device address, once looked up

// Device address of the current GPU's `scratch`, looked up on the first call
// on that GPU (with it current) and kept.  Caller holds g_scratch_mu[dev].
int scratch_address(int dev, unsigned char** out) {
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return KPM_EDEVICE;
    g_scratch_ptr[dev] = static_cast<unsigned char*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return KPM_OK;
}

// No C++ exception leaves the library (the C ABI has no way to carry one): a
// failed host allocation, here or in the planning thread, reports KPM_ENOMEM,
// any other exception KPM_EDEVICE; a size query reports 0.
template <typename F>
int guarded(F&& f) noexcept {
  try {
    return f();
  } catch (const std::bad_alloc&) {
    return KPM_ENOMEM;
  } catch (...) {
    return KPM_EDEVICE;
  }
}
template <typename F>
size_t guarded_size(F&& f) noexcept {
  try {
    return f();
  } catch (...) {
    return 0;
  }
}

}  // namespace

extern "C" {

const char* kpm_strerror(int code) {
  switch (code) {
    case KPM_OK: return "ok";
    case KPM_EINVAL: return "invalid argument";
    case KPM_ENOMEM: return "allocation failed";
    case KPM_EDEVICE: return "HIP runtime error";
    case KPM_EBOUNDS: return "spectral bounds do not enclose the spectrum (|mu_n| > mu_0)";
    case KPM_EWORKSPACE: return "workspace too small";
    case KPM_ETOOLARGE: return "needs more scratch than KPM_NOALLOC_MAX_BYTES (64 MiB) per GPU";
    default: return "unknown status";
  }
}

int kpm_site_relabel(const kpm_problem* p, int32_t L, int32_t* h_perm) {
  return guarded([&]() -> int {
    if (!p || !h_perm || check_problem(*p) != KPM_OK || two_s_of(*p) > 1 || L < 1 || L > 16) return KPM_EINVAL;
    std::vector<uint8_t> perm;
    const bool moved = choose_relabel(*p, std::min<int>(L, p->n_sites), perm);
    for (int i = 0; i < p->n_sites; ++i) h_perm[i] = moved ? perm[i] : i;
    return moved ? 1 : 0;
  });
}

uint64_t kpm_sector_dim(int32_t n_sites, int32_t n_up) {
  if (n_sites < 0 || n_sites > 64) return 0;
  return binom64(n_sites, n_up);
}

int kpm_autotune_reset(void) {
  return guarded([&]() -> int {
    std::lock_guard<std::mutex> lock(g_tune_mu);
    g_tune_cache.clear();
    return KPM_OK;
  });
}

int kpm_last_run_stats(kpm_run_stats* out) {
  return guarded([&]() -> int {
    if (!out) return KPM_EINVAL;
    *out = g_stats;
    return KPM_OK;
  });
}

int kpm_sector_states(int32_t n_sites, int32_t n_up, uint32_t* d_states, void* stream) {
  return guarded([&]() -> int {
    if (n_sites < 1 || n_sites > 32 || n_up < 0 || n_up > n_sites || !d_states) return KPM_EINVAL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    StreamSync guard{st};
    const int64_t dim = (int64_t)binom64(n_sites, n_up);
    const std::vector<uint32_t> bt = binom_table();
    DevBuf buf;
    int r = buf.alloc(bt.size() * 4);
    if (r != KPM_OK) return r;
    KPM_HIP(hipMemcpyAsync(buf.p, bt.data(), bt.size() * 4, hipMemcpyHostToDevice, st));
    KPM_HIP(launch_states(n_sites, n_up, static_cast<uint32_t*>(buf.p), d_states, dim, st));
    KPM_HIP(hipStreamSynchronize(st));
    return KPM_OK;
  });
}

int kpm_sector_matrix(const kpm_problem* p, int64_t row0, int64_t nrows, int32_t max_nb,
                      uint32_t* d_cols, int32_t* d_bond, int32_t* d_cnt, double* d_diag,
                      void* stream) {
  return guarded([&]() -> int {
    if (!p || check_problem(*p) != KPM_OK || two_s_of(*p) > 1) return KPM_EINVAL;
    const int64_t dim = (int64_t)binom64(p->n_sites, p->n_up);
    if (row0 < 0 || nrows < 0 || row0 + nrows > dim || max_nb < p->n_bonds || max_nb < 1)
      return KPM_EINVAL;
    if (nrows == 0) return KPM_OK;
    if (!d_cols || !d_bond || !d_cnt || !d_diag) return KPM_EINVAL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    StreamSync guard{st};
    RunShape s;
    s.precision = KPM_FP64;
    s.col_block = 1;
    s.allow_row = false;
    Planned P;
    const double one = 1.0, zero = 0.0;
    int r = make_plan(p, 1, s, &one, &zero, P);
    if (r != KPM_OK) return r;
    DevBuf buf;
    r = buf.alloc(P.bytes);
    if (r != KPM_OK) return r;
    std::vector<unsigned char> staging;
    r = upload_plan(P, static_cast<unsigned char*>(buf.p), staging, st);
    if (r != KPM_OK) return r;
    const DevicePlan& D = P.plan;
    MatrixArgs a{};
    a.probs = D.probs;
    a.tables = D.tables;
    a.bmask = D.bmask;
    a.boff = D.boff;
    a.bzz = D.bzz;
    a.binom = D.binom;
    a.row0 = row0;
    a.nrows = nrows;
    a.max_nb = max_nb;
    a.lds_tab = D.lds_tab;
    a.lds_bonds = D.lds_bonds;
    a.sub_rows = D.sub_rows;
    a.lds_nb = D.lds_nb;
    a.cols = d_cols;
    a.bond = d_bond;
    a.cnt = d_cnt;
    a.diag = d_diag;
    const int64_t grid = (nrows + D.sub_rows - 1) / D.sub_rows;
    if (grid > (1LL << 30)) return KPM_EINVAL;
    KPM_HIP(launch_matrix(a, step_lds_bytes(D), (int)grid, st));
    KPM_HIP(hipStreamSynchronize(st));
    return KPM_OK;
  });
}

int kpm_spectral_bounds(const kpm_problem* p, int32_t n, int32_t steps, double margin,
                        uint64_t seed, double* e_lo_hi, void* stream) {
  return guarded([&]() -> int {
    if (check_problems(p, n) != KPM_OK || steps < 1 || !(margin >= 0.0) || !e_lo_hi)
      return KPM_EINVAL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    StreamSync guard{st};
    DevBuf buf;
    int r = buf.alloc(lanczos_bytes(p, n, steps));
    if (r != KPM_OK) return r;
    return run_lanczos(p, n, steps, margin, seed, e_lo_hi, static_cast<unsigned char*>(buf.p), st);
  });
}

size_t chebyshev_moments_workspace_size(const kpm_problem* p, int32_t n, const kpm_params* q) {
  return guarded_size([&]() -> size_t {
    if (check_problems(p, n) != KPM_OK || !q || check_params_moments(*q) != KPM_OK) return 0;
    return moments_workspace(p, n, *q);
  });
}

int chebyshev_moments(const kpm_problem* p, int32_t n, const kpm_params* q, double* d_mu,
                      double* d_ab, void* d_work, size_t work_bytes, void* stream) {
  return guarded([&]() -> int {
    int r = check_problems(p, n);
    if (r != KPM_OK) return r;
    if (!q || check_params_moments(*q) != KPM_OK || !d_mu) return KPM_EINVAL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    StreamSync guard{st};
    const size_t need = moments_workspace(p, n, *q);
    if (need == 0) return KPM_EINVAL;
    DevBuf own;
    unsigned char* work = static_cast<unsigned char*>(d_work);
    if (!work) {
      r = own.alloc(need);
      if (r != KPM_OK) return r;
      work = static_cast<unsigned char*>(own.p);
    } else if (work_bytes < need) {
      return KPM_EWORKSPACE;
    }
    return moments_on_workspace(p, n, q, d_mu, d_ab, work, need, st, false);
  });
}

int chebyshev_moments_noalloc(const kpm_problem* p, int32_t n, const kpm_params* q, double* d_mu,
                              double* d_ab, void* stream) {
  return guarded([&]() -> int {
    int r = check_problems(p, n);
    if (r != KPM_OK) return r;
    if (!q || check_params_moments(*q) != KPM_OK || !d_mu || q->autotune != 0) return KPM_EINVAL;
    const size_t need = moments_workspace(p, n, *q);
    if (need == 0) return KPM_EINVAL;
    if (need > KPM_NOALLOC_MAX_BYTES) return KPM_ETOOLARGE;
    int dev = 0;
    KPM_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return KPM_EDEVICE;
    std::lock_guard<std::mutex> lock(g_scratch_mu[dev]);
    hipStream_t st = static_cast<hipStream_t>(stream);
    StreamSync guard{st};  // released before the lock: the array is idle when the next call starts
    unsigned char* work = nullptr;
    r = scratch_address(dev, &work);
    if (r != KPM_OK) return r;
    return moments_on_workspace(p, n, q, d_mu, d_ab, work, need, st, true);
  });
}

static kpm_params vectors_params(const kpm_params& q, int32_t n_vec) {
  kpm_params q2 = q;
  q2.M = std::max(2, 2 * n_vec);
  return q2;
}

size_t chebyshev_vectors_workspace_size(const kpm_problem* p, const kpm_params* q, int32_t n_vec) {
  return guarded_size([&]() -> size_t {
    if (check_problems(p, 1) != KPM_OK || !q || n_vec < 0) return 0;
    const kpm_params q2 = vectors_params(*q, n_vec);
    if (check_params(q2) != KPM_OK) return 0;
    return moments_workspace(p, 1, q2);
  });
}

int chebyshev_vectors(const kpm_problem* p, const kpm_params* q, int32_t n_vec, void* d_out,
                      double* d_ab, void* d_work, size_t work_bytes, void* stream) {
  return guarded([&]() -> int {
    int r = check_problems(p, 1);
    if (r != KPM_OK) return r;
    if (!q || n_vec < 0 || !d_out) return KPM_EINVAL;
    const kpm_params q2 = vectors_params(*q, n_vec);
    if (check_params(q2) != KPM_OK) return KPM_EINVAL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    StreamSync guard{st};
    const size_t need = moments_workspace(p, 1, q2);
    if (need == 0) return KPM_EINVAL;
    DevBuf own;
    unsigned char* work = static_cast<unsigned char*>(d_work);
    if (!work) {
      r = own.alloc(need);
      if (r != KPM_OK) return r;
      work = static_cast<unsigned char*>(own.p);
    } else if (work_bytes < need) {
      return KPM_EWORKSPACE;
    }
    Planned P0;
    r = make_plan(p, 1, shape_of(q2), nullptr, nullptr, P0);
    if (r != KPM_OK) return r;
    const MomLayout L0 = moments_layout(P0, n_steps(q2.M), 0);
    std::vector<double> a, b;
    r = resolve_scale(p, 1, q2, work + L0.lz, st, a, b);
    if (r != KPM_OK) return r;
    Planned P;
    r = make_plan(p, 1, shape_of(q2), a.data(), b.data(), P);
    if (r != KPM_OK) return r;
    const MomLayout L = moments_layout(P, n_steps(q2.M), 0);
    std::vector<unsigned char> staging;
    r = upload_plan(P, work + L.plan, staging, st);
    if (r != KPM_OK) return r;
    const double ab[2] = {a[0], b[0]};
    if (d_ab) KPM_HIP(hipMemcpyAsync(d_ab, ab, sizeof(ab), hipMemcpyHostToDevice, st));
    return run_vectors(P, L, work, q2, n_vec, d_out, st);
  });
}

int kpm_thermo(const double* d_mu, const double* d_ab, const kpm_problem* p, int32_t n,
               int32_t M, int32_t kernel, int32_t n_nodes, const double* d_T, int32_t n_T,
               double* d_lnZ, double* d_E, double* d_C, double* d_chi, uint8_t* d_znonpos,
               void* stream) {
  return guarded([&]() -> int {
    if (!d_lnZ || !d_E || !d_C || !d_chi) return KPM_EINVAL;
    ThermoDev TD;
    std::vector<ThermoProb> tp;
    int nc = 0;
    return thermo_forward(d_mu, d_ab, p, n, M, kernel, n_nodes, d_T, n_T, d_lnZ, d_E, d_C, d_chi,
                          d_znonpos, static_cast<hipStream_t>(stream), TD, tp, nc, false);
  });
}

int kpm_thermo_field(const double* d_mu, const double* d_ab, const kpm_problem* p, int32_t n,
                     int32_t M, int32_t kernel, int32_t n_nodes, const double* d_T,
                     const double* d_h, int32_t n_pts, double* d_lnZ, double* d_E, double* d_C,
                     double* d_chi, double* d_mag, uint8_t* d_znonpos, void* stream) {
  return guarded([&]() -> int {
    if (!d_h || !d_lnZ || !d_E || !d_C || !d_chi) return KPM_EINVAL;
    ThermoDev TD;
    std::vector<ThermoProb> tp;
    int nc = 0;
    return thermo_forward(d_mu, d_ab, p, n, M, kernel, n_nodes, d_T, n_pts, d_lnZ, d_E, d_C, d_chi,
                          d_znonpos, static_cast<hipStream_t>(stream), TD, tp, nc, false, d_h, d_mag);
  });
}

int kpm_thermo_vjp(const double* d_mu, const double* d_ab, const kpm_problem* p, int32_t n,
                   int32_t M, int32_t kernel, int32_t n_nodes, const double* d_T, int32_t n_T,
                   const double* d_wC, const double* d_wchi, double* d_lambda, void* stream) {
  return guarded([&]() -> int {
    if (!d_wC || !d_wchi || !d_lambda) return KPM_EINVAL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    std::vector<ThermoProb> tp;
    std::vector<int32_t> start, list;
    int nc = 0;
    if (thermo_meta(p, n, tp, start, list, nc) != KPM_OK) return KPM_EINVAL;
    StreamSync guard{st};
    DevBuf outs;
    int r = outs.alloc((size_t)4 * nc * n_T * 8);
    if (r != KPM_OK) return r;
    double* o = static_cast<double*>(outs.p);
    const size_t m = (size_t)nc * n_T;
    ThermoDev TD;
    r = thermo_forward(d_mu, d_ab, p, n, M, kernel, n_nodes, d_T, n_T, o, o + m, o + 2 * m, o + 3 * m,
                       nullptr, st, TD, tp, nc, true);
    if (r != KPM_OK) return r;
    ThermoVjpArgs va{};
    va.tp = TD.tp;
    va.ab = d_ab;
    va.stats = TD.stats;
    va.wC = d_wC;
    va.wchi = d_wchi;
    va.g = TD.g;
    va.node_adj = TD.adj;
    va.lambda = d_lambda;
    va.n_probs = n;
    va.M = M;
    va.n_nodes = n_nodes ? n_nodes : M;
    va.n_T = n_T;
    KPM_HIP(launch_thermo_vjp(va, st));
    KPM_HIP(hipStreamSynchronize(st));
    return KPM_OK;
  });
}

size_t chebyshev_moments_vjp_workspace_size(const kpm_problem* p, int32_t n, const kpm_params* q,
                                            int32_t ckpt_every) {
  return guarded_size([&]() -> size_t {
    if (check_problems(p, n) != KPM_OK || !q || check_params(*q) != KPM_OK || ckpt_every < 2)
      return 0;
    return vjp_workspace(p, n, *q, ckpt_every);
  });
}

int chebyshev_moments_vjp(const kpm_problem* p, int32_t n, const kpm_params* q,
                          const double* d_ab, const double* d_dmu, int32_t ckpt_every,
                          double* d_dJ, void* d_work, size_t work_bytes, void* stream) {
  return guarded([&]() -> int {
    int r = check_problems(p, n);
    if (r != KPM_OK) return r;
    if (!q || check_params(*q) != KPM_OK || !d_ab || !d_dmu || !d_dJ || ckpt_every < 2)
      return KPM_EINVAL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    StreamSync guard{st};
    const size_t need = vjp_workspace(p, n, *q, ckpt_every);
    if (need == 0) return KPM_EINVAL;
    DevBuf own;
    unsigned char* work = static_cast<unsigned char*>(d_work);
    if (!work) {
      r = own.alloc(need);
      if (r != KPM_OK) return r;
      work = static_cast<unsigned char*>(own.p);
    } else if (work_bytes < need) {
      return KPM_EWORKSPACE;
    }
    std::vector<double> h_ab(2 * n);
    KPM_HIP(hipMemcpyAsync(h_ab.data(), d_ab, h_ab.size() * 8, hipMemcpyDeviceToHost, st));
    KPM_HIP(hipStreamSynchronize(st));
    return run_vjp(p, n, *q, h_ab.data(), d_dmu, ckpt_every, d_dJ, work, st);
  });
}

size_t chebyshev_moments_ckpt_workspace_size(const kpm_problem* p, int32_t n, const kpm_params* q,
                                             int32_t ckpt_every) {
  return guarded_size([&]() -> size_t {
    if (check_problems(p, n) != KPM_OK || !q || check_params(*q) != KPM_OK || ckpt_every < 2) return 0;
    const size_t m = moments_workspace(p, n, *q);
    const size_t v = vjp_workspace(p, n, *q, ckpt_every);
    return (m && v) ? std::max(m, v) : 0;
  });
}

int chebyshev_moments_ckpt(const kpm_problem* p, int32_t n, const kpm_params* q, int32_t ckpt_every,
                           double* d_mu, double* d_ab, void* d_work, size_t work_bytes, void* stream) {
  return guarded([&]() -> int {
    int r = check_problems(p, n);
    if (r != KPM_OK) return r;
    if (!q || check_params(*q) != KPM_OK || !d_mu || !d_ab || !d_work || ckpt_every < 2) return KPM_EINVAL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    StreamSync guard{st};
    const size_t need = chebyshev_moments_ckpt_workspace_size(p, n, q, ckpt_every);
    if (need == 0) return KPM_EINVAL;
    if (work_bytes < need) return KPM_EWORKSPACE;
    unsigned char* work = static_cast<unsigned char*>(d_work);
    Planned P0;
    r = make_plan(p, n, shape_of(*q), nullptr, nullptr, P0);
    if (r != KPM_OK) return r;
    const MomLayout L0 = moments_layout(P0, n_steps(q->M), 0);
    std::vector<double> a, b;
    r = resolve_scale(p, n, *q, work + L0.lz, st, a, b);
    if (r != KPM_OK) return r;
    std::vector<double> h_ab(2 * n);
    for (int i = 0; i < n; ++i) {
      h_ab[2 * i] = a[i];
      h_ab[2 * i + 1] = b[i];
    }
    KPM_HIP(hipMemcpyAsync(d_ab, h_ab.data(), h_ab.size() * 8, hipMemcpyHostToDevice, st));
    return run_vjp(p, n, *q, h_ab.data(), nullptr, ckpt_every, nullptr, work, st, d_mu, {}, kVjpForward);
  });
}

int chebyshev_moments_vjp_resume(const kpm_problem* p, int32_t n, const kpm_params* q,
                                 const double* d_ab, const double* d_dmu, int32_t ckpt_every,
                                 double* d_dJ, void* d_work, size_t work_bytes, void* stream) {
  return guarded([&]() -> int {
    int r = check_problems(p, n);
    if (r != KPM_OK) return r;
    if (!q || check_params(*q) != KPM_OK || !d_ab || !d_dmu || !d_dJ || !d_work || ckpt_every < 2)
      return KPM_EINVAL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    StreamSync guard{st};
    const size_t need = chebyshev_moments_ckpt_workspace_size(p, n, q, ckpt_every);
    if (need == 0) return KPM_EINVAL;
    if (work_bytes < need) return KPM_EWORKSPACE;
    std::vector<double> h_ab(2 * n);
    KPM_HIP(hipMemcpyAsync(h_ab.data(), d_ab, h_ab.size() * 8, hipMemcpyDeviceToHost, st));
    KPM_HIP(hipStreamSynchronize(st));
    return run_vjp(p, n, *q, h_ab.data(), d_dmu, ckpt_every, d_dJ, static_cast<unsigned char*>(d_work), st,
                   nullptr, {}, kVjpReverse);
  });
}

int kpm_cluster_bond_grad(const kpm_problem* p, int32_t n, const double* d_dJ, double* d_dJ_cluster,
                          void* stream) {
  return guarded([&]() -> int {
    if (!p || n <= 0 || !d_dJ || !d_dJ_cluster) return KPM_EINVAL;
    if (const int e = check_problems(p, n)) return e;
    int nc = 0, max_b = 0;
    for (int i = 0; i < n; ++i) nc = std::max(nc, p[i].cluster + 1);
    std::vector<int32_t> info(2 * (size_t)n), cinfo(2 * (size_t)nc, 0), nb(nc, -1);
    int32_t off = 0;
    for (int i = 0; i < n; ++i) {
      const int c = p[i].cluster;
      if (nb[c] >= 0 && nb[c] != p[i].n_bonds) return KPM_EINVAL;   // one bond list per cluster
      nb[c] = p[i].n_bonds;
      info[2 * i] = c;
      info[2 * i + 1] = off;
      off += p[i].n_bonds;
    }
    int32_t out = 0;
    for (int c = 0; c < nc; ++c) {
      cinfo[2 * c] = out;
      cinfo[2 * c + 1] = std::max(nb[c], 0);
      out += cinfo[2 * c + 1];
      max_b = std::max(max_b, cinfo[2 * c + 1]);
    }
    if (max_b == 0) return KPM_OK;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    StreamSync sync{st};
    int32_t* d_tab = nullptr;
    const size_t bytes = (info.size() + cinfo.size()) * sizeof(int32_t);
    if (hipMalloc(&d_tab, bytes) != hipSuccess) return KPM_ENOMEM;
    int rc = KPM_OK;
    if (hipMemcpyAsync(d_tab, info.data(), info.size() * 4, hipMemcpyHostToDevice, st) != hipSuccess ||
        hipMemcpyAsync(d_tab + info.size(), cinfo.data(), cinfo.size() * 4, hipMemcpyHostToDevice, st) !=
            hipSuccess ||
        launch_cluster_grad(d_tab, n, d_tab + info.size(), nc, max_b, d_dJ, d_dJ_cluster, st) != hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      rc = KPM_EDEVICE;
    (void)hipFree(d_tab);
    return rc;
  });
}

int kpm_thermo_grad(const kpm_problem* p, int32_t n, const kpm_params* q, int32_t kernel,
                    int32_t n_nodes, const double* d_T, int32_t n_T, const double* d_wC,
                    const double* d_wchi, int32_t ckpt_every, double* d_L, double* d_dJ,
                    double* d_ab, void* d_work, size_t work_bytes, void* stream) {
  return guarded([&]() -> int {
    int r = check_problems(p, n);
    if (r != KPM_OK) return r;
    if (!q || check_params(*q) != KPM_OK || !d_T || n_T < 1 || !d_wC || !d_wchi || !d_L || !d_dJ ||
        ckpt_every < 2 || (kernel != 0 && kernel != 1) || n_nodes < 0)
      return KPM_EINVAL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    StreamSync guard{st};
    std::vector<ThermoProb> tp;
    std::vector<int32_t> start, list;
    int nc = 0;
    if (thermo_meta(p, n, tp, start, list, nc) != KPM_OK) return KPM_EINVAL;
    const size_t need_m = moments_workspace(p, n, *q);
    const size_t need_v = vjp_workspace(p, n, *q, ckpt_every);
    if (!need_m || !need_v) return KPM_EINVAL;
    const size_t need = std::max(need_m, need_v);
    DevBuf own;
    unsigned char* work = static_cast<unsigned char*>(d_work);
    if (!work) {
      r = own.alloc(need);
      if (r != KPM_OK) return r;
      work = static_cast<unsigned char*>(own.p);
    } else if (work_bytes < need) {
      return KPM_EWORKSPACE;
    }
    const size_t m = (size_t)nc * n_T;
    DevBuf tmp;
    r = tmp.alloc(align_up((size_t)n * q->M * 8) * 2 + align_up((size_t)n * 16) + 4 * align_up(m * 8));
    if (r != KPM_OK) return r;
    unsigned char* t8 = static_cast<unsigned char*>(tmp.p);
    double* mu = reinterpret_cast<double*>(t8);
    double* lam = reinterpret_cast<double*>(t8 + align_up((size_t)n * q->M * 8));
    double* ab = reinterpret_cast<double*>(t8 + 2 * align_up((size_t)n * q->M * 8));
    double* outs = reinterpret_cast<double*>(t8 + 2 * align_up((size_t)n * q->M * 8) + align_up((size_t)n * 16));
    const size_t ms = align_up(m * 8) / 8;
    // bounds and (a, b) as chebyshev_moments resolves them
    Planned P0;
    r = make_plan(p, n, shape_of(*q), nullptr, nullptr, P0);
    if (r != KPM_OK) return r;
    const MomLayout L0 = moments_layout(P0, n_steps(q->M), 0);
    std::vector<double> a, b;
    r = resolve_scale(p, n, *q, work + L0.lz, st, a, b);
    if (r != KPM_OK) return r;
    std::vector<double> h_ab(2 * n);
    for (int i = 0; i < n; ++i) {
      h_ab[2 * i] = a[i];
      h_ab[2 * i + 1] = b[i];
    }
    KPM_HIP(hipMemcpyAsync(ab, h_ab.data(), h_ab.size() * 8, hipMemcpyHostToDevice, st));
    if (d_ab) KPM_HIP(hipMemcpyAsync(d_ab, ab, (size_t)n * 16, hipMemcpyDeviceToDevice, st));
    // the adjoint's checkpointed forward pass gives the moments; between it and
    // the reverse sweep: dL/dmu, and L from the thermodynamics
    auto between = [&]() -> int {
      int rr = kpm_thermo_vjp(mu, ab, p, n, q->M, kernel, n_nodes, d_T, n_T, d_wC, d_wchi, lam, stream);
      if (rr != KPM_OK) return rr;
      rr = kpm_thermo(mu, ab, p, n, q->M, kernel, n_nodes, d_T, n_T, outs, outs + ms, outs + 2 * ms,
                      outs + 3 * ms, nullptr, stream);
      if (rr != KPM_OK) return rr;
      KPM_HIP(launch_loss(outs + 2 * ms, outs + 3 * ms, d_wC, d_wchi, (int)m, d_L, st));
      return KPM_OK;
    };
    return run_vjp(p, n, *q, h_ab.data(), lam, ckpt_every, d_dJ, work, st, mu, between);
  });
}

size_t kpm_ftlm_workspace_size(const kpm_problem* p, int32_t n, const kpm_params* q) {
  return guarded_size([&]() -> size_t {
    if (check_problems(p, n) != KPM_OK || !q || check_params(*q) != KPM_OK) return 0;
    if (q->precision != KPM_FP64) return 0;
    Planned P;
    const std::vector<double> two(n, 2.0), zero(n, 0.0);
    if (make_plan(p, n, ftlm_shape(*q, p, n), two.data(), zero.data(), P) != KPM_OK) return 0;
    return ftlm_layout(P, ftlm_steps(P, q->M)).total;
  });
}

int kpm_ftlm(const kpm_problem* p, int32_t n, const kpm_params* q, const double* d_T,
             const double* d_h, int32_t n_pts, double* d_lnZ, double* d_E, double* d_C,
             double* d_chi, double* d_mag, double* d_ritz, double* d_weight, void* d_work,
             size_t work_bytes, void* stream) {
  return guarded([&]() -> int {
    int r = check_problems(p, n);
    if (r != KPM_OK) return r;
    if (!q || check_params(*q) != KPM_OK || q->precision != KPM_FP64) return KPM_EINVAL;
    if (!d_T || n_pts < 1 || !d_lnZ || !d_E || !d_C || !d_chi) return KPM_EINVAL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    StreamSync guard{st};
    Planned P;
    // H' = H / 2 (a = 2, b = 0), so that the recursion step's 2 H' x - y is H q_j - beta_j q_{j-1}
    const std::vector<double> two(n, 2.0), zero_b(n, 0.0);
    r = make_plan(p, n, ftlm_shape(*q, p, n), two.data(), zero_b.data(), P);
    if (r != KPM_OK) return r;
    const int steps = ftlm_steps(P, q->M);
    const FtlmLayout L = ftlm_layout(P, steps);
    DevBuf own;
    unsigned char* work = static_cast<unsigned char*>(d_work);
    if (!work) {
      r = own.alloc(L.total);
      if (r != KPM_OK) return r;
      work = static_cast<unsigned char*>(own.p);
    } else if (work_bytes < L.total) {
      return KPM_EWORKSPACE;
    }
    std::vector<unsigned char> staging;
    r = upload_plan(P, work + L.plan, staging, st);
    if (r != KPM_OK) return r;
    DevicePlan& D = P.plan;
    D.err = reinterpret_cast<int*>(work + L.err);
    D.states = reinterpret_cast<uint32_t*>(work + L.states);
    KPM_HIP(hipMemsetAsync(D.err, 0, sizeof(int), st));
    if (D.row_ld || D.block || D.spin) KPM_HIP(fill_states(D, st));
    double* vec = reinterpret_cast<double*>(work + L.vec);
    double* part = reinterpret_cast<double*>(work + L.part);
    double* dots = reinterpret_cast<double*>(work + L.dots);
    double* b2 = reinterpret_cast<double*>(work + L.b2);
    double* norm = reinterpret_cast<double*>(work + L.norm);
    const int TC = D.total_cols;
    KPM_HIP(hipMemsetAsync(vec, 0, (size_t)D.vec_elems * 8, st));
    // unit-norm start columns (the random vectors of Eq. (7)), |column|^2 kept
    KPM_HIP(launch_init(D, vec, 0, q->vec_kind, q->seed, nullptr, part, st));
    KPM_HIP(launch_reduce(D, part, norm, nullptr, st));
    KPM_HIP(launch_init(D, vec, 2, q->vec_kind, q->seed, norm, part, st));
    // Lanczos per column (lanczos_turns)
    r = lanczos_turns(D, vec, part, dots, b2, reinterpret_cast<double*>(work + L.ww),
                      reinterpret_cast<double*>(work + L.fixed), reinterpret_cast<double*>(work + L.ybeta), steps, st);
    if (r != KPM_OK) return r;
    // thermodynamic metadata (sector weights, S^z, clusters)
    std::vector<ThermoProb> tp;
    std::vector<int32_t> start, list;
    int nc = 0;
    r = thermo_meta(p, n, tp, start, list, nc);
    if (r != KPM_OK) return r;
    DevBuf meta;
    const size_t otp = 0, ost = align_up(tp.size() * sizeof(ThermoProb)),
                 oli = ost + align_up(start.size() * 4);
    r = meta.alloc(oli + list.size() * 4);
    if (r != KPM_OK) return r;
    unsigned char* mb = static_cast<unsigned char*>(meta.p);
    KPM_HIP(hipMemcpyAsync(mb + otp, tp.data(), tp.size() * sizeof(ThermoProb), hipMemcpyHostToDevice, st));
    KPM_HIP(hipMemcpyAsync(mb + ost, start.data(), start.size() * 4, hipMemcpyHostToDevice, st));
    KPM_HIP(hipMemcpyAsync(mb + oli, list.data(), list.size() * 4, hipMemcpyHostToDevice, st));
    FtlmArgs fa{};
    fa.probs = D.probs;
    fa.units = D.units;
    fa.job_unit = D.job_unit;
    fa.prob_unit0 = D.prob_unit0;
    fa.dots = dots;
    fa.b2 = b2;
    fa.norms = norm;
    fa.ritz = reinterpret_cast<double*>(work + L.ritz);
    fa.escr = reinterpret_cast<double*>(work + L.escr);
    fa.weight = reinterpret_cast<double*>(work + L.weight);
    fa.len = reinterpret_cast<int32_t*>(work + L.len);
    fa.err = D.err;
    fa.total_cols = TC;
    fa.steps = steps;
    fa.vec_kind = q->vec_kind;
    fa.R = q->vec_kind == KPM_VEC_BASIS ? 0 : q->R;
    fa.tp = reinterpret_cast<ThermoProb*>(mb + otp);
    fa.cl_start = reinterpret_cast<int32_t*>(mb + ost);
    fa.cl_list = reinterpret_cast<int32_t*>(mb + oli);
    fa.T = d_T;
    fa.h = d_h;
    fa.lnZ = d_lnZ;
    fa.E = d_E;
    fa.C = d_C;
    fa.chi = d_chi;
    fa.mag = d_mag;
    fa.n_pts = n_pts;
    fa.n_clusters = nc;
    KPM_HIP(launch_ftlm_ritz(fa, st));
    KPM_HIP(launch_ftlm_thermo(fa, st));
    // real columns only (blocks may be padded), problem after problem
    if (d_ritz || d_weight) {
      size_t row = 0;
      for (const auto& u : P.units) {
        const size_t bytes = (size_t)u.ncols * steps * 8, src = (size_t)u.col_off * steps;
        if (d_ritz)
          KPM_HIP(hipMemcpyAsync(d_ritz + row * steps, fa.ritz + src, bytes, hipMemcpyDeviceToDevice, st));
        if (d_weight)
          KPM_HIP(hipMemcpyAsync(d_weight + row * steps, fa.weight + src, bytes, hipMemcpyDeviceToDevice, st));
        row += (size_t)u.ncols;
      }
    }
    int h_err = 0;
    KPM_HIP(hipMemcpyAsync(&h_err, D.err, sizeof(int), hipMemcpyDeviceToHost, st));
    KPM_HIP(hipStreamSynchronize(st));
    return h_err ? KPM_EDEVICE : KPM_OK;
  });
}

size_t kpm_sector_eigenvalues_workspace_size(const kpm_problem* p, int32_t n, int32_t max_dim) {
  return guarded_size([&]() -> size_t {
    EdPlan E;
    if (ed_plan(p, n, max_dim, E) != KPM_OK) return 0;
    return E.total;
  });
}

int kpm_sector_eigenvalues(const kpm_problem* p, int32_t n, int32_t max_dim, double* d_evals,
                           void* d_work, size_t work_bytes, void* stream) {
  return guarded([&]() -> int {
    EdPlan E;
    int r = ed_plan(p, n, max_dim, E);
    if (r != KPM_OK) return r;
    if (!d_evals) return KPM_EINVAL;
    hipStream_t st = static_cast<hipStream_t>(stream);
    StreamSync guard{st};
    DevBuf own;
    unsigned char* work = static_cast<unsigned char*>(d_work);
    if (!work) {
      r = own.alloc(E.total);
      if (r != KPM_OK) return r;
      work = static_cast<unsigned char*>(own.p);
    } else if (work_bytes < E.total) {
      return KPM_EWORKSPACE;
    }
    // NaN (all bits set) past each spectrum and in the rows of larger sectors
    KPM_HIP(hipMemsetAsync(d_evals, 0xFF, (size_t)n * max_dim * 8, st));
    const std::vector<uint32_t> bt = binom_table();
    std::vector<unsigned char> staging(E.o_mat, 0);
    std::memcpy(staging.data() + E.o_probs, E.probs.data(), E.probs.size() * sizeof(EigProb));
    std::memcpy(staging.data() + E.o_mask, E.bmask.data(), E.bmask.size() * 4);
    std::memcpy(staging.data() + E.o_J, E.J.data(), E.J.size() * 8);
    std::memcpy(staging.data() + E.o_binom, bt.data(), bt.size() * 4);
    if (!E.tables.empty()) std::memcpy(staging.data() + E.o_tab, E.tables.data(), E.tables.size() * 4);
    KPM_HIP(hipMemcpyAsync(work, staging.data(), E.o_mat, hipMemcpyHostToDevice, st));
    EigArgs a{};
    a.probs = reinterpret_cast<const EigProb*>(work + E.o_probs);
    a.bmask = reinterpret_cast<const uint32_t*>(work + E.o_mask);
    a.J = reinterpret_cast<const double*>(work + E.o_J);
    a.binom = reinterpret_cast<const uint32_t*>(work + E.o_binom);
    a.tables = reinterpret_cast<const uint32_t*>(work + E.o_tab);
    a.err = reinterpret_cast<int*>(work + E.o_err);
    a.mat = reinterpret_cast<double*>(work + E.o_mat);
    double* vecs = reinterpret_cast<double*>(work + E.o_vecs);
    a.hv = vecs;
    a.hp = vecs + E.vec_len;
    a.hd = vecs + 2 * E.vec_len;
    a.he = vecs + 3 * E.vec_len;
    a.evals = d_evals;
    a.ld = max_dim;
    a.max_dim = 1;
    std::vector<int> dims;
    for (const auto& e : E.probs) {
      a.max_dim = std::max(a.max_dim, e.dim);
      dims.push_back(e.dim);
    }
    // LDS: binomial table, bond masks and J values (build); the tridiagonal matrix (finish)
    a.o_bonds = (int32_t)align_up((size_t)(kBinomN * kBinomN + E.max_bonds) * 4, 16);
    const size_t lds_build = (size_t)a.o_bonds + (size_t)E.max_bonds * 8;
    const size_t lds_finish = (size_t)2 * a.max_dim * 8;   // d, e^2 (bisection)
    if (lds_build > 64 * 1024 || lds_finish > 64 * 1024) return KPM_EINVAL;
    KPM_HIP(hipMemsetAsync(a.err, 0, sizeof(int), st));
    KPM_HIP(launch_sector_eig(a, dims.data(), (int)E.probs.size(), lds_build, lds_finish, st));
    int h_err = 0;
    KPM_HIP(hipMemcpyAsync(&h_err, a.err, sizeof(int), hipMemcpyDeviceToHost, st));
    KPM_HIP(hipStreamSynchronize(st));
    return h_err ? KPM_EDEVICE : KPM_OK;
  });
}

int kpm_thermo_hybrid(const double* d_mu, const double* d_ab, const kpm_problem* p, int32_t n,
                      int32_t M, int32_t kernel, int32_t n_nodes, const double* d_evals,
                      int32_t evals_ld, const uint8_t* h_exact, const double* d_T, const double* d_h,
                      int32_t n_pts, double* d_lnZ, double* d_E, double* d_C, double* d_chi,
                      double* d_mag, uint8_t* d_znonpos, void* stream) {
  return guarded([&]() -> int {
    if (!d_mu || !d_ab || !d_T || !h_exact || !d_lnZ || !d_E || !d_C || !d_chi || M < 1 ||
        n_pts < 1 || n_nodes < 0 || (kernel != 0 && kernel != 1))
      return KPM_EINVAL;
    std::vector<ThermoProb> tp;
    std::vector<int32_t> start, list;
    int nc = 0;
    int r = thermo_meta(p, n, tp, start, list, nc);
    if (r != KPM_OK) return r;
    std::vector<int32_t> cnt(n, 0);
    for (int i = 0; i < n; ++i) {
      if (!h_exact[i]) continue;
      const uint64_t dim = prob_dim(p[i]);
      if (!d_evals || dim > (uint64_t)std::max(evals_ld, 0)) return KPM_EINVAL;
      cnt[i] = (int32_t)dim;
    }
    hipStream_t st = static_cast<hipStream_t>(stream);
    StreamSync guard{st};
    const int Nt = n_nodes ? n_nodes : M;
    size_t o = 0;
    auto put = [&](size_t bytes) {
      const size_t rr = o;
      o = align_up(o + bytes);
      return rr;
    };
    const size_t og = put((size_t)M * 8), ogam = put((size_t)n * Nt * 8),
                 otp = put(tp.size() * sizeof(ThermoProb)), ostart = put(start.size() * 4),
                 olist = put(list.size() * 4), ocnt = put(cnt.size() * 4);
    DevBuf buf;
    r = buf.alloc(o);
    if (r != KPM_OK) return r;
    unsigned char* w = static_cast<unsigned char*>(buf.p);
    KPM_HIP(hipMemcpyAsync(w + otp, tp.data(), tp.size() * sizeof(ThermoProb), hipMemcpyHostToDevice, st));
    KPM_HIP(hipMemcpyAsync(w + ostart, start.data(), start.size() * 4, hipMemcpyHostToDevice, st));
    KPM_HIP(hipMemcpyAsync(w + olist, list.data(), list.size() * 4, hipMemcpyHostToDevice, st));
    KPM_HIP(hipMemcpyAsync(w + ocnt, cnt.data(), cnt.size() * 4, hipMemcpyHostToDevice, st));
    double* g = reinterpret_cast<double*>(w + og);
    double* gamma = reinterpret_cast<double*>(w + ogam);
    KPM_HIP(launch_kernel_coef(M, kernel, g, st));
    KPM_HIP(launch_gamma(n, M, Nt, g, d_mu, gamma, st));
    ThermoArgs ta{};
    ta.tp = reinterpret_cast<const ThermoProb*>(w + otp);
    ta.cl_start = reinterpret_cast<const int32_t*>(w + ostart);
    ta.cl_list = reinterpret_cast<const int32_t*>(w + olist);
    ta.gamma = gamma;
    ta.ab = d_ab;
    ta.T = d_T;
    ta.lnZ = d_lnZ;
    ta.E = d_E;
    ta.C = d_C;
    ta.chi = d_chi;
    ta.znonpos = d_znonpos;
    ta.n_nodes = Nt;
    ta.n_T = n_pts;
    ta.n_clusters = nc;
    ta.h = d_h;
    ta.mag = d_mag;
    ta.ed_count = reinterpret_cast<const int32_t*>(w + ocnt);
    ta.evals = d_evals;
    ta.evals_ld = evals_ld;
    KPM_HIP(launch_thermo_hybrid(ta, st));
    KPM_HIP(hipStreamSynchronize(st));
    return KPM_OK;
  });
}

}  // extern "C"
