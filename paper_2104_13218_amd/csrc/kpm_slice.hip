// Slice step kernel: the recursion step v_{n+1} = 2 H' v_n - v_{n-1} (v_1 =
// H' v_0) with the fused dots (paper, Eqs. (4)-(7); the S^z-sector bit basis of
// Sec. II), for narrow column blocks (16-byte chunks, at most a few per row).
//
// Basis blocks are those of the block-table kernel: the states sharing their
// high word h = s >> L, member i of block h holding the i-th L-bit low word of
// its popcount class in colex order.  A bond between two high sites acts on
// every member of a block or on none and maps member i of block h to member i
// of block h ^ m; a bond between two low sites stays inside the block; a mixed
// bond (one low, one high site) moves a member to the block h ^ m_high, at the
// colex rank of the flipped low word.
//
// One wave per workgroup (nw = 1, no workgroup barriers) or nw waves sharing a
// tile.  A workgroup walks the blocks of its tile; per block it
//   1. copies the block's rows of v_n into LDS (row 0 of its LDS area stays
//      zero); with nw > 1 the whole tile's rows (consecutive ranks) are
//      copied once, before one barrier;
//   2. runs "slices" of 64 / nch members (nch = 16-byte chunks per row), one
//      member and chunk per lane; with nw > 1 the tile's slices, numbered
//      across its blocks, go round robin to the waves (slice k to wave
//      k mod nw).  Everything a block shares is scalar:
//      its high word, the acting high-high bonds (their target blocks' first
//      ranks and coefficients J_b/(2a) from per-block tables), and the
//      high-high part of the diagonal.  High-high rows are buffer loads whose
//      per-lane offset (member i, chunk c) is the same for every target block
//      and whose scalar offset is the target block's start.
// Per lane, one row of a per-call word table (indexed by the low word's
// position in its class) gives the low-low part of the diagonal, the low
// word l, the colex rank of l ^ m_low for each mixed bond, and per low-low
// bond the LDS row of the neighbour (0, the zero row, when the bond does not
// act).  Sum order per element: diagonal, low-low, high-high, mixed, each in
// bond order.
//
// Why nw > 1: the far high-high partners of a row are re-read from the L2
// only while their rows are still there.  The rows in use at any time span
// every tile open on an XCD; with one wave per tile that is every resident
// wave's tile, with nw waves per tile nw times fewer tiles, each finished nw
// times sooner, so more partner reads find their rows in the L2.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "kpm_device.h"
#include "kpm_internal.h"
#include "kpm_vec.h"

namespace kpm {

// Constant-address-space views: loads at wave-uniform indices become scalar
// loads (the tables are not written during a step).
template <typename T>
using cptr = const __attribute__((address_space(4))) T*;
template <typename T>
__device__ __forceinline__ cptr<T> cview(const T* p) {
  return (cptr<T>)(const void*)p;
}

// A plan struct at a wave-uniform address, word by word through scalar loads.
template <typename S>
__device__ __forceinline__ S sload(const S* p) {
  static_assert(sizeof(S) % 4 == 0, "word-sized struct");
  S out;
  const cptr<uint32_t> q = cview(reinterpret_cast<const uint32_t*>(p));
  uint32_t w[sizeof(S) / 4];
#pragma unroll
  for (int i = 0; i < (int)(sizeof(S) / 4); ++i) w[i] = q[i];
  __builtin_memcpy(&out, w, sizeof(S));
  return out;
}

// LDS ordering inside one wave (the block's rows are written by some lanes
// and read by others).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <typename T, int CPL>
__device__ __forceinline__ VecT<T, CPL> bload(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  VecT<T, CPL> v;
  constexpr int bytes = (int)sizeof(T) * CPL;
  if constexpr (bytes == 16) {
    const auto x = __builtin_amdgcn_raw_buffer_load_b128(r, voff, soff, 0);
    __builtin_memcpy(&v, &x, 16);
  } else if constexpr (bytes == 8) {
    const auto x = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0);
    __builtin_memcpy(&v, &x, 8);
  } else {
    const auto x = __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0);
    __builtin_memcpy(&v, &x, 4);
  }
  return v;
}

// v_{n-1} is read once and v_{n+1} written once per step: streaming (glc slc)
template <typename T, int CPL>
__device__ __forceinline__ VecT<T, CPL> bload_nt(__amdgpu_buffer_rsrc_t r, uint32_t voff) {
  VecT<T, CPL> v;
  constexpr int bytes = (int)sizeof(T) * CPL;
  if constexpr (bytes == 16) {
    const auto x = __builtin_amdgcn_raw_buffer_load_b128(r, voff, 0, 3);
    __builtin_memcpy(&v, &x, 16);
  } else if constexpr (bytes == 8) {
    const auto x = __builtin_amdgcn_raw_buffer_load_b64(r, voff, 0, 3);
    __builtin_memcpy(&v, &x, 8);
  } else {
    const auto x = __builtin_amdgcn_raw_buffer_load_b32(r, voff, 0, 3);
    __builtin_memcpy(&v, &x, 4);
  }
  return v;
}

template <typename T, int CPL>
__device__ __forceinline__ void bstore_nt(__amdgpu_buffer_rsrc_t r, uint32_t voff, const VecT<T, CPL>& v) {
  constexpr int bytes = (int)sizeof(T) * CPL;
  if constexpr (bytes == 16) {
    __attribute__((ext_vector_type(4))) uint32_t x;
    __builtin_memcpy(&x, &v, 16);
    __builtin_amdgcn_raw_buffer_store_b128(x, r, voff, 0, 3);
  } else if constexpr (bytes == 8) {
    __attribute__((ext_vector_type(2))) uint32_t x;
    __builtin_memcpy(&x, &v, 8);
    __builtin_amdgcn_raw_buffer_store_b64(x, r, voff, 0, 3);
  } else {
    uint32_t x;
    __builtin_memcpy(&x, &v, 4);
    __builtin_amdgcn_raw_buffer_store_b32(x, r, voff, 0, 3);
  }
}

// Residual parts of a row chunk (float32 + residual storage): CPL int16,
// two per word.
template <int CPL>
struct LoBits {
  uint32_t w[CPL >= 2 ? CPL / 2 : 1];
};
template <int CPL, int AUX>
__device__ __forceinline__ LoBits<CPL> bload_lo(__amdgpu_buffer_rsrc_t r, uint32_t voff, uint32_t soff) {
  static_assert(CPL == 2 || CPL == 4, "residual rows of 2 or 4 columns");
  LoBits<CPL> x;
  if constexpr (CPL == 4) {
    const auto v = __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, AUX);
    x.w[0] = v[0];
    x.w[1] = v[1];
  } else {
    x.w[0] = __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, AUX);
  }
  return x;
}
template <int CPL>
__device__ __forceinline__ void bstore_lo_nt(__amdgpu_buffer_rsrc_t r, uint32_t voff, const LoBits<CPL>& x) {
  if constexpr (CPL == 4) {
    __attribute__((ext_vector_type(2))) uint32_t v;
    v[0] = x.w[0];
    v[1] = x.w[1];
    __builtin_amdgcn_raw_buffer_store_b64(v, r, voff, 0, 3);
  } else {
    __builtin_amdgcn_raw_buffer_store_b32(x.w[0], r, voff, 0, 3);
  }
}
template <int CPL>
__device__ __forceinline__ int16_t lo_at(const LoBits<CPL>& x, int e) {
  return (int16_t)(x.w[e >> 1] >> ((e & 1) * 16));
}

// A row chunk as loaded: the stored values, and with RES their residuals.
template <typename T, int CPL, bool RES>
struct RowIn {
  VecT<T, CPL> v;
  LoBits<RES ? CPL : 2> lo;
};
// AUX 0: cached load (v_n); AUX 3: streaming load (v_{n-1}, no scalar offset)
template <typename T, int CPL, bool RES, int AUX>
__device__ __forceinline__ RowIn<T, CPL, RES> load_row(__amdgpu_buffer_rsrc_t rh, __amdgpu_buffer_rsrc_t rl,
                                                       uint32_t voff, uint32_t soff);
template <typename T, int CPL, bool RES>
__device__ __forceinline__ double row_val(const RowIn<T, CPL, RES>& r, int e) {
  if constexpr (RES) return res_decode(r.v.v[e], lo_at<CPL>(r.lo, e));
  else return (double)r.v.v[e];
}

__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)bytes, 0x00020000);
}

template <typename T, int CPL, bool RES, int AUX>
__device__ __forceinline__ RowIn<T, CPL, RES> load_row(__amdgpu_buffer_rsrc_t rh, __amdgpu_buffer_rsrc_t rl,
                                                       uint32_t voff, uint32_t soff) {
  RowIn<T, CPL, RES> r;
  if constexpr (AUX == 0) r.v = bload<T, CPL>(rh, voff, soff);
  else r.v = bload_nt<T, CPL>(rh, voff);
  if constexpr (RES) r.lo = bload_lo<CPL, AUX>(rl, voff >> 1, soff >> 1);
  return r;
}

// Word-table layout (one row of WB bytes per low word, indexed by the word's
// position koff[k] + i in the class-ordered list):
//   bytes 0..7       low-low part of the diagonal, sum_b (+-) J_b/(4a), float64
//   bytes 8..9       the low word l
//   bytes 12..       per mixed bond: colex rank of l ^ m_low (u16)
//   bytes kLlOff..   per low-low bond: LDS row of the neighbour (1 + its member
//                    index) when the bond acts on l, else 0 (u8)
template <int WB>
struct WordRow {
  static constexpr int kMx = WB == 32 ? 2 : 10;      // mixed bonds held
  static constexpr int kLlOff = WB == 32 ? 16 : 32;  // first low-low byte
  static constexpr int kLl = WB - kLlOff;            // low-low bonds held
};

int slice_word_bytes(int n_mx, int n_ll) {
  if (n_mx <= WordRow<32>::kMx && n_ll <= WordRow<32>::kLl) return 32;
  if (n_mx <= WordRow<64>::kMx && n_ll <= WordRow<64>::kLl) return 64;
  return 0;
}

__global__ __launch_bounds__(kThreads) void slice_words_kernel(const ProbDev* probs, const uint32_t* cmask,
                                                              const double* czz, const uint16_t* lunr,
                                                              const uint16_t* lrank, int words, int wb,
                                                              uint8_t* wtab) {
  const int w = blockIdx.x * kThreads + threadIdx.x;
  if (w >= words) return;
  const ProbDev P = probs[blockIdx.y];
  uint32_t* row = reinterpret_cast<uint32_t*>(wtab + ((size_t)blockIdx.y * words + w) * wb);
  uint32_t dw[16];
  for (int t = 0; t < 16; ++t) dw[t] = 0u;
  const uint32_t l = lunr[w];
  const int Lb = P.blk_L;
  if (Lb < 32 && (l >> Lb) == 0u) {
    const uint32_t* cm = cmask + P.bond_off;
    const double* cz = czz + P.bond_off;
    double d = 0.0;
    for (int q = 0; q < P.n_ll; ++q) {
      const uint32_t v = l & cm[q];
      d += (v == 0u || v == cm[q]) ? cz[q] : -cz[q];
    }
    uint64_t db;
    __builtin_memcpy(&db, &d, 8);
    dw[0] = (uint32_t)db;
    dw[1] = (uint32_t)(db >> 32);
    dw[2] = l;
    const uint32_t lmask = (1u << Lb) - 1u;
    const int mx0 = P.n_ll + P.n_hh;
    for (int q = 0; q < P.n_mx; ++q) {
      const uint32_t r = lrank[l ^ (cm[mx0 + q] & lmask)];
      const int byte = 12 + 2 * q;
      dw[byte >> 2] |= r << ((byte & 3) * 8);
    }
    const int llo = wb == 32 ? WordRow<32>::kLlOff : WordRow<64>::kLlOff;
    for (int q = 0; q < P.n_ll; ++q) {
      const uint32_t m = cm[q], v = l & m;
      const uint32_t r = (v == 0u || v == m) ? 0u : 1u + lrank[l ^ m];
      const int byte = llo + q;
      dw[byte >> 2] |= r << ((byte & 3) * 8);
    }
  }
  for (int t = 0; t < wb / 4; ++t) row[t] = dw[t];
}

hipError_t build_slice_words(const DevicePlan& p, uint8_t* wtab, hipStream_t st) {
  const int grid = (p.slice_words + kThreads - 1) / kThreads;
  hipLaunchKernelGGL(slice_words_kernel, dim3(grid, p.n_probs), dim3(kThreads), 0, st, p.probs, p.cmask,
                     p.czz, p.lunr, p.lrank, p.slice_words, p.slice_wb, wtab);
  return hipGetLastError();
}

// LDS of the slice kernel: the low-low coefficients of the tile's problem
// (kLlMax doubles, zero past its count), then the rows of the largest block
// (at most 254 members, storage precision) after the zero row.
constexpr int kLlMax = 32;

size_t slice_lds_bytes(const DevicePlan& p) {
  const size_t rowb = (size_t)p.ld_max * (p.fp32 ? 4 : 8);
  // nw > 1: one buffer of the largest tile's rows after the zero row, then
  // each wave's partial dots (2 ld doubles per wave)
  if (p.slice_nw > 1 && p.resid)   // decoded float64 rows, staged through registers
    return (size_t)kLlMax * 8 + (size_t)(p.slice_tile_rows + 1) * p.ld_max * 8 + (size_t)p.slice_nw * 2 * p.ld_max * 8;
  if (p.slice_nw > 1)
    return (size_t)kLlMax * 8 + rowb + ((size_t)p.slice_tile_rows * rowb + 1023) / 1024 * 1024 +
           (size_t)p.slice_nw * 2 * p.ld_max * 8;
  // rows of a multiple of 16 bytes: two buffers for direct staging, each the
  // zero row plus the largest block rounded up to whole 1 KB loads
  if (!p.resid && rowb % 16 == 0)
    return (size_t)kLlMax * 8 + 2 * (rowb + ((size_t)p.blk_lds_rows * rowb + 1023) / 1024 * 1024);
  // float32 + residual storage: the block's rows are staged decoded (float64)
  return (size_t)kLlMax * 8 + (size_t)(p.blk_lds_rows + 1) * p.ld_max * (p.fp32 && !p.resid ? 4 : 8);
}

template <int WB>
__device__ __forceinline__ uint32_t row_byte(const uint32_t (&w)[WB / 4], int byte) {
  return (w[byte >> 2] >> ((byte & 3) * 8)) & 0xFFu;
}
template <int WB>
__device__ __forceinline__ uint32_t row_u16(const uint32_t (&w)[WB / 4], int byte) {
  return (w[byte >> 2] >> ((byte & 3) * 8)) & 0xFFFFu;
}

// The double held by lane (lane ^ M) of the wave, M a power of two below 64:
// quad permutes for 1 and 2, a rotation by 8 inside rows of 16 lanes for 8,
// swizzles inside halves of 32 lanes for 4 and 16, a lane permute for 32.
template <int M>
__device__ __forceinline__ double lane_xor(double x) {
  int lo = __double2loint(x), hi = __double2hiint(x);
  if constexpr (M == 1 || M == 2 || M == 8) {
    constexpr int ctrl = M == 1 ? 0xB1 : (M == 2 ? 0x4E : 0x128);
    lo = __builtin_amdgcn_mov_dpp(lo, ctrl, 0xF, 0xF, false);
    hi = __builtin_amdgcn_mov_dpp(hi, ctrl, 0xF, 0xF, false);
  } else if constexpr (M == 4 || M == 16) {
    constexpr int pat = 0x1F | (M << 10);
    lo = __builtin_amdgcn_ds_swizzle(lo, pat);
    hi = __builtin_amdgcn_ds_swizzle(hi, pat);
  } else {
    return __shfl_xor(x, M, 64);
  }
  return __hiloint2double(hi, lo);
}

// V values per lane folded to one: at step t the lanes that differ in bit
// M << t swap halves of what they hold and add, so each lane ends with one
// value, of index sum_t b_t * V / 2^(t+1) (b_t = its bit M << t), summed
// over the V lanes that differ from it only in those bits.
template <int M, int V>
__device__ __forceinline__ double fold_lanes(const double (&v)[V], int lane) {
  if constexpr (V == 1) {
    return v[0];
  } else {
    constexpr int H = V / 2;
    const bool up = (lane & M) != 0;
    double nv[H];
#pragma unroll
    for (int j = 0; j < H; ++j) {
      const double keep = up ? v[j + H] : v[j];
      const double send = up ? v[j] : v[j + H];
      nv[j] = keep + lane_xor<M>(send);
    }
    return fold_lanes<2 * M, H>(nv, lane);
  }
}

// s * y rounded on its own (the product a caller would have stored as the
// scaled v_{n-1}), not fused into the subtraction that follows.
__device__ __forceinline__ double scaled_term(double s, double y) {
#pragma clang fp contract(off)
  return s * y;
}

template <typename T, int CPL, int NCH, int GH, int WB, bool RES, int NW, bool YS = false>
__global__ __launch_bounds__(64 * NW) void slice_kernel(const StepArgs a) {
  static_assert(!RES || (sizeof(T) == 4 && (CPL == 2 || CPL == 4)), "residual storage: float32 chunks of 2 or 4");
  static_assert(!YS || (sizeof(T) == 8 && !RES), "scaled v_{n-1}: float64 storage");
  extern __shared__ __align__(16) unsigned char smem[];
  using RowT = WordRow<WB>;
  using LT = typename std::conditional<RES, double, T>::type;   // LDS copy of v_n
  constexpr int LD = NCH * CPL;          // columns per row (every unit of the plan)
  constexpr int RPS = 64 / NCH;          // members per slice
  constexpr uint32_t ROWB = LD * sizeof(T);
  static_assert(NW == 1 || NW == 2 || NW == 4, "waves per workgroup: 1, 2 or 4");
  static_assert(NW == 1 || RES || ROWB % 16u == 0u, "shared tiles: direct loads, or decoded residual rows");
  const int lane = (int)threadIdx.x & 63;
  const int wid = NW > 1 ? __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6) : 0;

  if (a.n_jobs > 0) {
    // the previous step's partial dots: one column sum per job, fixed order
    const int64_t s = (a.step_base ? *a.step_base : 0) + a.step_add;
    for (int job = (int)blockIdx.x * NW + wid; job < a.n_jobs; job += (int)gridDim.x * NW) {
      const UnitDev U = sload(a.units + cview(a.job_unit)[job]);
      const int v = job - 2 * U.col_off;
      const double* p = a.part_in + U.part_off + (int64_t)v * U.ntiles;
      double acc = strided_sum(p, U.ntiles, lane, 64);
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) acc += __shfl_down(acc, off, 64);
      if (lane == 0) {
        if (v < U.ld) a.alpha[s * a.total_cols + U.col_off + v] = acc;
        else a.beta[(s - 1) * a.total_cols + U.col_off + (v - U.ld)] = acc;
      }
    }
  }

  // the workgroup's record names its tile, column block, problem and blocks,
  // so that the unit, problem and first block record load side by side
  const SliceWg R = sload(a.wg_rec + blockIdx.x);
  const int tile = R.tile;
  if (tile < 0 || tile >= a.n_tiles) return;
  const UnitDev U = sload(a.units + R.unit);
  const ProbDev P = sload(a.probs + R.prob);
  SliceBlk Bn = sload(a.blk_rec + R.g0);
  const int rl = lane / NCH;
  const int c = lane - rl * NCH;
  const uint32_t cc = (uint32_t)(c * CPL);
  // YS: v_{n-1} enters scaled per column (the FTLM's beta_j q_{j-1})
  double ysc[YS ? CPL : 1];
  if constexpr (YS) {
#pragma unroll
    for (int e = 0; e < CPL; ++e) ysc[e] = a.yscale[U.col_off + cc + e];
  }
  const int Lb = P.blk_L, nll = P.n_ll, nhh = P.n_hh, nmx = P.n_mx;
  const uint32_t lmask = (1u << Lb) - 1u;

  T* base = reinterpret_cast<T*>(a.vec) + U.vec_off;
  const T* X = base + a.x_slot * a.slot_stride;
  const T* Yin = base + a.yin_slot * a.slot_stride;
  T* Y = base + a.yout_slot * a.slot_stride;
  const uint32_t slot_bytes = (uint32_t)((uint64_t)P.dim * ROWB);
  const __amdgpu_buffer_rsrc_t rx = make_rsrc(X, slot_bytes);
  // the first step reads v_n in place of v_{n-1} and ignores it
  const __amdgpu_buffer_rsrc_t ry = make_rsrc(a.first ? X : Yin, slot_bytes);
  const __amdgpu_buffer_rsrc_t ro = make_rsrc(Y, slot_bytes);
  const __amdgpu_buffer_rsrc_t rw =
      make_rsrc(a.wtab + (size_t)U.prob * a.slice_words * WB, (uint32_t)a.slice_words * WB);
  // residual planes: same element index, 2 bytes per element
  __amdgpu_buffer_rsrc_t rxl = rx, ryl = ry, rol = ro;
  if constexpr (RES) {
    int16_t* lbase = a.vec_lo + U.vec_off;
    const int16_t* Xl = lbase + a.x_slot * a.slot_stride;
    rxl = make_rsrc(Xl, slot_bytes / 2);
    ryl = make_rsrc(a.first ? Xl : lbase + a.yin_slot * a.slot_stride, slot_bytes / 2);
    rol = make_rsrc(lbase + a.yout_slot * a.slot_stride, slot_bytes / 2);
  }

  // bonds in class order (padded with zeros past the last problem)
  const cptr<uint32_t> cm = cview(a.cmask) + P.bond_off;
  const cptr<double> co = cview(a.coff) + P.bond_off;
  const cptr<double> cz = cview(a.czz) + P.bond_off;

  // LDS: low-low coefficients, then the staged rows of v_n ([1 + members][LD],
  // row 0 = 0).  Rows of a multiple of 16 bytes are staged by direct
  // buffer-to-LDS loads into two buffers, the next block's while the current
  // one is computed; other rows go through registers into one buffer.
  constexpr bool DIRECT = !RES && (ROWB % 16u == 0u);
  double* lco = reinterpret_cast<double*>(smem);
  LT* xs0 = reinterpret_cast<LT*>(lco + kLlMax);
  // (nw > 1 with rows staged through registers: the zero row and the tile's rows)
  const int buf_elems = DIRECT ? (int)(LD + (((uint32_t)a.blk_lds_rows * ROWB + 1023u) / 1024u) * 1024u / sizeof(T))
                               : (NW > 1 ? LD + a.blk_lds_rows * LD : 0);
  LT* xs1 = xs0 + buf_elems;
  // nw > 1: each wave's partial dots after the one buffer
  double* red = reinterpret_cast<double*>(xs1);
  if (wid == 0) {
    for (int e = lane; e < LD; e += 64) {
      xs0[e] = LT(0);
      if constexpr (DIRECT && NW == 1) xs1[e] = LT(0);
    }
    for (int q = lane; q < kLlMax; q += 64) lco[q] = q < nll ? a.coff[P.bond_off + q] : 0.0;
  }
  // a run of rows, contiguous in v_n, to LDS rows 1.. of buf: 1 KB per
  // instruction (lane i writes bytes 16i..16i+15 of the instruction's 1 KB);
  // lanes past the run's end re-read its last 16 bytes into the buffer's
  // rounded-up capacity, so every read stays inside the run.  The wave issues
  // the instructions o0, o0 + ostep, ... (bytes).
  auto stage_rows = [&](uint32_t start, uint32_t rows, LT* buf, uint32_t o0, uint32_t ostep) {
    const uint32_t bytes = rows * ROWB, soff = start * ROWB;
    for (uint32_t o = o0; o < bytes; o += ostep)
      __builtin_amdgcn_raw_ptr_buffer_load_lds(
          rx, (__attribute__((address_space(3))) void*)(reinterpret_cast<unsigned char*>(buf + LD) + o), 16,
          min(o + (uint32_t)lane * 16u, bytes - 16u), soff, 0, 0);
  };
  auto stage_direct = [&](const SliceBlk& b, LT* buf) { stage_rows(b.start, b.size, buf, 0u, 1024u); };
  // nw > 1: the tile's rows [tstart, tstart + trows) staged once, by all waves
  uint32_t tstart = 0u;
  bool tile_ok = true;
  if constexpr (NW > 1) {
    const SliceBlk Bl = sload(a.blk_rec + R.g0 + R.ng - 1);
    tstart = Bn.start;
    const uint32_t trows = Bl.start + Bl.size - Bn.start;
    tile_ok = R.ng > 0 && Bl.start >= Bn.start && trows <= (uint32_t)a.blk_lds_rows;
    if constexpr (DIRECT) {
      if (tile_ok) stage_rows(tstart, trows, xs0, (uint32_t)wid * 1024u, (uint32_t)NW * 1024u);
    } else if (tile_ok) {
      // residual rows, decoded to float64 through registers by all waves
      const int ne = (int)trows * NCH;
      const int tid = wid * 64 + lane;
      for (int e0 = 0; e0 < ne; e0 += 4 * NW * 64) {
        RowIn<T, CPL, RES> v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const uint32_t e = (uint32_t)min(e0 + u * NW * 64 + tid, ne - 1);
          v[u] = load_row<T, CPL, RES, 0>(rx, rxl, (tstart * LD + e * CPL) * (uint32_t)sizeof(T), 0);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int e = e0 + u * NW * 64 + tid;
          if (e < ne) {
            VecT<LT, CPL> d;
#pragma unroll
            for (int k = 0; k < CPL; ++k) d.v[k] = (LT)row_val(v[u], k);
            *reinterpret_cast<VecT<LT, CPL>*>(xs0 + LD + e * CPL) = d;
          }
        }
      }
    }
    __builtin_amdgcn_s_waitcnt(0);
    __syncthreads();
  }
  auto valid = [&](const SliceBlk& b) {
    if constexpr (NW > 1) return tile_ok && b.size != 0u;
    return b.size != 0u && (int)b.size <= a.blk_lds_rows;
  };

  // the dots <v_{n+1}, v_{n+1}> and <v_{n+1}, v_n> of the wave's rows: per
  // slice the 2 CPL products of each lane are folded over 2 CPL lanes
  // (fold_lanes), so one sum per lane carries them from slice to slice
  double dacc = 0.0;

  {
    const int gend = R.g0 + R.ng;
    // records: the current block's and the next one's are at hand, the one
    // after is requested while the current block runs
    SliceBlk Bx = R.ng > 1 ? sload(a.blk_rec + R.g0 + 1) : Bn;
    if constexpr (DIRECT && NW == 1)
      if (valid(Bn)) stage_direct(Bn, xs0);
    int soff = 0;        // nw > 1: the tile's slices before the current block
    for (int g = R.g0; g < gend; ++g) {
      const SliceBlk B = Bn;
      Bn = Bx;
      if (g + 2 < gend) Bx = sload(a.blk_rec + g + 2);
      LT* xs = DIRECT && NW == 1 && ((g - R.g0) & 1) ? xs1 : xs0;
      if constexpr (DIRECT && NW == 1) {
        // this block's rows (and every earlier memory operation) complete,
        // the other buffer's last readers done: stage the next block there
        __builtin_amdgcn_s_waitcnt(0);
        wave_sync();
        if (g + 1 < gend && valid(Bn)) stage_direct(Bn, ((g + 1 - R.g0) & 1) ? xs1 : xs0);
      }
      const uint32_t h = B.h;
      const uint32_t st = B.start;
      const int bsz = (int)B.size;
      const int nsl = (bsz + RPS - 1) / RPS;
      // this wave's first slice of the block (slice soff + s of the tile)
      const int s_first = NW > 1 ? ((wid - soff) & (NW - 1)) : 0;
      soff += nsl;
      if (!valid(B)) {
        if (lane == 0 && wid == 0 && a.err) atomicOr(a.err, 4);
        continue;
      }
      // LDS row of member 0 is 1 + xbase (nw > 1: the block's place in the tile)
      const uint32_t xbase = NW > 1 ? st - tstart : 0u;
      const int nh = min((int)B.nh, nhh);
      const double dhh = B.dhh;
      const uint32_t kofs = B.kofs;
      const cptr<uint32_t> hs = cview(a.meta_hstart) + (int64_t)g * a.meta_hh;
      const cptr<double> hc = cview(a.meta_hcoef) + (int64_t)g * a.meta_hh;
      const cptr<uint32_t> ms = cview(a.meta_mstart) + (int64_t)g * a.meta_mx;

      // 1. the block's rows of v_n into LDS rows 1..bsz (direct staging: done)
      if constexpr (!DIRECT && NW == 1) {
        const int ne = bsz * NCH;
        for (int e0 = 0; e0 < ne; e0 += 4 * 64) {
          RowIn<T, CPL, RES> v[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const uint32_t e = (uint32_t)min(e0 + u * 64 + lane, ne - 1);
            v[u] = load_row<T, CPL, RES, 0>(rx, rxl, (st * LD + e * CPL) * (uint32_t)sizeof(T), 0);
          }
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int e = e0 + u * 64 + lane;
            if (e < ne) {
              if constexpr (RES) {
                VecT<double, CPL> d;
#pragma unroll
                for (int k = 0; k < CPL; ++k) d.v[k] = row_val(v[u], k);
                *reinterpret_cast<VecT<double, CPL>*>(xs + LD + e * CPL) = d;
              } else {
                *reinterpret_cast<VecT<T, CPL>*>(xs + LD + e * CPL) = v[u].v;
              }
            }
          }
        }
        wave_sync();
      }

      // 2. slices of the block.  A slice's v_{n+1} is stored after the next
      // slice's loads are issued (its data registers are then not the next
      // loads' targets, so those loads need not wait for the store).
      RowIn<T, CPL, RES> pend;
      uint32_t pend_off = 0u;
      bool pend_on = false;
      // the word-table row of a member (requested at its slice's start: a row
      // requested a slice ahead held 4-5 more VGPRs, one wave per SIMD fewer,
      // and was 1 % slower)
      auto wload = [&](uint32_t kof, int nmem, int sl, uint32_t (&wr)[WB / 4]) {
        const int i = sl * RPS + rl;
        const uint32_t ii = i < nmem ? (uint32_t)i : 0u;
#pragma unroll
        for (int t = 0; t < WB / 16; ++t) {
          const auto q = __builtin_amdgcn_raw_buffer_load_b128(rw, (kof + ii) * WB + 16 * t, 0, 0);
          wr[4 * t] = q[0];
          wr[4 * t + 1] = q[1];
          wr[4 * t + 2] = q[2];
          wr[4 * t + 3] = q[3];
        }
      };
      for (int s = s_first; s < nsl; s += NW) {
        const int i = s * RPS + rl;
        const bool on = i < bsz;
        const uint32_t ii = on ? (uint32_t)i : 0u;
        uint32_t w[WB / 4];
        wload(kofs, bsz, s, w);
        const uint32_t own = st + ii;
        const uint32_t voff_own = own * ROWB + cc * (uint32_t)sizeof(T);
        const uint32_t voff_m = ii * ROWB + cc * (uint32_t)sizeof(T);
        const RowIn<T, CPL, RES> yv = load_row<T, CPL, RES, 3>(ry, ryl, voff_own, 0);
        // first batch of high-high rows: starts and coefficients by scalar
        // loads (entries past the block's count are read, not used)
        RowIn<T, CPL, RES> hv[GH];
        double hcf[GH];
#pragma unroll
        for (int j = 0; j < GH; ++j) {
          const uint32_t tj = hs[j];
          const double cj = hc[j];
          const uint32_t t = j < nh ? tj : st;    // past the count: own member, coefficient 0
          hcf[j] = j < nh ? cj : 0.0;
          hv[j] = load_row<T, CPL, RES, 0>(rx, rxl, voff_m, t * ROWB);
        }
        if (pend_on) {
          bstore_nt<T, CPL>(ro, pend_off, pend.v);
          if constexpr (RES) bstore_lo_nt<CPL>(rol, pend_off >> 1, pend.lo);
        }

        const uint32_t l = w[2] & 0xFFFFu;
        double dll;
        {
          const uint64_t db = (uint64_t)w[0] | ((uint64_t)w[1] << 32);
          __builtin_memcpy(&dll, &db, 8);
        }
        // mixed bonds act where their low and high sites differ
        bool mact[RowT::kMx];
        double d = dhh + dll;
#pragma unroll
        for (int q = 0; q < RowT::kMx; ++q) {
          mact[q] = false;
          if (q < nmx) {
            const uint32_t m = cm[nll + nhh + q];
            mact[q] = ((l & m & lmask) != 0u) != ((h & (m >> Lb)) != 0u);
            d = fma(mact[q] ? -1.0 : 1.0, cz[nll + nhh + q], d);
          }
        }
        double acc[CPL];
        {
          const VecT<LT, CPL> xv = *reinterpret_cast<const VecT<LT, CPL>*>(xs + (1 + xbase + ii) * LD + cc);
#pragma unroll
          for (int e = 0; e < CPL; ++e) acc[e] = d * (double)xv.v[e];
        }
        // low-low neighbours in batches of four: the word table names the LDS
        // row (0 = the zero row for a bond that does not act, and for the
        // slots past the problem's count)
#pragma unroll
        for (int q0 = 0; q0 < RowT::kLl; q0 += 4) {
          if (q0 < nll) {
            VecT<LT, CPL> xv[4];
            double cf[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
              const uint32_t r0 = row_byte<WB>(w, RowT::kLlOff + q0 + u);
              const uint32_t r = NW > 1 && r0 != 0u ? r0 + xbase : r0;
              cf[u] = lco[q0 + u];
              xv[u] = *reinterpret_cast<const VecT<LT, CPL>*>(xs + r * LD + cc);
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
#pragma unroll
              for (int e = 0; e < CPL; ++e) acc[e] = fma(cf[u], (double)xv[u].v[e], acc[e]);
            }
          }
        }
        // mixed rows (requested now; their latency overlaps the high-high sums)
        RowIn<T, CPL, RES> mv[2];
        auto mx_issue = [&](int q0) {
#pragma unroll
          for (int u = 0; u < 2; ++u) {
            const int q = q0 + u;
            uint32_t row = own;
            if (q < nmx && q < RowT::kMx) {
              const uint32_t stq = ms[q];
              if (mact[q] && stq == kNoRun) {
                if (a.err) atomicOr(a.err, 2);
                mact[q] = false;
              }
              if (mact[q]) row = stq + row_u16<WB>(w, 12 + 2 * q);
            }
            mv[u] = load_row<T, CPL, RES, 0>(rx, rxl, row * ROWB + cc * (uint32_t)sizeof(T), 0);
          }
        };
        mx_issue(0);
        // high-high rows
#pragma unroll
        for (int j = 0; j < GH; ++j) {
#pragma unroll
          for (int e = 0; e < CPL; ++e) acc[e] = fma(hcf[j], row_val(hv[j], e), acc[e]);
        }
        for (int k0 = GH; k0 < nh; k0 += GH) {
#pragma unroll
          for (int j = 0; j < GH; ++j) {
            const uint32_t tj = hs[k0 + j];
            const double cj = hc[k0 + j];
            const uint32_t t = k0 + j < nh ? tj : st;
            hcf[j] = k0 + j < nh ? cj : 0.0;
            hv[j] = load_row<T, CPL, RES, 0>(rx, rxl, voff_m, t * ROWB);
          }
#pragma unroll
          for (int j = 0; j < GH; ++j) {
#pragma unroll
            for (int e = 0; e < CPL; ++e) acc[e] = fma(hcf[j], row_val(hv[j], e), acc[e]);
          }
        }
#pragma unroll
        for (int q0 = 0; q0 < RowT::kMx; q0 += 2) {
          if (q0 < nmx) {
            if (q0 > 0) mx_issue(q0);
#pragma unroll
            for (int u = 0; u < 2; ++u) {
              const int q = q0 + u;
              const double cq = co[nll + nhh + q];
              const double cf = (q < nmx && mact[q]) ? cq : 0.0;
#pragma unroll
              for (int e = 0; e < CPL; ++e) acc[e] = fma(cf, row_val(mv[u], e), acc[e]);
            }
          }
        }
        pend_on = on;
        pend_off = voff_own;
        {
          // v_{n+1} as stored (lanes past the block: member 0's rows, not
          // stored); the dots are of the stored values
          const VecT<LT, CPL> xv = *reinterpret_cast<const VecT<LT, CPL>*>(xs + (1 + xbase + ii) * LD + cc);
          double fv[2 * CPL];
#pragma unroll
          for (int e = 0; e < CPL; ++e) {
            double yt = row_val(yv, e);
            if constexpr (YS) yt = scaled_term(ysc[e], yt);
            const double val = a.first ? acc[e] : 2.0 * acc[e] - yt;
            double o;
            if constexpr (RES) {
              float hi;
              int16_t q;
              res_encode(val, hi, q);
              pend.v.v[e] = hi;
              const uint32_t bits = (uint32_t)(uint16_t)q << ((e & 1) * 16);
              if (e & 1) pend.lo.w[e >> 1] |= bits;
              else pend.lo.w[e >> 1] = bits;
              o = res_decode(hi, q);
            } else {
              pend.v.v[e] = (T)val;
              o = (double)pend.v.v[e];
            }
            fv[e] = on ? o * o : 0.0;
            fv[CPL + e] = on ? o * (double)xv.v[e] : 0.0;
          }
          dacc += fold_lanes<NCH, 2 * CPL>(fv, lane);
        }
      }
      if (pend_on) {
        bstore_nt<T, CPL>(ro, pend_off, pend.v);
        if constexpr (RES) bstore_lo_nt<CPL>(rol, pend_off >> 1, pend.lo);
      }
      wave_sync();
    }
  }

  // dots: the lanes' sums over the member bits not folded per slice (fixed
  // order); lane l < 2 CPL * NCH then holds chunk l % NCH's value of index
  // bit-reversed(l / NCH)
  {
    constexpr int V = 2 * CPL;
    double dv = dacc;
#pragma unroll
    for (int m = NCH * V; m < 64; m <<= 1) dv += __shfl_xor(dv, m, 64);
    if (lane < NCH * V) {
      const int r = lane / NCH;
      int idx = 0;
#pragma unroll
      for (int t = 0; (1 << t) < V; ++t) idx += ((r >> t) & 1) * (V >> (t + 1));
      const int dot = idx < CPL ? 0 : 1;
      const int col = (lane % NCH) * CPL + idx - dot * CPL;
      if constexpr (NW == 1) a.part_out[U.part_off + (int64_t)(dot * LD + col) * U.ntiles + (tile - U.tile0)] = dv;
      else red[wid * 2 * LD + dot * LD + col] = dv;
    }
  }
  if constexpr (NW > 1) {
    // then over the waves, in wave order
    __syncthreads();
    if (wid == 0 && lane < 2 * LD) {
      double sum = red[lane];
      for (int w = 1; w < NW; ++w) sum += red[w * 2 * LD + lane];
      a.part_out[U.part_off + (int64_t)lane * U.ntiles + (tile - U.tile0)] = sum;
    }
  }
}

template <typename T, int CPL, int NCH, int WB, bool RES, int NW, bool YS>
static hipError_t launch_slice_w(const StepArgs& a, size_t lds, int grid, int gh, hipStream_t st) {
  if (gh == 4)
    hipLaunchKernelGGL((slice_kernel<T, CPL, NCH, 4, WB, RES, NW, YS>), dim3(grid), dim3(64 * NW), lds, st, a);
  else
    hipLaunchKernelGGL((slice_kernel<T, CPL, NCH, 8, WB, RES, NW, YS>), dim3(grid), dim3(64 * NW), lds, st, a);
  return hipGetLastError();
}

template <typename T, int CPL, int NCH, bool RES, int NW, bool YS>
static hipError_t launch_slice_n(const StepArgs& a, size_t lds, int grid, int gh, int wb, hipStream_t st) {
  if (wb == 32) return launch_slice_w<T, CPL, NCH, 32, RES, NW, YS>(a, lds, grid, gh, st);
  return launch_slice_w<T, CPL, NCH, 64, RES, NW, YS>(a, lds, grid, gh, st);
}

// waves per workgroup: 1, or 2 / 4 for rows of 16 or 32 bytes (direct staging)
template <typename T, int CPL, int NCH, bool RES = false, bool YS = false>
static hipError_t launch_slice_t(const StepArgs& a, size_t lds, int grid, int gh, int wb, int nw, hipStream_t st) {
  if constexpr (RES || (NCH * CPL * sizeof(T)) % 16 == 0) {
    if (nw == 4) return launch_slice_n<T, CPL, NCH, RES, 4, YS>(a, lds, grid, gh, wb, st);
    if (nw == 2) return launch_slice_n<T, CPL, NCH, RES, 2, YS>(a, lds, grid, gh, wb, st);
  }
  if (nw != 1) return hipErrorInvalidValue;
  return launch_slice_n<T, CPL, NCH, RES, 1, YS>(a, lds, grid, gh, wb, st);
}

// Every unit of a slice plan has ld = cpl * nch with nch 1 or 2.
hipError_t launch_slice(const DevicePlan& p, const StepArgs& a, hipStream_t st) {
  const size_t lds = slice_lds_bytes(p);
  const int grid = p.slice_grid > 0 ? p.slice_grid : p.grid_tiles;
  const int gh = p.gather_batch;
  const int wb = p.slice_wb;
  const int nw = p.slice_nw;
  const int nch = p.ld_max / p.cpl;
  if (p.ld_max != nch * p.cpl || (nch != 1 && nch != 2)) return hipErrorInvalidValue;
  if (a.yscale && p.fp32) return hipErrorInvalidValue;   // scaled v_{n-1}: float64 storage only
  if (p.resid) {
    if (!p.fp32 || !a.vec_lo) return hipErrorInvalidValue;
    if (p.cpl == 4) return nch == 1 ? launch_slice_t<float, 4, 1, true>(a, lds, grid, gh, wb, nw, st)
                                    : launch_slice_t<float, 4, 2, true>(a, lds, grid, gh, wb, nw, st);
    if (p.cpl == 2 && nch == 1) return launch_slice_t<float, 2, 1, true>(a, lds, grid, gh, wb, nw, st);
    return hipErrorInvalidValue;
  }
  if (p.fp32) {
    if (p.cpl == 4) return nch == 1 ? launch_slice_t<float, 4, 1>(a, lds, grid, gh, wb, nw, st)
                                    : launch_slice_t<float, 4, 2>(a, lds, grid, gh, wb, nw, st);
    if (p.cpl == 2 && nch == 1) return launch_slice_t<float, 2, 1>(a, lds, grid, gh, wb, nw, st);
    if (p.cpl == 1 && nch == 1) return launch_slice_t<float, 1, 1>(a, lds, grid, gh, wb, nw, st);
    return hipErrorInvalidValue;
  }
  if (a.yscale) {   // float64 with v_{n-1} scaled per column
    if (p.cpl == 2) return nch == 1 ? launch_slice_t<double, 2, 1, false, true>(a, lds, grid, gh, wb, nw, st)
                                    : launch_slice_t<double, 2, 2, false, true>(a, lds, grid, gh, wb, nw, st);
    if (p.cpl == 1 && nch == 1) return launch_slice_t<double, 1, 1, false, true>(a, lds, grid, gh, wb, nw, st);
    return hipErrorInvalidValue;
  }
  if (p.cpl == 2) return nch == 1 ? launch_slice_t<double, 2, 1>(a, lds, grid, gh, wb, nw, st)
                                  : launch_slice_t<double, 2, 2>(a, lds, grid, gh, wb, nw, st);
  if (p.cpl == 1 && nch == 1) return launch_slice_t<double, 1, 1>(a, lds, grid, gh, wb, nw, st);
  return hipErrorInvalidValue;
}

}  // namespace kpm
