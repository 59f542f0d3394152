// Device helpers shared by the gfx950 kernels: basis unranking and ranking in
// the combinatorial number system of an S^z sector.
#pragma once

#include <hip/hip_runtime.h>

#include "kpm_internal.h"

namespace kpm {

// Word of rank r among N-bit words with k set bits (combinatorial number
// system, colex order = ascending integer order): greedily take the highest
// position p with C(p, j) <= remaining rank, for j = k .. 1.
__device__ __forceinline__ uint32_t unrank(uint32_t r, int N, int k, const uint32_t* binom) {
  uint32_t s = 0;
  int j = k;
  for (int p = N - 1; p >= 0 && j > 0; --p) {
    const uint32_t cv = binom[p * kBinomN + j];
    if (cv <= r) {
      s |= 1u << p;
      r -= cv;
      --j;
    }
  }
  return s;
}

// Rank of word s: the bits split as x0 (B0 low bits), x1 (next B1), x2 (rest);
// rank = T0[x0] + T1[x1][popcount(x0)] + T2[x2] (T2 already knows the sector's
// popcount, so the number of set bits below x2 is implied).
struct RankTables {
  const uint32_t* T0;
  const uint32_t* T1;
  const uint32_t* T2;
  uint32_t m0, m1;
  int B0, sh2;
  __device__ __forceinline__ uint32_t rank(uint32_t s) const {
    const uint32_t x0 = s & m0;
    const uint32_t x1 = (s >> B0) & m1;
    const uint32_t x2 = s >> sh2;
    return T0[x0] + T1[x1 * (uint32_t)(B0 + 1) + __popc(x0)] + T2[x2];
  }
};

__device__ __forceinline__ RankTables make_tables(const uint32_t* tab, const ProbDev& P) {
  RankTables R;
  R.T0 = tab;
  R.T1 = tab + (1u << P.B0);
  R.T2 = R.T1 + (1u << P.B1) * (uint32_t)(P.B0 + 1);
  R.m0 = (1u << P.B0) - 1u;
  R.m1 = (1u << P.B1) - 1u;
  R.B0 = P.B0;
  R.sh2 = P.B0 + P.B1;
  return R;
}

// Colex (= ascending-integer) rank of word s among the words of its popcount.
__device__ __forceinline__ uint32_t word_rank(uint32_t s, const uint32_t* binom) {
  uint32_t r = 0;
  int j = 0;
  for (uint32_t x = s; x; x &= x - 1u) {
    ++j;
    r += binom[(__ffs(x) - 1) * kBinomN + j];
  }
  return r;
}

// Relabelled sites: the word with bit i moved to bit perm[i] (to_kernel) or
// back (from the kernels' labels to the problem's).
__device__ __forceinline__ uint32_t relabel_word(uint32_t w, const uint8_t* perm, int N, bool to_kernel) {
  uint32_t o = 0;
  for (int i = 0; i < N; ++i) {
    if (to_kernel) o |= ((w >> i) & 1u) << perm[i];
    else o |= ((w >> perm[i]) & 1u) << i;
  }
  return o;
}

// Spin-s sites: rank of the digit string dg (4 bits per site, digit sum n)
// in its sector, from the table P[i][r][d] (strings of sites 0..i with sum r
// and digit < d at site i): the entries of each site's digit, from the most
// significant site down, with r the sum still left.
__device__ __forceinline__ uint32_t spin_rank(uint64_t dg, int N, int n, int R1, int B,
                                              const uint32_t* tab) {
  uint32_t rank = 0;
  int r = n;
  for (int i = N - 1; i >= 0; --i) {
    const int d = (int)((dg >> (4 * i)) & 15u);
    rank += tab[(i * R1 + r) * B + d];
    r -= d;
  }
  return rank;
}

}  // namespace kpm
