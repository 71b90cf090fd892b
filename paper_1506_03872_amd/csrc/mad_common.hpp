// mad_common.hpp -- device-side building blocks shared by the kernels of the
// diamond-sampling library (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mad {

// Sums and prefix sums of non-negative FP64 weights use a two-level order:
// runs of kRun consecutive terms are summed left to right, and the run
// offsets are accumulated left to right (E_0 = 0, E_{c+1} = E_c + S_c).
// The prefix at item r of run c is E_c + l_r, l_r the run-local sum.  This
// order is non-decreasing and keeps a zero weight's prefix equal to its
// predecessor's, so integer quanta of zero-weight items are exactly zero.
constexpr int kRun = 128;

// Alias tables: 2^L slots of capacity 2^31; a draw uses the top L bits of a
// 64-bit random word as the slot and its low 31 bits as the coin.
constexpr int kCapBits = 31;
constexpr uint64_t kCap = 1ull << kCapBits;
constexpr uint32_t kLow31 = 0x7FFFFFFFu;

constexpr uint64_t kEmptyKey = ~0ull;

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds, each two
// 64x64->128 products with the published multipliers, key bumped by the
// published Weyl constants between rounds.
// ---------------------------------------------------------------------------
struct Philox4 {
  uint64_t w0, w1, w2, w3;
};

__device__ __forceinline__ Philox4 philox4x64_10(uint64_t c0, uint64_t c1,
                                                 uint64_t c2, uint64_t c3,
                                                 uint64_t k0, uint64_t k1) {
  constexpr uint64_t M0 = 0xD2E7470EE14C6C93ull;
  constexpr uint64_t M1 = 0xCA5A826395121157ull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    // each 64 x 64 -> 128-bit product formed once (both halves share the
    // partial products)
    const __uint128_t p0 = (__uint128_t)M0 * c0;
    const __uint128_t p1 = (__uint128_t)M1 * c2;
    const uint64_t n0 = (uint64_t)(p1 >> 64) ^ c1 ^ k0;
    const uint64_t n2 = (uint64_t)(p0 >> 64) ^ c3 ^ k1;
    c0 = n0;
    c1 = (uint64_t)p1;
    c2 = n2;
    c3 = (uint64_t)p0;
    k0 += 0x9E3779B97F4A7C15ull;
    k1 += 0xBB67AE8584CAA73Bull;
  }
  return {c0, c1, c2, c3};
}

// ---------------------------------------------------------------------------
// Alias-table entry (64 bits):
//   bits  0..30  thr      item = slot when coin < thr
//   bit   31     sign bit of the slot's own item (sign of its A or B value)
//   bits 32..62  alias    item when coin >= thr
//   bit   63     sign bit of the alias item
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint64_t pack_entry(uint32_t thr, uint32_t sgn_self,
                                               uint32_t alias,
                                               uint32_t sgn_alias) {
  const uint32_t lo = (thr & kLow31) | (sgn_self << 31);
  const uint32_t hi = (alias & kLow31) | (sgn_alias << 31);
  return (uint64_t)lo | ((uint64_t)hi << 32);
}

__device__ __forceinline__ uint32_t slot_of(uint64_t U, int L) {
  return L ? (uint32_t)(U >> (64 - L)) : 0u;
}

struct Drawn {
  uint32_t pos;  // table position (item index for dense tables)
  uint32_t sgn;  // sign bit of the drawn item's value
};

__device__ __forceinline__ Drawn draw_entry(uint64_t e, uint32_t slot,
                                            uint64_t U) {
  const uint32_t lo = (uint32_t)e, hi = (uint32_t)(e >> 32);
  const uint32_t coin = (uint32_t)U & kLow31;
  const bool self = coin < (lo & kLow31);
  const uint32_t w = self ? lo : hi;
  return {self ? slot : (hi & kLow31), w >> 31};
}

// 64-bit mixer for hash slots: the output function of SplitMix64 (Steele,
// Lea, Flood, OOPSLA 2014) with Stafford's "Mix13" constants.
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__device__ __forceinline__ uint32_t sign_bit(float x) {
  return __float_as_uint(x) >> 31;
}

// Fixed-point exponent of the score increments: F = 62 - e - ceil(log2 s')
// with s' = max(s, 2) and max|b| < 2^e (frexp exponent of max|b|).
__host__ __device__ inline int fix_exponent(float bmax, int64_t s) {
  int e;
  (void)frexpf(bmax, &e);
  int64_t v = s > 2 ? s : 2;
  int ls = 0;
  while ((int64_t(1) << ls) < v) ++ls;
  return 62 - e - ls;
}

// ---------------------------------------------------------------------------
// wave64 helpers
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    T u = __shfl_up(v, off, 64);
    if (lane >= off) v += u;
  }
  return v;
}

// Inclusive scan over the 64 lanes by DPP moves (GFX9 controls: row_shr
// by 1, 2, 4 and 8 within each row of 16 lanes, then row_bcast:15 into
// rows 1 and 3 and row_bcast:31 into rows 2 and 3); lanes without a source
// add 0.  No LDS round trip per step, unlike the shuffle scan above.  Every
// lane of the wave must be active.
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp_from(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xF,
                                               false);
}

template <int CTRL, int ROWS>
__device__ __forceinline__ uint64_t dpp_from(uint64_t v) {
  const uint32_t lo = dpp_from<CTRL, ROWS>((uint32_t)v);
  const uint32_t hi = dpp_from<CTRL, ROWS>((uint32_t)(v >> 32));
  return ((uint64_t)hi << 32) | lo;
}

template <typename T>
__device__ __forceinline__ T wave_scan_dpp(T v) {
  v += dpp_from<0x111, 0xF>(v);  // row_shr:1
  v += dpp_from<0x112, 0xF>(v);  // row_shr:2
  v += dpp_from<0x114, 0xF>(v);  // row_shr:4
  v += dpp_from<0x118, 0xF>(v);  // row_shr:8
  v += dpp_from<0x142, 0xA>(v);  // row_bcast:15
  v += dpp_from<0x143, 0xC>(v);  // row_bcast:31
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

}  // namespace mad
