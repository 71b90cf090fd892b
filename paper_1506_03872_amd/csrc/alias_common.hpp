// alias_common.hpp -- the one-wave alias-table builder shared by the dense
// and sparse table builders (see tables.hip for the construction: lights
// and heavies in index order, closed form of the sequential sweep).
#pragma once

#include "mad_common.hpp"

namespace mad {

constexpr uint64_t kQMask = ~(1ull << 63);

// Integer quanta in FP64: while K = L + 31 <= 52, every F_r, q_r, deficit
// and excess and each of their sums is an integer below 2^52, so FP64 holds
// them exactly and its adds, subtractions and comparisons are exact;
// exact_u52 turns such an integer into its u64 with one add and one mask.
constexpr int kF64MaxL = 52 - kCapBits;
constexpr double kCapD = 2147483648.0;  // 2^31

__device__ __forceinline__ uint64_t exact_u52(double x) {
  return (uint64_t)__double_as_longlong(x + 4503599627370496.0) &
         ((1ull << 52) - 1);
}

// One wave builds the alias table of one table from its quanta qv (lane
// holds slots lane*SPL ..) and sign bits sg; LDS scratch Ld/He (2^L u64
// each) and Hi (2^L u32) belongs to this wave.  Every wave of the block
// calls this (it synchronises the block once).  Each slot r is handed to
// emit(r, thr, sign_self, alias_position, sign_alias).  With HAVE_F the
// caller passes Fb = F before the lane's first slot (the sum of all quanta
// before it): the excess before the lane then follows from the deficit
// before it, sum (C - q) = first C - Fb, and one 64-bit scan suffices.
template <int SPL, bool HAVE_F = false, class Emit>
__device__ void wave_alias(const uint64_t (&qv)[SPL], const uint32_t (&sg)[SPL],
                           bool active, int L, uint64_t* Ld, uint64_t* He,
                           uint32_t* Hi, Emit emit, uint64_t Fb = 0) {
  const int Np = 1 << L;
  const int lane = threadIdx.x & 63;
  uint32_t nl = 0, nh = 0;
  uint64_t sd = 0, se = 0;
#pragma unroll
  for (int s = 0; s < SPL; ++s) {
    const int r = lane * SPL + s;
    if (active && r < Np) {
      if (qv[s] < kCap) { ++nl; sd += kCap - qv[s]; }
      else { ++nh; se += qv[s] - kCap; }
    }
  }
  uint32_t NL, NH, lp, hp;
  uint64_t da, ea;
  if (HAVE_F) {
    const uint32_t c_in = wave_scan_dpp(nl);
    const uint64_t sd_in = wave_scan_dpp(sd);
    NL = __shfl(c_in, 63, 64);
    lp = c_in - nl;
    const uint32_t first = active ? (uint32_t)(lane * SPL) : 0u;
    const uint32_t before = first < (uint32_t)Np ? first : (uint32_t)Np;
    NH = active ? (uint32_t)Np - NL : 0u;
    hp = before - lp;
    da = sd_in - sd;
    ea = da - (uint64_t)before * kCap + Fb;
  } else {
    // light and heavy counts share one scan (each total is at most 2^L <=
    // 512, so 16 bits apiece)
    const uint32_t c_in = wave_incl_scan(nl | (nh << 16));
    const uint64_t sd_in = wave_incl_scan(sd), se_in = wave_incl_scan(se);
    const uint32_t c_all = __shfl(c_in, 63, 64);
    NL = c_all & 0xFFFFu;
    NH = c_all >> 16;
    lp = (c_in & 0xFFFFu) - nl;
    hp = (c_in >> 16) - nh;
    da = sd_in - sd;
    ea = se_in - se;
  }
  uint32_t mypos[SPL];
#pragma unroll
  for (int s = 0; s < SPL; ++s) {
    const int r = lane * SPL + s;
    mypos[s] = 0;
    if (active && r < Np) {
      if (qv[s] < kCap) {
        da += kCap - qv[s];
        Ld[lp] = da;
        mypos[s] = lp++;
      } else {
        ea += qv[s] - kCap;
        He[hp] = ea;
        Hi[hp] = (uint32_t)r | (sg[s] << 31);
        mypos[s] = hp++;
      }
    }
  }
  __syncthreads();
  // Each slot searches the other list once, with the same branch-free
  // lower bound (a uniform loop of L + 1 halving steps): a light the first
  // heavy whose inclusive excess reaches its exclusive deficit Dx, i.e.
  // the count of heavies with He < Dx; a heavy the first light whose
  // inclusive deficit exceeds its excess Eh, i.e. the count of lights with
  // Ld < Eh + 1.
#pragma unroll
  for (int s = 0; s < SPL; ++s) {
    const int r = lane * SPL + s;
    const bool ok = active && r < Np;
    const bool light = qv[s] < kCap;
    const uint64_t own = ok ? (light ? Ld[mypos[s]] : He[mypos[s]]) : 0ull;
    const uint64_t key = light ? own - (kCap - qv[s]) : own + 1;
    const uint64_t* lst = light ? He : Ld;
    const uint32_t n = ok ? (light ? NH : NL) : 0u;
    uint32_t lo = 0;
    for (uint32_t step = (uint32_t)Np; step > 0; step >>= 1)
      if (lo + step <= n && lst[lo + step - 1] < key) lo += step;
    if (!ok) continue;
    if (light) {
      const uint32_t a = NH ? Hi[lo < NH ? lo : NH - 1]
                            : (uint32_t)r | (sg[s] << 31);
      emit(r, (uint32_t)qv[s], sg[s], a & kLow31, a >> 31);
    } else if (lo < NL && mypos[s] + 1 < NH) {
      const uint32_t a = Hi[mypos[s] + 1];
      emit(r, (uint32_t)(own + kCap - Ld[lo]), sg[s], a & kLow31, a >> 31);
    } else {
      emit(r, 0u, sg[s], (uint32_t)r, sg[s]);
    }
  }
}

// alias statistics of a run of slots: light / heavy counts, total deficit
// (C - q over lights) and total excess (q - C over heavies)
struct Quad {
  uint64_t nl, nh, sd, se;
};

__device__ __forceinline__ void slot_stats(uint64_t q, Quad& a) {
  if (q < kCap) { a.nl += 1; a.sd += kCap - q; }
  else { a.nh += 1; a.se += q - kCap; }
}

// merge-path split: how many of the first di merged elements are lights,
// merging the light deficits D (exclusive prefixes) before the heavy
// excesses E (inclusive prefixes) on ties
__device__ __forceinline__ int64_t merge_split(const uint64_t* D, int64_t NL,
                                               const uint64_t* E, int64_t NH,
                                               int64_t di) {
  int64_t lo = di - NH > 0 ? di - NH : 0;
  int64_t hi = di < NL ? di : NL;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (D[mid] <= E[di - mid - 1]) lo = mid + 1; else hi = mid;
  }
  return lo;
}

// emitter of packed 8-byte entries into et[r]
struct EmitPacked {
  uint64_t* et;
  __device__ void operator()(int r, uint32_t thr, uint32_t ss, uint32_t al,
                             uint32_t sa) const {
    et[r] = pack_entry(thr, ss, al, sa);
  }
};

}  // namespace mad
