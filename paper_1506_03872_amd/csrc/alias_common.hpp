// alias_common.hpp -- the one-wave alias-table builder shared by the dense
// and sparse table builders (see tables.hip for the construction: lights
// and heavies in index order, closed form of the sequential sweep).
#pragma once

#include "mad_common.hpp"

namespace mad {

constexpr uint64_t kQMask = ~(1ull << 63);

// One wave builds the alias table of one table from its quanta qv (lane
// holds slots lane*SPL ..) and sign bits sg; LDS scratch Ld/He (2^L u64
// each) and Hi (2^L u32) belongs to this wave.  Every wave of the block
// calls this (it synchronises the block once).  Each slot r is handed to
// emit(r, thr, sign_self, alias_position, sign_alias).
template <int SPL, class Emit>
__device__ void wave_alias(const uint64_t (&qv)[SPL], const uint32_t (&sg)[SPL],
                           bool active, int L, uint64_t* Ld, uint64_t* He,
                           uint32_t* Hi, Emit emit) {
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
  const uint32_t nl_in = wave_incl_scan(nl), nh_in = wave_incl_scan(nh);
  const uint64_t sd_in = wave_incl_scan(sd), se_in = wave_incl_scan(se);
  const uint32_t NL = __shfl(nl_in, 63, 64), NH = __shfl(nh_in, 63, 64);
  uint32_t lp = nl_in - nl, hp = nh_in - nh;
  uint64_t da = sd_in - sd, ea = se_in - se;
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
#pragma unroll
  for (int s = 0; s < SPL; ++s) {
    const int r = lane * SPL + s;
    if (!(active && r < Np)) continue;
    if (qv[s] < kCap) {
      const uint64_t Dx = Ld[mypos[s]] - (kCap - qv[s]);
      uint32_t lo = 0, hi = NH;
      while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (He[mid] >= Dx) hi = mid; else lo = mid + 1;
      }
      const uint32_t a = NH ? Hi[lo < NH ? lo : NH - 1]
                            : (uint32_t)r | (sg[s] << 31);
      emit(r, (uint32_t)qv[s], sg[s], a & kLow31, a >> 31);
    } else {
      const uint64_t Eh = He[mypos[s]];
      uint32_t lo = 0, hi = NL;
      while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (Ld[mid] > Eh) hi = mid; else lo = mid + 1;
      }
      if (lo < NL && mypos[s] + 1 < NH) {
        const uint32_t a = Hi[mypos[s] + 1];
        emit(r, (uint32_t)(Eh + kCap - Ld[lo]), sg[s], a & kLow31, a >> 31);
      } else {
        emit(r, 0u, sg[s], (uint32_t)r, sg[s]);
      }
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
