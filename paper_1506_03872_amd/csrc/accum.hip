// accum.hip -- the score matrix X, filled by the score update of Alg. 3, built
// from the closed samples without per-sample global atomics.
//
// Sample l writes its pair at index l of two arrays: the key i*n + j
// (EMPTY when the three-path is open) and the fourth edge b_k'j as fp32 with
// the sign of a_ki b_kj a_k'i applied, v; its increment is rne(v 2^F)
// (exact in int64, rint is odd).  So the sampler needs no atomics and a
// pair takes 12 bytes.  X is the sum of the increments per key, computed
// as:
//   count    per group of tiles of pairs, a histogram of the bin = top B1
//            bits of mix64(key) (bins are disjoint in keys); open samples
//            dropped;
//   scan     exclusive prefix of the group counts in bin-major order;
//   place    every closed pair written into its bin's range;
//   split    (large s) one workgroup per bin partitions it again by the next
//            B2 hash bits, so that bins hold about 512 pairs; above 8 bits
//            in two splits (each storing runs of ~16+ pairs per sub-bin);
//   reduce   one workgroup per bin sums equal keys in an LDS hash table and
//            appends the distinct (key, x) to the output list.  A bin with
//            more distinct keys than the LDS table holds is split by the
//            next hash bits into sub-bins, each reduced on its own, so the
//            output never holds a key twice.
// The sums are int64 fixed point, so X is the same in any order.
#include <stdlib.h>

#include "mad_common.hpp"
#include "plan.hpp"

namespace mad {

constexpr int kAccThreads = 512;
constexpr int kAccPer = 8;                // pairs per thread of a tile
constexpr int kAccTile = kAccThreads * kAccPer;  // count / place tile
constexpr int kAccMaxBits = 8;            // first level: up to 256 bins
constexpr int kAcc2MaxBits = 12;          // one split: up to 4096 sub-bins
constexpr int kAccSplitBits = 8;          // above this, two splits
constexpr int kAccMaxTotalBits = kAccMaxBits + 14;
constexpr int kRedThreads = 256;
// LDS table of a reduce workgroup: 1024 slots, 4096 or 8192 when the bins
// hold more pairs than the partition bits can bring below ~400
constexpr int kRedSlots = 1024;
constexpr int kRedPer = 4;                // pairs loaded per thread at once

static inline unsigned acc_blocks(int64_t n, int per) {
  int64_t g = (n + per - 1) / per;
  return (unsigned)(g < 1 ? 1 : g);
}

// pairs per final bin aimed at (MAD_ACC_TARGET overrides it: 256 .. 4096,
// read once; the result does not depend on it)
static int64_t acc_target() {
  static const int64_t v = [] {
    const char* e = getenv("MAD_ACC_TARGET");
    const long x = e ? atol(e) : 512;
    return (int64_t)(x >= 256 && x <= 4096 ? x : 512);
  }();
  return v;
}

// bits of the bin index: B1 for the global partition, B2 for the second
// partition inside each first-level bin, so that bins hold about
// acc_target() pairs
static int acc_total_bits(int64_t s) {
  int b = 0;
  while (b < kAccMaxTotalBits && (acc_target() << b) < s) ++b;
  return b;
}

static int acc_b1(int64_t s) {
  const int b = acc_total_bits(s);
  return b < kAccMaxBits ? b : kAccMaxBits;
}

static int acc_b2(int64_t s) { return acc_total_bits(s) - acc_b1(s); }

size_t accum_bytes(int64_t s) {
  const int B1 = acc_b1(s), B2 = acc_b2(s);
  const int64_t tiles = (s + kAccTile - 1) / kAccTile;
  const size_t cnt = (size_t)(tiles << B1) + 1;
  const size_t starts = ((size_t)1 << (B1 + B2)) + 1;
  return (size_t)s * 12 + cnt * 8 * 2 + starts * 8 * 3 + 8192;
}

__device__ __forceinline__ uint32_t bin_of(uint64_t key, int B) {
  return B ? (uint32_t)(mix64(key) >> (64 - B)) : 0u;
}

// Count and place walk the pairs in tiles of kAccTile; a workgroup takes a
// group of consecutive tiles (about kAccGroups groups in all, enough to
// fill the chip), so that the per-(bin, group) counts and offsets are
// written and read once per group instead of once per tile: a tile's share
// of a bin follows the shares of the group's earlier tiles, through a
// per-bin cursor kept in LDS.
constexpr int64_t kAccGroups = 2048;

static inline int64_t acc_group_tiles(int64_t tiles) {
  const int64_t g = tiles / kAccGroups;
  return g < 1 ? 1 : g;
}

// count: per group, histogram of bins -> cnt[bin * groups + group]; the
// entry after the last, cnt[groups << B], is set to 0 so that the
// exclusive scan leaves the number of closed pairs there.  Each thread
// loads its kAccPer pairs of a tile before any of them is counted.
__global__ __launch_bounds__(kAccThreads) void k_acc_count(
    const uint64_t* pk, int64_t n, int B, int64_t gt, int64_t groups,
    uint64_t* cnt) {
  // pk: the keys; gt: tiles per group
  __shared__ unsigned h[1 << kAccMaxBits];
  const int nb = 1 << B;
  for (int b = threadIdx.x; b < nb; b += kAccThreads) h[b] = 0;
  __syncthreads();
  const int64_t tiles = (n + kAccTile - 1) / kAccTile;
  const int64_t tl0 = (int64_t)blockIdx.x * gt;
  const int64_t tl1 = tl0 + gt < tiles ? tl0 + gt : tiles;
  for (int64_t tile = tl0; tile < tl1; ++tile) {
    const int64_t t0 = tile * kAccTile + threadIdx.x;
    uint64_t key[kAccPer];
#pragma unroll
    for (int u = 0; u < kAccPer; ++u) {
      const int64_t e = t0 + (int64_t)u * kAccThreads;
      key[u] = e < n ? pk[e] : kEmptyKey;
    }
#pragma unroll
    for (int u = 0; u < kAccPer; ++u)
      if (key[u] != kEmptyKey) atomicAdd(&h[bin_of(key[u], B)], 1u);
  }
  __syncthreads();
  for (int b = threadIdx.x; b < nb; b += kAccThreads)
    cnt[(int64_t)b * groups + blockIdx.x] = h[b];
  if (blockIdx.x == 0 && threadIdx.x == 0) cnt[groups << B] = 0;
}

// place: every pair into its bin's range.  Each tile is first sorted by bin
// in LDS (the order inside a tile's share of a bin does not matter), so
// that each bin's share is stored as one contiguous run at the bin's
// cursor, which then advances by the share.
__global__ __launch_bounds__(kAccThreads) void k_acc_place(
    const uint64_t* pk, const float* pv, int64_t n, int B, int64_t gt,
    int64_t groups, const uint64_t* offs, uint64_t* ok, float* ov) {
  __shared__ unsigned long long base[1 << kAccMaxBits];
  __shared__ unsigned h[(1 << kAccMaxBits) + 1];  // h[nb]: the tile's total
  __shared__ unsigned long long sk[kAccTile];
  __shared__ float sv[kAccTile];
  __shared__ unsigned char sb[kAccTile];
  const int nb = 1 << B;
  for (int b = threadIdx.x; b < nb; b += kAccThreads)
    base[b] = offs[(int64_t)b * groups + blockIdx.x];
  const int64_t tiles = (n + kAccTile - 1) / kAccTile;
  const int64_t tl0 = (int64_t)blockIdx.x * gt;
  const int64_t tl1 = tl0 + gt < tiles ? tl0 + gt : tiles;
  for (int64_t tile = tl0; tile < tl1; ++tile) {
    for (int b = threadIdx.x; b < nb; b += kAccThreads) h[b] = 0;
    const int64_t t0 = tile * kAccTile;
    uint64_t key[kAccPer];
    float val[kAccPer];
    uint32_t bin[kAccPer], rank[kAccPer];
#pragma unroll
    for (int u = 0; u < kAccPer; ++u) {
      const int64_t e = t0 + u * kAccThreads + threadIdx.x;
      key[u] = e < n ? pk[e] : kEmptyKey;
      val[u] = e < n ? pv[e] : 0.0f;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kAccPer; ++u) {
      bin[u] = key[u] == kEmptyKey ? 0u : bin_of(key[u], B);
      rank[u] = key[u] == kEmptyKey ? 0u : atomicAdd(&h[bin[u]], 1u);
    }
    __syncthreads();
    // local starts: exclusive prefix of h (nb <= 256: one wave, 4 per
    // lane); h[nb] = the tile's closed pairs
    if (threadIdx.x < 64) {
      const int lane = threadIdx.x;
      unsigned v[4], sum = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int b = lane * 4 + q;
        v[q] = b < nb ? h[b] : 0u;
        sum += v[q];
      }
      unsigned ex = wave_incl_scan(sum) - sum;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int b = lane * 4 + q;
        if (b < nb) h[b] = ex;
        ex += v[q];
      }
      if (lane == 63) h[nb] = ex;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kAccPer; ++u) {
      if (key[u] == kEmptyKey) continue;
      const unsigned p = h[bin[u]] + rank[u];
      sk[p] = key[u];
      sv[p] = val[u];
      sb[p] = (unsigned char)bin[u];
    }
    __syncthreads();
    const unsigned total = h[nb];
    for (unsigned i = threadIdx.x; i < total; i += kAccThreads) {
      const unsigned b = sb[i];
      const int64_t d = (int64_t)base[b] + (int64_t)(i - h[b]);
      ok[d] = sk[i];
      ov[d] = sv[i];
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nb; b += kAccThreads)
      base[b] += h[b + 1] - h[b];
    __syncthreads();
  }
}

// one workgroup per bin: sum equal keys in an LDS table and write the
// distinct (key, x) at the front of the bin's own range [lo, hi) of the
// output (a bin has no more distinct keys than pairs), EMPTY after them, so
// the output is a table of n entries and no global atomics are needed.  The
// bin's keys share the top B hash bits.  The thread that claims a slot for
// a new key stores its increment; increments of keys already present are
// added after a barrier, so most pairs cost one LDS atomic.
template <int SLOTS>
__global__ __launch_bounds__(kRedThreads) void k_acc_reduce(
    const uint64_t* pk, const float* pv, const uint64_t* starts, int B,
    const float* bmax, int64_t s_for_F, uint64_t* okey, int64_t* oval,
    uint64_t* bin_distinct) {
  constexpr int kPer = SLOTS / kRedThreads;  // slots owned per thread
  constexpr int kW = kRedThreads / 64;
  __shared__ unsigned long long sk[SLOTS];
  __shared__ unsigned long long sv[SLOTS];
  __shared__ int full;
  __shared__ unsigned wc[kPer][kW];
  const int64_t bin = blockIdx.x;
  const int64_t lo = (int64_t)starts[bin];
  const int64_t hi = (int64_t)starts[bin + 1];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int F = bmax ? fix_exponent(*bmax, s_for_F) : (int)s_for_F;
  int64_t wpos = lo;  // next output position (uniform)
  // sub-bins: the hash bits below the bin's B bits
  int R = 1;  // sub-bins in the current split (a power of two)
  int64_t sub = 0;
  while (hi > lo && sub < R) {
    for (int q = threadIdx.x; q < SLOTS; q += kRedThreads)
      sk[q] = kEmptyKey;
    if (threadIdx.x == 0) full = 0;
    __syncthreads();
    const int rb = 31 - __clz(R);  // log2 R
    for (int64_t b0 = lo; b0 < hi; b0 += kRedThreads * kRedPer) {
      uint64_t pkey[kRedPer];
      int64_t pinc[kRedPer];
#pragma unroll
      for (int u = 0; u < kRedPer; ++u) {
        const int64_t e = b0 + threadIdx.x + (int64_t)u * kRedThreads;
        pkey[u] = e < hi ? pk[e] : kEmptyKey;
        pinc[u] = e < hi ? (int64_t)rint(ldexp((double)pv[e], F)) : 0;
      }
      int dq[kRedPer];  // slot of a key found present (-1: none)
#pragma unroll
      for (int u = 0; u < kRedPer; ++u) {
        dq[u] = -1;
        const uint64_t key = pkey[u];
        if (key == kEmptyKey) continue;
        const uint64_t h = mix64(key);
        if (rb && (int64_t)((h << B) >> (64 - rb)) != sub) continue;
        uint32_t q = (uint32_t)(h ^ (h >> 29)) & (SLOTS - 1);
        int probes = 0;
        while (true) {
          const unsigned long long prev =
              atomicCAS(&sk[q], (unsigned long long)kEmptyKey,
                        (unsigned long long)key);
          if (prev == kEmptyKey) {
            sv[q] = (unsigned long long)pinc[u];
            break;
          }
          if (prev == key) {
            dq[u] = (int)q;
            break;
          }
          if (++probes == SLOTS / 2) {  // table nearly full: split finer
            full = 1;
            break;
          }
          q = (q + 1) & (SLOTS - 1);
        }
      }
      __syncthreads();
#pragma unroll
      for (int u = 0; u < kRedPer; ++u)
        if (dq[u] >= 0) atomicAdd(&sv[dq[u]], (unsigned long long)pinc[u]);
      __syncthreads();
    }
    if (full) {
      // sub-bin `sub` of R becomes sub-bins 2 sub and 2 sub + 1 of 2R (the
      // hash bits are taken from the top, so the ranges nest)
      __syncthreads();
      if (rb + B >= 60) break;  // cannot split further (not reachable)
      R *= 2;
      sub *= 2;
      continue;
    }
    // compact the table: thread t owns slots u kRedThreads + t
    uint64_t ball[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      ball[u] = __ballot(sk[u * kRedThreads + threadIdx.x] != kEmptyKey);
      if (lane == 0) wc[u][wv] = (unsigned)__popcll(ball[u]);
    }
    __syncthreads();
    int64_t base = wpos;
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      unsigned before = 0, all = 0;
#pragma unroll
      for (int w = 0; w < kW; ++w) {
        before += w < wv ? wc[u][w] : 0u;
        all += wc[u][w];
      }
      const int q = u * kRedThreads + threadIdx.x;
      if ((ball[u] >> lane) & 1) {
        const int64_t o =
            base + before + __popcll(ball[u] & ((1ull << lane) - 1));
        okey[o] = sk[q];
        oval[o] = (int64_t)sv[q];
      }
      base += all;
    }
    wpos = base;
    __syncthreads();
    ++sub;
  }
  for (int64_t e = wpos + threadIdx.x; e < hi; e += kRedThreads) {
    okey[e] = kEmptyKey;
    oval[e] = 0;
  }
  // one count per bin: atomics of every workgroup on one counter would
  // serialize
  if (threadIdx.x == 0) bin_distinct[bin] = (uint64_t)(wpos - lo);
}

// *out = sum of v[0 .. n), *len = *last (one workgroup)
__global__ __launch_bounds__(1024) void k_acc_sum(const uint64_t* v, int64_t n,
                                                  int64_t* out,
                                                  const uint64_t* last,
                                                  int64_t* len) {
  __shared__ unsigned long long ws[16];
  unsigned long long x = 0;
  for (int64_t e = threadIdx.x; e < n; e += 1024) x += v[e];
  x = wave_sum(x);
  if ((threadIdx.x & 63) == 0) ws[threadIdx.x >> 6] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long t = 0;
    for (int w = 0; w < 16; ++w) t += ws[w];
    *out = (int64_t)t;
    *len = (int64_t)*last;
  }
}

// exclusive prefix of a u64 array (one 1024-thread workgroup per 4096
// values, then the tile sums recursively)
__global__ __launch_bounds__(1024) void k_acc_scan_tiles(const uint64_t* in,
                                                        uint64_t* out,
                                                        int64_t n,
                                                        uint64_t* sums) {
  __shared__ uint64_t ws[16];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int64_t base = (int64_t)blockIdx.x * 4096 + (int64_t)t * 4;
  uint64_t v[4], sum = 0;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    v[u] = base + u < n ? in[base + u] : 0ull;
    sum += v[u];
  }
  const uint64_t inc = wave_incl_scan(sum);
  if (lane == 63) ws[wv] = inc;
  __syncthreads();
  uint64_t off = 0, all = 0;
  for (int w = 0; w < 16; ++w) {
    off += w < wv ? ws[w] : 0ull;
    all += ws[w];
  }
  uint64_t run = off + inc - sum;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    if (base + u < n) out[base + u] = run;
    run += v[u];
  }
  if (t == 0) sums[blockIdx.x] = all;
}

__global__ void k_acc_scan_add(uint64_t* out, int64_t n,
                               const uint64_t* offs) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) out[e] += offs[e / 4096];
}

static hipError_t acc_scan(uint64_t* a, int64_t n, uint64_t* tmp,
                           hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int64_t nt = (n + 4095) / 4096;
  k_acc_scan_tiles<<<(unsigned)nt, 1024, 0, st>>>(a, a, n, tmp);
  if (nt > 1) {
    hipError_t e = acc_scan(tmp, nt, tmp + nt, st);
    if (e != hipSuccess) return e;
    k_acc_scan_add<<<acc_blocks(n, 256), 256, 0, st>>>(a, n, tmp);
  }
  return hipGetLastError();
}

// first-level bin starts: starts[b] = offs[b * groups] (b <= nb; the last
// is the number of closed pairs)
__global__ void k_acc_starts1(const uint64_t* offs, int64_t groups, int B1,
                              uint64_t* starts) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (b <= (int64_t(1) << B1)) starts[b] = offs[b * groups];
}

// second level: one workgroup per first-level bin partitions its pairs by
// the B2 hash bits below the B1 bits already used (LDS counts, scan, place)
// and writes the sub-bin starts; starts2[(b << B2) + r] for every sub-bin,
// starts2[bins << B2] = the end of the last bin
constexpr int kAcc2Threads = 1024;
constexpr int kChunk2 = 4 * kAcc2Threads;

__global__ __launch_bounds__(kAcc2Threads) void k_acc_split2(
    const uint64_t* ik, const float* iv, const uint64_t* starts1, int B1,
    int B2, uint64_t* ok, float* ov, uint64_t* starts2) {
  __shared__ unsigned h[1 << kAcc2MaxBits];
  __shared__ unsigned cc[1 << kAcc2MaxBits];
  __shared__ unsigned wt[kAcc2Threads / 64];
  __shared__ unsigned long long sk[kChunk2];
  __shared__ float sv[kChunk2];
  __shared__ unsigned short sr[kChunk2];
  const int64_t b = blockIdx.x;
  const int64_t lo = (int64_t)starts1[b], hi = (int64_t)starts1[b + 1];
  const int nb2 = 1 << B2;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  for (int r = t; r < nb2; r += kAcc2Threads) h[r] = 0;
  __syncthreads();
  for (int64_t e0 = lo + t; e0 < hi; e0 += kAcc2Threads * 8) {
    uint64_t key[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t e = e0 + (int64_t)u * kAcc2Threads;
      key[u] = e < hi ? ik[e] : 0ull;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u)
      if (e0 + (int64_t)u * kAcc2Threads < hi)
        atomicAdd(&h[(uint32_t)((mix64(key[u]) << B1) >> (64 - B2))], 1u);
  }
  __syncthreads();
  // exclusive scan of h: thread t owns sub-bins [t kPer2, (t + 1) kPer2)
  constexpr int kPer2 = (1 << kAcc2MaxBits) / kAcc2Threads;
  unsigned v[kPer2], sum = 0;
#pragma unroll
  for (int u = 0; u < kPer2; ++u) {
    const int r = t * kPer2 + u;
    v[u] = r < nb2 ? h[r] : 0u;
    sum += v[u];
  }
  const unsigned inc = wave_incl_scan(sum);
  if (lane == 63) wt[wv] = inc;
  __syncthreads();
  unsigned ex = inc - sum;
  for (int w = 0; w < wv; ++w) ex += wt[w];
  __syncthreads();
#pragma unroll
  for (int u = 0; u < kPer2; ++u) {
    const int r = t * kPer2 + u;
    if (r < nb2) {
      h[r] = ex;  // cursor
      starts2[(b << B2) + r] = (uint64_t)(lo + ex);
    }
    ex += v[u];
  }
  if (b == (int64_t)gridDim.x - 1 && t == 0)
    starts2[(b + 1) << B2] = starts1[b + 1];
  __syncthreads();
  // place, a chunk of kChunk2 pairs at a time: the chunk is sorted by
  // sub-bin in LDS, then each sub-bin's share is stored as one run at its
  // cursor (h[r], relative to lo), which then advances by that share
  // the next chunk's pairs are loaded while this one is placed (clamped
  // to the bin's last pair, so the loads carry no branch)
  uint64_t nkey[4] = {0ull, 0ull, 0ull, 0ull};
  float nval[4] = {0.0f, 0.0f, 0.0f, 0.0f};
  if (hi > lo) {  // uniform: an empty bin loads nothing
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      int64_t e = lo + (int64_t)u * kAcc2Threads + t;
      e = e < hi ? e : hi - 1;
      nkey[u] = ik[e];
      nval[u] = iv[e];
    }
  }
  for (int64_t c0 = lo; c0 < hi; c0 += kChunk2) {
    uint64_t key[4];
    float val[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      key[u] = nkey[u];
      val[u] = nval[u];
      int64_t e = c0 + kChunk2 + (int64_t)u * kAcc2Threads + t;
      e = e < hi ? e : hi - 1;
      nkey[u] = ik[e];
      nval[u] = iv[e];
    }
    for (int r = t; r < nb2; r += kAcc2Threads) cc[r] = 0;
    __syncthreads();
    uint32_t sub[4], rank[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t e = c0 + (int64_t)u * kAcc2Threads + t;
      const bool in = e < hi;
      sub[u] = in ? (uint32_t)((mix64(key[u]) << B1) >> (64 - B2)) : 0u;
      rank[u] = in ? atomicAdd(&cc[sub[u]], 1u) : 0u;
    }
    __syncthreads();
    unsigned cv[kPer2], csum = 0;
#pragma unroll
    for (int u = 0; u < kPer2; ++u) {
      const int r = t * kPer2 + u;
      cv[u] = r < nb2 ? cc[r] : 0u;
      csum += cv[u];
    }
    const unsigned cinc = wave_incl_scan(csum);
    if (lane == 63) wt[wv] = cinc;
    __syncthreads();
    unsigned cex = cinc - csum;
    for (int w = 0; w < wv; ++w) cex += wt[w];
#pragma unroll
    for (int u = 0; u < kPer2; ++u) {
      const int r = t * kPer2 + u;
      if (r < nb2) cc[r] = cex;  // the chunk's start of sub-bin r
      cex += cv[u];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      if (c0 + (int64_t)u * kAcc2Threads + t >= hi) continue;
      const unsigned q = cc[sub[u]] + rank[u];
      sk[q] = key[u];
      sv[q] = val[u];
      sr[q] = (unsigned short)sub[u];
    }
    __syncthreads();
    const int nc = hi - c0 < kChunk2 ? (int)(hi - c0) : kChunk2;
    for (int i = t; i < nc; i += kAcc2Threads) {
      const unsigned r = sr[i];
      const int64_t d = lo + (int64_t)h[r] + (int64_t)(i - (int)cc[r]);
      ok[d] = sk[i];
      ov[d] = sv[i];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kPer2; ++u) {
      const int r = t * kPer2 + u;
      if (r < nb2) h[r] += cv[u];
    }
    __syncthreads();
  }
}

// the LDS table size for bins of about `per_bin` pairs (load <= ~0.5);
// MAD_ACC_SLOTS = 1024, 4096 or 8192 forces one (the result is the same)
static int reduce_slots(int64_t per_bin) {
  if (const char* e = getenv("MAD_ACC_SLOTS")) {
    const int v = atoi(e);
    if (v == 1024 || v == 4096 || v == 8192) return v;
  }
  return per_bin <= 512 ? 1024 : per_bin <= 1536 ? 4096 : 8192;
}

static void launch_reduce(int64_t per_bin, int64_t bins, const uint64_t* pk,
                          const float* pv, const uint64_t* starts, int B,
                          const float* bmax, int64_t s_for_F, uint64_t* okey,
                          int64_t* oval, uint64_t* bin_distinct,
                          hipStream_t st) {
  const int slots = reduce_slots(per_bin);
  if (slots == kRedSlots)
    k_acc_reduce<kRedSlots><<<(unsigned)bins, kRedThreads, 0, st>>>(
        pk, pv, starts, B, bmax, s_for_F, okey, oval, bin_distinct);
  else if (slots == 4096)
    k_acc_reduce<4096><<<(unsigned)bins, kRedThreads, 0, st>>>(
        pk, pv, starts, B, bmax, s_for_F, okey, oval, bin_distinct);
  else
    k_acc_reduce<8192><<<(unsigned)bins, kRedThreads, 0, st>>>(
        pk, pv, starts, B, bmax, s_for_F, okey, oval, bin_distinct);
}

// pairs: n (key, inc) pairs, key EMPTY for none; work: accum_bytes(n);
// output: okey / oval, *o_len (device) entries = closed pairs holding the
// *o_count (device) distinct keys, EMPTY elsewhere.  The pair array is
// overwritten.
hipError_t launch_accumulate(uint64_t* keys, float* vals, int64_t n,
                             const float* bmax, int64_t s_for_F, void* work,
                             size_t work_bytes, uint64_t* okey, int64_t* oval,
                             int64_t* o_count, int64_t* o_len, hipStream_t st) {
  hipError_t e;
  if (n <= 0) {  // otherwise k_acc_sum writes both
    FillBatch f{};
    f.p[0] = (uint64_t*)o_count;
    f.p[1] = (uint64_t*)o_len;
    f.n[0] = f.n[1] = 1;
    f.count = 2;
    return launch_fill_multi(f, st);
  }
  if (work_bytes < accum_bytes(n)) return hipErrorInvalidValue;
  const int B1 = acc_b1(n), B2 = acc_b2(n);
  const int64_t tiles = (n + kAccTile - 1) / kAccTile;
  const int64_t gt = acc_group_tiles(tiles);
  const int64_t groups = (tiles + gt - 1) / gt;
  const int64_t ncnt = groups << B1;
  const int64_t nb1 = int64_t(1) << B1;
  char* p = (char*)work;
  uint64_t* placed = (uint64_t*)p;
  p += (size_t)n * 8;
  float* placed_v = (float*)p;
  p += ((size_t)n * 4 + 15) / 16 * 16;
  uint64_t* cnt = (uint64_t*)p;
  p += ((size_t)(tiles << B1) + 1) * 8;  // room for one group per tile
  uint64_t* starts = (uint64_t*)p;
  p += (((size_t)1 << (B1 + B2)) + 1) * 8;
  uint64_t* starts1 = (uint64_t*)p;
  p += (((size_t)1 << (B1 + B2)) + 1) * 8;
  uint64_t* bin_distinct = (uint64_t*)p;
  p += (((size_t)1 << (B1 + B2)) + 1) * 8;
  uint64_t* tmp = (uint64_t*)p;  // scan partial sums
  k_acc_count<<<(unsigned)groups, kAccThreads, 0, st>>>(keys, n, B1, gt,
                                                        groups, cnt);
  if ((e = acc_scan(cnt, ncnt + 1, tmp, st)) != hipSuccess) return e;
  k_acc_place<<<(unsigned)groups, kAccThreads, 0, st>>>(
      keys, vals, n, B1, gt, groups, cnt, placed, placed_v);
  if (B2 == 0) {
    k_acc_starts1<<<acc_blocks(nb1 + 1, 256), 256, 0, st>>>(cnt, groups, B1,
                                                            starts);
    launch_reduce(n >> B1, nb1, placed, placed_v, starts, B1, bmax, s_for_F,
                  okey, oval, bin_distinct, st);
  } else if (B2 <= kAccSplitBits) {
    k_acc_starts1<<<acc_blocks(nb1 + 1, 256), 256, 0, st>>>(cnt, groups, B1,
                                                            starts1);
    k_acc_split2<<<(unsigned)nb1, kAcc2Threads, 0, st>>>(
        placed, placed_v, starts1, B1, B2, keys, vals, starts);
    launch_reduce(n >> (B1 + B2), nb1 << B2, keys, vals, starts, B1 + B2,
                  bmax, s_for_F, okey, oval, bin_distinct, st);
  } else {
    // two splits of at most kAccSplitBits bits each, so that a chunk of
    // kChunk2 pairs still stores runs of ~16 or more pairs per sub-bin;
    // the middle starts live in bin_distinct until the reduce writes it
    const int Ba = (B2 + 1) / 2, Bb = B2 - Ba;
    uint64_t* starts_mid = bin_distinct;
    k_acc_starts1<<<acc_blocks(nb1 + 1, 256), 256, 0, st>>>(cnt, groups, B1,
                                                            starts1);
    k_acc_split2<<<(unsigned)nb1, kAcc2Threads, 0, st>>>(
        placed, placed_v, starts1, B1, Ba, keys, vals, starts_mid);
    k_acc_split2<<<(unsigned)(nb1 << Ba), kAcc2Threads, 0, st>>>(
        keys, vals, starts_mid, B1 + Ba, Bb, placed, placed_v, starts);
    launch_reduce(n >> (B1 + B2), nb1 << B2, placed, placed_v, starts,
                  B1 + B2, bmax, s_for_F, okey, oval, bin_distinct, st);
  }
  // entries written = closed pairs = the end of the last bin
  k_acc_sum<<<1, 1024, 0, st>>>(bin_distinct, nb1 << B2, o_count,
                                starts + (nb1 << B2), o_len);
  return hipGetLastError();
}

hipError_t launch_accumulate_grouped(uint64_t* keys, float* vals, int64_t n,
                                     const uint64_t* gstarts, int64_t G,
                                     const float* bmax, int64_t s_for_F,
                                     void* work, size_t work_bytes,
                                     uint64_t* okey, int64_t* oval,
                                     int64_t* o_count, int64_t* o_len,
                                     hipStream_t st) {
  if (n <= 0 || G < 1 || !gstarts)
    return launch_accumulate(keys, vals, n, bmax, s_for_F, work, work_bytes,
                             okey, oval, o_count, o_len, st);
  if (work_bytes < accum_bytes(n)) return hipErrorInvalidValue;
  // the groups stand for the first gb bits of the hashed form: split each
  // by the hash bits that bring its bins to about acc_target() pairs
  int gb = 0;
  while ((int64_t(1) << gb) < G) ++gb;
  const int T = acc_total_bits(n);
  // more groups than bins of the hashed form (few pairs): its layout would
  // not hold the group starts, and the groups would be tiny anyway
  if (gb > T)
    return launch_accumulate(keys, vals, n, bmax, s_for_F, work, work_bytes,
                             okey, oval, o_count, o_len, st);
  const int B2 = T - gb;
  char* p = (char*)work;
  uint64_t* placed = (uint64_t*)p;
  p += (size_t)n * 8;
  float* placed_v = (float*)p;
  p += ((size_t)n * 4 + 15) / 16 * 16;
  const int B1h = acc_b1(n);
  const int64_t tiles = (n + kAccTile - 1) / kAccTile;
  p += ((size_t)(tiles << B1h) + 1) * 8;  // the count array of the other form
  uint64_t* starts = (uint64_t*)p;
  p += (((size_t)1 << T) + 1) * 8;
  p += (((size_t)1 << T) + 1) * 8;  // first-level starts of the other form
  uint64_t* bin_distinct = (uint64_t*)p;
  const int64_t bins = G << B2;
  if (B2 == 0) {
    launch_reduce(n / G, G, keys, vals, gstarts, 0, bmax, s_for_F, okey, oval,
                  bin_distinct, st);
    k_acc_sum<<<1, 1024, 0, st>>>(bin_distinct, G, o_count, gstarts + G,
                                  o_len);
    return hipGetLastError();
  }
  if (B2 <= kAccSplitBits) {
    k_acc_split2<<<(unsigned)G, kAcc2Threads, 0, st>>>(
        keys, vals, gstarts, 0, B2, placed, placed_v, starts);
    launch_reduce(n / bins, bins, placed, placed_v, starts, B2, bmax, s_for_F,
                  okey, oval, bin_distinct, st);
  } else {
    const int Ba = (B2 + 1) / 2, Bb = B2 - Ba;
    uint64_t* starts_mid = bin_distinct;
    k_acc_split2<<<(unsigned)G, kAcc2Threads, 0, st>>>(
        keys, vals, gstarts, 0, Ba, placed, placed_v, starts_mid);
    k_acc_split2<<<(unsigned)(G << Ba), kAcc2Threads, 0, st>>>(
        placed, placed_v, starts_mid, Ba, Bb, keys, vals, starts);
    launch_reduce(n / bins, bins, keys, vals, starts, B2, bmax, s_for_F, okey,
                  oval, bin_distinct, st);
  }
  k_acc_sum<<<1, 1024, 0, st>>>(bin_distinct, bins, o_count, starts + bins,
                                o_len);
  return hipGetLastError();
}

}  // namespace mad
