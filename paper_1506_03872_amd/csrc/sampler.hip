// sampler.hip -- the sampling loop of Alg. 3 (its draws and score update) for dense
// inputs.  Each sample either writes its (key, increment) pair at its own
// index (pair form; X is then summed by accum.hip) or adds its increment to
// an open-addressing hash table X (hash form).  Samples can run in k order
// (the grouping of Sec. 5.2) so that T1[k] and T2[k] stay in L2.
//
// Sample l uses the Philox4x64-10 block with counter (l, qid, 0, 0) and key
// (seed, 0): word 0 draws k from T0, word 1 draws i from T1[k], word 2 draws
// j from T2[k], word 3 draws k' from T3[i] (the two-stage form of line
// the draw of (k, i): k with weight ||B_k*||_1 v_k, then i with weight |a_ki| ||a_i||_1).
// The alias entries carry the sign bits of a_ki, b_kj and a_k'i, so the only
// value read from the inputs is the fourth edge b_k'j.  A closed three-path
// (b_k'j != 0) adds sgn(a_ki b_kj a_k'i) * rne(b_k'j * 2^F) to the int64
// score of key i*n + j; integer sums make X independent of the order in
// which the increments are added.
#include <stdlib.h>

#include "mad_common.hpp"
#include "plan.hpp"

namespace mad {

constexpr int kT0Lds = 4096;  // stage-0 table kept in LDS up to this size
constexpr int64_t kOrderMaxD = 1024;          // k ordering for d up to this
constexpr int64_t kOrderChunkMin = int64_t(1) << 12;
constexpr int64_t kOrderChunkMax = int64_t(1) << 28;  // samples per ordering

struct DenseSampleArgs {
  const uint64_t* T0;
  const uint64_t* T1;
  const uint64_t* T2;
  const uint64_t* T3;
  int L0, L1, L2, L3;
  const float* B;
  int64_t d, n;
  uint64_t seed, qid;
  int64_t l0, count;
  int gram;  // B = A: key of the pair with i < j, diagonal left out
  // squared variant (Sec. 3.2.3): the second pair of sample e, keyed by
  // (k, k') like the first, goes to pk2[e] / pv2[e] (pair form only)
  uint64_t* pk2;
  float* pv2;
  // binary B (Alg. 1): when *bbin == 1 the fourth edge is bit j*d + k' of
  // bbits, an array of n*d bits that stays in L2, instead of B[j*d + k']
  const uint32_t* bbits;
  const int* bbin;
};

// the fourth edge b_k'j: from the bitmap of a binary B, else from B
__device__ __forceinline__ float fourth_edge(const float* B,
                                             const uint32_t* bbits, bool bin,
                                             int64_t d, uint32_t j,
                                             uint32_t kp) {
  const int64_t e = (int64_t)j * d + kp;
  if (bin) return (float)((bbits[e >> 5] >> (e & 31)) & 1u);
  return B[e];
}

// key of an update of x_ab: a*n + b, or for symmetrised scores the key of
// (min, max) with the diagonal left out (kEmptyKey)
__device__ __forceinline__ uint64_t pair_key(uint64_t a, uint64_t b,
                                             uint64_t n, int gram,
                                             bool closed) {
  if (!closed) return kEmptyKey;
  if (gram) {
    if (a == b) return kEmptyKey;
    if (a > b) {
      const uint64_t t = a;
      a = b;
      b = t;
    }
  }
  return a * n + b;
}

struct OneSample {
  uint32_t k, i, j, kp;
  int64_t inc;
  bool closed;
};

// Samples in k order (the first reordering of the locality scheme of Sec. 5.2): `ell` lists sample offsets sorted by their stage-0 draw k.  The
// sampling launch then gives each XCD (workgroups are dispatched to the 8
// XCDs round robin) a contiguous eighth of that list, walked in order by
// its workgroups, so the rows T1[k] and T2[k] being drawn from stay in that
// XCD's L2.  Results do not depend on the order.
struct GroupOrder {
  const uint32_t* ell;  // sample offsets (from l0), sorted by k
  int64_t chunk;        // samples per workgroup step (256 * U)
};

template <int U, bool DEBUG, bool GROUPED>
__global__ __launch_bounds__(256) void k_sample_dense(
    DenseSampleArgs a, const double* wtot, const float* bmax, int64_t s_for_F,
    int F_debug,
    uint64_t* hkeys, int64_t* hvals, uint64_t hmask, uint64_t* pkeys,
    float* pvals, SampleCounters* ctr, int32_t* ok, int32_t* oi, int32_t* oj,
    int32_t* okp, int64_t* oinc, GroupOrder go) {
  extern __shared__ uint64_t t0s[];  // T0 when it fits (kT0Lds entries)
  if (!(wtot[0] > 0.0)) {  // ||W||_1 = 0: nothing can be sampled
    if (pkeys)
      for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
           e < a.count; e += (int64_t)gridDim.x * blockDim.x) {
        pkeys[e] = kEmptyKey;
        if (a.pk2) a.pk2[e] = kEmptyKey;
      }
    return;
  }
  const int N0 = 1 << a.L0;
  const bool t0_lds = N0 <= kT0Lds;
  if (t0_lds)
    for (int e = threadIdx.x; e < N0; e += blockDim.x) t0s[e] = a.T0[e];
  __syncthreads();
  const uint64_t* T0 = t0_lds ? t0s : a.T0;
  const int F = DEBUG ? F_debug : fix_exponent(*bmax, s_for_F);
  const bool binB = a.bbin && *a.bbin == 1;

  // ungrouped: grid-stride over samples; grouped: chunks of the k-sorted
  // list, XCD x = blockIdx % 8 takes chunks [x, x+1) * nch / 8 in order
  const int64_t nthreads = GROUPED ? 256 : (int64_t)gridDim.x * blockDim.x;
  const int64_t nch = GROUPED ? (a.count + go.chunk - 1) / go.chunk : 0;
  const int64_t xcd = blockIdx.x & 7, g8 = gridDim.x >> 3;
  const int64_t ch_lo = GROUPED ? xcd * nch / 8 : 0;
  const int64_t ch_hi = GROUPED ? (xcd + 1) * nch / 8 : 0;
  int64_t ch = GROUPED ? ch_lo + (blockIdx.x >> 3) : 0;
  int64_t base = GROUPED ? ch * go.chunk + threadIdx.x
                         : (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long nclosed = 0, ncreated = 0;
  while (GROUPED ? ch < ch_hi : base < a.count) {
    OneSample smp[U];
    uint64_t U1[U], U2[U], U3[U];
    // the samples' indices l - l0 (positions e = base + 256 u)
    uint64_t ls[U];
    if constexpr (GROUPED) {
      // from the k-sorted list: each thread loads U consecutive entries in
      // one 16-byte load and passes them through LDS, so the U entries a
      // thread draws arrive with one memory latency (separate loads were
      // issued one after another, each waited for before the next)
      static_assert(U == 4, "the grouped sampler takes four samples a thread");
      __shared__ __attribute__((aligned(16))) uint32_t ell_s[256 * U];
      const int64_t cb = ch * go.chunk;  // go.chunk == 256 U
      const int64_t p = cb + (int64_t)threadIdx.x * U;
      uint4 q;
      if (p + U <= a.count) {
        q = *(const uint4*)(go.ell + p);
      } else {  // the last, partial chunk: entries past the end read as 0
        q.x = p < a.count ? go.ell[p] : 0u;
        q.y = p + 1 < a.count ? go.ell[p + 1] : 0u;
        q.z = p + 2 < a.count ? go.ell[p + 2] : 0u;
        q.w = p + 3 < a.count ? go.ell[p + 3] : 0u;
      }
      __syncthreads();  // the previous step's reads of ell_s are done
      *(uint4*)(ell_s + threadIdx.x * U) = q;
      __syncthreads();
#pragma unroll
      for (int u = 0; u < U; ++u)
        ls[u] = (uint64_t)(a.l0 + (int64_t)ell_s[threadIdx.x + u * 256]);
    } else {
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t e = base + (int64_t)u * nthreads;
        ls[u] = (uint64_t)(a.l0 + (e < a.count ? e : 0));
      }
    }
    // draw of k (stage 0): from the LDS copy of T0
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint64_t l = ls[u];
      const Philox4 r = philox4x64_10(l, a.qid, 0ull, 0ull, a.seed, 0ull);
      const uint32_t s0 = slot_of(r.w0, a.L0);
      smp[u].k = draw_entry(T0[s0], s0, r.w0).pos;
      U1[u] = r.w1;
      U2[u] = r.w2;
      U3[u] = r.w3;
    }
    // draws of i (stage 1) and j: i from T1[k], j from T2[k]
    uint64_t e1[U], e2[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      e1[u] = a.T1[((uint64_t)smp[u].k << a.L1) + slot_of(U1[u], a.L1)];
      e2[u] = a.T2[((uint64_t)smp[u].k << a.L2) + slot_of(U2[u], a.L2)];
    }
    uint32_t sgn[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const Drawn di = draw_entry(e1[u], slot_of(U1[u], a.L1), U1[u]);
      const Drawn dj = draw_entry(e2[u], slot_of(U2[u], a.L2), U2[u]);
      smp[u].i = di.pos;
      smp[u].j = dj.pos;
      sgn[u] = di.sgn ^ dj.sgn;
    }
    // draw of k': from T3[i]
    uint64_t e3[U];
#pragma unroll
    for (int u = 0; u < U; ++u)
      e3[u] = a.T3[((uint64_t)smp[u].i << a.L3) + slot_of(U3[u], a.L3)];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const Drawn dk = draw_entry(e3[u], slot_of(U3[u], a.L3), U3[u]);
      smp[u].kp = dk.pos;
      sgn[u] ^= dk.sgn;
    }
    // dx: the fourth edge b_k'j and the increment
    float v[U];
#pragma unroll
    for (int u = 0; u < U; ++u)
      v[u] = fourth_edge(a.B, a.bbits, binB, a.d, smp[u].j, smp[u].kp);
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t e = base + (int64_t)u * nthreads;
      const bool live = e < a.count;
      smp[u].closed = live && v[u] != 0.0f;
      int64_t inc = 0;
      if (smp[u].closed) {
        const int64_t mag = (int64_t)rint(ldexp((double)v[u], F));
        inc = sgn[u] ? -mag : mag;
      }
      smp[u].inc = inc;
      if (DEBUG && live) {
        ok[e] = (int32_t)smp[u].k;
        oi[e] = (int32_t)smp[u].i;
        oj[e] = (int32_t)smp[u].j;
        okp[e] = (int32_t)smp[u].kp;
        oinc[e] = inc;
      }
    }
    if (!DEBUG) {
      // score updates: the U compare-and-swaps go out together, then the
      // adds; a slot's key changes from EMPTY to its final value once, so a
      // swap that finds EMPTY or the key itself owns the slot
      uint64_t key[U], slot[U];
      bool pend[U], ins[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        uint64_t ii = smp[u].i, jj = smp[u].j;
        ins[u] = smp[u].closed;
        if (a.gram) {  // Sec. 3.2.2: X + X^T on i < j, diagonal dropped
          if (ii == jj) ins[u] = false;
          if (ii > jj) {
            const uint64_t tmp = ii;
            ii = jj;
            jj = tmp;
          }
        }
        key[u] = ii * (uint64_t)a.n + jj;
        slot[u] = mix64(key[u]) & hmask;
        pend[u] = ins[u];
        nclosed += smp[u].closed;
      }
      if (pkeys) {
        // pair form: the key and the signed fourth edge at the sample's
        // place in the walk, which is one-to-one with the samples of this
        // launch; streamed once, kept out of the caches that hold T3 and B
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int64_t e = base + (int64_t)u * nthreads;
          if (e < a.count) {
            __builtin_nontemporal_store(
                (unsigned long long)(ins[u] ? key[u] : kEmptyKey),
                (unsigned long long*)(pkeys + e));
            __builtin_nontemporal_store(sgn[u] ? -v[u] : v[u], pvals + e);
            if (a.pk2) {  // Sec. 3.2.3: the same increment to x_kk'
              __builtin_nontemporal_store(
                  (unsigned long long)pair_key(smp[u].k, smp[u].kp, a.n,
                                               a.gram, smp[u].closed),
                  (unsigned long long*)(a.pk2 + e));
              __builtin_nontemporal_store(sgn[u] ? -v[u] : v[u], a.pv2 + e);
            }
          }
          pend[u] = false;
        }
      }
      bool any = !pkeys;
      while (any) {
        uint64_t prev[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
          prev[u] = pend[u] ? atomicCAS((unsigned long long*)(hkeys + slot[u]),
                                        (unsigned long long)kEmptyKey,
                                        (unsigned long long)key[u])
                            : 0ull;
        any = false;
#pragma unroll
        for (int u = 0; u < U; ++u) {
          if (!pend[u]) continue;
          if (prev[u] == kEmptyKey || prev[u] == key[u]) {
            ncreated += prev[u] == kEmptyKey;
            pend[u] = false;
          } else {
            slot[u] = (slot[u] + 1) & hmask;
            any = true;
          }
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (!pkeys && ins[u] && smp[u].inc != 0)
          atomicAdd((unsigned long long*)(hvals + slot[u]),
                    (unsigned long long)smp[u].inc);
    }
    if (GROUPED) {
      ch += g8;
      base = ch * go.chunk + threadIdx.x;
    } else {
      base += nthreads * U;
    }
  }
  if (!DEBUG) {
    // one pair of counter atomics per block
    __shared__ unsigned long long part[2][4];
    nclosed = wave_sum(nclosed);
    ncreated = wave_sum(ncreated);
    if ((threadIdx.x & 63) == 0) {
      part[0][threadIdx.x >> 6] = nclosed;
      part[1][threadIdx.x >> 6] = ncreated;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      const unsigned long long c = part[0][0] + part[0][1] + part[0][2] +
                                   part[0][3];
      const unsigned long long dd = part[1][0] + part[1][1] + part[1][2] +
                                    part[1][3];
      if (c) atomicAdd(&ctr->closed, c);
      if (dd) atomicAdd(&ctr->distinct, dd);
    }
  }
}

// the fourth edge of a binary B from its bitmap (default), or from B
// itself with MAD_BINARY_BITMAP=0 (for measurement; same results)
static bool binary_bitmap_enabled() {
  static const bool v = [] {
    const char* e = getenv("MAD_BINARY_BITMAP");
    return !(e && atoi(e) == 0);
  }();
  return v;
}

static DenseSampleArgs dense_args(const DenseTables& t, const float* B,
                                  uint64_t seed, uint64_t qid, int64_t l0,
                                  int64_t count) {
  DenseSampleArgs a;
  a.T0 = t.T0.ent;
  a.T1 = t.T1.ent;
  a.T2 = t.T2.ent;
  a.T3 = t.T3.ent;
  a.L0 = t.T0.L;
  a.L1 = t.T1.L;
  a.L2 = t.T2.L;
  a.L3 = t.T3.L;
  a.B = B;
  a.d = t.d;
  a.n = t.n;
  a.seed = seed;
  a.qid = qid;
  a.l0 = l0;
  a.count = count;
  a.gram = t.gram;
  a.pk2 = nullptr;
  a.pv2 = nullptr;
  a.bbits = t.bbits;
  a.bbin = t.bad && binary_bitmap_enabled() ? t.bad + 6 : nullptr;
  return a;
}

// most workgroups of a sampling launch (result-invariant;
// MAD_SAMPLER_GRID overrides for tuning)
static int64_t sampler_max_grid() {
  static const int64_t g = [] {
    const char* e = getenv("MAD_SAMPLER_GRID");
    const long long v = e ? atoll(e) : 8192;
    return (int64_t)(v >= 8 && v <= 65536 ? v : 8192);
  }();
  return g;
}

static unsigned sample_grid(int64_t count, int per_thread) {
  int64_t blocks = (count + 256LL * per_thread - 1) / (256LL * per_thread);
  if (blocks > sampler_max_grid()) blocks = sampler_max_grid();
  return (unsigned)(blocks < 1 ? 1 : blocks);
}

// samples in flight per thread (result-invariant; MAD_SAMPLER_UNROLL
// selects 1, 2, 4 or 8 for tuning)
static int sampler_unroll() {
  static int u = [] {
    const char* e = getenv("MAD_SAMPLER_UNROLL");
    const int v = e ? atoi(e) : 4;
    return (v == 1 || v == 2 || v == 4 || v == 8) ? v : 4;
  }();
  return u;
}

static size_t t0_lds_bytes(const DenseTables& t) {
  const int64_t N0 = int64_t(1) << t.T0.L;
  return N0 <= kT0Lds ? (size_t)N0 * 8 : 0;
}

// ---------------------------------------------------------------------------
// the k order: per block of kOrdPer consecutive samples, each sample's k
// and the counts of each k (pass 1); per k, exclusive prefix of those
// counts over the blocks and the k's total (pass 2); the start of each k's
// range (pass 3); every sample's offset written into its k's range (pass
// 4).  The order inside one block's share of a k does not matter.
// ---------------------------------------------------------------------------
constexpr int kOrdU = 16;
constexpr int kOrdPer = 256 * kOrdU;

// pass 1: each sample's k (Philox word 0 on T0) stored as 16 bits, and the
// counts of each k per block of kOrdPer samples
__global__ __launch_bounds__(256) void k_order_count(DenseSampleArgs a,
                                                    uint32_t* cnt,
                                                    uint16_t* kbuf) {
  extern __shared__ uint64_t sm[];
  const int N0 = 1 << a.L0;
  uint64_t* t0s = sm;
  uint32_t* lc = (uint32_t*)(sm + N0);
  const int64_t d = a.d;
  for (int e = threadIdx.x; e < N0; e += 256) t0s[e] = a.T0[e];
  for (int64_t k = threadIdx.x; k < d; k += 256) lc[k] = 0;
  __syncthreads();
  const int64_t b0 = (int64_t)blockIdx.x * kOrdPer;
#pragma unroll 4
  for (int u = 0; u < kOrdU; ++u) {
    const int64_t e = b0 + u * 256 + threadIdx.x;
    if (e < a.count) {
      const Philox4 r = philox4x64_10((uint64_t)(a.l0 + e), a.qid, 0ull, 0ull,
                                      a.seed, 0ull);
      const uint32_t s0 = slot_of(r.w0, a.L0);
      const uint32_t k = draw_entry(t0s[s0], s0, r.w0).pos;
      kbuf[e] = (uint16_t)k;
      atomicAdd(&lc[k], 1u);
    }
  }
  __syncthreads();
  for (int64_t k = threadIdx.x; k < d; k += 256)
    cnt[(int64_t)blockIdx.x * d + k] = lc[k];
}

// pass 4: every sample's offset into its k's range.  The block's samples
// are first sorted by k in LDS (the order inside one block's share of a k
// does not matter), so that each k's share is stored as one contiguous run.
__global__ __launch_bounds__(256) void k_order_place(DenseSampleArgs a,
                                                    const uint32_t* cnt,
                                                    const uint32_t* start,
                                                    const uint16_t* kbuf,
                                                    uint32_t* ell) {
  extern __shared__ uint64_t sm[];
  const int64_t d = a.d;
  uint32_t* lc = (uint32_t*)sm;        // d: counts, then local starts
  uint32_t* gs = lc + d;               // d: global start of the share
  uint32_t* se = gs + d;               // kOrdPer: sorted sample offsets
  uint16_t* sk = (uint16_t*)(se + kOrdPer);  // kOrdPer: their k
  __shared__ uint32_t wt[4];
  for (int64_t k = threadIdx.x; k < d; k += 256) {
    lc[k] = 0;
    gs[k] = start[k] + cnt[(int64_t)blockIdx.x * d + k];
  }
  __syncthreads();
  const int64_t b0 = (int64_t)blockIdx.x * kOrdPer;
  const int n = a.count - b0 < kOrdPer ? (int)(a.count - b0) : kOrdPer;
  uint32_t kk[kOrdU], rank[kOrdU];
#pragma unroll
  for (int u = 0; u < kOrdU; ++u) {
    const int i = u * 256 + threadIdx.x;
    kk[u] = i < n ? kbuf[b0 + i] : 0u;
  }
#pragma unroll
  for (int u = 0; u < kOrdU; ++u) {
    const int i = u * 256 + threadIdx.x;
    rank[u] = i < n ? atomicAdd(&lc[kk[u]], 1u) : 0u;
  }
  __syncthreads();
  // local starts: exclusive prefix of lc, 256 ks at a time
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint32_t carry = 0;
  for (int64_t k0 = 0; k0 < d; k0 += 256) {
    const int64_t k = k0 + threadIdx.x;
    const uint32_t v = k < d ? lc[k] : 0u;
    const uint32_t inc = wave_incl_scan(v);
    if (lane == 63) wt[wv] = inc;
    __syncthreads();
    uint32_t off = 0, all = 0;
    for (int w = 0; w < 4; ++w) {
      off += w < wv ? wt[w] : 0u;
      all += wt[w];
    }
    if (k < d) lc[k] = carry + off + inc - v;
    carry += all;
    __syncthreads();
  }
#pragma unroll
  for (int u = 0; u < kOrdU; ++u) {
    const int i = u * 256 + threadIdx.x;
    if (i < n) {
      const uint32_t p = lc[kk[u]] + rank[u];
      se[p] = (uint32_t)(b0 + i);
      sk[p] = (uint16_t)kk[u];
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < kOrdU; ++u) {
    const int i = u * 256 + threadIdx.x;
    if (i < n) {
      const uint32_t k = sk[i];
      ell[gs[k] + (uint32_t)i - lc[k]] = se[i];
    }
  }
}

// per k: exclusive prefix of the block counts (one workgroup per k)
__global__ __launch_bounds__(256) void k_order_colscan(uint32_t* cnt,
                                                      int64_t nblk,
                                                      int64_t d,
                                                      uint32_t* tot) {
  __shared__ uint32_t wt[4];
  const int64_t k = blockIdx.x;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint32_t carry = 0;
  for (int64_t b0 = 0; b0 < nblk; b0 += 256) {
    const int64_t b = b0 + threadIdx.x;
    const uint32_t v = b < nblk ? cnt[b * d + k] : 0u;
    const uint32_t inc = wave_incl_scan(v);
    if (lane == 63) wt[wv] = inc;
    __syncthreads();
    uint32_t off = 0, all = 0;
    for (int w = 0; w < 4; ++w) {
      off += w < wv ? wt[w] : 0u;
      all += wt[w];
    }
    if (b < nblk) cnt[b * d + k] = carry + off + inc - v;
    carry += all;
    __syncthreads();
  }
  if (threadIdx.x == 0) tot[k] = carry;
}

// start of each k's range: exclusive prefix of the totals (one workgroup)
__global__ __launch_bounds__(256) void k_order_starts(const uint32_t* tot,
                                                     int64_t d,
                                                     uint32_t* start) {
  __shared__ uint32_t wt[4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  uint32_t carry = 0;
  for (int64_t k0 = 0; k0 < d; k0 += 256) {
    const int64_t k = k0 + threadIdx.x;
    const uint32_t v = k < d ? tot[k] : 0u;
    const uint32_t inc = wave_incl_scan(v);
    if (lane == 63) wt[wv] = inc;
    __syncthreads();
    uint32_t off = 0, all = 0;
    for (int w = 0; w < 4; ++w) {
      off += w < wv ? wt[w] : 0u;
      all += wt[w];
    }
    if (k < d) start[k] = carry + off + inc - v;
    carry += all;
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// The locality pipeline (Sec. 5.2): after the k order, each sample is drawn
// in three passes, each over records grouped for the table it reads:
//   pass A (k order)   Philox, k (T0), i (T1[k]), j (T2[k]); record
//                      R1 = {U3, i, j | sign} grouped by the block of i;
//   pass B (i groups)  k' (T3[i]); record R2 = {i, j | sign, k'} grouped
//                      by the block of j;
//   pass C (j groups)  the fourth edge b_k'j (row j of B) and the sample's
//                      (key, signed fourth edge) pair.
// A pass writes each tile of records sorted by group, with the tile's group
// counts; a column scan of the counts gives every (group, tile) run its
// place in the grouped stream, and a scatter moves the runs there.  The
// next pass reads that stream in order, the tiles of each XCD contiguous,
// so the table rows of the groups it works on stay in that XCD's L2.  The
// pairs come out grouped by j, which the score accumulation takes as its
// first partition level.  Results do not depend on any of this: every
// sample is a function of (seed, l) and X is an exact int64 sum.
// ---------------------------------------------------------------------------
constexpr int kPipeU = 8;
constexpr int kPipeTile = 256 * kPipeU;  // records per tile
constexpr int kPipeMaxG = 1024;          // groups per pass
// table bytes per group: T3 rows of an i group, B rows of a j group (the j
// groups are also the first level of the score accumulation, whose
// per-group split wants a few hundred of them)
constexpr int64_t kPipeSliceT3 = 1 << 20;
constexpr int64_t kPipeSliceB = 1 << 18;

struct PipeR1 {
  uint64_t u3;  // Philox word 3 (slot and coin of the k' draw)
  uint32_t i;
  uint32_t js;  // j | sign(a_ki b_kj) << 31
};

struct PipeR2 {
  uint32_t i;
  uint32_t js;  // j | sign(a_ki b_kj a_k'i) << 31
  uint32_t kp;
};

// group shifts: rows per group a power of two with about kPipeSliceBytes
// of table rows, and at most kPipeMaxG groups
static int pipe_shift(int64_t rows, int64_t row_bytes, int64_t slice) {
  int sh = 0;
  while (sh < 31 && ((int64_t(2) << sh) * row_bytes <= slice)) ++sh;
  while (((rows + (int64_t(1) << sh) - 1) >> sh) > kPipeMaxG) ++sh;
  return sh;
}

struct PipeShape {
  int gsh_i = 0, gsh_j = 0;
  int64_t Gi = 1, Gj = 1;
};

static PipeShape pipe_shape(const DenseTables& t) {
  PipeShape p;
  p.gsh_i = pipe_shift(t.m, (int64_t)8 << t.T3.L, kPipeSliceT3);
  p.gsh_j = pipe_shift(t.n, 4 * t.d, kPipeSliceB);
  p.Gi = (t.m + (int64_t(1) << p.gsh_i) - 1) >> p.gsh_i;
  p.Gj = (t.n + (int64_t(1) << p.gsh_j) - 1) >> p.gsh_j;
  return p;
}

// exclusive prefix of c[0 .. G) in place (G <= kPipeMaxG, 256 threads, 4
// per thread); returns nothing, c[g] becomes the start of group g
__device__ __forceinline__ void pipe_block_scan(uint32_t* c, int G,
                                                uint32_t* wt) {
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  uint32_t v[4], sum = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int g = t * 4 + q;
    v[q] = g < G ? c[g] : 0u;
    sum += v[q];
  }
  const uint32_t inc = wave_incl_scan(sum);
  if (lane == 63) wt[wv] = inc;
  __syncthreads();
  uint32_t ex = inc - sum;
  for (int w = 0; w < wv; ++w) ex += wt[w];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int g = t * 4 + q;
    if (g < G) c[g] = ex;
    ex += v[q];
  }
  __syncthreads();
}

// tile index of a workgroup's q-th step: each XCD (blockIdx % 8) walks a
// contiguous eighth of the tiles
struct XcdWalk {
  int64_t t, t_hi, step;
  __device__ XcdWalk(int64_t ntiles) {
    const int64_t xcd = blockIdx.x & 7;
    t = xcd * ntiles / 8 + (blockIdx.x >> 3);
    t_hi = (xcd + 1) * ntiles / 8;
    step = gridDim.x >> 3;
  }
};

// pass A: draws of k, i, j in k order; R1 tiles sorted by the group of i,
// counts cnt[tile * G + g]
__global__ __launch_bounds__(256) void k_pipe_ij(DenseSampleArgs a,
                                                 const double* wtot,
                                                 const uint32_t* ell,
                                                 int64_t ntiles, int gsh,
                                                 int G, PipeR1* out,
                                                 uint32_t* cnt) {
  __shared__ uint64_t t0s[kOrderMaxD];
  __shared__ PipeR1 srec[kPipeTile];
  __shared__ uint32_t gc[kPipeMaxG];
  __shared__ uint32_t wt[4];
  // ||W||_1 = 0: nothing can be drawn; records carry i = j = 0 (in range)
  // and the last pass writes no pair
  const bool live_w = wtot[0] > 0.0;
  const int N0 = 1 << a.L0;
  for (int e = threadIdx.x; e < N0; e += 256) t0s[e] = a.T0[e];
  for (XcdWalk w(ntiles); w.t < w.t_hi; w.t += w.step) {
    for (int g = threadIdx.x; g < G; g += 256) gc[g] = 0;
    __syncthreads();
    const int64_t base = w.t * kPipeTile;
    PipeR1 rec[kPipeU];
    uint32_t grp[kPipeU], rank[kPipeU];
    uint64_t U1[kPipeU], U2[kPipeU];
    uint32_t kk[kPipeU];
#pragma unroll
    for (int u = 0; u < kPipeU; ++u) {
      const int64_t e = base + u * 256 + threadIdx.x;
      const int64_t ec = e < a.count ? e : 0;
      const uint64_t l = (uint64_t)(a.l0 + (int64_t)ell[ec]);
      const Philox4 r = philox4x64_10(l, a.qid, 0ull, 0ull, a.seed, 0ull);
      const uint32_t s0 = slot_of(r.w0, a.L0);
      kk[u] = draw_entry(t0s[s0], s0, r.w0).pos;
      U1[u] = r.w1;
      U2[u] = r.w2;
      rec[u].u3 = r.w3;
    }
    uint64_t e1[kPipeU], e2[kPipeU];
#pragma unroll
    for (int u = 0; u < kPipeU; ++u) {
      e1[u] = a.T1[((uint64_t)kk[u] << a.L1) + slot_of(U1[u], a.L1)];
      e2[u] = a.T2[((uint64_t)kk[u] << a.L2) + slot_of(U2[u], a.L2)];
    }
#pragma unroll
    for (int u = 0; u < kPipeU; ++u) {
      const int64_t e = base + u * 256 + threadIdx.x;
      Drawn di = draw_entry(e1[u], slot_of(U1[u], a.L1), U1[u]);
      Drawn dj = draw_entry(e2[u], slot_of(U2[u], a.L2), U2[u]);
      if (!live_w) di.pos = dj.pos = 0;
      rec[u].i = di.pos;
      rec[u].js = dj.pos | ((di.sgn ^ dj.sgn) << 31);
      grp[u] = di.pos >> gsh;
      rank[u] = e < a.count ? atomicAdd(&gc[grp[u]], 1u) : 0u;
    }
    __syncthreads();
    for (int g = threadIdx.x; g < G; g += 256)
      cnt[w.t * G + g] = gc[g];
    __syncthreads();
    pipe_block_scan(gc, G, wt);
#pragma unroll
    for (int u = 0; u < kPipeU; ++u) {
      const int64_t e = base + u * 256 + threadIdx.x;
      if (e < a.count) srec[gc[grp[u]] + rank[u]] = rec[u];
    }
    __syncthreads();
    const int64_t n = a.count - base < kPipeTile ? a.count - base : kPipeTile;
    for (int p = threadIdx.x; p < n; p += 256) out[base + p] = srec[p];
    __syncthreads();
  }
}

// pass B: k' from T3[i] over the i-grouped stream; R2 tiles sorted by the
// group of j
__global__ __launch_bounds__(256) void k_pipe_kp(const uint64_t* T3, int L3,
                                                 const double* wtot,
                                                 const PipeR1* in,
                                                 int64_t count, int64_t ntiles,
                                                 int gsh, int G, PipeR2* out,
                                                 uint32_t* cnt) {
  __shared__ PipeR2 srec[kPipeTile];
  __shared__ uint32_t gc[kPipeMaxG];
  __shared__ uint32_t wt[4];
  const bool live_w = wtot[0] > 0.0;
  for (XcdWalk w(ntiles); w.t < w.t_hi; w.t += w.step) {
    for (int g = threadIdx.x; g < G; g += 256) gc[g] = 0;
    __syncthreads();
    const int64_t base = w.t * kPipeTile;
    PipeR1 r1[kPipeU];
#pragma unroll
    for (int u = 0; u < kPipeU; ++u) {
      const int64_t e = base + u * 256 + threadIdx.x;
      r1[u] = in[e < count ? e : 0];
    }
    uint64_t e3[kPipeU];
#pragma unroll
    for (int u = 0; u < kPipeU; ++u)
      e3[u] = T3[((uint64_t)r1[u].i << L3) + slot_of(r1[u].u3, L3)];
    PipeR2 rec[kPipeU];
    uint32_t grp[kPipeU], rank[kPipeU];
#pragma unroll
    for (int u = 0; u < kPipeU; ++u) {
      const int64_t e = base + u * 256 + threadIdx.x;
      const Drawn dk = draw_entry(e3[u], slot_of(r1[u].u3, L3), r1[u].u3);
      rec[u].i = r1[u].i;
      rec[u].js = r1[u].js ^ (dk.sgn << 31);
      rec[u].kp = live_w ? dk.pos : 0u;
      grp[u] = (r1[u].js & kLow31) >> gsh;
      rank[u] = e < count ? atomicAdd(&gc[grp[u]], 1u) : 0u;
    }
    __syncthreads();
    for (int g = threadIdx.x; g < G; g += 256)
      cnt[w.t * G + g] = gc[g];
    __syncthreads();
    pipe_block_scan(gc, G, wt);
#pragma unroll
    for (int u = 0; u < kPipeU; ++u) {
      const int64_t e = base + u * 256 + threadIdx.x;
      if (e < count) srec[gc[grp[u]] + rank[u]] = rec[u];
    }
    __syncthreads();
    const int64_t n = count - base < kPipeTile ? count - base : kPipeTile;
    for (int p = threadIdx.x; p < n; p += 256) out[base + p] = srec[p];
    __syncthreads();
  }
}

__device__ __forceinline__ uint32_t pipe_group(const PipeR1& r, int gsh) {
  return r.i >> gsh;
}
__device__ __forceinline__ uint32_t pipe_group(const PipeR2& r, int gsh) {
  return (r.js & kLow31) >> gsh;
}

// the runs of each tile (sorted by group) to their places in the grouped
// stream: run (g, tile) starts at start[g] + pre[tile * G + g], where pre
// is the column prefix of the tile counts
template <typename R>
__global__ __launch_bounds__(256) void k_pipe_scatter(
    const R* in, int64_t count, int gsh, int G, const uint32_t* pre,
    const uint32_t* start, R* out) {
  __shared__ uint16_t sg[kPipeTile];
  __shared__ uint32_t first[kPipeMaxG];
  const int64_t tile = blockIdx.x;
  const int64_t base = tile * kPipeTile;
  const int n = count - base < kPipeTile ? (int)(count - base) : kPipeTile;
  R rec[kPipeU];
  uint32_t grp[kPipeU];
#pragma unroll
  for (int u = 0; u < kPipeU; ++u) {
    const int p = u * 256 + threadIdx.x;
    if (p < n) {
      rec[u] = in[base + p];
      grp[u] = pipe_group(rec[u], gsh);
      sg[p] = (uint16_t)grp[u];
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < kPipeU; ++u) {
    const int p = u * 256 + threadIdx.x;
    if (p < n && (p == 0 || sg[p - 1] != grp[u])) first[grp[u]] = (uint32_t)p;
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < kPipeU; ++u) {
    const int p = u * 256 + threadIdx.x;
    if (p < n) {
      const uint32_t g = grp[u];
      const uint64_t d = (uint64_t)start[g] + pre[tile * G + g] +
                         (uint32_t)p - first[g];
      out[d] = rec[u];
    }
  }
}

// pass C: the fourth edge over the j-grouped stream and each sample's pair
__global__ __launch_bounds__(256) void k_pipe_edge(const PipeR2* in,
                                                   int64_t count,
                                                   int64_t ntiles,
                                                   const float* B, int64_t d,
                                                   int64_t n, int gram,
                                                   const double* wtot,
                                                   const uint32_t* bbits,
                                                   const int* bbin,
                                                   uint64_t* pkeys,
                                                   float* pvals,
                                                   SampleCounters* ctr) {
  const bool live_w = wtot[0] > 0.0;
  const bool binB = bbin && *bbin == 1;
  unsigned long long nclosed = 0;
  for (XcdWalk w(ntiles); w.t < w.t_hi; w.t += w.step) {
    const int64_t base = w.t * kPipeTile;
    PipeR2 r[kPipeU];
#pragma unroll
    for (int u = 0; u < kPipeU; ++u) {
      const int64_t e = base + u * 256 + threadIdx.x;
      r[u] = in[e < count ? e : 0];
    }
    float v[kPipeU];
#pragma unroll
    for (int u = 0; u < kPipeU; ++u)
      v[u] = fourth_edge(B, bbits, binB, d, r[u].js & kLow31, r[u].kp);
#pragma unroll
    for (int u = 0; u < kPipeU; ++u) {
      const int64_t e = base + u * 256 + threadIdx.x;
      if (e >= count) continue;
      uint64_t ii = r[u].i, jj = r[u].js & kLow31;
      const bool closed = live_w && v[u] != 0.0f;
      bool ins = closed;
      if (gram) {  // Sec. 3.2.2: X + X^T on i < j, diagonal dropped
        if (ii == jj) ins = false;
        if (ii > jj) {
          const uint64_t tmp = ii;
          ii = jj;
          jj = tmp;
        }
      }
      nclosed += closed;
      __builtin_nontemporal_store(
          (unsigned long long)(ins ? ii * (uint64_t)n + jj : kEmptyKey),
          (unsigned long long*)(pkeys + e));
      __builtin_nontemporal_store((r[u].js >> 31) ? -v[u] : v[u], pvals + e);
    }
  }
  __shared__ unsigned long long part[4];
  nclosed = wave_sum(nclosed);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = nclosed;
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned long long c = part[0] + part[1] + part[2] + part[3];
    if (c) atomicAdd(&ctr->closed, c);
  }
}

// first-level bins of the score accumulation: the j groups' starts as
// 64-bit offsets, starts[G] = count
__global__ void k_pipe_starts64(const uint32_t* start, int G, int64_t count,
                                uint64_t* out) {
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g < G) out[g] = start[g];
  if (g == G) out[g] = (uint64_t)count;
}

// workspace of the pipeline passes for a chunk of c samples
struct PipeLayout {
  PipeR1* ra;      // tile-major records of pass A, then of pass B
  PipeR1* rb;      // the i-grouped stream, then the j-grouped one
  uint32_t *ca, *ta, *sa;  // pass A: tile counts, group totals, starts
  uint32_t *cb, *tb, *sb;  // pass B
  uint64_t* starts64;      // first-level bins of the accumulation
  size_t bytes;
};

static size_t align256(size_t b) { return (b + 255) / 256 * 256; }

static PipeLayout pipe_layout(char* base, int64_t c, const PipeShape& ps) {
  PipeLayout L;
  const int64_t nt = (c + kPipeTile - 1) / kPipeTile;
  char* p = base;
  L.ra = (PipeR1*)p; p += align256((size_t)c * sizeof(PipeR1));
  L.rb = (PipeR1*)p; p += align256((size_t)c * sizeof(PipeR1));
  L.ca = (uint32_t*)p; p += align256((size_t)nt * ps.Gi * 4);
  L.ta = (uint32_t*)p; p += align256((size_t)ps.Gi * 4);
  L.sa = (uint32_t*)p; p += align256((size_t)ps.Gi * 4);
  L.cb = (uint32_t*)p; p += align256((size_t)nt * ps.Gj * 4);
  L.tb = (uint32_t*)p; p += align256((size_t)ps.Gj * 4);
  L.sb = (uint32_t*)p; p += align256((size_t)ps.Gj * 4);
  L.starts64 = (uint64_t*)p; p += align256((size_t)(ps.Gj + 1) * 8);
  L.bytes = (size_t)(p - base);
  return L;
}

static size_t korder_bytes(int64_t c, int64_t d) {
  const int64_t nblk = (c + kOrdPer - 1) / kOrdPer;
  return align256((size_t)c * 4) + align256((size_t)c * 2) +
         (size_t)nblk * d * 4 + (size_t)d * 8 + 2048;
}

size_t sample_order_bytes(const DenseTables& t, int64_t count,
                          const SampleOptions& o) {
  if (t.d > kOrderMaxD || o.order == 0) return 0;
  const int64_t c = count < o.chunk ? count : o.chunk;
  size_t b = align256(korder_bytes(c, t.d));
  if (o.order == 2) b += pipe_layout(nullptr, c, pipe_shape(t)).bytes;
  return b;
}

// Samples run in k order by default for d <= kOrderMaxD: one sampling
// kernel whose T1[k], T2[k] rows stay in the XCD's L2 (on dense 1e5 x 1e5
// x 100 with s = 1e7 it takes the kernel from 0.75 to 0.50 ms for 0.1 ms of
// ordering passes).  Order 2, the three passes grouped by k, i and j,
// moves 216 instead of 348 bytes per sample there but takes longer: HBM
// serves random 128-byte lines nearly at its streaming rate, so the
// records, scans and scatters of the grouping cost more than the random
// lines they save.  Order 0 draws in index order.  The process default
// comes from MAD_SAMPLER_ORDER; a plan can change it (mad_plan_set_option).
// MAD_SAMPLER_G8 and MAD_PIPE_G8 set workgroups per XCD.  None changes a
// result.
SampleOptions sample_options_default() {
  static const SampleOptions v = [] {
    SampleOptions o;
    const char* e = getenv("MAD_SAMPLER_ORDER");
    o.order = e ? atoi(e) : 1;
    if (o.order < 0 || o.order > 2) o.order = 1;
    return o;
  }();
  return v;
}

bool sample_options_valid(const SampleOptions& o) {
  return o.order >= 0 && o.order <= 2 && o.chunk >= kOrderChunkMin &&
         o.chunk <= kOrderChunkMax && (o.chunk & (o.chunk - 1)) == 0;
}

// workgroups per XCD of the pipeline passes (MAD_PIPE_G8, 8 .. 1024;
// result-invariant)
static int pipe_g8() {
  static int v = [] {
    const char* e = getenv("MAD_PIPE_G8");
    const int x = e ? atoi(e) : 96;
    return x >= 8 && x <= 1024 ? x : 96;
  }();
  return v;
}

static int order_g8() {
  static int v = [] {
    const char* e = getenv("MAD_SAMPLER_G8");
    const int x = e ? atoi(e) : 32;
    return x >= 1 && x <= 4096 ? x : 32;
  }();
  return v;
}

hipError_t launch_sample_dense(const DenseTables& t, const float* B,
                               uint64_t seed, uint64_t qid, int64_t l0,
                               int64_t count, int64_t s_for_F, HashTable h,
                               SampleCounters* ctr, void* order_ws,
                               size_t order_bytes, const SampleOptions& o,
                               PairGroups* groups, hipEvent_t main_start,
                               hipStream_t st) {
  if (groups) *groups = PairGroups{};
  if (count <= 0) return hipSuccess;
  const size_t lds = t0_lds_bytes(t);
  const uint64_t hm = (uint64_t)h.cap - 1;
  const int64_t chunk = o.chunk;
  const bool ordered = o.order >= 1 && t.d <= kOrderMaxD && order_ws &&
                       order_bytes >= sample_order_bytes(t, count, o) &&
                       (int64_t(1) << t.T0.L) <= kT0Lds;
  // the pipeline writes one pair per sample, so it needs the pair form of
  // X and not the squared variant
  const bool pipe = ordered && o.order == 2 && h.pkeys != nullptr &&
                    !t.square;
  if (!ordered) {
    if (main_start) (void)hipEventRecord(main_start, st);
    DenseSampleArgs a = dense_args(t, B, seed, qid, l0, count);
    a.pk2 = h.pkeys2;
    a.pv2 = h.pvals2;
    switch (sampler_unroll()) {
#define MAD_SAMPLE_CASE(UU)                                                \
  case UU:                                                                 \
    k_sample_dense<UU, false, false>                                       \
        <<<sample_grid(count, UU), 256, lds, st>>>(                        \
            a, t.T0.tot, t.bmax, s_for_F, 0, h.keys, h.vals, hm, h.pkeys,  \
            h.pvals, ctr, nullptr, nullptr, nullptr, nullptr, nullptr,     \
            GroupOrder{});                                                 \
    break;
      MAD_SAMPLE_CASE(1)
      MAD_SAMPLE_CASE(2)
      MAD_SAMPLE_CASE(8)
      default:
      MAD_SAMPLE_CASE(4)
#undef MAD_SAMPLE_CASE
    }
    return hipGetLastError();
  }
  // ordered: chunks of at most `chunk` samples
  const int64_t d = t.d;
  const size_t lds_ord = ((size_t)8 << t.T0.L) + 4 * (size_t)d;
  const PipeShape ps = pipe_shape(t);
  for (int64_t c0 = 0; c0 < count; c0 += chunk) {
    const int64_t c = count - c0 < chunk ? count - c0 : chunk;
    DenseSampleArgs a = dense_args(t, B, seed, qid, l0 + c0, c);
    a.pk2 = h.pkeys2 ? h.pkeys2 + c0 : nullptr;
    a.pv2 = h.pvals2 ? h.pvals2 + c0 : nullptr;
    const int64_t nblk = (c + kOrdPer - 1) / kOrdPer;
    char* p = (char*)order_ws;
    uint32_t* ell = (uint32_t*)p;
    uint16_t* kbuf = (uint16_t*)(p + align256((size_t)c * 4));
    uint32_t* cnt = (uint32_t*)((char*)kbuf + align256((size_t)c * 2));
    uint32_t* tot = cnt + nblk * d;
    uint32_t* start = tot + d;
    // the first chunk's order needs only T0: when the build put T0 on the
    // aux stream, the order passes follow it there, beside the rest of the
    // table build, once the previous launch has sampled from the buffers
    const bool on_aux = t.t0_aux && c0 == 0;
    hipStream_t os = on_aux ? t.aux : st;
    if (on_aux) {
      const hipError_t ew = hipStreamWaitEvent(t.aux, t.sampled, 0);
      if (ew != hipSuccess) return ew;
    }
    k_order_count<<<(unsigned)nblk, 256, lds_ord, os>>>(a, cnt, kbuf);
    k_order_colscan<<<(unsigned)d, 256, 0, os>>>(cnt, nblk, d, tot);
    k_order_starts<<<1, 256, 0, os>>>(tot, d, start);
    const size_t lds_place = 8 * (size_t)d + 6 * (size_t)kOrdPer;
    k_order_place<<<(unsigned)nblk, 256, lds_place, os>>>(a, cnt, start, kbuf,
                                                         ell);
    if (on_aux) {
      hipError_t ew = hipEventRecord(t.order_done, t.aux);
      if (ew == hipSuccess) ew = hipStreamWaitEvent(st, t.order_done, 0);
      if (ew != hipSuccess) return ew;
    }
    if (main_start && c0 == 0) (void)hipEventRecord(main_start, st);
    int64_t g8 = order_g8();
    if (pipe) {
      const PipeLayout L =
          pipe_layout((char*)order_ws + align256(korder_bytes(c, d)), c, ps);
      const int64_t nt = (c + kPipeTile - 1) / kPipeTile;
      int64_t gp = pipe_g8();
      if (gp * 8 > nt) gp = (nt + 7) / 8;
      if (gp < 1) gp = 1;
      const unsigned grid = (unsigned)(8 * gp);
      const int Gi = (int)ps.Gi, Gj = (int)ps.Gj;
      // pass A, then the i-grouped stream
      k_pipe_ij<<<grid, 256, 0, st>>>(a, t.T0.tot, ell, nt, ps.gsh_i, Gi,
                                      L.ra, L.ca);
      k_order_colscan<<<(unsigned)Gi, 256, 0, st>>>(L.ca, nt, Gi, L.ta);
      k_order_starts<<<1, 256, 0, st>>>(L.ta, Gi, L.sa);
      k_pipe_scatter<PipeR1><<<(unsigned)nt, 256, 0, st>>>(
          L.ra, c, ps.gsh_i, Gi, L.ca, L.sa, L.rb);
      // pass B, then the j-grouped stream
      PipeR2* r2t = (PipeR2*)L.ra;
      PipeR2* r2s = (PipeR2*)L.rb;
      k_pipe_kp<<<grid, 256, 0, st>>>(t.T3.ent, t.T3.L, t.T0.tot, L.rb, c, nt,
                                      ps.gsh_j, Gj, r2t, L.cb);
      k_order_colscan<<<(unsigned)Gj, 256, 0, st>>>(L.cb, nt, Gj, L.tb);
      k_order_starts<<<1, 256, 0, st>>>(L.tb, Gj, L.sb);
      k_pipe_scatter<PipeR2><<<(unsigned)nt, 256, 0, st>>>(
          r2t, c, ps.gsh_j, Gj, L.cb, L.sb, r2s);
      // pass C: the pairs, in j-grouped order
      k_pipe_edge<<<grid, 256, 0, st>>>(r2s, c, nt, B, d, t.n, t.gram,
                                        t.T0.tot, a.bbits, a.bbin,
                                        h.pkeys + c0, h.pvals + c0, ctr);
      if (groups && c == count && !t.gram) {
        k_pipe_starts64<<<(unsigned)((Gj + 256) / 256), 256, 0, st>>>(
            L.sb, Gj, c, L.starts64);
        groups->starts = L.starts64;
        groups->G = Gj;
      }
    } else {
      GroupOrder go{ell, 256 * 4};
      const int64_t nch = (c + go.chunk - 1) / go.chunk;
      if (g8 * 8 > nch) g8 = (nch + 7) / 8;
      if (g8 < 1) g8 = 1;
      k_sample_dense<4, false, true><<<(unsigned)(8 * g8), 256, lds, st>>>(
          a, t.T0.tot, t.bmax, s_for_F, 0, h.keys, h.vals, hm,
          h.pkeys ? h.pkeys + c0 : nullptr, h.pvals ? h.pvals + c0 : nullptr,
          ctr, nullptr, nullptr, nullptr, nullptr, nullptr, go);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  // the order buffers are free again once this launch's samplers are done
  return t.t0_aux ? hipEventRecord(t.sampled, st) : hipSuccess;
}

hipError_t launch_sample_dense_debug(const DenseTables& t, const float* B,
                                     uint64_t seed, uint64_t qid, int64_t l0,
                                     int64_t count, int F, int32_t* k,
                                     int32_t* i, int32_t* j, int32_t* kp,
                                     int64_t* inc, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  const DenseSampleArgs a = dense_args(t, B, seed, qid, l0, count);
  k_sample_dense<2, true, false>
      <<<sample_grid(count, 2), 256, t0_lds_bytes(t), st>>>(
      a, t.T0.tot, t.bmax, 0, F, nullptr, nullptr, 0, nullptr, nullptr, nullptr,
      k, i, j, kp, inc, GroupOrder{});
  return hipGetLastError();
}

}  // namespace mad
