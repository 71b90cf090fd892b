// select.hip -- Alg. 2 postprocessing on the GPU.
//
//   candidate selection  Omega_s = pairs with x_ij > 0; Omega_t' = the t'
//                        largest by x, ties by key (i*n + j) ascending;
//   verification         c_ij = a_i . b_j in fp32 for each candidate;
//   final selection      Omega_t = the t largest by |c|, ties by key
//                        ascending, written in that order.
//
// Each selection of k elements by (primary descending, key ascending) runs
// in three steps, with every count kept in device memory:
//   1. while the elements are produced (the score table scan for candidate selection, the
//      verification kernel for final selection) a 2048-bin histogram of a monotone
//      "float" digit of the primary (its highest set bit and the 5 bits
//      below it) is accumulated;
//   2. one pass splits the elements: bins above the bin that holds the k-th
//      element are taken outright, that bin's elements go to a boundary list;
//   3. one workgroup selects exactly the remaining count from the boundary
//      list with 11-bit radix passes over the primary and then the key.
// A boundary list of more than kRefineMin elements first gets one such
// radix pass on the whole grid (histogram, decision, split), so that step 3
// reads one digit's bin of it.
#include "mad_common.hpp"
#include "plan.hpp"

namespace mad {

constexpr int kBins = 2048;
constexpr int kDigit = 11;
constexpr uint64_t kDigitMask = kBins - 1;

// SelectWork::counts slots
enum {
  kCntPos = kCountPos,           // |Omega_s|
  kCntDistinct = kCountDistinct, // nnz(X) (filled by the sampler)
  kCntCand = kCountCand,         // |Omega_t'|
  kCntFinal = kCountFinal,       // |Omega_t|
  kCntBound = 4,                 // boundary list length
  kCntWin = 5,                   // elements taken outright
  kCntPreFilter = 7,             // |Omega_t'| before the low-precision filter
  kCntReranked = 8               // candidates left for fp32 verification
};

// coarse decision of one selection
struct Coarse {
  int64_t n;      // elements
  int64_t k;      // to select
  int64_t k_rem;  // still to select inside the boundary bin
  int64_t bin;    // boundary bin (-1: take everything)
};

// candidate selection boundary refinement: one full-grid radix pass over a long boundary
// list (ties of x leave millions of elements in one coarse bin), so that the
// single-workgroup step 3 starts from one digit's bin of it
struct Refine {
  uint64_t mask, prefix;           // the chosen digit's bin and bits above
  int64_t key_phase;               // 1: the digit is one of the key's
  int64_t active;                  // refined list in use
  unsigned long long nout;         // refined list length
  int64_t pad[3];
};
// select state: three Coarse (candidate selection, final selection,
// low-precision filter), then a Refine for each of the two selections
static_assert(3 * sizeof(Coarse) + 2 * sizeof(Refine) <= kSelStateBytes,
              "select state");
constexpr int kRefineMin = 4096;   // shorter lists go to step 3 as they are
constexpr int kRefineThreads = 1024;
constexpr int kRefineThreadsMax = 1024;
constexpr int64_t kRefineFinalMin = 16384;  // t' above which the final
                                            // selection may refine

static inline unsigned blocks_for(int64_t n, int per_block, int cap) {
  int64_t g = (n + per_block - 1) / per_block;
  if (g > cap) g = cap;
  return (unsigned)(g < 1 ? 1 : g);
}

// monotone 11-bit digit of a positive value: (msb, next 5 bits)
__device__ __forceinline__ int fbin(uint64_t p) {
  if (p == 0) return 0;
  const int msb = 63 - __clzll((long long)p);
  const uint64_t mant = msb >= 5 ? (p >> (msb - 5)) : (p << (5 - msb));
  return msb * 32 + (int)(mant & 31);
}

// monotone 11-bit digit of a non-negative float given as its bits: the
// exponent and the top 3 mantissa bits (1/8-octave bins)
__device__ __forceinline__ int fbin_float(uint64_t bits) {
  return (int)(bits >> 20) & (kBins - 1);
}

__device__ void block_hist_flush(unsigned* lds, unsigned* gh) {
  __syncthreads();
  for (int b = threadIdx.x; b < kBins; b += blockDim.x)
    if (lds[b]) atomicAdd(&gh[b], lds[b]);
}

// ---------------------------------------------------------------------------
// candidate selection step 1: histogram of x > 0 straight from the score table (the
// number of positive scores is the histogram's total)
// ---------------------------------------------------------------------------
// The grid is small (kHistBlocks workgroups of 1024 threads): every block
// ends with one global atomic per non-empty bin, and the few bins that hold
// most scores would serialise one atomic per block.
constexpr int kHistBlocks = 256;
constexpr int kHistThreads = 1024;

__global__ __launch_bounds__(kHistThreads) void k_score_hist(
    const int64_t* hvals, int64_t cap, const int64_t* live, unsigned* hist) {
  __shared__ unsigned h[kBins];
  for (int b = threadIdx.x; b < kBins; b += blockDim.x) h[b] = 0;
  __syncthreads();
  if (live && *live < cap) cap = *live;
  constexpr int kU = 4;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x * kU;
  for (int64_t e0 = (int64_t)blockIdx.x * blockDim.x * kU + threadIdx.x;
       e0 < cap; e0 += stride) {
    int64_t v[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int64_t e = e0 + (int64_t)u * blockDim.x;
      v[u] = e < cap ? hvals[e] : 0;
    }
#pragma unroll
    for (int u = 0; u < kU; ++u)
      if (v[u] > 0) atomicAdd(&h[fbin((uint64_t)v[u])], 1u);
  }
  block_hist_flush(h, hist);
}

// step 2a (one block): the boundary bin from the histogram, then clear it.
// The element count is *n_ptr, or the histogram's total when n_ptr is
// null; n_store (if set) receives it.
__global__ __launch_bounds__(256) void k_coarse_decide(
    unsigned* hist, const int64_t* n_ptr, int64_t k, Coarse* out,
    int64_t* n_store, Refine* rf = nullptr) {
  __shared__ unsigned long long wsum[4];
  __shared__ int chosen;
  __shared__ unsigned long long before;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  if (t == 0) chosen = -1;
  // thread t owns 8 consecutive bins in descending order
  unsigned v[8];
  unsigned long long sum = 0;
  for (int q = 0; q < 8; ++q) {
    v[q] = hist[kBins - 1 - (t * 8 + q)];
    sum += v[q];
  }
  const unsigned long long winc = wave_incl_scan(sum);
  if (lane == 63) wsum[wv] = winc;
  __syncthreads();
  unsigned long long woff = 0, total = 0;
  for (int w = 0; w < 4; ++w) {
    woff += w < wv ? wsum[w] : 0ull;
    total += wsum[w];
  }
  const int64_t n = n_ptr ? *n_ptr : (int64_t)total;
  if (n > k) {
    unsigned long long acc = woff + winc - sum;
    for (int q = 0; q < 8; ++q) {
      if ((long long)acc < k && (long long)(acc + v[q]) >= k) {
        chosen = kBins - 1 - (t * 8 + q);
        before = acc;
      }
      acc += v[q];
    }
  }
  __syncthreads();
  for (int b = t; b < kBins; b += 256) hist[b] = 0;  // ready for reuse
  if (t == 0) {
    if (rf) {
      rf->active = 0;
      rf->nout = 0ull;
    }
    if (n_store) *n_store = n;
    out->n = n;
    out->k = k;
    if (n <= k || chosen < 0) {
      out->bin = -1;
      out->k_rem = 0;
    } else {
      out->bin = chosen;
      out->k_rem = k - (int64_t)before;
    }
  }
}

// block-aggregated append (256 threads): this thread's slot when take
__device__ __forceinline__ int64_t block_append(bool take,
                                                unsigned long long* ctr,
                                                unsigned* wcount,
                                                unsigned long long* wbase) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const uint64_t ball = __ballot(take);
  if (lane == 0) wcount[wv] = (unsigned)__popcll(ball);
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long tot = 0;
    for (int w = 0; w < 4; ++w) {
      const unsigned c = wcount[w];
      wbase[w] = tot;
      tot += c;
    }
    wbase[4] = tot ? atomicAdd(ctr, tot) : 0ull;
  }
  __syncthreads();
  const int64_t slot = (int64_t)(wbase[4] + wbase[wv] +
                                 __popcll(ball & ((1ull << lane) - 1)));
  __syncthreads();
  return slot;
}

// and / or of a block's boundary elements (256 threads, all of them) into
// its own slot part[4 * blockIdx.x ..]: no atomics (a few hundred blocks
// on the same four words would serialise); the refinement kernels reduce
// the slots when they run
__device__ void block_and_or(uint64_t xa, uint64_t xo, uint64_t ka,
                             uint64_t ko, unsigned long long (*red)[4],
                             uint64_t* part) {
  const int t = threadIdx.x;
  for (int off = 32; off > 0; off >>= 1) {
    xa &= __shfl_xor(xa, off, 64);
    xo |= __shfl_xor(xo, off, 64);
    ka &= __shfl_xor(ka, off, 64);
    ko |= __shfl_xor(ko, off, 64);
  }
  const int wv = t >> 6;
  if ((t & 63) == 0) {
    red[0][wv] = xa;
    red[1][wv] = xo;
    red[2][wv] = ka;
    red[3][wv] = ko;
  }
  __syncthreads();
  if (t == 0) {
    for (int w = 1; w < 4; ++w) {
      xa &= red[0][w];
      xo |= red[1][w];
      ka &= red[2][w];
      ko |= red[3][w];
    }
    uint64_t* o = part + 4 * (int64_t)blockIdx.x;
    o[0] = xa;
    o[1] = xo;
    o[2] = ka;
    o[3] = ko;
  }
}

// ---------------------------------------------------------------------------
// candidate selection step 2b: split the score table (winners -> w*, boundary -> b*).
// Each block stages its finds in LDS and reserves output space once per
// flush: one global atomic per list and flush, not per wave or element.
// ---------------------------------------------------------------------------
constexpr int kSplitU = 4;       // elements per thread and step
constexpr int kStage = 2048;     // staged entries per list

__global__ __launch_bounds__(256) void k_score_split(
    const uint64_t* hkeys, const int64_t* hvals, int64_t cap,
    const int64_t* live, const Coarse* cz, uint64_t* wx, uint64_t* wkey,
    int64_t wcap, uint64_t* bx, uint64_t* bkey, int64_t bcap,
    int64_t* counts, uint64_t* part) {
  __shared__ unsigned long long sx[2][kStage];
  __shared__ unsigned long long sk[2][kStage];
  __shared__ unsigned scnt[2];
  __shared__ unsigned long long gbase[2];
  __shared__ unsigned long long red[4][4];
  uint64_t xa = ~0ull, xo = 0ull, ka = ~0ull, ko = 0ull;
  const Coarse c = *cz;
  if (live && *live < cap) cap = *live;
  const int t = threadIdx.x;
  if (t == 0) scnt[0] = scnt[1] = 0;
  __syncthreads();
  uint64_t* ox[2] = {wx, bx};
  uint64_t* ok[2] = {wkey, bkey};
  const int64_t ocap[2] = {wcap, bcap};
  const int64_t step = 256 * kSplitU;
  const int64_t stride = (int64_t)gridDim.x * step;
  for (int64_t b0 = (int64_t)blockIdx.x * step; b0 < cap + stride;
       b0 += stride) {
    const bool last = b0 >= cap;  // one extra (uniform) round to flush
    if (!last) {
      int64_t v[kSplitU];
#pragma unroll
      for (int u = 0; u < kSplitU; ++u) {
        const int64_t e = b0 + t + (int64_t)u * 256;
        v[u] = e < cap ? hvals[e] : 0;
      }
#pragma unroll
      for (int u = 0; u < kSplitU; ++u) {
        if (v[u] <= 0) continue;
        const int bin = fbin((uint64_t)v[u]);
        const int L = (c.bin < 0 || bin > c.bin) ? 0 : (bin == c.bin ? 1 : -1);
        if (L < 0) continue;
        const unsigned p = atomicAdd(&scnt[L], 1u);
        const uint64_t kk = hkeys[b0 + t + (int64_t)u * 256];
        sx[L][p] = (unsigned long long)v[u];
        sk[L][p] = kk;
        if (L) {
          xa &= (uint64_t)v[u];
          xo |= (uint64_t)v[u];
          ka &= kk;
          ko |= kk;
        }
      }
    }
    __syncthreads();
    const unsigned n0 = scnt[0], n1 = scnt[1];
    if (last || n0 > kStage - step || n1 > kStage - step) {
      if (t < 2) {
        const unsigned nl = t ? n1 : n0;
        gbase[t] = nl ? atomicAdd((unsigned long long*)&counts[t ? kCntBound
                                                                 : kCntWin],
                                  (unsigned long long)nl)
                      : 0ull;
      }
      __syncthreads();
      for (int L = 0; L < 2; ++L) {
        const unsigned nl = L ? n1 : n0;
        for (unsigned i = t; i < nl; i += 256) {
          const int64_t d = (int64_t)gbase[L] + i;
          if (d < ocap[L]) {
            ox[L][d] = sx[L][i];
            ok[L][d] = sk[L][i];
          }
        }
      }
      __syncthreads();
      if (t == 0) scnt[0] = scnt[1] = 0;
      __syncthreads();
    }
  }
  block_and_or(xa, xo, ka, ko, red, part);
}

// the refinement digit: the 11 bits below the highest bit in which the
// boundary list's x values differ, or its keys when every x is equal
struct RefineDigit {
  bool key_phase;
  int shift;
  uint64_t above;   // bits above the digit, shared by the whole list
  uint64_t common;  // their value
};

// the digit from the split blocks' and / or slots (every thread of the
// block calls it; blocks without boundary elements hold the identities)
__device__ RefineDigit refine_digit(const uint64_t* part, int nblk) {
  __shared__ unsigned long long r4[4][kRefineThreadsMax / 64];
  uint64_t xa = ~0ull, xo = 0ull, ka = ~0ull, ko = 0ull;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) {
    xa &= part[4 * b];
    xo |= part[4 * b + 1];
    ka &= part[4 * b + 2];
    ko |= part[4 * b + 3];
  }
  for (int off = 32; off > 0; off >>= 1) {
    xa &= __shfl_xor(xa, off, 64);
    xo |= __shfl_xor(xo, off, 64);
    ka &= __shfl_xor(ka, off, 64);
    ko |= __shfl_xor(ko, off, 64);
  }
  const int wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if ((threadIdx.x & 63) == 0) {
    r4[0][wv] = xa;
    r4[1][wv] = xo;
    r4[2][wv] = ka;
    r4[3][wv] = ko;
  }
  __syncthreads();
  for (int w = 0; w < nw; ++w) {
    xa &= r4[0][w];
    xo |= r4[1][w];
    ka &= r4[2][w];
    ko |= r4[3][w];
  }
  RefineDigit g;
  const uint64_t dx = xa ^ xo;
  g.key_phase = dx == 0ull;
  const uint64_t diff = g.key_phase ? (ka ^ ko) : dx;
  const int hd = diff ? 63 - __clzll((long long)diff) : 0;
  g.shift = hd >= kDigit - 1 ? hd - (kDigit - 1) : 0;
  g.above = hd < 63 ? ~0ull << (hd + 1) : 0ull;
  g.common = (g.key_phase ? ka : xa) & g.above;
  return g;
}

// is the boundary list refined: long, and not taken whole
__device__ __forceinline__ bool refine_wanted(const Coarse& c, int64_t nb) {
  return c.bin >= 0 && c.k_rem > 0 && c.k_rem < nb && nb > kRefineMin;
}

// refinement 1/3: histogram of the digit over the boundary list

__global__ __launch_bounds__(kRefineThreads) void k_refine_hist(
    const Coarse* cz, const uint64_t* part, int nblk, const uint64_t* bx,
    const uint64_t* bkey, int64_t bcap, const int64_t* counts,
    unsigned* hist) {
  __shared__ unsigned h[kBins];
  int64_t nb = counts[kCntBound];
  if (nb > bcap) nb = bcap;
  if (!refine_wanted(*cz, nb)) return;
  const RefineDigit g = refine_digit(part, nblk);
  const uint64_t* v = g.key_phase ? bkey : bx;
  for (int b = threadIdx.x; b < kBins; b += kRefineThreads) h[b] = 0;
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * kRefineThreads;
  for (int64_t e = (int64_t)blockIdx.x * kRefineThreads + threadIdx.x;
       e < nb; e += stride)
    atomicAdd(&h[(v[e] >> g.shift) & kDigitMask], 1u);
  block_hist_flush(h, hist);
}

// refinement 2/3 (one block): the bin of the digit that holds the k_rem-th
// element in selection order (x descending, or key ascending); clears the
// histogram
__global__ __launch_bounds__(kRefineThreads) void k_refine_decide(
    Coarse* cz, Refine* rf, const uint64_t* part, int nblk,
    const int64_t* counts, int64_t bcap, int64_t rcap, unsigned* hist) {
  __shared__ unsigned long long wsum[kRefineThreads / 64];
  __shared__ int chosen;
  __shared__ unsigned long long before;
  int64_t nb = counts[kCntBound];
  if (nb > bcap) nb = bcap;
  const Coarse c = *cz;
  if (!refine_wanted(c, nb)) return;
  const RefineDigit g = refine_digit(part, nblk);
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  // thread t owns positions 2t and 2t+1 of the selection order
  const int b0 = g.key_phase ? 2 * t : kBins - 1 - 2 * t;
  const int b1 = g.key_phase ? 2 * t + 1 : kBins - 2 - 2 * t;
  const unsigned v0 = hist[b0], v1 = hist[b1];
  const unsigned long long pair = (unsigned long long)v0 + v1;
  const unsigned long long winc = wave_incl_scan(pair);
  if (lane == 63) wsum[wv] = winc;
  if (t == 0) chosen = -1;
  __syncthreads();
  unsigned long long woff = 0;
  for (int w = 0; w < wv; ++w) woff += wsum[w];
  const unsigned long long excl = woff + winc - pair;
  const int64_t k = c.k_rem;
  if ((int64_t)excl < k && (int64_t)(excl + v0) >= k) {
    chosen = b0;
    before = excl;
  } else if ((int64_t)(excl + v0) < k && (int64_t)(excl + v0 + v1) >= k) {
    chosen = b1;
    before = excl + v0;
  }
  __syncthreads();
  const int b = chosen;
  const unsigned nbin = b >= 0 ? hist[b] : 0u;
  __syncthreads();
  hist[b0] = 0;
  hist[b1] = 0;
  // a bin longer than the refined list's room stays unrefined (step 3 then
  // reads the whole list)
  if (t == 0 && b >= 0 && (int64_t)nbin <= rcap) {
    rf->mask = g.above | (kDigitMask << g.shift);
    rf->prefix = g.common | ((uint64_t)b << g.shift);
    rf->key_phase = g.key_phase ? 1 : 0;
    rf->active = 1;
    cz->k_rem = k - (int64_t)before;
  }
}

// refinement 3/3: elements ordered before the chosen bin join the winners,
// the bin's elements form the refined list (the final selection's lists
// also carry x and c: bextra / bc, when set).  Elements are classified from
// the one column that orders them; each block stages the indices it keeps
// in LDS and reserves output space once per flush (kept elements are rare:
// a global atomic per block and round would serialise on the counters),
// then gathers the kept elements' columns.
constexpr int kRsU = 4;          // elements per thread and round
constexpr int kRsStage = 2048;   // staged indices per list

__global__ __launch_bounds__(256) void k_refine_split(
    const Refine* rf, const uint64_t* bx, const uint64_t* bkey,
    const uint64_t* bextra, const float* bc, int64_t bcap, int64_t* counts,
    uint64_t* wx, uint64_t* wkey, uint64_t* wextra, float* wc, int64_t wcap,
    unsigned long long* nout, uint64_t* rx, uint64_t* rkey, uint64_t* rextra,
    float* rc, int64_t rcap) {
  __shared__ long long sidx[2][kRsStage];
  __shared__ unsigned scnt[2];
  __shared__ unsigned long long gbase[2];
  if (!rf->active) return;
  int64_t nb = counts[kCntBound];
  if (nb > bcap) nb = bcap;
  const uint64_t mask = rf->mask, prefix = rf->prefix;
  const bool kp = rf->key_phase != 0;
  const uint64_t* ord = kp ? bkey : bx;
  const int t = threadIdx.x;
  if (t == 0) scnt[0] = scnt[1] = 0;
  __syncthreads();
  uint64_t* ox[2] = {wx, rx};
  uint64_t* okey[2] = {wkey, rkey};
  uint64_t* oext[2] = {wextra, rextra};
  float* oc[2] = {wc, rc};
  const int64_t ocap[2] = {wcap, rcap};
  unsigned long long* ctr[2] = {(unsigned long long*)&counts[kCntWin], nout};
  const int64_t step = 256 * kRsU;
  const int64_t stride = (int64_t)gridDim.x * step;
  for (int64_t b0 = (int64_t)blockIdx.x * step; b0 < nb + stride;
       b0 += stride) {
    const bool last = b0 >= nb;  // one extra (uniform) round to flush
    if (!last) {
      uint64_t v[kRsU];
#pragma unroll
      for (int u = 0; u < kRsU; ++u) {
        const int64_t e = b0 + t + (int64_t)u * 256;
        v[u] = e < nb ? ord[e] : 0ull;
      }
#pragma unroll
      for (int u = 0; u < kRsU; ++u) {
        const int64_t e = b0 + t + (int64_t)u * 256;
        if (e >= nb) continue;
        const uint64_t m = v[u] & mask;
        const int L = (kp ? m < prefix : m > prefix) ? 0 : (m == prefix ? 1 : -1);
        if (L < 0) continue;
        sidx[L][atomicAdd(&scnt[L], 1u)] = (long long)e;
      }
    }
    __syncthreads();
    const unsigned n0 = scnt[0], n1 = scnt[1];
    if (last || n0 > kRsStage - step || n1 > kRsStage - step) {
      if (t < 2) {
        const unsigned nl = t ? n1 : n0;
        gbase[t] = nl ? atomicAdd(ctr[t], (unsigned long long)nl) : 0ull;
      }
      __syncthreads();
      for (int L = 0; L < 2; ++L) {
        const unsigned nl = L ? n1 : n0;
        for (unsigned i = t; i < nl; i += 256) {
          const int64_t e = (int64_t)sidx[L][i];
          const int64_t d = (int64_t)gbase[L] + i;
          if (d < ocap[L]) {
            ox[L][d] = bx[e];
            okey[L][d] = bkey[e];
            if (bextra) oext[L][d] = bextra[e];
            if (bc) oc[L][d] = bc[e];
          }
        }
      }
      __syncthreads();
      if (t == 0) scnt[0] = scnt[1] = 0;
      __syncthreads();
    }
  }
}

// ---------------------------------------------------------------------------
// step 3: one workgroup selects k_rem of the boundary list exactly, by
// (primary desc, key asc), and appends them after the winners
// ---------------------------------------------------------------------------
constexpr int kFineThreads = 1024;

constexpr int kFineLds = 4096;  // boundary lists up to this size sit in LDS

__global__ __launch_bounds__(kFineThreads) void k_fine_select(
    const Coarse* cz, const uint64_t* bx, const uint64_t* bkey,
    const uint64_t* bextra, const float* bc, int64_t bcap, int64_t* counts,
    int win_slot, uint64_t* ox, uint64_t* okey, uint64_t* oextra, float* oc,
    int64_t ocap, int out_count_slot, const Refine* rf = nullptr,
    const uint64_t* rx = nullptr, const uint64_t* rkey = nullptr,
    const uint64_t* rextra = nullptr, const float* rc = nullptr,
    int64_t rcap = 0) {
  __shared__ unsigned h[kBins];
  __shared__ unsigned long long wsum[kFineThreads / 64];
  __shared__ uint64_t lx[kFineLds], lk[kFineLds];
  __shared__ unsigned long long red_and, red_or;
  __shared__ int chosen;
  __shared__ unsigned long long before;
  __shared__ unsigned long long emitted;
  const Coarse c = *cz;
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int64_t nwin = counts[win_slot] < ocap ? counts[win_slot] : ocap;
  int64_t nb = counts[kCntBound];
  if (nb > bcap) nb = bcap;
  if (rf && rf->active) {  // the refined list
    bx = rx;
    bkey = rkey;
    bextra = rextra;
    bc = rc;
    nb = (int64_t)rf->nout < rcap ? (int64_t)rf->nout : rcap;
  }
  const bool none = c.bin < 0 || c.k_rem <= 0;
  int64_t k_rem = none ? 0 : c.k_rem;
  // the list in LDS when it fits
  const bool in_lds = nb <= kFineLds;
  if (in_lds)
    for (int64_t e = t; e < nb; e += kFineThreads) {
      lx[e] = bx[e];
      lk[e] = bkey[e];
    }
  const uint64_t* X = in_lds ? lx : bx;
  const uint64_t* Kk = in_lds ? lk : bkey;
  // bits shared by every primary value: the radix passes start below them
  if (t == 0) {
    red_and = ~0ull;
    red_or = 0ull;
  }
  __syncthreads();
  {
    uint64_t va = ~0ull, vo = 0ull;
    for (int64_t e = t; e < nb; e += kFineThreads) {
      va &= X[e];
      vo |= X[e];
    }
    for (int off = 32; off > 0; off >>= 1) {
      va &= __shfl_xor(va, off, 64);
      vo |= __shfl_xor(vo, off, 64);
    }
    if (lane == 0 && nb > 0) {
      atomicAnd(&red_and, (unsigned long long)va);
      atomicOr(&red_or, (unsigned long long)vo);
    }
  }
  __syncthreads();
  const uint64_t diff = nb > 0 ? (uint64_t)(red_and ^ red_or) : 0ull;
  uint64_t pp = 0, pm = 0, kp = 0, km = 0;
  bool key_phase = diff == 0;
  int shift = 64 - kDigit;
  if (diff != 0) {
    const int hd = 63 - __clzll((long long)diff);  // highest differing bit
    shift = hd >= kDigit - 1 ? hd - (kDigit - 1) : 0;
    pm = hd < 63 ? ~0ull << (hd + 1) : 0ull;
    pp = (uint64_t)red_and & pm;
  }
  bool done = none || k_rem >= nb;
  // primary digits from the highest differing bit down, then key digits
  while (!done) {
    for (int b = t; b < kBins; b += kFineThreads) h[b] = 0;
    __syncthreads();
    for (int64_t e = t; e < nb; e += kFineThreads) {
      const uint64_t p = X[e];
      if ((p & pm) != pp) continue;
      if (!key_phase) {
        atomicAdd(&h[(p >> shift) & kDigitMask], 1u);
      } else {
        const uint64_t kk = Kk[e];
        if ((kk & km) != kp) continue;
        atomicAdd(&h[(kk >> shift) & kDigitMask], 1u);
      }
    }
    __syncthreads();
    // bins in selection order (descending primary, ascending key); thread t
    // owns positions 2t and 2t+1 of that order
    const int b0 = key_phase ? 2 * t : kBins - 1 - 2 * t;
    const int b1 = key_phase ? 2 * t + 1 : kBins - 2 - 2 * t;
    const unsigned v0 = h[b0], v1 = h[b1];
    const unsigned long long pair = (unsigned long long)v0 + v1;
    const unsigned long long winc = wave_incl_scan(pair);
    if (lane == 63) wsum[wv] = winc;
    if (t == 0) chosen = -1;
    __syncthreads();
    unsigned long long woff = 0;
    for (int w = 0; w < wv; ++w) woff += wsum[w];
    const unsigned long long excl = woff + winc - pair;
    if ((long long)excl < k_rem && (long long)(excl + v0) >= k_rem) {
      chosen = b0;
      before = excl;
    } else if ((long long)(excl + v0) < k_rem &&
               (long long)(excl + v0 + v1) >= k_rem) {
      chosen = b1;
      before = excl + v0;
    }
    __syncthreads();
    const int b = chosen;
    const unsigned nbin = b >= 0 ? h[b] : 0u;
    const unsigned long long bef = before;
    __syncthreads();
    if (b < 0) break;  // cannot happen while k_rem <= matching count
    k_rem -= (int64_t)bef;
    if (!key_phase) {
      pp |= (uint64_t)b << shift;
      pm |= kDigitMask << shift;
    } else {
      kp |= (uint64_t)b << shift;
      km |= kDigitMask << shift;
    }
    if ((int64_t)nbin == k_rem) {
      done = true;
    } else if (shift == 0) {
      if (key_phase) done = true;  // keys are unique: cannot recur
      key_phase = true;
      shift = 64 - kDigit;
    } else {
      shift = shift > kDigit ? shift - kDigit : 0;
    }
  }
  // emit the boundary elements ordered before the threshold and those
  // matching it (exactly k_rem of the original count in total)
  if (t == 0) emitted = 0;
  __syncthreads();
  for (int64_t e = t; e < nb && !none; e += kFineThreads) {
    const uint64_t p = X[e];
    const uint64_t kk = Kk[e];
    const uint64_t pmv = p & pm;
    bool take;
    if (pmv != pp) take = pmv > pp;
    else if (!key_phase) take = true;
    else take = (kk & km) <= kp;
    if (!take) continue;
    const int64_t slot = nwin + (int64_t)atomicAdd(&emitted, 1ull);
    if (slot >= ocap) continue;
    ox[slot] = p;
    okey[slot] = kk;
    if (oextra) oextra[slot] = bextra[e];
    if (oc) oc[slot] = bc[e];
  }
  __syncthreads();
  if (t == 0) {
    const int64_t tot = nwin + (int64_t)emitted;
    counts[out_count_slot] = tot < ocap ? tot : ocap;
  }
}

// ---------------------------------------------------------------------------
// verification: c = a_i . b_j in fp32, 16 lanes per candidate (four per
// wave), 16-byte loads when the rows allow them; histogram of |c|
__global__ __launch_bounds__(256) void k_verify(const uint64_t* key2,
                                                const int64_t* counts,
                                                const float* A, const float* B,
                                                int64_t n, int64_t d,
                                                int64_t cap2, float* c,
                                                uint64_t* absbits,
                                                unsigned* hist) {
  __shared__ unsigned h[kBins];
  for (int b = threadIdx.x; b < kBins; b += blockDim.x) h[b] = 0;
  __syncthreads();
  const int64_t ncand = counts[kCntCand] < cap2 ? counts[kCntCand] : cap2;
  const int q = threadIdx.x & 15;
  const int64_t grp = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 4;
  const int64_t ngrp = ((int64_t)gridDim.x * blockDim.x) >> 4;
  const bool vec = (d & 3) == 0 && ((uintptr_t)A & 15) == 0 &&
                   ((uintptr_t)B & 15) == 0;
  // the 16 lanes of a group share e, so they run the same rounds
  for (int64_t e = grp; e < ncand; e += ngrp) {
    float acc = 0.0f;
    {
      const uint64_t kk = key2[e];
      const int64_t i = (int64_t)(kk / (uint64_t)n);
      const int64_t j = (int64_t)(kk % (uint64_t)n);
      const float* a = A + i * d;
      const float* b = B + j * d;
      if (vec) {
        const float4* a4 = (const float4*)a;
        const float4* b4 = (const float4*)b;
        for (int64_t k = q; k < d / 4; k += 16) {
          const float4 x = a4[k], y = b4[k];
          acc = fmaf(x.x, y.x, acc);
          acc = fmaf(x.y, y.y, acc);
          acc = fmaf(x.z, y.z, acc);
          acc = fmaf(x.w, y.w, acc);
        }
      } else {
        for (int64_t k = q; k < d; k += 16) acc = fmaf(a[k], b[k], acc);
      }
    }
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 16);
    if (q == 0) {
      c[e] = acc;
      const uint64_t ab = __float_as_uint(fabsf(acc));
      absbits[e] = ab;
      atomicAdd(&h[fbin_float(ab)], 1u);
    }
  }
  block_hist_flush(h, hist);
}

// verification for sparse vectors: one wave per candidate, each lane takes entries
// of a_i and finds their coordinate in b_j by binary search
__global__ __launch_bounds__(256) void k_verify_csr(const uint64_t* key2,
                                                    const int64_t* counts,
                                                    CsrView v, int64_t n,
                                                    int64_t cap2, float* c,
                                                    uint64_t* absbits,
                                                    unsigned* hist) {
  __shared__ unsigned h[kBins];
  for (int b = threadIdx.x; b < kBins; b += blockDim.x) h[b] = 0;
  __syncthreads();
  const int64_t ncand = counts[kCntCand] < cap2 ? counts[kCntCand] : cap2;
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t e = wave; e < ncand; e += nwaves) {
    const uint64_t kk = key2[e];
    const int64_t i = (int64_t)(kk / (uint64_t)n);
    const int64_t j = (int64_t)(kk % (uint64_t)n);
    const int64_t a0 = v.a_ptr[i], a1 = v.a_ptr[i + 1];
    const int64_t b0 = v.b_ptr[j], b1 = v.b_ptr[j + 1];
    float acc = 0.0f;
    for (int64_t p = a0 + lane; p < a1; p += 64) {
      const int32_t k = v.a_idx[p];
      int64_t lo = b0, hi = b1;
      while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (v.b_idx[mid] < k) lo = mid + 1; else hi = mid;
      }
      if (lo < b1 && v.b_idx[lo] == k) acc = fmaf(v.a_val[p], v.b_val[lo], acc);
    }
    acc = wave_sum(acc);
    if (lane == 0) {
      c[e] = acc;
      const uint64_t ab = __float_as_uint(fabsf(acc));
      absbits[e] = ab;
      atomicAdd(&h[fbin_float(ab)], 1u);
    }
  }
  block_hist_flush(h, hist);
}


// ---------------------------------------------------------------------------
// low-precision filter of Omega_t' (between candidate selection and verification): c^ from the
// bf16 / fp8 copies with an a-priori bound mg on |c^ - c_fp32| (input
// rounding, fp32 accumulation, and the fp32 re-rank's own error).  With
// tau <= the t-th largest lower bound |c^| - mg, a candidate whose upper
// bound |c^| + mg is below tau has |c_fp32| < tau while t others have
// |c_fp32| >= tau, so dropping it leaves the fp32 top t unchanged.
// 16 lanes per candidate, 16-byte loads.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_verify_lowp(const uint64_t* key2,
                                                     int64_t* counts,
                                                     LowpView v, int64_t n,
                                                     int64_t cap2, float* hi,
                                                     unsigned* hist) {
  __shared__ unsigned h[kBins];
  __shared__ unsigned long long part[4];
  for (int b = threadIdx.x; b < kBins; b += blockDim.x) h[b] = 0;
  __syncthreads();
  const int64_t ncand = counts[kCntCand] < cap2 ? counts[kCntCand] : cap2;
  const int lane = threadIdx.x & 63, grp = lane >> 4, gl = lane & 15;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  const int eb = v.prec == 1 ? 2 : 1;
  const int64_t row_bytes = v.Kp * eb;
  unsigned long long npos = 0;
  for (int64_t e0 = wave * 4; e0 < ncand; e0 += nwaves * 4) {
    const int64_t e = e0 + grp;
    const bool ok = e < ncand;
    const uint64_t kk = key2[ok ? e : e0];
    const int64_t i = (int64_t)(kk / (uint64_t)n);
    const int64_t j = (int64_t)(kk % (uint64_t)n);
    const char* ar = (const char*)v.A + i * row_bytes;
    const char* br = (const char*)v.B + j * row_bytes;
    float acc = 0.0f;
    for (int64_t b0 = (int64_t)gl * 16; b0 < row_bytes; b0 += 256) {
      const uint4 x = *(const uint4*)(ar + b0);
      const uint4 y = *(const uint4*)(br + b0);
      acc = lowp_dot16(x, y, v.prec, acc);
    }
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (ok && gl == 0) {
      const VecInfo va = v.ia[i], vb = v.ib[j];
      const float c = acc * va.inv_s * vb.inv_s;
      const float mg = v.kappa * va.n2 * vb.n2 +
                       v.onepu * (va.eta * vb.n1 + vb.eta * va.n1) +
                       v.d_f * va.eta * vb.eta;
      const float lo = fabsf(c) - mg;
      hi[e] = fabsf(c) + mg;
      if (lo > 0.0f) {
        ++npos;
        atomicAdd(&h[fbin_float(__float_as_uint(lo))], 1u);
      }
    }
  }
  block_hist_flush(h, hist);
  npos = wave_sum(npos);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = npos;
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned long long tt = part[0] + part[1] + part[2] + part[3];
    if (tt) atomicAdd((unsigned long long*)&counts[kCntWin], tt);
  }
}

// the screen value c^ and its margin mg of given pairs (the arithmetic of
// k_verify_lowp, for measuring c^ against FP64 next to its bound)
__global__ __launch_bounds__(256) void k_lowp_screen_values(
    const uint64_t* keys, int64_t count, LowpView v, int64_t n, float* chat,
    float* margin) {
  const int lane = threadIdx.x & 63, grp = lane >> 4, gl = lane & 15;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  const int eb = v.prec == 1 ? 2 : 1;
  const int64_t row_bytes = v.Kp * eb;
  for (int64_t e0 = wave * 4; e0 < count; e0 += nwaves * 4) {
    const int64_t e = e0 + grp;
    const bool ok = e < count;
    const uint64_t kk = keys[ok ? e : e0];
    const int64_t i = (int64_t)(kk / (uint64_t)n);
    const int64_t j = (int64_t)(kk % (uint64_t)n);
    const char* ar = (const char*)v.A + i * row_bytes;
    const char* br = (const char*)v.B + j * row_bytes;
    float acc = 0.0f;
    for (int64_t b0 = (int64_t)gl * 16; b0 < row_bytes; b0 += 256) {
      const uint4 x = *(const uint4*)(ar + b0);
      const uint4 y = *(const uint4*)(br + b0);
      acc = lowp_dot16(x, y, v.prec, acc);
    }
#pragma unroll
    for (int off = 8; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if (ok && gl == 0) {
      const VecInfo va = v.ia[i], vb = v.ib[j];
      chat[e] = acc * va.inv_s * vb.inv_s;
      margin[e] = v.kappa * va.n2 * vb.n2 +
                  v.onepu * (va.eta * vb.n1 + vb.eta * va.n1) +
                  v.d_f * va.eta * vb.eta;
    }
  }
}

hipError_t launch_lowp_screen_values(const uint64_t* keys, int64_t count,
                                     const LowpView& v, int64_t n,
                                     float* chat, float* margin,
                                     hipStream_t st) {
  if (count <= 0) return hipSuccess;
  k_lowp_screen_values<<<blocks_for(count * 16, 256, 2048), 256, 0, st>>>(
      keys, count, v, n, chat, margin);
  return hipGetLastError();
}

// keep the candidates whose upper bound reaches tau (lower edge of the bin
// of the t-th largest lower bound; 0 when fewer than t are positive)
__global__ __launch_bounds__(256) void k_lowp_filter(
    const Coarse* cz, const uint64_t* key2, const uint64_t* x2,
    const float* hi, int64_t cap2, uint64_t* okey, uint64_t* ox,
    int64_t* counts) {
  __shared__ unsigned wcount[4];
  __shared__ unsigned long long wbase[5];
  const Coarse c = *cz;
  const float tau = c.bin >= 0 ? __uint_as_float((uint32_t)c.bin << 20) : 0.0f;
  const int64_t n = counts[kCntCand] < cap2 ? counts[kCntCand] : cap2;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t b0 = (int64_t)blockIdx.x * blockDim.x; b0 < n; b0 += stride) {
    const int64_t e = b0 + threadIdx.x;
    const bool keep = e < n && hi[e] >= tau;
    const int64_t p = block_append(
        keep, (unsigned long long*)&counts[kCntBound], wcount, wbase);
    if (keep) {
      okey[p] = key2[e];
      ox[p] = x2[e];
    }
  }
}

// the kept candidates become Omega for verification / final selection
__global__ void k_lowp_copy(const uint64_t* key, const uint64_t* x,
                            uint64_t* key2, uint64_t* x2, int64_t* counts) {
  const int64_t kept = counts[kCntBound];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < kept;
       e += stride) {
    key2[e] = key[e];
    x2[e] = x[e];
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    counts[kCntPreFilter] = counts[kCntCand];
    counts[kCntReranked] = kept;
    counts[kCntCand] = kept;
  }
}

// final selection step 2b: split the candidates
__global__ __launch_bounds__(256) void k_cand_split(
    const Coarse* cz, const uint64_t* absbits, const uint64_t* key2,
    const uint64_t* x2, const float* c, int64_t cap2, uint64_t* fp,
    uint64_t* fkey, uint64_t* fx, float* fc, int64_t tcap, uint64_t* bp,
    uint64_t* bkey, uint64_t* bx, float* bc, int64_t bcap, int64_t* counts,
    uint64_t* part = nullptr) {
  __shared__ unsigned wcount[4];
  __shared__ unsigned long long wbase[5];
  __shared__ unsigned long long red[4][4];
  uint64_t xa = ~0ull, xo = 0ull, ka = ~0ull, ko = 0ull;
  const Coarse cc = *cz;
  const int64_t n = counts[kCntCand] < cap2 ? counts[kCntCand] : cap2;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t b0 = (int64_t)blockIdx.x * blockDim.x; b0 < n; b0 += stride) {
    const int64_t e = b0 + threadIdx.x;
    const bool live = e < n;
    const uint64_t p = live ? absbits[e] : 0;
    const int bin = fbin_float(p);
    const bool win = live && (cc.bin < 0 || bin > cc.bin);
    const bool bnd = live && cc.bin >= 0 && bin == cc.bin;
    const int64_t ws = block_append(
        win, (unsigned long long*)&counts[kCntWin], wcount, wbase);
    if (win && ws < tcap) {
      fp[ws] = p;
      fkey[ws] = key2[e];
      fx[ws] = x2[e];
      fc[ws] = c[e];
    }
    const int64_t bs = block_append(
        bnd, (unsigned long long*)&counts[kCntBound], wcount, wbase);
    if (bnd && bs < bcap) {
      const uint64_t kk = key2[e];
      bp[bs] = p;
      bkey[bs] = kk;
      bx[bs] = x2[e];
      bc[bs] = c[e];
      xa &= p;
      xo |= p;
      ka &= kk;
      ko |= kk;
    }
  }
  if (part) block_and_or(xa, xo, ka, ko, red, part);
}

// rank sort of the final set by (|c| desc, key asc) into mad_pair order
struct PairOut {
  int64_t i, j;
  float c, x;
};

// the final set ordered by (|c| desc, key asc): each element's rank is the
// number of elements before it, counted against the set staged in LDS in
// chunks
constexpr int kSortChunk = 2048;

__global__ __launch_bounds__(256) void k_final_sort(
    const uint64_t* fkey, const uint64_t* fx, const float* fc,
    const int64_t* counts, int64_t tcap, int64_t n, const float* bmax,
    int64_t s_for_F, int x_shift, PairOut* out, int64_t* n_out) {
  __shared__ float sa[kSortChunk];
  __shared__ uint64_t sk[kSortChunk];
  const int64_t nf = counts[kCntFinal] < tcap ? counts[kCntFinal] : tcap;
  const int F = (bmax ? fix_exponent(*bmax, s_for_F) : 0) + x_shift;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const float ae = e < nf ? fabsf(fc[e]) : 0.0f;
  const uint64_t ke = e < nf ? fkey[e] : 0ull;
  int64_t rank = 0;
  for (int64_t o0 = 0; o0 < nf; o0 += kSortChunk) {
    const int64_t no = nf - o0 < kSortChunk ? nf - o0 : kSortChunk;
    __syncthreads();
    for (int64_t o = threadIdx.x; o < no; o += blockDim.x) {
      sa[o] = fabsf(fc[o0 + o]);
      sk[o] = fkey[o0 + o];
    }
    __syncthreads();
    if (e < nf) {
      const int nn = (int)no;
      int r = 0;
#pragma unroll 8
      for (int o = 0; o < nn; ++o)
        r += (sa[o] > ae || (sa[o] == ae && sk[o] < ke)) ? 1 : 0;
      rank += r;
    }
  }
  if (e < nf) {
    PairOut p;
    p.i = (int64_t)(ke / (uint64_t)n);
    p.j = (int64_t)(ke % (uint64_t)n);
    p.c = fc[e];
    p.x = (float)ldexp((double)(int64_t)fx[e], -F);
    out[rank] = p;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) *n_out = nf;
}

// every key of X (closed diamonds), for parity checks
__global__ void k_dump_scores(const uint64_t* hkeys, const int64_t* hvals,
                              int64_t cap, const int64_t* live, int64_t* keys,
                              int64_t* xfix, int64_t out_cap, int64_t* count) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  if (live && *live < cap) cap = *live;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < cap;
       e += stride) {
    const uint64_t kk = hkeys[e];
    if (kk == kEmptyKey) continue;
    const unsigned long long p =
        atomicAdd((unsigned long long*)count, 1ull);
    if ((int64_t)p < out_cap) {
      keys[p] = (int64_t)kk;
      xfix[p] = hvals[e];
    }
  }
}

hipError_t launch_dump_scores(const HashTable& h, int64_t* keys,
                              int64_t* xfix, int64_t out_cap, int64_t* count,
                              hipStream_t st) {
  hipError_t e = launch_fill_u64((uint64_t*)count, 1, 0ull, st);
  if (e != hipSuccess) return e;
  k_dump_scores<<<blocks_for(h.cap, 256, 4096), 256, 0, st>>>(
      h.keys, h.vals, h.cap, h.live, keys, xfix, out_cap, count);
  return hipGetLastError();
}

// histogram of |v| (float digit) and |v| bits, for a selection on values
__global__ __launch_bounds__(256) void k_absval_hist(const float* v,
                                                     int64_t n,
                                                     uint64_t* absbits,
                                                     unsigned* hist) {
  __shared__ unsigned h[kBins];
  for (int b = threadIdx.x; b < kBins; b += blockDim.x) h[b] = 0;
  __syncthreads();
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += stride) {
    const uint64_t ab = __float_as_uint(fabsf(v[e]));
    absbits[e] = ab;
    atomicAdd(&h[fbin_float(ab)], 1u);
  }
  block_hist_flush(h, hist);
}

hipError_t launch_select_keys_by_absval(const uint64_t* keys, const float* v,
                                        int64_t count, int64_t k,
                                        DeviceBuffer& buf, uint64_t* out_keys,
                                        hipStream_t st) {
  const int64_t cnt = count > 1 ? count : 1;
  const size_t need = 256 + 256 + kBins * 4 + (size_t)cnt * (8 + 8) +
                      (size_t)(4 * k + 4 * cnt) * 8 + 1024;
  hipError_t e = dev_alloc(buf, need);
  if (e != hipSuccess) return e;
  char* p = (char*)buf.p;
  int64_t* counts = (int64_t*)p; p += 256;
  Coarse* cz = (Coarse*)p; p += 256;
  unsigned* hist = (unsigned*)p; p += kBins * 4;
  uint64_t* x2 = (uint64_t*)p; p += (size_t)cnt * 8;
  uint64_t* absbits = (uint64_t*)p; p += (size_t)cnt * 8;
  uint64_t* key = (uint64_t*)p;
  if ((e = launch_fill_u64((uint64_t*)counts, 32, 0ull, st)) != hipSuccess ||
      (e = launch_fill_u64((uint64_t*)hist, kBins / 2, 0ull, st)) != hipSuccess ||
      (e = launch_fill_u64(x2, cnt, 0ull, st)) != hipSuccess ||
      (e = launch_fill_u64((uint64_t*)&counts[kCntCand], 1, (uint64_t)count,
                           st)) != hipSuccess)
    return e;
  k_absval_hist<<<blocks_for(cnt, 256 * 8, 2048), 256, 0, st>>>(v, count,
                                                                absbits, hist);
  k_coarse_decide<<<1, 256, 0, st>>>(hist, &counts[kCntCand], k, cz,
                                     nullptr);
  uint64_t* fp = key;
  uint64_t* fkey = out_keys;
  uint64_t* fx = key + k;
  float* fc = (float*)(key + 2 * k);
  const int64_t bcap = cnt;
  uint64_t* bp = key + 4 * k;
  uint64_t* bkey = bp + bcap;
  uint64_t* bx = bkey + bcap;
  float* bc = (float*)(bx + bcap);
  k_cand_split<<<blocks_for(cnt, 256 * 4, 1024), 256, 0, st>>>(
      cz, absbits, keys, x2, v, cnt, fp, fkey, fx, fc, k, bp, bkey, bx, bc,
      bcap, counts);
  k_fine_select<<<1, kFineThreads, 0, st>>>(cz, bp, bkey, bx, bc, bcap,
                                            counts, kCntWin, fp, fkey, fx, fc,
                                            k, kCntFinal);
  return hipGetLastError();
}

hipError_t launch_rerank_topk(const uint64_t* keys, int64_t count,
                              const float* A, const float* B, int64_t n,
                              int64_t d, int64_t t, DeviceBuffer& buf,
                              void* out, int64_t* n_out, const CsrView* csr,
                              hipStream_t st) {
  // layout: counts, Coarse, hist, x2 (zeros), c, |c| bits, final + boundary
  const int64_t cnt = count > 1 ? count : 1;
  const size_t need = 256 + 256 + kBins * 4 + (size_t)cnt * (8 + 4 + 8) +
                      (size_t)(4 * t + 4 * cnt) * 8 + 1024;
  hipError_t e = dev_alloc(buf, need);
  if (e != hipSuccess) return e;
  char* p = (char*)buf.p;
  int64_t* counts = (int64_t*)p; p += 256;
  Coarse* cz = (Coarse*)p; p += 256;
  unsigned* hist = (unsigned*)p; p += kBins * 4;
  uint64_t* x2 = (uint64_t*)p; p += (size_t)cnt * 8;
  float* c = (float*)p; p += (size_t)cnt * 4;
  p = (char*)(((uintptr_t)p + 15) & ~(uintptr_t)15);
  uint64_t* absbits = (uint64_t*)p; p += (size_t)cnt * 8;
  uint64_t* key = (uint64_t*)p;
  if ((e = launch_fill_u64((uint64_t*)counts, 32, 0ull, st)) != hipSuccess ||
      (e = launch_fill_u64((uint64_t*)hist, kBins / 2, 0ull, st)) != hipSuccess ||
      (e = launch_fill_u64(x2, cnt, 0ull, st)) != hipSuccess)
    return e;
  // the candidate count goes where the verification kernel reads it
  e = launch_fill_u64((uint64_t*)&counts[kCntCand], 1, (uint64_t)count, st);
  if (e != hipSuccess) return e;
  if (csr)
    k_verify_csr<<<blocks_for(cnt * 64, 256, 2048), 256, 0, st>>>(
        keys, counts, *csr, n, cnt, c, absbits, hist);
  else
    k_verify<<<blocks_for(cnt * 16, 256, 2048), 256, 0, st>>>(
        keys, counts, A, B, n, d, cnt, c, absbits, hist);
  k_coarse_decide<<<1, 256, 0, st>>>(hist, &counts[kCntCand], t, cz,
                                     nullptr);
  uint64_t* fp = key;
  uint64_t* fkey = key + t;
  uint64_t* fx = key + 2 * t;
  float* fc = (float*)(key + 3 * t);
  const int64_t bcap = cnt;
  uint64_t* bp = key + 4 * t;
  uint64_t* bkey = bp + bcap;
  uint64_t* bx = bkey + bcap;
  float* bc = (float*)(bx + bcap);
  k_cand_split<<<blocks_for(cnt, 256 * 4, 1024), 256, 0, st>>>(
      cz, absbits, keys, x2, c, cnt, fp, fkey, fx, fc, t, bp, bkey, bx, bc,
      bcap, counts);
  k_fine_select<<<1, kFineThreads, 0, st>>>(cz, bp, bkey, bx, bc, bcap,
                                            counts, kCntWin, fp, fkey, fx, fc,
                                            t, kCntFinal);
  // x = 0 for brute-force results (no sampler score); F is irrelevant
  k_final_sort<<<blocks_for(t, 256, 1 << 30), 256, 0, st>>>(
      fkey, fx, fc, counts, t, n, nullptr, 0, 0, (PairOut*)out, n_out);
  return hipGetLastError();
}

// The clears postprocessing starts from: the counts it accumulates and the
// histogram (cleared by each decision, and here as well so that a fresh or
// previously interrupted workspace starts from zero).  Appends 3 fills.
void post_fills(SelectWork& w, FillBatch& f) {
  f.p[f.count] = (uint64_t*)w.counts;
  f.n[f.count++] = 1;
  f.p[f.count] = (uint64_t*)&w.counts[kCntCand];
  f.n[f.count++] = 4;
  f.p[f.count] = (uint64_t*)w.hist;
  f.n[f.count++] = kBins / 2;
}

hipError_t launch_postprocess(const HashTable& h, const float* A,
                              const float* B, const CsrView* csr,
                              const LowpView* lowp, int64_t n, int64_t d,
                              int64_t t_prime, int64_t t, const float* bmax,
                              int64_t s, int x_shift, SelectWork& w,
                              void* out, int64_t* n_out, bool cleared,
                              hipStream_t st) {
  Coarse* cz = (Coarse*)w.state;
  int64_t* counts = w.counts;
  // keep counts[kCntDistinct] (the sampler's), clear the others
  hipError_t e = hipSuccess;
  if (!cleared) {
    FillBatch f{};
    post_fills(w, f);
    if ((e = launch_fill_multi(f, st)) != hipSuccess) return e;
  }
  // ---- candidate selection: top t' of x over x > 0 ------------------------------------
  k_score_hist<<<blocks_for(h.cap, kHistThreads * 16, kHistBlocks),
                 kHistThreads, 0, st>>>(h.vals, h.cap, h.live, w.hist);
  Refine* rf = (Refine*)(cz + 3);
  k_coarse_decide<<<1, 256, 0, st>>>(w.hist, nullptr, t_prime, cz,
                                     &counts[kCntPos], rf);
  // winners go straight to (x2, key2); the boundary bin to (x, key)
  const unsigned nsplit = blocks_for(h.cap, 256 * 16, 512);
  static_assert(512 <= kPartBlocks, "one and / or slot per split block");
  k_score_split<<<nsplit, 256, 0, st>>>(h.keys, h.vals, h.cap, h.live, cz,
                                        w.x2, w.key2, w.cap2, w.x, w.key,
                                        w.cap, counts, w.part);
  // a long boundary list: one digit of it on the whole grid (each kernel
  // returns at once otherwise)
  k_refine_hist<<<256, kRefineThreads, 0, st>>>(
      cz, w.part, (int)nsplit, w.x, w.key, w.cap, counts, w.hist);
  k_refine_decide<<<1, kRefineThreads, 0, st>>>(
      cz, rf, w.part, (int)nsplit, counts, w.cap, w.rcap, w.hist);
  k_refine_split<<<1024, 256, 0, st>>>(
      rf, w.x, w.key, nullptr, nullptr, w.cap, counts, w.x2, w.key2, nullptr,
      nullptr, w.cap2, &rf->nout, w.rx, w.rkey, nullptr, nullptr, w.rcap);
  k_fine_select<<<1, kFineThreads, 0, st>>>(
      cz, w.x, w.key, nullptr, nullptr, w.cap, counts, kCntWin, w.x2, w.key2,
      nullptr, nullptr, w.cap2, kCntCand, rf, w.rx, w.rkey, nullptr, nullptr,
      w.rcap);
  // ---- low-precision filter of Omega_t' ----------------------------------
  if (lowp) {
    e = launch_fill_u64((uint64_t*)&counts[kCntBound], 2, 0ull, st);
    if (e != hipSuccess) return e;
    k_verify_lowp<<<blocks_for(t_prime * 16, 256, 2048), 256, 0, st>>>(
        w.key2, counts, *lowp, n, w.cap2, w.c, w.hist);
    k_coarse_decide<<<1, 256, 0, st>>>(w.hist, &counts[kCntWin], t, cz + 2,
                                       nullptr);
    k_lowp_filter<<<blocks_for(t_prime, 256 * 4, 1024), 256, 0, st>>>(
        cz + 2, w.key2, w.x2, w.c, w.cap2, w.x, w.key, counts);
    k_lowp_copy<<<blocks_for(t_prime, 256 * 4, 1024), 256, 0, st>>>(
        w.x, w.key, w.key2, w.x2, counts);
  }
  // ---- verification: fp32 dot products and the |c| histogram --------------------
  // (|c| bits go to w.x, free after candidate selection)
  if (csr)
    k_verify_csr<<<blocks_for(t_prime * 64, 256, 2048), 256, 0, st>>>(
        w.key2, counts, *csr, n, w.cap2, w.c, w.x, w.hist);
  else
    k_verify<<<blocks_for(t_prime * 16, 256, 2048), 256, 0, st>>>(
        w.key2, counts, A, B, n, d, w.cap2, w.c, w.x, w.hist);
  // ---- final selection: top t by |c| ----------------------------------------------
  e = launch_fill_u64((uint64_t*)&counts[kCntBound], 2, 0ull, st);
  if (e != hipSuccess) return e;
  Refine* rf2 = rf + 1;
  k_coarse_decide<<<1, 256, 0, st>>>(w.hist, &counts[kCntCand], t, cz + 1,
                                     nullptr, rf2);
  // final set in w.key[0 .. 4t): |c| bits, key, x, c; boundary after it
  uint64_t* fp = w.key;
  uint64_t* fkey = w.key + t;
  uint64_t* fx = w.key + 2 * t;
  float* fc = (float*)(w.key + 3 * t);
  const int64_t bcap = (w.cap - 4 * t) / 4;
  uint64_t* bp = w.key + 4 * t;
  uint64_t* bkey = bp + bcap;
  uint64_t* bx = bkey + bcap;
  float* bc = (float*)(bx + bcap);
  const unsigned ncs = blocks_for(t_prime, 256 * 4, 1024);
  static_assert(1024 <= kPartBlocks, "one and / or slot per split block");
  uint64_t* part2 = w.part + 4 * kPartBlocks;
  k_cand_split<<<ncs, 256, 0, st>>>(cz + 1, w.x, w.key2, w.x2, w.c, w.cap2,
                                    fp, fkey, fx, fc, t, bp, bkey, bx, bc,
                                    bcap, counts, part2);
  // a long boundary list of tied |c|: one digit of it on the whole grid;
  // the refined list (|c| bits, key, x, c) in the refinement buffer, half
  // as many entries as for the candidate selection.  The boundary holds at
  // most t' entries: below kRefineFinalMin the three launches (which would
  // return at once or save little) are left out.
  const int64_t rcap2 = w.rcap / 2;
  uint64_t* rp = w.rx;
  uint64_t* rk = rp + rcap2;
  uint64_t* rxx = rk + rcap2;
  float* rc = (float*)(rxx + rcap2);
  if (t_prime > kRefineFinalMin) {
    k_refine_hist<<<256, kRefineThreads, 0, st>>>(
        cz + 1, part2, (int)ncs, bp, bkey, bcap, counts, w.hist);
    k_refine_decide<<<1, kRefineThreads, 0, st>>>(
        cz + 1, rf2, part2, (int)ncs, counts, bcap, rcap2, w.hist);
    k_refine_split<<<1024, 256, 0, st>>>(rf2, bp, bkey, bx, bc, bcap, counts,
                                         fp, fkey, fx, fc, t, &rf2->nout, rp,
                                         rk, rxx, rc, rcap2);
  }
  k_fine_select<<<1, kFineThreads, 0, st>>>(
      cz + 1, bp, bkey, bx, bc, bcap, counts, kCntWin, fp, fkey, fx, fc, t,
      kCntFinal, rf2, rp, rk, rxx, rc, rcap2);
  k_final_sort<<<blocks_for(t, 256, 1 << 30), 256, 0, st>>>(
      fkey, fx, fc, counts, t, n, bmax, s, x_shift, (PairOut*)out, n_out);
  return hipGetLastError();
}

}  // namespace mad
