// select.hip -- Alg. 3 postprocessing on the GPU.
//
//   post1  Omega_s = pairs with x_ij > 0; Omega_t' = the t' largest by x,
//          ties by key (i*n + j) ascending;
//   post2  c_ij = a_i . b_j in fp32 for each candidate;
//   post3  Omega_t = the t largest by |c|, ties by key ascending, written in
//          that order.
//
// Both selections are radix selects on a (primary descending, key
// ascending) order: 11-bit digits of the primary from its highest set bit
// down, each pass a histogram of the elements that still match the chosen
// prefix; when the chosen bin holds exactly the number still needed, or the
// primary is fully fixed, the ties are split the same way on the key.  Every
// count lives in device memory, so the sequence of launches needs no host
// synchronisation.
#include "mad_common.hpp"
#include "plan.hpp"

namespace mad {

constexpr int kDigit = 11;
constexpr int kBins = 1 << kDigit;
constexpr uint64_t kDigitMask = kBins - 1;

struct SelState {
  int64_t n;          // elements
  int64_t k;          // how many to select
  int64_t k_rem;      // still to take among the matching elements
  uint64_t maxp;      // largest primary
  uint64_t pprefix, pmask;  // fixed primary bits
  uint64_t kprefix, kmask;  // fixed key bits (tie split)
  int shift;          // current digit position
  int phase;          // 0 primary digits, 1 key digits, 2 done
  int take_all;       // n <= k
  int key_split;      // ties at the primary threshold split on the key
};

// counters in SelectWork::counts
enum {
  kCntPos = 0,      // |Omega_s|
  kCntDistinct = 1, // nnz(X)
  kCntCand = 2,     // |Omega_t'|
  kCntFinal = 3,    // |Omega_t|
  kCntMax = 4       // largest primary (as u64) of the current selection
};

static inline unsigned blocks_for(int64_t n, int per_block, int cap) {
  int64_t g = (n + per_block - 1) / per_block;
  if (g > cap) g = cap;
  return (unsigned)(g < 1 ? 1 : g);
}

// ---------------------------------------------------------------------------
// post1 input: compact the hash table to (x, key) with x > 0
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_compact_scores(
    const uint64_t* hkeys, const int64_t* hvals, int64_t cap, uint64_t* x,
    uint64_t* key, int64_t* counts) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int lane = threadIdx.x & 63;
  unsigned long long distinct = 0;
  uint64_t mx = 0;
  for (int64_t b = (int64_t)blockIdx.x * blockDim.x; b < cap; b += stride) {
    const int64_t e = b + threadIdx.x;
    uint64_t kk = kEmptyKey;
    int64_t v = 0;
    if (e < cap) {
      kk = hkeys[e];
      v = hvals[e];
    }
    distinct += kk != kEmptyKey;
    const bool take = kk != kEmptyKey && v > 0;
    const uint64_t ball = __ballot(take);
    const int cnt = __popcll(ball);
    unsigned long long base = 0;
    if (cnt) {
      if (lane == 0)
        base = atomicAdd((unsigned long long*)&counts[kCntPos],
                         (unsigned long long)cnt);
      base = __shfl(base, 0, 64);
    }
    if (take) {
      const int r = __popcll(ball & ((1ull << lane) - 1));
      x[base + r] = (uint64_t)v;
      key[base + r] = kk;
      mx = (uint64_t)v > mx ? (uint64_t)v : mx;
    }
  }
  distinct = wave_sum(distinct);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    const uint64_t o = __shfl_xor(mx, off, 64);
    mx = o > mx ? o : mx;
  }
  if (lane == 0) {
    if (distinct)
      atomicAdd((unsigned long long*)&counts[kCntDistinct], distinct);
    if (mx) atomicMax((unsigned long long*)&counts[kCntMax], mx);
  }
}

// ---------------------------------------------------------------------------
// radix select
// ---------------------------------------------------------------------------
__global__ void k_sel_init(SelState* s, const int64_t* n_ptr, int64_t k,
                           const int64_t* counts, unsigned* hist) {
  const int64_t n = *n_ptr;
  for (int b = threadIdx.x; b < kBins; b += blockDim.x) hist[b] = 0;
  if (threadIdx.x != 0) return;
  s->n = n;
  s->k = k;
  s->k_rem = k;
  s->maxp = (uint64_t)counts[kCntMax];
  s->pprefix = s->pmask = s->kprefix = s->kmask = 0;
  s->take_all = n <= k;
  s->key_split = 0;
  s->phase = n <= k ? 2 : 0;
  const int hi = s->maxp ? 64 - __clzll((long long)s->maxp) : 1;
  s->shift = hi > kDigit ? hi - kDigit : 0;
}

__global__ __launch_bounds__(256) void k_sel_hist(const SelState* s,
                                                  const uint64_t* prim,
                                                  const uint64_t* key,
                                                  unsigned* hist) {
  const int phase = s->phase;
  if (phase == 2) return;
  __shared__ unsigned h[kBins];
  for (int b = threadIdx.x; b < kBins; b += blockDim.x) h[b] = 0;
  __syncthreads();
  const int64_t n = s->n;
  const int shift = s->shift;
  const uint64_t pp = s->pprefix, pm = s->pmask;
  const uint64_t kp = s->kprefix, km = s->kmask;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += stride) {
    const uint64_t p = prim[e];
    if ((p & pm) != pp) continue;
    if (phase == 0) {
      atomicAdd(&h[(p >> shift) & kDigitMask], 1u);
    } else {
      const uint64_t kk = key[e];
      if ((kk & km) != kp) continue;
      atomicAdd(&h[(kk >> shift) & kDigitMask], 1u);
    }
  }
  __syncthreads();
  for (int b = threadIdx.x; b < kBins; b += blockDim.x)
    if (h[b]) atomicAdd(&hist[b], h[b]);
}

// one block: pick the digit, update the state, clear the histogram
__global__ __launch_bounds__(256) void k_sel_decide(SelState* s,
                                                    unsigned* hist) {
  __shared__ unsigned long long part[256];
  __shared__ int chosen;
  __shared__ unsigned long long before;
  if (s->phase == 2) return;
  const int phase = s->phase;
  // phase 0 counts from the top bin down (descending primary); phase 1 from
  // the bottom up (ascending key).  Each thread owns 8 consecutive bins in
  // scan order.
  const int t = threadIdx.x;
  if (t == 0) chosen = -1;
  unsigned v[8];
  unsigned long long sum = 0;
  for (int q = 0; q < 8; ++q) {
    const int idx = t * 8 + q;
    const int b = phase == 0 ? kBins - 1 - idx : idx;
    v[q] = hist[b];
    sum += v[q];
  }
  part[t] = sum;
  __syncthreads();
  if (t == 0) {
    unsigned long long acc = 0;
    for (int u = 0; u < 256; ++u) {
      const unsigned long long x = part[u];
      part[u] = acc;
      acc += x;
    }
  }
  __syncthreads();
  const long long need = s->k_rem;
  {
    unsigned long long acc = part[t];
    for (int q = 0; q < 8; ++q) {
      if ((long long)acc < need && (long long)(acc + v[q]) >= need) {
        const int idx = t * 8 + q;
        chosen = phase == 0 ? kBins - 1 - idx : idx;
        before = acc;
      }
      acc += v[q];
    }
  }
  __syncthreads();
  const int b = chosen;
  if (b < 0) {  // cannot happen when k_rem <= matching count; stop safely
    if (t == 0) s->phase = 2;
    return;
  }
  const unsigned nb = hist[b];
  __syncthreads();
  for (int q = t; q < kBins; q += 256) hist[q] = 0;
  if (t != 0) return;
  const int shift = s->shift;
  const int64_t k_rem = need - (long long)before;
  s->k_rem = k_rem;
  if (phase == 0) {
    s->pprefix |= (uint64_t)b << shift;
    s->pmask |= kDigitMask << shift;
    if ((int64_t)nb == k_rem) {
      s->phase = 2;  // every element matching the prefix is taken
    } else if (shift == 0) {
      s->phase = 1;  // primary fixed: split the ties on the key
      s->key_split = 1;
      s->shift = 64 - kDigit;
    } else {
      s->shift = shift > kDigit ? shift - kDigit : 0;
    }
  } else {
    s->kprefix |= (uint64_t)b << shift;
    s->kmask |= kDigitMask << shift;
    if ((int64_t)nb == k_rem || shift == 0) s->phase = 2;
    else s->shift = shift > kDigit ? shift - kDigit : 0;
  }
}

__device__ __forceinline__ bool sel_take(const SelState& s, uint64_t p,
                                         uint64_t kk) {
  if (s.take_all) return true;
  const uint64_t pm = p & s.pmask;
  if (pm != s.pprefix) return pm > s.pprefix;
  if (!s.key_split) return true;
  const uint64_t km = kk & s.kmask;
  return km <= s.kprefix;
}

// post1 emit: copy the selected (x, key) pairs
__global__ __launch_bounds__(256) void k_emit_candidates(
    const SelState* sp, const uint64_t* x, const uint64_t* key, uint64_t* x2,
    uint64_t* key2, int64_t cap2, int64_t* counts) {
  const SelState s = *sp;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int lane = threadIdx.x & 63;
  for (int64_t b = (int64_t)blockIdx.x * blockDim.x; b < s.n; b += stride) {
    const int64_t e = b + threadIdx.x;
    bool take = false;
    uint64_t xv = 0, kv = 0;
    if (e < s.n) {
      xv = x[e];
      kv = key[e];
      take = sel_take(s, xv, kv);
    }
    const uint64_t ball = __ballot(take);
    const int cnt = __popcll(ball);
    if (!cnt) continue;
    unsigned long long base = 0;
    if (lane == 0)
      base = atomicAdd((unsigned long long*)&counts[kCntCand],
                       (unsigned long long)cnt);
    base = __shfl(base, 0, 64);
    if (take) {
      const int64_t r = base + __popcll(ball & ((1ull << lane) - 1));
      if (r < cap2) {  // the select takes exactly min(n, t') elements
        x2[r] = xv;
        key2[r] = kv;
      }
    }
  }
}

// post2: c = a_i . b_j in fp32, one wave per candidate; also |c| as bits
__global__ __launch_bounds__(256) void k_verify(const uint64_t* key2,
                                                const int64_t* counts,
                                                const float* A, const float* B,
                                                int64_t n, int64_t d,
                                                int64_t cap2, float* c,
                                                uint64_t* absbits,
                                                int64_t* maxbits) {
  const int64_t ncand = counts[kCntCand] < cap2 ? counts[kCntCand] : cap2;
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  uint64_t mx = 0;
  for (int64_t e = wave; e < ncand; e += nwaves) {
    const uint64_t kk = key2[e];
    const int64_t i = (int64_t)(kk / (uint64_t)n), j = (int64_t)(kk % (uint64_t)n);
    const float* a = A + i * d;
    const float* b = B + j * d;
    float acc = 0.0f;
    for (int64_t k = lane; k < d; k += 64) acc = fmaf(a[k], b[k], acc);
    acc = wave_sum(acc);
    if (lane == 0) {
      c[e] = acc;
      const uint64_t ab = __float_as_uint(fabsf(acc));
      absbits[e] = ab;
      mx = ab > mx ? ab : mx;
    }
  }
  if (lane == 0 && mx) atomicMax((unsigned long long*)maxbits, mx);
}

// post3 emit: the selected candidates into the final buffer
__global__ __launch_bounds__(256) void k_emit_final(
    const SelState* sp, const uint64_t* absbits, const uint64_t* key2,
    const uint64_t* x2, const float* c, uint64_t* fkey, uint64_t* fx,
    float* fc, int64_t tcap, int64_t* counts) {
  const SelState s = *sp;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < s.n;
       e += stride) {
    if (!sel_take(s, absbits[e], key2[e])) continue;
    const unsigned long long p =
        atomicAdd((unsigned long long*)&counts[kCntFinal], 1ull);
    if ((int64_t)p >= tcap) continue;
    fkey[p] = key2[e];
    fx[p] = x2[e];
    fc[p] = c[e];
  }
}

// rank sort of the final set by (|c| desc, key asc) into mad_pair order
struct PairOut {
  int64_t i, j;
  float c, x;
};

__global__ void k_final_sort(const uint64_t* fkey, const uint64_t* fx,
                             const float* fc, const int64_t* counts,
                             int64_t tcap, int64_t n, const float* bmax,
                             int64_t s_for_F, PairOut* out, int64_t* n_out) {
  const int64_t nf = counts[kCntFinal] < tcap ? counts[kCntFinal] : tcap;
  const int F = fix_exponent(*bmax, s_for_F);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nf;
       e += stride) {
    const float ae = fabsf(fc[e]);
    const uint64_t ke = fkey[e];
    int64_t rank = 0;
    for (int64_t o = 0; o < nf; ++o) {
      const float ao = fabsf(fc[o]);
      rank += ao > ae || (ao == ae && fkey[o] < ke);
    }
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
                              int64_t cap, int64_t* keys, int64_t* xfix,
                              int64_t out_cap, int64_t* count) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
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
      h.keys, h.vals, h.cap, keys, xfix, out_cap, count);
  return hipGetLastError();
}

static hipError_t run_select(SelState* st_dev, const int64_t* n_ptr,
                             int64_t k, const int64_t* counts,
                             const uint64_t* prim, const uint64_t* key,
                             unsigned* hist, int64_t n_ub, hipStream_t st) {
  k_sel_init<<<1, 256, 0, st>>>(st_dev, n_ptr, k, counts, hist);
  const unsigned g = blocks_for(n_ub, 256 * 16, 1024);
  // up to 6 primary digits and 6 key digits; idle passes return at once
  for (int pass = 0; pass < 12; ++pass) {
    k_sel_hist<<<g, 256, 0, st>>>(st_dev, prim, key, hist);
    k_sel_decide<<<1, 256, 0, st>>>(st_dev, hist);
  }
  return hipGetLastError();
}

hipError_t launch_postprocess(const HashTable& h, const float* A,
                              const float* B, int64_t n, int64_t d,
                              int64_t t_prime, int64_t t, const float* bmax,
                              int64_t s, SelectWork& w, void* out,
                              int64_t* n_out, hipStream_t st) {
  SelState* ss = (SelState*)w.state;
  int64_t* counts = w.counts;
  hipError_t e = launch_fill_u64((uint64_t*)counts, 8, 0ull, st);
  if (e != hipSuccess) return e;
  // post1
  k_compact_scores<<<blocks_for(h.cap, 256 * 8, 4096), 256, 0, st>>>(
      h.keys, h.vals, h.cap, w.x, w.key, counts);
  const int64_t n_ub = w.cap;
  e = run_select(ss, &counts[kCntPos], t_prime, counts, w.x, w.key, w.hist,
                 n_ub, st);
  if (e != hipSuccess) return e;
  k_emit_candidates<<<blocks_for(n_ub, 256 * 8, 4096), 256, 0, st>>>(
      ss, w.x, w.key, w.x2, w.key2, w.cap2, counts);
  // post2: |c| bits go to w.x (free now), the running max to counts[kCntMax]
  e = launch_fill_u64((uint64_t*)&counts[kCntMax], 1, 0ull, st);
  if (e != hipSuccess) return e;
  k_verify<<<blocks_for(t_prime * 64, 256, 4096), 256, 0, st>>>(
      w.key2, counts, A, B, n, d, w.cap2, w.c, w.x, &counts[kCntMax]);
  // post3
  e = run_select(ss, &counts[kCntCand], t, counts, w.x, w.key2, w.hist,
                 t_prime, st);
  if (e != hipSuccess) return e;
  uint64_t* fkey = w.key;  // reuse: first t entries
  uint64_t* fx = w.key + t;
  float* fc = (float*)(w.key + 2 * t);
  k_emit_final<<<blocks_for(t_prime, 256, 1024), 256, 0, st>>>(
      ss, w.x, w.key2, w.x2, w.c, fkey, fx, fc, t, counts);
  k_final_sort<<<blocks_for(t, 256, 1024), 256, 0, st>>>(
      fkey, fx, fc, counts, t, n, bmax, s, (PairOut*)out, n_out);
  return hipGetLastError();
}

}  // namespace mad
