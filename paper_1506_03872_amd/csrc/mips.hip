// mips.hip -- batched maximum inner product search (MIPS) with diamond
// sampling.
//
// A MIPS query is the MAD problem with a single vector on the B side
// (Sec. 2: a one-column matrix gives MIPS; Sec. 6 runs Alg. 3 once per
// query column).  Query q with budget s_q is exactly the general plan with
// B = {q}: the database tables T1 (i given k) and T3 (k' given i) are shared,
// stage 0 draws k with weight |q_k| v_k from the query's own table, the j
// draw of a one-vector B always returns 0 (its random word is still
// consumed, so sample l of query q uses the Philox block with counter
// (l, q, 0, 0) as in the general plan), the sign of b_kj is the sign of
// q_k, and the fourth edge is q_k'.  Scores are keyed by i alone.
//
// Each query's scores live in an open-addressing table of 64-bit slots
// that hold the key i + 1 in the low kb bits (kb = bits of m) and x in the
// high 64 - kb bits, two's complement: adding inc << kb to a slot never
// changes its key bits, and x stays exact as long as it fits in 64 - kb
// bits, which the exponent F = (general F) - kb guarantees (s_q increments
// of at most max|q| 2^F sum to at most 2^(62 - kb)).  A new key costs one
// compare-and-swap that writes key and first increment together, instead
// of a swap on a key array followed by an add on a value array.
//
// Three launches serve a whole batch of queries with uneven budgets:
//   k_mips_query_info   per query: fixed-point exponent, finiteness;
//   k_sample_mips       persistent: workgroups walk a list of sample chunks
//                       (contiguous l ranges of one query), with the query
//                       row and its stage-0 table staged in LDS;
//   k_mips_post         one workgroup per query (largest budgets first):
//                       Alg. 2 on the query's score table -- keys with
//                       x > 0, the t'_q largest (ties by i), fp32 dot
//                       products, the t largest |c| (ties by i), in order.
#include "mad_common.hpp"
#include "plan.hpp"

namespace mad {

constexpr int kPostThreads = 1024;
constexpr int kPostWaves = kPostThreads / 64;
constexpr int kSelBinsM = 2048;
constexpr int kSelDigit = 11;
constexpr int kMaxOutT = 1024;  // t per query
constexpr int kFinCap = 2048;   // final selection list in LDS

// ---------------------------------------------------------------------------
// per query: F from max |q_k| and s_q; live = all entries finite
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_mips_query_info(const float* Q,
                                                         int64_t nq,
                                                         int64_t d, int kb,
                                                         MipsQuery* qi) {
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t q = (int64_t)blockIdx.x * 4 + wv;
  if (q >= nq) return;
  float mx = 0.0f;
  int nonfinite = 0;
  for (int64_t k = lane; k < d; k += 64) {
    const float v = Q[q * d + k];
    nonfinite |= !isfinite(v);
    mx = fmaxf(mx, fabsf(v));
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    mx = fmaxf(mx, __shfl_xor(mx, off, 64));
    nonfinite |= __shfl_xor(nonfinite, off, 64);
  }
  if (lane == 0) {
    qi[q].F = fix_exponent(mx, qi[q].s) - kb;  // x shares a slot with i
    qi[q].live = nonfinite ? 0 : 1;
  }
}

hipError_t launch_mips_query_info(const float* Q, int64_t nq, int64_t d,
                                  int kb, MipsQuery* qi, hipStream_t st) {
  if (nq <= 0) return hipSuccess;
  k_mips_query_info<<<(unsigned)((nq + 3) / 4), 256, 0, st>>>(Q, nq, d, kb,
                                                              qi);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// sampling: a persistent grid over the chunk list
// ---------------------------------------------------------------------------
size_t mips_sample_lds_bytes(int L0, int64_t d) {
  return ((size_t)8 << L0) + (size_t)4 * (size_t)d;
}

template <int U>
__global__ __launch_bounds__(256) void k_sample_mips(MipsArgs a) {
  extern __shared__ uint64_t sm[];
  const int N0 = 1 << a.L0;
  uint64_t* t0s = sm;
  float* qs = (float*)(sm + N0);
  unsigned long long nclosed = 0, ncreated = 0;
  for (int64_t c = blockIdx.x; c < a.nchunks; c += gridDim.x) {
    const MipsChunk ch = a.chunks[c];
    const MipsQuery qi = a.qi[ch.q];
    if (!qi.live || !(a.t0tot[ch.q] > 0.0)) continue;  // uniform per block
    __syncthreads();  // the previous chunk is done with the LDS copies
    const uint64_t* t0g = a.T0q + ((int64_t)ch.q << a.L0);
    for (int e = threadIdx.x; e < N0; e += blockDim.x) t0s[e] = t0g[e];
    for (int64_t k = threadIdx.x; k < a.d; k += blockDim.x)
      qs[k] = a.Q[(int64_t)ch.q * a.d + k];
    __syncthreads();
    unsigned long long* hs = (unsigned long long*)(a.hslot + qi.hoff);
    const uint32_t hmask = qi.hmask;
    const int kb = a.kb;
    const uint64_t kmask = (1ull << kb) - 1;
    for (int base = threadIdx.x; base < ch.count; base += 256 * U) {
      uint32_t key[U], slot[U];
      int64_t inc[U];
      bool closed[U];
      uint64_t e1[U], e3[U], U1[U], U3[U];
      uint32_t sg[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int e = base + u * 256;
        const uint64_t l = (uint64_t)(ch.l0 + (e < ch.count ? e : 0));
        const Philox4 r = philox4x64_10(l, (uint64_t)ch.q, 0ull, 0ull,
                                        a.seed, 0ull);
        const uint32_t s0 = slot_of(r.w0, a.L0);
        const uint32_t k = draw_entry(t0s[s0], s0, r.w0).pos;
        U1[u] = r.w1;
        U3[u] = r.w3;
        sg[u] = sign_bit(qs[k]);  // b_kj of the one-vector B is q_k
        e1[u] = a.T1[((uint64_t)k << a.L1) + slot_of(r.w1, a.L1)];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const Drawn di = draw_entry(e1[u], slot_of(U1[u], a.L1), U1[u]);
        key[u] = di.pos;
        sg[u] ^= di.sgn;
        e3[u] = a.T3[((uint64_t)di.pos << a.L3) + slot_of(U3[u], a.L3)];
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const Drawn dk = draw_entry(e3[u], slot_of(U3[u], a.L3), U3[u]);
        const float v = qs[dk.pos];
        sg[u] ^= dk.sgn;
        closed[u] = base + u * 256 < ch.count && v != 0.0f;
        inc[u] = 0;
        if (closed[u]) {
          const int64_t mag = (int64_t)rint(ldexp((double)v, qi.F));
          inc[u] = sg[u] ? -mag : mag;
        }
        slot[u] = (uint32_t)mix64(key[u]) & hmask;
        nclosed += closed[u];
      }
      // claim an empty slot with key and increment in one swap; a slot
      // that already holds the key takes the increment by an add
      bool pend[U], add[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        pend[u] = closed[u];
        add[u] = false;
      }
      bool any = true;
      while (any) {
        unsigned long long prev[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
          prev[u] = pend[u] ? atomicCAS(hs + slot[u], 0ull,
                                        ((uint64_t)inc[u] << kb) |
                                            ((uint64_t)key[u] + 1))
                            : 0ull;
        any = false;
#pragma unroll
        for (int u = 0; u < U; ++u) {
          if (!pend[u]) continue;
          if (prev[u] == 0ull) {
            ++ncreated;
            pend[u] = false;
          } else if ((prev[u] & kmask) == (uint64_t)key[u] + 1) {
            add[u] = inc[u] != 0;
            pend[u] = false;
          } else {
            slot[u] = (slot[u] + 1) & hmask;
            any = true;
          }
        }
      }
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (add[u]) atomicAdd(hs + slot[u], (uint64_t)inc[u] << kb);
    }
  }
  __shared__ unsigned long long part[2][4];
  nclosed = wave_sum(nclosed);
  ncreated = wave_sum(ncreated);
  if ((threadIdx.x & 63) == 0) {
    part[0][threadIdx.x >> 6] = nclosed;
    part[1][threadIdx.x >> 6] = ncreated;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const unsigned long long cc = part[0][0] + part[0][1] + part[0][2] +
                                  part[0][3];
    const unsigned long long dd = part[1][0] + part[1][1] + part[1][2] +
                                  part[1][3];
    if (cc) atomicAdd(&a.ctr->closed, cc);
    if (dd) atomicAdd(&a.ctr->distinct, dd);
  }
}

hipError_t launch_sample_mips(const MipsArgs& a, int unroll, int grid,
                              hipStream_t st) {
  if (a.nchunks <= 0) return hipSuccess;
  const size_t lds = mips_sample_lds_bytes(a.L0, a.d);
  int64_t g = grid < a.nchunks ? grid : a.nchunks;
  if (g < 1) g = 1;
  switch (unroll) {
    case 1: k_sample_mips<1><<<(unsigned)g, 256, lds, st>>>(a); break;
    case 2: k_sample_mips<2><<<(unsigned)g, 256, lds, st>>>(a); break;
    case 8: k_sample_mips<8><<<(unsigned)g, 256, lds, st>>>(a); break;
    default: k_sample_mips<4><<<(unsigned)g, 256, lds, st>>>(a); break;
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// postprocessing helpers (1024 threads)
// ---------------------------------------------------------------------------
struct PostShared {
  unsigned h[kSelBinsM];
  unsigned long long scan[kPostThreads];
  unsigned wcnt[kPostWaves];
  unsigned long long base;
  int chosen;
  unsigned long long before;
};

// Slot of this thread among the takers of one round of the whole block, in
// thread order, after `ps.base`; advances ps.base by the round's count.
__device__ int64_t block_take(bool take, PostShared& ps) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const uint64_t ball = __ballot(take);
  if (lane == 0) ps.wcnt[wv] = (unsigned)__popcll(ball);
  __syncthreads();
  unsigned before = 0, total = 0;
  for (int w = 0; w < kPostWaves; ++w) {
    const unsigned c = ps.wcnt[w];
    before += w < wv ? c : 0u;
    total += c;
  }
  const int64_t slot = (int64_t)ps.base + before +
                       __popcll(ball & ((1ull << lane) - 1));
  __syncthreads();
  if (threadIdx.x == 0) ps.base += total;
  __syncthreads();
  return slot;
}

// First slot of this thread's `cnt` takers among those of one round of the
// whole block, in thread order, after `ps.base`; advances ps.base by the
// round's count.
__device__ int64_t block_take_n(unsigned cnt, PostShared& ps) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const unsigned incl = wave_incl_scan(cnt);
  if (lane == 63) ps.wcnt[wv] = incl;
  __syncthreads();
  unsigned before = 0, total = 0;
  for (int w = 0; w < kPostWaves; ++w) {
    const unsigned c = ps.wcnt[w];
    before += w < wv ? c : 0u;
    total += c;
  }
  const int64_t slot = (int64_t)ps.base + before + (incl - cnt);
  __syncthreads();
  if (threadIdx.x == 0) ps.base += total;
  __syncthreads();
  return slot;
}

// Threshold of an exact selection of k of n elements by (primary desc,
// key asc): the elements taken are those with take(p, key) true.  Digits
// of kSelDigit bits, from bit `top` of the primary down, then the 32-bit
// key.  Keys are unique, so the key phase always ends the search.
struct SelThr {
  uint64_t pp, pm;
  uint32_t kp, km;
  int key_phase;
};

__device__ __forceinline__ bool sel_take(uint64_t p, uint32_t kk,
                                         const SelThr& s) {
  const uint64_t pmv = p & s.pm;
  if (pmv != s.pp) return pmv > s.pp;
  if (!s.key_phase) return true;
  return (kk & s.km) <= s.kp;
}

__device__ SelThr block_select(const uint64_t* prim, const uint32_t* key,
                               int64_t n, int64_t k, int top,
                               PostShared& ps) {
  const int t = threadIdx.x;
  SelThr s{0, 0, 0, 0, 0};
  int64_t k_rem = k;
  int shift = top - kSelDigit > 0 ? top - kSelDigit : 0;
  bool done = k_rem >= n;
  while (!done) {
    for (int b = t; b < kSelBinsM; b += kPostThreads) ps.h[b] = 0;
    __syncthreads();
    for (int64_t e = t; e < n; e += kPostThreads) {
      const uint64_t p = prim[e];
      if ((p & s.pm) != s.pp) continue;
      if (!s.key_phase) {
        atomicAdd(&ps.h[(p >> shift) & (kSelBinsM - 1)], 1u);
      } else {
        const uint32_t kk = key[e];
        if ((kk & s.km) != s.kp) continue;
        atomicAdd(&ps.h[(kk >> shift) & (kSelBinsM - 1)], 1u);
      }
    }
    __syncthreads();
    // bins in selection order; thread t owns positions 2t, 2t + 1
    const int b0 = s.key_phase ? 2 * t : kSelBinsM - 1 - 2 * t;
    const int b1 = s.key_phase ? 2 * t + 1 : kSelBinsM - 2 - 2 * t;
    const unsigned v0 = ps.h[b0], v1 = ps.h[b1];
    ps.scan[t] = (unsigned long long)v0 + v1;
    if (t == 0) ps.chosen = -1;
    __syncthreads();
    for (int off = 1; off < kPostThreads; off <<= 1) {
      const unsigned long long o = t >= off ? ps.scan[t - off] : 0ull;
      __syncthreads();
      ps.scan[t] += o;
      __syncthreads();
    }
    const unsigned long long excl = ps.scan[t] - v0 - v1;
    if ((long long)excl < k_rem && (long long)(excl + v0) >= k_rem) {
      ps.chosen = b0;
      ps.before = excl;
    } else if ((long long)(excl + v0) < k_rem &&
               (long long)(excl + v0 + v1) >= k_rem) {
      ps.chosen = b1;
      ps.before = excl + v0;
    }
    __syncthreads();
    const int b = ps.chosen;
    const unsigned nbin = b >= 0 ? ps.h[b] : 0u;
    const unsigned long long bef = ps.before;
    __syncthreads();
    if (b < 0) break;  // cannot happen while k_rem <= matching count
    k_rem -= (int64_t)bef;
    if (!s.key_phase) {
      s.pp |= (uint64_t)b << shift;
      s.pm |= (uint64_t)(kSelBinsM - 1) << shift;
    } else {
      s.kp |= (uint32_t)b << shift;
      s.km |= (uint32_t)(kSelBinsM - 1) << shift;
    }
    if ((int64_t)nbin == k_rem) {
      done = true;
    } else if (shift == 0) {
      if (s.key_phase) done = true;
      s.key_phase = 1;
      shift = 32 - kSelDigit;
    } else {
      shift = shift > kSelDigit ? shift - kSelDigit : 0;
    }
  }
  return s;
}

// Histograms over the bits of a float >= 0 shifted right by 20 (exponent
// and three mantissa bits, kSelBinsM bins): bin(v) is monotone in v, and
// every v in bin b is at least edge(b), the float with bits b << 20.
__device__ __forceinline__ unsigned fbin(uint32_t bits) { return bits >> 20; }
__device__ __forceinline__ float fbin_edge(int b) {
  return __uint_as_float((uint32_t)b << 20);
}

// The bin b of the histogram ps.h that holds the k-th largest value: bins
// above b hold fewer than k values, bins from b up at least k.  Wave 0
// searches (32 bins per lane, from the top); ps.chosen = b (-1 when the
// histogram holds fewer than k values) and ps.before = the count in bins
// >= b.  The histogram must be complete; synchronise before reading.
__device__ void hist_kth_bin(PostShared& ps, int64_t k) {
  if (threadIdx.x >= 64) return;
  const int lane = threadIdx.x;
  const int hi = kSelBinsM - 1 - 32 * lane;
  unsigned long long sum = 0;
  for (int b = hi; b > hi - 32; --b) sum += ps.h[b];
  const unsigned long long incl = wave_incl_scan(sum);
  const uint64_t reach = __ballot((long long)incl >= k);
  if (lane == 0 && reach == 0) ps.chosen = -1;
  if (reach == 0) return;
  if (lane != __builtin_ctzll(reach)) return;
  unsigned long long acc = incl - sum;
  for (int b = hi; b > hi - 32; --b) {
    acc += ps.h[b];
    if ((long long)acc >= k) {
      ps.chosen = b;
      ps.before = acc;
      return;
    }
  }
}

// ---------------------------------------------------------------------------
// post: one workgroup per query
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(kPostThreads) void k_mips_post(MipsArgs a) {
  extern __shared__ float qs[];  // the query row (d floats)
  __shared__ PostShared ps;
  __shared__ uint32_t fk[kMaxOutT];
  __shared__ uint64_t fx[kMaxOutT];
  __shared__ float fc[kMaxOutT];
  __shared__ uint32_t lk[kFinCap];  // final-selection list: keys,
  __shared__ float lc[kFinCap];     // c,
  __shared__ int32_t le[kFinCap];   // positions in the verified arrays
  __shared__ unsigned nl;
  const int t = threadIdx.x;
  const int64_t q = a.order[blockIdx.x];
  const MipsQuery qi = a.qi[q];
  if (!qi.live || !(a.t0tot[q] > 0.0) || qi.s <= 0) {
    if (t == 0) {
      a.n_out[q] = qi.live ? 0 : -1;
      a.qstats[q].n_pos = 0;
      a.qstats[q].n_cand = 0;
      a.qstats[q].n_fp32 = 0;
    }
    return;
  }
  for (int64_t k = t; k < a.d; k += kPostThreads) qs[k] = a.Q[q * a.d + k];
  // candidate selection (Omega_s): keys with x > 0, compacted in slot order
  const uint64_t* hs = a.hslot + qi.hoff;
  const uint64_t kmask = (1ull << a.kb) - 1;
  uint64_t* cx = a.cx + qi.coff;
  uint32_t* ck = a.ck + qi.coff;
  const int64_t cap = (int64_t)qi.hmask + 1;
  if (t == 0) ps.base = 0;
  __syncthreads();
  // kScanPer consecutive slots per thread and round (the table capacity is
  // a power of two of at least 1024 slots, so rounds are whole)
  constexpr int kScanPer = 8;
  for (int64_t r0 = 0; r0 < cap; r0 += kPostThreads * kScanPer) {
    const int64_t e0 = r0 + (int64_t)t * kScanPer;
    uint64_t w[kScanPer];
    unsigned cnt = 0;
#pragma unroll
    for (int u = 0; u < kScanPer; ++u) {
      w[u] = e0 + u < cap ? hs[e0 + u] : 0ull;
      cnt += w[u] != 0ull && (int64_t)w[u] >> a.kb > 0;
    }
    int64_t pos = block_take_n(cnt, ps);
#pragma unroll
    for (int u = 0; u < kScanPer; ++u) {
      const int64_t v = (int64_t)w[u] >> a.kb;  // sign-extended x
      if (w[u] != 0ull && v > 0) {
        if (pos < qi.ccap) {
          cx[pos] = (uint64_t)v;
          ck[pos] = (uint32_t)(w[u] & kmask) - 1u;
        }
        ++pos;
      }
    }
  }
  int64_t npos = (int64_t)ps.base;
  if (npos > qi.ccap) npos = qi.ccap;  // cannot happen: distinct <= s_q, m
  // candidate selection (Omega_t'): the t'_q largest x, ties by i
  // ascending; when all are taken, the candidate arrays serve as they are
  const bool cut = npos > qi.tp;
  uint64_t* sx = cut ? a.sx + qi.soff : cx;
  uint32_t* sk = cut ? a.sk + qi.soff : ck;
  float* sc = a.sc + qi.soff;
  uint64_t* sab = a.sab + qi.soff;
  int64_t nsel = npos;
  if (cut) {
    const SelThr thr = block_select(cx, ck, npos, qi.tp, 64, ps);
    nsel = qi.tp;
    __syncthreads();
    if (t == 0) ps.base = 0;
    __syncthreads();
    for (int64_t r0 = 0; r0 < npos; r0 += kPostThreads) {
      const int64_t e = r0 + t;
      const bool live = e < npos;
      const uint64_t p = live ? cx[e] : 0;
      const uint32_t kk = live ? ck[e] : 0;
      const bool take = live && sel_take(p, kk, thr);
      const int64_t pos = block_take(take, ps);
      if (take && pos < qi.scap) {
        sx[pos] = p;
        sk[pos] = kk;
      }
    }
  }
  if (nsel > qi.scap) nsel = qi.scap;
  __syncthreads();
  const int lane = t & 63, wv = t >> 6, grp = lane >> 4, gl = lane & 15;
  const int64_t tq = a.t < nsel ? a.t : nsel;
  // low-precision screen (when the plan asks for one and more than t
  // candidates remain): c^ of every candidate from the bf16 / fp8 rows and
  // the bound mg on |c^ - c_fp32|; tau <= the t-th largest lower bound
  // |c^| - mg; only candidates with |c^| + mg >= tau are verified in fp32.
  // Every other candidate has |c_fp32| < tau <= the fp32 |c| of t others,
  // so the top t is the one the fp32 verification of all of them gives.
  // tau is the lower edge of the histogram bin that holds the t-th largest
  // lower bound (at most that bound), from a histogram the screen pass
  // fills as it goes.
  const bool screen = a.lp != 0 && nsel > tq;
  float tau = 0.0f;
  for (int b = t; b < kSelBinsM; b += kPostThreads) ps.h[b] = 0;
  __syncthreads();
  if (screen) {
    const int64_t rowb = a.Kp * (a.lp == 1 ? 2 : 1);  // bytes per row
    const uint4* qrow = (const uint4*)((const char*)a.Qlp + q * rowb);
    const VecInfo vq = a.iq[q];
    // kScrU rounds of 4 candidates per wave at once, as in verification below
    constexpr int kScrU = 4;
    const int64_t round = kPostWaves * 4;
    for (int64_t e0 = (int64_t)wv * 4; e0 < nsel; e0 += round * kScrU) {
      const uint4* arow[kScrU];
      int64_t iu[kScrU];
      float acc[kScrU];
      VecInfo va[kScrU];  // loaded with the rows, used by lane gl = 0
#pragma unroll
      for (int u = 0; u < kScrU; ++u) {
        const int64_t e = e0 + grp + u * round;
        iu[u] = (int64_t)sk[e < nsel ? e : e0];
        arow[u] = (const uint4*)((const char*)a.Alp + iu[u] * rowb);
        acc[u] = 0.0f;
        if (gl == 0) va[u] = a.ia[iu[u]];
      }
      for (int64_t c16 = gl; c16 < rowb / 16; c16 += 16) {
        const uint4 y = qrow[c16];
        uint4 x[kScrU];
#pragma unroll
        for (int u = 0; u < kScrU; ++u) x[u] = arow[u][c16];
#pragma unroll
        for (int u = 0; u < kScrU; ++u)
          acc[u] = lowp_dot16(x[u], y, a.lp, acc[u]);
      }
#pragma unroll
      for (int u = 0; u < kScrU; ++u) {
#pragma unroll
        for (int off = 8; off > 0; off >>= 1)
          acc[u] += __shfl_xor(acc[u], off, 64);
        const int64_t e = e0 + grp + u * round;
        if (e < nsel && gl == 0) {
          const float c = acc[u] * va[u].inv_s * vq.inv_s;
          const float mg = a.kappa * va[u].n2 * vq.n2 +
                           a.onepu * (va[u].eta * vq.n1 + vq.eta * va[u].n1) +
                           a.d_f * va[u].eta * vq.eta;
          const float lo = fabsf(c) - mg;
          atomicAdd(&ps.h[fbin(__float_as_uint(lo > 0.0f ? lo : 0.0f))], 1u);
          sab[e] = 0;  // |c| of the candidates verified below
          sc[e] = fabsf(c) + mg;
        }
      }
    }
    __syncthreads();
    hist_kth_bin(ps, tq);
    __syncthreads();
    tau = ps.chosen > 0 ? fbin_edge(ps.chosen) : 0.0f;
    if (t == 0) nl = 0;
    __syncthreads();
    for (int b = t; b < kSelBinsM; b += kPostThreads) ps.h[b] = 0;
    // the candidates left to verify (upper bound >= tau), listed in LDS
    for (int64_t e = t; e < nsel; e += kPostThreads)
      if (sc[e] >= tau) {
        const unsigned p = atomicAdd(&nl, 1u);
        if (p < (unsigned)kFinCap) le[p] = (int32_t)e;
      }
  }
  if (t == 0) ps.base = 0;
  __syncthreads();
  // verify the listed candidates, or (no screen, or a list that did not
  // fit) every candidate whose bound reaches tau
  const bool via_list = screen && nl <= (unsigned)kFinCap;
  const int64_t nv = via_list ? (int64_t)nl : nsel;
  // verification: c = a_i . q in fp32; 16 lanes per candidate, 4 candidates per
  // wave and kVerU rounds of them at once (their row loads in flight
  // together), rows read as float4 when d is a multiple of 4; a histogram
  // of |c| is filled as the values come
  constexpr int kVerU = 4;
  const int64_t round = kPostWaves * 4;  // candidates per block round
  const bool vec = (a.d & 3) == 0 && ((uintptr_t)a.A & 15) == 0;
  unsigned nfp = 0;
  for (int64_t r0 = (int64_t)wv * 4; r0 < nv; r0 += round * kVerU) {
    bool need[kVerU];
    int64_t ev[kVerU];
    const float* ar[kVerU];
    float acc[kVerU];
#pragma unroll
    for (int u = 0; u < kVerU; ++u) {
      const int64_t r = r0 + grp + u * round;
      ev[u] = r < nv ? (via_list ? (int64_t)le[r] : r) : 0;
      need[u] = r < nv && (via_list || !screen || sc[ev[u]] >= tau);
      ar[u] = a.A + (int64_t)sk[ev[u]] * a.d;
      acc[u] = 0.0f;
    }
    if (vec) {
      for (int64_t k = gl * 4; k < a.d; k += 64) {
        const float4 y = *(const float4*)(qs + k);
        float4 x[kVerU];
#pragma unroll
        for (int u = 0; u < kVerU; ++u)
          x[u] = need[u] ? *(const float4*)(ar[u] + k)
                         : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
#pragma unroll
        for (int u = 0; u < kVerU; ++u) {
          acc[u] = fmaf(x[u].x, y.x, acc[u]);
          acc[u] = fmaf(x[u].y, y.y, acc[u]);
          acc[u] = fmaf(x[u].z, y.z, acc[u]);
          acc[u] = fmaf(x[u].w, y.w, acc[u]);
        }
      }
    } else {
#pragma unroll
      for (int u = 0; u < kVerU; ++u)
        if (need[u])
          for (int64_t k = gl; k < a.d; k += 16)
            acc[u] = fmaf(ar[u][k], qs[k], acc[u]);
    }
#pragma unroll
    for (int u = 0; u < kVerU; ++u) {
#pragma unroll
      for (int off = 8; off > 0; off >>= 1)
        acc[u] += __shfl_xor(acc[u], off, 64);
      if (need[u] && gl == 0) {
        const int64_t e = ev[u];
        const uint32_t ab = __float_as_uint(fabsf(acc[u]));
        sc[e] = acc[u];
        sab[e] = ab;
        atomicAdd(&ps.h[fbin(ab)], 1u);
        ++nfp;
      }
    }
  }
  if (nfp) atomicAdd((unsigned long long*)&ps.base, (unsigned long long)nfp);
  __syncthreads();
  const int64_t n_fp32 = (int64_t)ps.base;
  // final selection: the t largest |c|, ties by i ascending.  The
  // histogram gives the bin b of the t-th largest |c|; the candidates of
  // bins >= b (every one verified: a screened-out candidate keeps |c| = 0
  // and b >= 1) go to an LDS list where each one's rank is counted
  // directly.  A list that would not fit, or b = 0, takes the digit
  // selection over all candidates instead.
  const bool cut3 = nsel > tq;
  bool listed = false;
  if (cut3) {
    hist_kth_bin(ps, tq);
    if (t == 0) nl = 0;
    __syncthreads();
    const int b3 = ps.chosen;
    listed = b3 >= 1 && ps.before <= (unsigned long long)kFinCap;
    __syncthreads();
    if (listed) {
      for (int64_t e = t; e < nsel; e += kPostThreads) {
        const uint32_t ab = (uint32_t)sab[e];
        if ((int)fbin(ab) >= b3) {
          const unsigned p = atomicAdd(&nl, 1u);
          lk[p] = sk[e];
          lc[p] = sc[e];
          le[p] = (int32_t)e;
        }
      }
      __syncthreads();
      const int n = (int)nl;
      for (int e = t; e < n; e += kPostThreads) {
        const uint32_t ae = __float_as_uint(fabsf(lc[e]));
        const uint32_t ke = lk[e];
        int rank = 0;
        for (int u = 0; u < n; ++u) {
          const uint32_t au = __float_as_uint(fabsf(lc[u]));
          rank += au > ae || (au == ae && lk[u] < ke);
        }
        if (rank < tq) {
          fk[rank] = ke;
          fx[rank] = sx[le[e]];
          fc[rank] = lc[e];
        }
      }
      __syncthreads();
    }
  }
  if (!listed) {
    SelThr thr3{0, 0, 0, 0, 0};
    if (cut3) thr3 = block_select(sab, sk, nsel, tq, 32, ps);
    __syncthreads();
    if (t == 0) ps.base = 0;
    __syncthreads();
    for (int64_t r0 = 0; r0 < nsel; r0 += kPostThreads) {
      const int64_t e = r0 + t;
      const bool live = e < nsel;
      const uint64_t p = live ? sab[e] : 0;
      const uint32_t kk = live ? sk[e] : 0;
      const bool take = live && (!cut3 || sel_take(p, kk, thr3));
      const int64_t pos = block_take(take, ps);
      if (take && pos < tq) {
        fk[pos] = kk;
        fx[pos] = sx[e];
        fc[pos] = sc[e];
      }
    }
    __syncthreads();
  }
  // rank order (|c| desc, i asc) and output
  struct Pair {
    int64_t i, j;
    float c, x;
  };
  Pair* o = (Pair*)a.out + q * a.t;
  for (int64_t e = t; e < tq; e += kPostThreads) {
    const float ae = fabsf(fc[e]);
    const uint32_t ke = fk[e];
    int64_t rank = 0;
    for (int64_t u = 0; u < tq; ++u) {
      const float au = fabsf(fc[u]);
      rank += au > ae || (au == ae && fk[u] < ke);
    }
    Pair pr;
    pr.i = (int64_t)ke;
    pr.j = q;
    pr.c = fc[e];
    pr.x = (float)ldexp((double)(int64_t)fx[e], -qi.F);
    o[rank] = pr;
  }
  if (t == 0) {
    a.n_out[q] = tq;
    a.qstats[q].n_pos = npos;
    a.qstats[q].n_cand = nsel;
    a.qstats[q].n_fp32 = n_fp32;
  }
}

hipError_t launch_mips_post(const MipsArgs& a, hipStream_t st) {
  if (a.nq <= 0) return hipSuccess;
  if (a.t > kMaxOutT) return hipErrorInvalidValue;
  k_mips_post<<<(unsigned)a.nq, kPostThreads, (size_t)4 * a.d, st>>>(a);
  return hipGetLastError();
}

// every key of query q's score table, for parity checks
__global__ void k_mips_dump(const uint64_t* hs, int kb, int64_t cap,
                            int64_t* keys, int64_t* xfix, int64_t out_cap,
                            int64_t* count) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const uint64_t kmask = (1ull << kb) - 1;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < cap;
       e += stride) {
    const uint64_t w = hs[e];
    if (w == 0) continue;
    const unsigned long long p = atomicAdd((unsigned long long*)count, 1ull);
    if ((int64_t)p < out_cap) {
      keys[p] = (int64_t)(w & kmask) - 1;
      xfix[p] = (int64_t)w >> kb;
    }
  }
}

hipError_t launch_mips_dump(const MipsArgs& a, int64_t q, int64_t* keys,
                            int64_t* xfix, int64_t cap, int64_t* count,
                            hipStream_t st) {
  MipsQuery qi;
  hipError_t e = hipMemcpy(&qi, a.qi + q, sizeof qi, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return e;
  if ((e = launch_fill_u64((uint64_t*)count, 1, 0ull, st)) != hipSuccess)
    return e;
  const int64_t hcap = (int64_t)qi.hmask + 1;
  int64_t blocks = (hcap + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  k_mips_dump<<<(unsigned)blocks, 256, 0, st>>>(a.hslot + qi.hoff, a.kb,
                                                hcap, keys, xfix, cap, count);
  return hipGetLastError();
}

}  // namespace mad
