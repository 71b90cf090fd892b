// tables.hip -- preprocessing of Alg. 2 (line "dw") on the GPU: FP64 norms
// and stage weights, integer quanta from the normalised cumulative sums
// (Sec. 3.3 "Preprocessing", Sec. 5.2), and alias tables (the alias method
// named in Sec. 5.1) built in parallel.
//
// Quanta.  A table of N items with FP64 weights w_r gets L = ceil(log2 N),
// K = L + 31 and the integer CDF F_r = floor(2^K * P_r / T), where P_r is
// the two-level prefix of mad_common.hpp and T = P_{N-1}; q_r = F_r -
// F_{r-1}.  q sums to exactly 2^K and is zero for zero weights.
//
// Alias construction.  Slots of capacity C = 2^31; light slots (q < C) and
// heavy slots (q >= C) are each taken in index order, and the result equals
// the sequential sweep "the current heavy slot fills each light slot in
// turn; once its residual drops below C it is closed as a light slot and
// the next heavy slot takes over".  With D_l the deficit (C - q) of the
// lights before light l and E_h the excess (q - C) of heavies up to and
// including heavy h, that sweep gives in closed form
//   light l : thr = q_l, alias = first heavy h with E_h >= D_l,
//   heavy h : with l* the first light whose inclusive deficit exceeds E_h,
//             thr = E_h + C - (D_l* + C - q_l*), alias = the next heavy;
//             no such l* means the slot is full (thr = 0, alias = itself).
// Both are a prefix sum plus a binary search per slot, i.e. exact integer
// work that any parallel schedule reproduces bit for bit (the
// prefix-sum formulation of the sweep follows Huebschle-Schneider and
// Sanders, "Parallel Weighted Random Sampling", ACM TOMS 2022).
#include "mad_common.hpp"
#include "plan.hpp"

namespace mad {

// ---------------------------------------------------------------------------
// weight and sign functors: seg = table index, r = item position
// ---------------------------------------------------------------------------
struct WColAbs {  // table per coordinate k over vectors r: |X[r][k]| * scale_r
  const float* X;
  int64_t d;
  const double* scale;
  __device__ double operator()(int64_t seg, int64_t r) const {
    const double w = fabs((double)X[r * d + seg]);
    return scale ? w * scale[r] : w;
  }
};

struct WRowAbs {  // table per vector i over coordinates r: |X[i][r]|
  const float* X;
  int64_t d;
  __device__ double operator()(int64_t seg, int64_t r) const {
    return fabs((double)X[seg * d + r]);
  }
};

struct WExplicit {  // one table over explicit FP64 weights
  const double* w;
  __device__ double operator()(int64_t, int64_t r) const { return w[r]; }
};

struct SignCol {
  const float* X;
  int64_t d;
  __device__ uint32_t operator()(int64_t seg, int64_t r) const {
    return sign_bit(X[r * d + seg]);
  }
};

struct SignRow {
  const float* X;
  int64_t d;
  __device__ uint32_t operator()(int64_t seg, int64_t r) const {
    return sign_bit(X[seg * d + r]);
  }
};

struct SignNone {
  __device__ uint32_t operator()(int64_t, int64_t) const { return 0u; }
};

static inline int ceil_log2_host(int64_t N) {
  int L = 0;
  while ((int64_t(1) << L) < N) ++L;
  return L;
}

static inline unsigned grid_for(int64_t n, int block) {
  int64_t g = (n + block - 1) / block;
  return (unsigned)(g < 1 ? 1 : g);
}

// ---------------------------------------------------------------------------
// small utility kernels
// ---------------------------------------------------------------------------
__global__ void k_fill_u64(uint64_t* p, int64_t n, uint64_t v) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += stride)
    p[e] = v;
}

hipError_t launch_fill_u64(uint64_t* p, int64_t n, uint64_t v,
                           hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int64_t blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  k_fill_u64<<<(unsigned)blocks, 256, 0, st>>>(p, n, v);
  return hipGetLastError();
}

// max |x| (as float bits, atomically) and a flag for non-finite entries
__global__ void k_scan_inputs(const float* X, int64_t n, float* amax,
                              int* bad) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  float mx = 0.0f;
  int nonfinite = 0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += stride) {
    const float v = X[e];
    nonfinite |= !isfinite(v);
    mx = fmaxf(mx, fabsf(v));
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    mx = fmaxf(mx, __shfl_xor(mx, off, 64));
    nonfinite |= __shfl_xor(nonfinite, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    if (amax && !nonfinite) atomicMax((unsigned int*)amax, __float_as_uint(mx));
    if (nonfinite) atomicOr(bad, 1);
  }
}

__global__ void k_stage0_weights(const double* nb, const double* v,
                                 int64_t d, double* om) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < d) om[k] = nb[k] * v[k];
}

// ---------------------------------------------------------------------------
// two-level sums and quanta for S equal tables of N items (R runs each)
// thread t handles run c = t / S of table seg = t % S
// ---------------------------------------------------------------------------
template <class W>
__global__ void k_run_sums(W w, int64_t S, int64_t N, int64_t R,
                           double* Ssum) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= S * R) return;
  const int64_t seg = t % S, c = t / S;
  const int64_t r0 = c * kRun;
  const int64_t r1 = N < r0 + kRun ? N : r0 + kRun;
  double l = w(seg, r0);
#pragma unroll 8
  for (int64_t r = r0 + 1; r < r1; ++r) l = l + w(seg, r);
  Ssum[c * S + seg] = l;
}

__global__ void k_run_offsets(const double* Ssum, int64_t S, int64_t R,
                              double* E, double* tot) {
  const int64_t seg = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (seg >= S) return;
  double e = 0.0;
  for (int64_t c = 0; c < R; ++c) {
    E[c * S + seg] = e;
    e = e + Ssum[c * S + seg];
  }
  tot[seg] = e;
}

template <class W>
__global__ void k_quantize(W w, int64_t S, int64_t N, int64_t R, int L,
                           const double* E, const double* tot, uint64_t* q) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= S * R) return;
  const int64_t seg = t % S, c = t / S;
  const double T = tot[seg];
  if (!(T > 0.0)) return;  // dead table: quanta stay zero
  const int K = L + kCapBits;
  const double e = E[c * S + seg];
  const int64_t r0 = c * kRun;
  const int64_t r1 = N < r0 + kRun ? N : r0 + kRun;
  // the prefix before this run is exactly E_c (end of the previous run)
  uint64_t Fprev = c == 0 ? 0ull : (uint64_t)floor(ldexp(e / T, K));
  uint64_t* qs = q + (seg << L);
  double l = 0.0;
  for (int64_t r = r0; r < r1; ++r) {
    const double wr = w(seg, r);
    l = r == r0 ? wr : l + wr;
    const double P = e + l;
    const uint64_t F = (uint64_t)floor(ldexp(P / T, K));
    qs[r] = F - Fprev;
    Fprev = F;
  }
}

template <class W>
static hipError_t uniform_quanta(W w, int64_t S, int64_t N, int L,
                                 double* tot, uint64_t* q, double* runbuf,
                                 hipStream_t st) {
  const int64_t R = (N + kRun - 1) / kRun;
  double* Ssum = runbuf;          // R * S
  double* E = runbuf + R * S;     // R * S
  hipError_t e = launch_fill_u64(q, S << L, 0ull, st);
  if (e != hipSuccess) return e;
  k_run_sums<W><<<grid_for(S * R, 256), 256, 0, st>>>(w, S, N, R, Ssum);
  k_run_offsets<<<grid_for(S, 256), 256, 0, st>>>(Ssum, S, R, E, tot);
  k_quantize<W><<<grid_for(S * R, 256), 256, 0, st>>>(w, S, N, R, L, E, tot,
                                                        q);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// alias construction, one wave per table (2^L <= 64 * SPL <= 512 slots;
// 4 tables per block use at most 40 KB of LDS)
// ---------------------------------------------------------------------------
template <int SPL, class Sign>
__global__ __launch_bounds__(256) void k_alias_wave(const uint64_t* q,
                                                    const double* tot,
                                                    int64_t S, int64_t N,
                                                    int L, Sign sign,
                                                    uint64_t* ent) {
  extern __shared__ uint64_t smem64[];
  const int Np = 1 << L;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t seg = (int64_t)blockIdx.x * 4 + wv;
  const bool active = seg < S && tot[seg < S ? seg : 0] > 0.0;
  uint64_t* Ld = smem64 + (int64_t)wv * 2 * Np;  // inclusive light deficits
  uint64_t* He = Ld + Np;                         // inclusive heavy excesses
  uint32_t* Hi = (uint32_t*)(smem64 + 8 * Np) + (int64_t)wv * Np;  // heavy ids

  uint64_t qv[SPL];
  uint32_t nl = 0, nh = 0;
  uint64_t sd = 0, se = 0;
#pragma unroll
  for (int s = 0; s < SPL; ++s) {
    const int r = lane * SPL + s;
    const bool ok = active && r < Np;
    qv[s] = ok ? q[(seg << L) + r] : 0ull;
    if (ok) {
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
        Hi[hp] = (uint32_t)r;
        mypos[s] = hp++;
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int s = 0; s < SPL; ++s) {
    const int r = lane * SPL + s;
    if (!(active && r < Np)) continue;
    const uint32_t sg = r < N ? sign(seg, r) : 0u;
    uint64_t e;
    if (qv[s] < kCap) {
      const uint64_t Dx = Ld[mypos[s]] - (kCap - qv[s]);
      uint32_t lo = 0, hi = NH;
      while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (He[mid] >= Dx) hi = mid; else lo = mid + 1;
      }
      const uint32_t a = NH ? Hi[lo < NH ? lo : NH - 1] : (uint32_t)r;
      e = pack_entry((uint32_t)qv[s], sg, a, sign(seg, a));
    } else {
      const uint64_t Eh = He[mypos[s]];
      uint32_t lo = 0, hi = NL;
      while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (Ld[mid] > Eh) hi = mid; else lo = mid + 1;
      }
      if (lo < NL && mypos[s] + 1 < NH) {
        const uint32_t a = Hi[mypos[s] + 1];
        e = pack_entry((uint32_t)(Eh + kCap - Ld[lo]), sg, a, sign(seg, a));
      } else {
        e = pack_entry(0u, sg, (uint32_t)r, sg);
      }
    }
    ent[(seg << L) + r] = e;
  }
}

template <class Sign>
static hipError_t alias_small(const uint64_t* q, const double* tot, int64_t S,
                              int64_t N, int L, Sign sign, uint64_t* ent,
                              hipStream_t st) {
  const int Np = 1 << L;
  const size_t lds = (size_t)4 * Np * 20;
  const unsigned blocks = grid_for(S, 4);
  if (Np <= 64)
    k_alias_wave<1, Sign><<<blocks, 256, lds, st>>>(q, tot, S, N, L, sign, ent);
  else if (Np <= 128)
    k_alias_wave<2, Sign><<<blocks, 256, lds, st>>>(q, tot, S, N, L, sign, ent);
  else if (Np <= 256)
    k_alias_wave<4, Sign><<<blocks, 256, lds, st>>>(q, tot, S, N, L, sign, ent);
  else
    k_alias_wave<8, Sign><<<blocks, 256, lds, st>>>(q, tot, S, N, L, sign, ent);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// alias construction for large tables (2^L >= 1024 slots): blocks of 1024
// slots (256 threads x 4) never straddle a table.
// ---------------------------------------------------------------------------
constexpr int kAliasBlk = 1024;

struct Quad {
  uint64_t nl, nh, sd, se;
};

__device__ __forceinline__ void slot_stats(uint64_t q, Quad& a) {
  if (q < kCap) { a.nl += 1; a.sd += kCap - q; }
  else { a.nh += 1; a.se += q - kCap; }
}

// block-wide exclusive scan of a Quad (256 threads); returns the block total
__device__ Quad block_excl_scan(Quad& v) {
  __shared__ Quad wtot[4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  Quad inc{wave_incl_scan(v.nl), wave_incl_scan(v.nh), wave_incl_scan(v.sd),
           wave_incl_scan(v.se)};
  if (lane == 63) wtot[wv] = inc;
  __syncthreads();
  Quad off{0, 0, 0, 0}, all{0, 0, 0, 0};
  for (int w = 0; w < 4; ++w) {
    if (w < wv) {
      off.nl += wtot[w].nl; off.nh += wtot[w].nh;
      off.sd += wtot[w].sd; off.se += wtot[w].se;
    }
    all.nl += wtot[w].nl; all.nh += wtot[w].nh;
    all.sd += wtot[w].sd; all.se += wtot[w].se;
  }
  __syncthreads();
  v = Quad{off.nl + inc.nl - v.nl, off.nh + inc.nh - v.nh,
           off.sd + inc.sd - v.sd, off.se + inc.se - v.se};
  return all;
}

__global__ __launch_bounds__(256) void k_alias_blocksum(const uint64_t* q,
                                                        Quad* bs) {
  const int64_t base = (int64_t)blockIdx.x * kAliasBlk + threadIdx.x * 4;
  Quad a{0, 0, 0, 0};
#pragma unroll
  for (int s = 0; s < 4; ++s) slot_stats(q[base + s], a);
  Quad all = block_excl_scan(a);
  if (threadIdx.x == 0) bs[blockIdx.x] = all;
}

// per table: exclusive scan of its block sums, and its light/heavy counts
__global__ void k_alias_blockscan(Quad* bs, int64_t S, int64_t B,
                                  uint64_t* NL, uint64_t* NH) {
  const int64_t seg = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (seg >= S) return;
  Quad acc{0, 0, 0, 0};
  for (int64_t b = seg * B; b < (seg + 1) * B; ++b) {
    const Quad v = bs[b];
    bs[b] = acc;
    acc.nl += v.nl; acc.nh += v.nh; acc.sd += v.sd; acc.se += v.se;
  }
  NL[seg] = acc.nl;
  NH[seg] = acc.nh;
}

// scatter light inclusive deficits (Ld) and heavy inclusive excesses/ids
// (He/Hi) into per-table lists; pos[slot] = rank among lights or heavies
__global__ __launch_bounds__(256) void k_alias_scatter(
    const uint64_t* q, const Quad* bo, int L, uint64_t* Ld, uint64_t* He,
    uint32_t* Hi, uint32_t* pos) {
  const int64_t base = (int64_t)blockIdx.x * kAliasBlk + threadIdx.x * 4;
  const int64_t tb = (base >> L) << L;  // first slot of the table
  uint64_t qv[4];
  Quad a{0, 0, 0, 0};
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    qv[s] = q[base + s];
    slot_stats(qv[s], a);
  }
  (void)block_excl_scan(a);
  const Quad o = bo[blockIdx.x];
  uint64_t lp = o.nl + a.nl, hp = o.nh + a.nh;
  uint64_t da = o.sd + a.sd, ea = o.se + a.se;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int64_t slot = base + s;
    if (qv[s] < kCap) {
      da += kCap - qv[s];
      Ld[tb + lp] = da;
      pos[slot] = (uint32_t)lp++;
    } else {
      ea += qv[s] - kCap;
      He[tb + hp] = ea;
      Hi[tb + hp] = (uint32_t)(slot - tb);
      pos[slot] = (uint32_t)hp++;
    }
  }
}

template <class Sign>
__global__ void k_alias_resolve(const uint64_t* q, const uint64_t* Ld,
                                const uint64_t* He, const uint32_t* Hi,
                                const uint32_t* pos, const uint64_t* NLa,
                                const uint64_t* NHa, const double* tot,
                                int64_t seg0, int64_t nslots, int L,
                                int64_t N, Sign sign, uint64_t* ent) {
  const int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (slot >= nslots) return;
  const int64_t segl = slot >> L;  // table index within the batch
  const int64_t seg = seg0 + segl;
  if (!(tot[seg] > 0.0)) return;
  const int64_t tb = segl << L;
  const uint32_t r = (uint32_t)(slot - tb);
  const uint64_t NL = NLa[segl], NH = NHa[segl];
  const uint64_t qv = q[slot];
  const uint32_t sg = (int64_t)r < N ? sign(seg, r) : 0u;
  const uint32_t p = pos[slot];
  uint64_t e;
  if (qv < kCap) {
    const uint64_t Dx = Ld[tb + p] - (kCap - qv);
    uint64_t lo = 0, hi = NH;
    while (lo < hi) {
      const uint64_t mid = (lo + hi) >> 1;
      if (He[tb + mid] >= Dx) hi = mid; else lo = mid + 1;
    }
    const uint32_t a = NH ? Hi[tb + (lo < NH ? lo : NH - 1)] : r;
    e = pack_entry((uint32_t)qv, sg, a, sign(seg, a));
  } else {
    const uint64_t Eh = He[tb + p];
    uint64_t lo = 0, hi = NL;
    while (lo < hi) {
      const uint64_t mid = (lo + hi) >> 1;
      if (Ld[tb + mid] > Eh) hi = mid; else lo = mid + 1;
    }
    if (lo < NL && (uint64_t)p + 1 < NH) {
      const uint32_t a = Hi[tb + p + 1];
      e = pack_entry((uint32_t)(Eh + kCap - Ld[tb + lo]), sg, a, sign(seg, a));
    } else {
      e = pack_entry(0u, sg, r, sg);
    }
  }
  ent[(seg0 << L) + slot] = e;
}

// scratch layout for a batch of `slots` slots and `tables` tables
static size_t alias_scratch_bytes(int64_t slots, int64_t tables) {
  return (size_t)slots * (8 + 8 + 4 + 4) + (size_t)(slots / kAliasBlk) *
         sizeof(Quad) + (size_t)tables * 16 + 256;
}

template <class Sign>
static hipError_t alias_large(const uint64_t* q, const double* tot, int64_t S,
                              int64_t N, int L, Sign sign, uint64_t* ent,
                              void* scratch, size_t scratch_bytes,
                              hipStream_t st) {
  const int64_t Np = int64_t(1) << L;
  int64_t per = (int64_t)(scratch_bytes / (alias_scratch_bytes(Np, 1)));
  if (per < 1) return hipErrorOutOfMemory;
  for (int64_t s0 = 0; s0 < S; s0 += per) {
    const int64_t ns = S - s0 < per ? S - s0 : per;
    const int64_t slots = ns * Np;
    const int64_t nblk = slots / kAliasBlk;
    char* p = (char*)scratch;
    uint64_t* Ld = (uint64_t*)p; p += slots * 8;
    uint64_t* He = (uint64_t*)p; p += slots * 8;
    uint32_t* Hi = (uint32_t*)p; p += slots * 4;
    uint32_t* pos = (uint32_t*)p; p += slots * 4;
    Quad* bs = (Quad*)p; p += nblk * sizeof(Quad);
    uint64_t* NL = (uint64_t*)p; p += ns * 8;
    uint64_t* NH = (uint64_t*)p;
    const uint64_t* qb = q + (s0 << L);
    k_alias_blocksum<<<(unsigned)nblk, 256, 0, st>>>(qb, bs);
    k_alias_blockscan<<<grid_for(ns, 64), 64, 0, st>>>(bs, ns, Np / kAliasBlk,
                                                       NL, NH);
    k_alias_scatter<<<(unsigned)nblk, 256, 0, st>>>(qb, bs, L, Ld, He, Hi, pos);
    k_alias_resolve<Sign><<<grid_for(slots, 256), 256, 0, st>>>(
        qb, Ld, He, Hi, pos, NL, NH, tot, s0, slots, L, N, sign, ent);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <class Sign>
static hipError_t build_alias(const uint64_t* q, const double* tot, int64_t S,
                              int64_t N, int L, Sign sign, uint64_t* ent,
                              void* scratch, size_t scratch_bytes,
                              hipStream_t st) {
  hipError_t e = launch_fill_u64(ent, S << L, 0ull, st);
  if (e != hipSuccess) return e;
  if (L <= 9) return alias_small(q, tot, S, N, L, sign, ent, st);
  return alias_large(q, tot, S, N, L, sign, ent, scratch, scratch_bytes, st);
}

// ---------------------------------------------------------------------------
// dense plan tables
// ---------------------------------------------------------------------------
hipError_t dev_alloc(DeviceBuffer& b, size_t bytes) {
  if (b.bytes >= bytes && b.p) return hipSuccess;
  dev_free(b);
  if (bytes == 0) return hipSuccess;
  hipError_t e = hipMalloc(&b.p, bytes);
  if (e != hipSuccess) {
    b.p = nullptr;
    b.bytes = 0;
    return e;
  }
  b.bytes = bytes;
  return hipSuccess;
}

void dev_free(DeviceBuffer& b) {
  if (b.p) (void)hipFree(b.p);
  b.p = nullptr;
  b.bytes = 0;
}

static hipError_t family_alloc(Family& f, int64_t S, int64_t N) {
  f.S = S;
  f.N = N;
  f.L = ceil_log2_host(N);
  hipError_t e = hipMalloc(&f.ent, sizeof(uint64_t) * (size_t)(S << f.L));
  if (e != hipSuccess) return e;
  return hipMalloc(&f.tot, sizeof(double) * (size_t)S);
}

static void family_free(Family& f) {
  if (f.ent) (void)hipFree(f.ent);
  if (f.tot) (void)hipFree(f.tot);
  f.ent = nullptr;
  f.tot = nullptr;
}

hipError_t dense_tables_alloc(DenseTables& t, int64_t m, int64_t n,
                              int64_t d) {
  t.m = m;
  t.n = n;
  t.d = d;
  hipError_t e;
  if ((e = family_alloc(t.T0, 1, d)) != hipSuccess) return e;
  if ((e = family_alloc(t.T1, d, m)) != hipSuccess) return e;
  if ((e = family_alloc(t.T2, d, n)) != hipSuccess) return e;
  if ((e = family_alloc(t.T3, m, d)) != hipSuccess) return e;
  t.na = t.T3.tot;
  t.v = t.T1.tot;
  t.nb = t.T2.tot;
  if ((e = hipMalloc(&t.om, sizeof(double) * (size_t)d)) != hipSuccess)
    return e;
  if ((e = hipMalloc(&t.bmax, 256)) != hipSuccess) return e;
  return hipMalloc(&t.bad, 256);
}

void dense_tables_free(DenseTables& t) {
  family_free(t.T0);
  family_free(t.T1);
  family_free(t.T2);
  family_free(t.T3);
  if (t.om) (void)hipFree(t.om);
  if (t.bmax) (void)hipFree(t.bmax);
  if (t.bad) (void)hipFree(t.bad);
  t.om = nullptr;
  t.bmax = nullptr;
  t.bad = nullptr;
}

// scratch: quanta of the largest family, run sums, alias lists
struct BuildBuffers {
  uint64_t* q;
  double* runs;
  void* alias;
  size_t alias_bytes;
};

static size_t run_doubles(int64_t S, int64_t N) {
  const int64_t R = (N + kRun - 1) / kRun;
  return (size_t)(2 * R * S);
}

hipError_t dense_tables_build(DenseTables& t, const float* A, const float* B,
                              bool check, DeviceBuffer& scratch_buf,
                              hipStream_t st) {
  const int64_t m = t.m, n = t.n, d = t.d;
  // scratch sizes
  size_t qslots = 0, runs = 0;
  const Family* fams[4] = {&t.T0, &t.T1, &t.T2, &t.T3};
  for (const Family* f : fams) {
    const size_t s = (size_t)(f->S << f->L);
    if (s > qslots) qslots = s;
    const size_t r = run_doubles(f->S, f->N);
    if (r > runs) runs = r;
  }
  // alias lists for large families, batched to at most 2^26 slots
  size_t alias_slots = 0;
  for (const Family* f : fams)
    if (f->L > 9) {
      size_t s = (size_t)(f->S << f->L);
      if (s > alias_slots) alias_slots = s;
    }
  if (alias_slots > ((size_t)1 << 26)) alias_slots = (size_t)1 << 26;
  for (const Family* f : fams)  // at least one table per batch
    if (f->L > 9 && alias_slots < ((size_t)1 << f->L))
      alias_slots = (size_t)1 << f->L;
  const size_t alias_bytes =
      alias_slots ? alias_scratch_bytes((int64_t)alias_slots,
                                        (int64_t)alias_slots / kAliasBlk) : 0;
  const size_t total = qslots * 8 + runs * 8 + alias_bytes + 1024;
  hipError_t e = dev_alloc(scratch_buf, total);
  if (e != hipSuccess) return e;
  char* scratch = (char*)scratch_buf.p;
  uint64_t* q = (uint64_t*)scratch;
  double* runbuf = (double*)(scratch + qslots * 8);
  void* abuf = scratch + qslots * 8 + runs * 8;

  if ((e = launch_fill_u64((uint64_t*)t.bmax, 1, 0ull, st)) != hipSuccess ||
      (e = launch_fill_u64((uint64_t*)t.bad, 1, 0ull, st)) != hipSuccess)
    return e;
  if (check)
    k_scan_inputs<<<grid_for(m * d, 256) > 4096 ? 4096 : grid_for(m * d, 256),
                    256, 0, st>>>(A, m * d, nullptr, t.bad);
  k_scan_inputs<<<grid_for(n * d, 256) > 4096 ? 4096 : grid_for(n * d, 256),
                  256, 0, st>>>(B, n * d, t.bmax, t.bad);

  // T3[i]: k' given i, weight |a_k'i|; totals na_i (Alg. 2 line "ds3")
  e = uniform_quanta(WRowAbs{A, d}, m, d, t.T3.L, t.T3.tot, q, runbuf, st);
  if (e == hipSuccess)
    e = build_alias(q, t.T3.tot, m, d, t.T3.L, SignRow{A, d}, t.T3.ent, abuf,
                    alias_bytes, st);
  // T1[k]: i given k, weight |a_ki| na_i; totals v_k
  if (e == hipSuccess)
    e = uniform_quanta(WColAbs{A, d, t.na}, d, m, t.T1.L, t.T1.tot, q, runbuf,
                       st);
  if (e == hipSuccess)
    e = build_alias(q, t.T1.tot, d, m, t.T1.L, SignCol{A, d}, t.T1.ent, abuf,
                    alias_bytes, st);
  // T2[k]: j given k, weight |b_kj|; totals nb_k (Alg. 2 line "ds2")
  if (e == hipSuccess)
    e = uniform_quanta(WColAbs{B, d, nullptr}, d, n, t.T2.L, t.T2.tot, q,
                       runbuf, st);
  if (e == hipSuccess)
    e = build_alias(q, t.T2.tot, d, n, t.T2.L, SignCol{B, d}, t.T2.ent, abuf,
                    alias_bytes, st);
  // T0: k with weight nb_k v_k; total ||W||_1 (Alg. 2 lines "dw", "ds1")
  if (e == hipSuccess) {
    k_stage0_weights<<<grid_for(d, 256), 256, 0, st>>>(t.nb, t.v, d, t.om);
    e = uniform_quanta(WExplicit{t.om}, 1, d, t.T0.L, t.T0.tot, q, runbuf, st);
  }
  if (e == hipSuccess)
    e = build_alias(q, t.T0.tot, 1, d, t.T0.L, SignNone{}, t.T0.ent, abuf,
                    alias_bytes, st);
  return e;
}

}  // namespace mad
