// tables.hip -- preprocessing for the weights w_ki of Alg. 3 on the GPU: FP64
// norms and stage weights, integer quanta from the normalised cumulative sums
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
#include <stdlib.h>

#include "alias_common.hpp"
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
  __device__ uint32_t sgn(int64_t seg, int64_t r) const {
    return sign_bit(X[r * d + seg]);
  }
};

struct WRowAbs {  // table per vector i over coordinates r: |X[i][r]|
  const float* X;
  int64_t d;
  __device__ double operator()(int64_t seg, int64_t r) const {
    return fabs((double)X[seg * d + r]);
  }
  __device__ uint32_t sgn(int64_t seg, int64_t r) const {
    return sign_bit(X[seg * d + r]);
  }
};

struct WQuery {  // MIPS stage 0 of query seg over coordinates r: |q_r| v_r
  const float* Q;   // nq x d, row-major
  int64_t d;
  const double* v;  // d
  __device__ double operator()(int64_t seg, int64_t r) const {
    return fabs((double)Q[seg * d + r]) * v[r];
  }
  __device__ uint32_t sgn(int64_t, int64_t) const { return 0u; }
};

struct WExplicit {  // one table over explicit FP64 weights
  const double* w;
  __device__ double operator()(int64_t, int64_t r) const { return w[r]; }
  __device__ uint32_t sgn(int64_t, int64_t) const { return 0u; }
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

// up to kFillMax fills in one launch (small clears would otherwise each pay
// a launch)
__global__ void k_fill_multi(FillBatch f) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int q = 0; q < f.count; ++q) {
    for (; e < f.n[q]; e += stride) f.p[q][e] = f.v[q];
    e -= f.n[q];
  }
}

hipError_t launch_fill_multi(const FillBatch& f, hipStream_t st) {
  int64_t tot = 0;
  for (int q = 0; q < f.count; ++q) tot += f.n[q] > 0 ? f.n[q] : 0;
  if (tot <= 0) return hipSuccess;
  int64_t blocks = (tot + 255) / 256;
  if (blocks > 1024) blocks = 1024;
  k_fill_multi<<<(unsigned)blocks, 256, 0, st>>>(f);
  return hipGetLastError();
}

// max |x| (as float bits, atomically) and a flag for non-finite entries;
// float4 loads when X is 16-byte aligned
__global__ __launch_bounds__(1024) void k_scan_inputs(const float* X,
                                                     int64_t n, float* amax,
                                                     int* bad) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  float mx = 0.0f;
  int nonfinite = 0;
  int64_t done = 0;
  if (((uintptr_t)X & 15) == 0) {
    const float4* X4 = (const float4*)X;
    const int64_t n4 = n / 4;
    for (int64_t e0 = tid; e0 < n4; e0 += 4 * stride) {
      float4 v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t e = e0 + u * stride;
        v[u] = e < n4 ? X4[e] : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        nonfinite |= (int)!isfinite(v[u].x) | (int)!isfinite(v[u].y) |
                     (int)!isfinite(v[u].z) | (int)!isfinite(v[u].w);
        mx = fmaxf(mx, fmaxf(fmaxf(fabsf(v[u].x), fabsf(v[u].y)),
                             fmaxf(fabsf(v[u].z), fabsf(v[u].w))));
      }
    }
    done = n4 * 4;
  }
  for (int64_t e = done + tid; e < n; e += stride) {
    const float v = X[e];
    nonfinite |= !isfinite(v);
    mx = fmaxf(mx, fabsf(v));
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    mx = fmaxf(mx, __shfl_xor(mx, off, 64));
    nonfinite |= __shfl_xor(nonfinite, off, 64);
  }
  // one pair of atomics per block (a small grid: all blocks' atomics hit
  // the same two words)
  __shared__ float bmx[16];
  __shared__ int bnf[16];
  if ((threadIdx.x & 63) == 0) {
    bmx[threadIdx.x >> 6] = mx;
    bnf[threadIdx.x >> 6] = nonfinite;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    mx = 0.0f;
    nonfinite = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
      mx = fmaxf(mx, bmx[w]);
      nonfinite |= bnf[w];
    }
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
constexpr int kRowGroup = 16;

template <class W>
__global__ void k_run_sums(W w, int64_t S, int64_t N, int64_t R,
                           double* Ssum) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= S * R) return;
  const int64_t seg = t % S, c = t / S;
  const int64_t r0 = c * kRun;
  const int64_t r1 = N < r0 + kRun ? N : r0 + kRun;
  double l = 0.0;
  for (int64_t g0 = r0; g0 < r1; g0 += kRowGroup) {
    double v[kRowGroup];
#pragma unroll
    for (int q = 0; q < kRowGroup; ++q)
      v[q] = w(seg, g0 + q < r1 ? g0 + q : r1 - 1);
#pragma unroll
    for (int q = 0; q < kRowGroup; ++q)
      if (g0 + q < r1) l = g0 + q == r0 ? v[q] : l + v[q];
  }
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

// quanta with the item's sign bit in bit 63 (quanta are below 2^62)
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
  for (int64_t g0 = r0; g0 < r1; g0 += kRowGroup) {
    double v[kRowGroup];
    uint32_t sg[kRowGroup];
#pragma unroll
    for (int u = 0; u < kRowGroup; ++u) {
      const int64_t r = g0 + u < r1 ? g0 + u : r1 - 1;
      v[u] = w(seg, r);
      sg[u] = w.sgn(seg, r);
    }
#pragma unroll
    for (int u = 0; u < kRowGroup; ++u) {
      const int64_t r = g0 + u;
      if (r >= r1) continue;
      l = r == r0 ? v[u] : l + v[u];
      const double P = e + l;
      const uint64_t F = (uint64_t)floor(ldexp(P / T, K));
      qs[r] = (F - Fprev) | ((uint64_t)sg[u] << 63);
      Fprev = F;
    }
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
// alias construction.  Each quantum carries its item's sign bit in bit 63;
// the lists below carry it in bit 31 of the slot id.
// ---------------------------------------------------------------------------
// Small tables (N <= 2^L <= 512 items), entirely on chip, TB tables per
// 256-thread block (small_tables picks TB for the LDS budget):
//   phase 1  the block loads its tables' weights (with the sign bits in
//            bit 63; weights are >= 0) into LDS together; then lanes of wave
//            0, one per table, walk the items left to right and overwrite
//            them with the run-local prefixes l_r (sign bits kept); the
//            totals of the runs of kRun items go to LDS as well;
//   phase 2  each wave takes a table at a time: E_c and T from the run
//            totals in the two-level order (E_0 = 0, E_{c+1} = E_c + l of
//            run c's last item, T = E_R), then per slot in parallel P_r =
//            E_c + l_r (0 + l_r = l_r exactly in the first run), F_r =
//            floor(2^K P_r / T) and q_r = F_r - F_{r-1} (F of the slot
//            before a lane's first comes from the previous lane), and the
//            alias table from the quanta in registers.
// Padding slots and dead tables get q = 0.
template <int SPL, class W>
__global__ __launch_bounds__(256) void k_small_tables(W w, int64_t S,
                                                      int64_t N, int L,
                                                      int TB, double* tot,
                                                      uint64_t* ent) {
  extern __shared__ uint64_t smem64[];
  const int Np = 1 << L;
  const int ld = Np + 1;  // row stride of the prefixes (bank spread)
  const int R = (int)((N + kRun - 1) / kRun);
  uint64_t* lb = smem64;                        // TB x ld
  double* rt = (double*)(smem64 + TB * ld);     // TB x 4 run totals
  uint64_t* ascr = smem64 + TB * ld + TB * 4;   // alias scratch, 4 waves
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int K = L + kCapBits;
  uint64_t* Ld = ascr + (int64_t)wv * 2 * Np;
  uint64_t* He = Ld + Np;
  uint32_t* Hi = (uint32_t*)(ascr + 8 * Np) + (int64_t)wv * Np;
  {  // this block's chunk of TB tables
    const int64_t chunk = blockIdx.x;
    const int64_t seg0 = chunk * TB;
    // ---- phase 1 -----------------------------------------------------------
    // the block's weights and sign bits, kLoadPer loads per thread in
    // flight together
    constexpr int kLoadPer = 4;
    const int ntab = S - seg0 < TB ? (int)(S - seg0) : TB;
    const int total = ntab * (int)N;
    for (int i0 = threadIdx.x; i0 < total; i0 += 256 * kLoadPer) {
      double wv[kLoadPer];
      uint32_t sv[kLoadPer];
      int at[kLoadPer];
#pragma unroll
      for (int u = 0; u < kLoadPer; ++u) {
        const int i = i0 + u * 256;
        const int ic = i < total ? i : total - 1;
        const int tb = ic / (int)N, r = ic - tb * (int)N;
        wv[u] = w(seg0 + tb, r);
        sv[u] = w.sgn(seg0 + tb, r);
        at[u] = i < total ? tb * ld + r : -1;
      }
#pragma unroll
      for (int u = 0; u < kLoadPer; ++u)
        if (at[u] >= 0)
          lb[at[u]] = (uint64_t)__double_as_longlong(wv[u]) |
                      ((uint64_t)sv[u] << 63);
    }
    __syncthreads();
    if (wv == 0 && lane < ntab) {
      uint64_t* row = lb + lane * ld;
      double l = 0.0;
      for (int r0 = 0; r0 < N; r0 += 8) {
        uint64_t x[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) x[u] = row[r0 + u < N ? r0 + u : N - 1];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int r = r0 + u;
          if (r < N) {
            const double wr = __longlong_as_double((long long)(x[u] & kQMask));
            l = r % kRun == 0 ? wr : l + wr;
            row[r] = (uint64_t)__double_as_longlong(l) | (x[u] & ~kQMask);
            if (r % kRun == kRun - 1 || r == N - 1) rt[lane * 4 + r / kRun] = l;
          }
        }
      }
    }
    __syncthreads();
    // ---- phase 2 -----------------------------------------------------------
    // every wave runs every round (ntab is the same for the whole block)
    for (int t0 = 0; t0 < ntab; t0 += 4) {
      const int tb = t0 + wv;
      const int64_t seg = seg0 + tb;
      const bool have = tb < TB && seg < S;
      double Ec[4] = {0.0, 0.0, 0.0, 0.0};
      double T = 0.0;
      if (have)
        for (int c = 0; c < R; ++c) {
          Ec[c] = T;
          T = T + rt[tb * 4 + c];
        }
      const bool live = have && T > 0.0;
      if (have && lane == 0 && tot) tot[seg] = T;  // tot may be null
      if (have && !live)  // dead table: never sampled, entries zero
        for (int r = lane; r < Np; r += 64) ent[(seg << L) + r] = 0ull;
      // F_r exact in FP64 (K <= 40 here); slots past the items keep F of
      // the last item, 2^K, so their quanta are zero
      uint64_t F[SPL];
      uint32_t sg[SPL];
#pragma unroll
      for (int s = 0; s < SPL; ++s) {
        const int r = lane * SPL + s;
        F[s] = live ? (uint64_t)1 << K : 0ull;
        sg[s] = 0;
        if (live && r < N) {
          const uint64_t raw = lb[tb * ld + r];
          const double lr = __longlong_as_double((long long)(raw & kQMask));
          F[s] = exact_u52(floor(ldexp((Ec[r / kRun] + lr) / T, K)));
          sg[s] = (uint32_t)(raw >> 63);
        }
      }
      uint64_t Fp = __shfl_up(F[SPL - 1], 1, 64);
      if (lane == 0) Fp = 0;
      const uint64_t Fb = Fp;  // the sum of the quanta before this lane
      uint64_t qv[SPL];
#pragma unroll
      for (int s = 0; s < SPL; ++s) {
        qv[s] = F[s] - Fp;
        Fp = F[s];
      }
      wave_alias<SPL, true>(qv, sg, live, L, Ld, He, Hi,
                            EmitPacked{ent + ((have ? seg : 0) << L)}, Fb);
      __syncthreads();  // the wave's alias scratch is reused next round
    }
  }
}

template <class W>
static hipError_t small_tables(W w, int64_t S, int64_t N, int L, double* tot,
                               uint64_t* ent, hipStream_t st) {
  if (S <= 0 || N <= 0) return hipSuccess;
  const int Np = 1 << L;
  // the most tables per block (a power of two, 4 .. 64) within the LDS
  // budget; about 32 KB measured best (MAD_SMALL_LDS overrides it for
  // tuning)
  static const size_t budget = [] {
    const char* e = getenv("MAD_SMALL_LDS");
    const long v = e ? atol(e) : 32768;
    return (size_t)(v >= 4096 && v <= 65536 ? v : 32768);
  }();
  auto lds_for = [Np](int tb) {
    return ((size_t)tb * (Np + 1) + (size_t)tb * 4 + (size_t)Np * 10) * 8;
  };
  int TB = 64;
  while (TB > 4 && lds_for(TB) > budget) TB /= 2;
  const size_t lds = lds_for(TB);
  const unsigned blocks = grid_for(S, TB);
  if (Np <= 64)
    k_small_tables<1, W><<<blocks, 256, lds, st>>>(w, S, N, L, TB, tot, ent);
  else if (Np <= 128)
    k_small_tables<2, W><<<blocks, 256, lds, st>>>(w, S, N, L, TB, tot, ent);
  else if (Np <= 256)
    k_small_tables<4, W><<<blocks, 256, lds, st>>>(w, S, N, L, TB, tot, ent);
  else
    k_small_tables<8, W><<<blocks, 256, lds, st>>>(w, S, N, L, TB, tot, ent);
  return hipGetLastError();
}

// Workgroups go to the 8 XCDs in turn; this remaps block b so that each
// XCD takes a contiguous run of logical blocks (when the grid is a
// multiple of 8), which keeps neighbouring blocks' writes to a shared line,
// and their reads of a shared line, in one L2.
__device__ __forceinline__ int64_t xcd_block() {
  const int64_t nbk = gridDim.x, b = blockIdx.x;
  return nbk % 8 == 0 ? (b % 8) * (nbk / 8) + b / 8 : b;
}

// large tables (2^L >= 1024 slots): blocks of 1024 slots (256 threads x 4)
// never straddle a table
constexpr int kAliasBlk = 1024;

// block-wide exclusive scan of a Quad (256 threads); returns the block total
__device__ Quad block_excl_scan(Quad& v) {
  __shared__ Quad wtot[4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  Quad inc{wave_scan_dpp(v.nl), wave_scan_dpp(v.nh), wave_scan_dpp(v.sd),
           wave_scan_dpp(v.se)};
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
  for (int s = 0; s < 4; ++s) slot_stats(q[base + s] & kQMask, a);
  Quad all = block_excl_scan(a);
  if (threadIdx.x == 0) bs[blockIdx.x] = all;
}

// per table: exclusive scan of its block sums; light/heavy counts and the
// total deficit (one 256-thread block per table)
__global__ __launch_bounds__(256) void k_alias_blockscan(Quad* bs, int64_t S,
                                                         int64_t B,
                                                         uint64_t* NL,
                                                         uint64_t* NH,
                                                         uint64_t* Dt) {
  const int64_t seg = blockIdx.x;
  Quad carry{0, 0, 0, 0};
  for (int64_t c0 = 0; c0 < B; c0 += 256) {
    const int64_t b = c0 + threadIdx.x;
    Quad v = b < B ? bs[seg * B + b] : Quad{0, 0, 0, 0};
    const Quad all = block_excl_scan(v);
    if (b < B)
      bs[seg * B + b] = Quad{carry.nl + v.nl, carry.nh + v.nh,
                             carry.sd + v.sd, carry.se + v.se};
    carry.nl += all.nl;
    carry.nh += all.nh;
    carry.sd += all.sd;
    carry.se += all.se;
  }
  if (threadIdx.x == 0) {
    NL[seg] = carry.nl;
    NH[seg] = carry.nh;
    Dt[seg] = carry.sd;
  }
}

// per table lists in index order: lights with their exclusive deficit
// prefix (Ld) and slot id (Li); heavies with their inclusive excess prefix
// (He) and slot id (Hi); ids carry the item's sign in bit 31
__global__ __launch_bounds__(256) void k_alias_scatter(
    const uint64_t* q, const Quad* bo, int L, uint64_t* Ld, uint32_t* Li,
    uint64_t* He, uint32_t* Hi) {
  const int64_t base = (int64_t)blockIdx.x * kAliasBlk + threadIdx.x * 4;
  const int64_t tb = (base >> L) << L;  // first slot of the table
  uint64_t qv[4];
  uint32_t sg[4];
  Quad a{0, 0, 0, 0};
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const uint64_t raw = q[base + s];
    qv[s] = raw & kQMask;
    sg[s] = (uint32_t)(raw >> 63);
    slot_stats(qv[s], a);
  }
  (void)block_excl_scan(a);
  const Quad o = bo[blockIdx.x];
  uint64_t lp = o.nl + a.nl, hp = o.nh + a.nh;
  uint64_t da = o.sd + a.sd, ea = o.se + a.se;
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const uint32_t id = (uint32_t)(base + s - tb) | (sg[s] << 31);
    if (qv[s] < kCap) {
      Ld[tb + lp] = da;
      Li[tb + lp] = id;
      da += kCap - qv[s];
      ++lp;
    } else {
      ea += qv[s] - kCap;
      He[tb + hp] = ea;
      Hi[tb + hp] = id;
      ++hp;
    }
  }
}

// The sweep as a merge of the light deficits D (exclusive) and the heavy
// excesses E (inclusive), a light first on ties: light l is filled by the
// heavy that follows all heavies merged before it; heavy h closes against
// the light merged right after it.  A block merges kMergeBlk consecutive
// positions: one merge-path search per block edge in global memory, the
// block's slices of both lists in LDS, one search per thread in LDS, then
// kMergeP sequential merge steps per thread.
constexpr int kMergeP = 4;
constexpr int kMergeBlk = 256 * kMergeP;

// merge-path split of every block edge (kMergeBlk positions apart), one
// binary search per thread (a 64-lane search per edge was tried: it reads
// 64 scattered lines per round and took twice as long)
__global__ void k_alias_edges(const uint64_t* Ld, const uint64_t* He,
                              const uint64_t* NLa, const uint64_t* NHa,
                              int64_t ntab, int L, int64_t* edges) {
  const int64_t Np = int64_t(1) << L;
  const int64_t per = Np / kMergeBlk + 1;
  const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= ntab * per) return;
  const int64_t segl = gid / per, b = gid % per;
  const int64_t tb = segl << L;
  edges[gid] = merge_split(Ld + tb, (int64_t)NLa[segl], He + tb,
                           (int64_t)NHa[segl], b * kMergeBlk);
}

// (A persistent version that loaded the next block's slices while merging
// the current one needed 146 VGPRs, held half as many waves and took 106
// against 83 us per C2 family.)
__global__ __launch_bounds__(256) void k_alias_merge(
    const uint64_t* Ld, const uint32_t* Li, const uint64_t* He,
    const uint32_t* Hi, const uint64_t* NLa, const uint64_t* NHa,
    const uint64_t* Dta, const int64_t* edges, const double* tot,
    int64_t seg0, int L, uint64_t* ent) {
  __shared__ uint64_t sD[kMergeBlk + 1], sE[kMergeBlk + 1];
  __shared__ uint32_t sLi[kMergeBlk + 1], sHi[kMergeBlk + 1];
  const int64_t Np = int64_t(1) << L;
  const int64_t blocks_per = Np / kMergeBlk;
  // each XCD takes a contiguous run of blocks, so that a table's scattered
  // entry writes meet in one L2
  const int64_t lb = xcd_block();
  const int64_t segl = lb / blocks_per;
  const int64_t bi = lb % blocks_per;
  const int64_t seg = seg0 + segl;
  const int64_t d0 = bi * kMergeBlk;
  uint64_t* et = ent + (seg << L);
  // the table's figures and the block's edges in one round of loads
  const int64_t* ed = edges + segl * (blocks_per + 1) + bi;
  const double tt = tot[seg];
  const int64_t NL = (int64_t)NLa[segl], NH = (int64_t)NHa[segl];
  const uint64_t Dt = Dta[segl];
  const int64_t e0 = ed[0], e1 = ed[1];
  if (!(tt > 0.0)) {  // dead table: never sampled, entries zero
    for (int u = threadIdx.x; u < kMergeBlk; u += 256) et[d0 + u] = 0ull;
    return;
  }
  const int64_t tb = segl << L;
  const uint64_t* D = Ld + tb;
  const uint64_t* E = He + tb;
  const int64_t a0 = e0, b0 = d0 - e0;
  const int64_t na = e1 - a0, nb = (d0 + kMergeBlk - e1) - b0;
  // slices, plus one element past each end (the next D bounds a light's
  // quantum; the next heavy id closes a heavy): every load issued before
  // the first LDS store
  constexpr int kSl = (kMergeBlk + 1 + 255) / 256;
  uint64_t rD[kSl], rE[kSl];
  uint32_t rL[kSl], rH[kSl];
#pragma unroll
  for (int k = 0; k < kSl; ++k) {
    const int64_t u = threadIdx.x + 256 * k;
    const bool la = u <= na && a0 + u < NL, hb = u <= nb && b0 + u < NH;
    rD[k] = la ? D[a0 + u] : Dt;
    rL[k] = la ? Li[tb + a0 + u] : 0u;
    rE[k] = hb ? E[b0 + u] : ~0ull;
    rH[k] = hb ? Hi[tb + b0 + u] : 0u;
  }
#pragma unroll
  for (int k = 0; k < kSl; ++k) {
    const int64_t u = threadIdx.x + 256 * k;
    if (u <= na) {
      sD[u] = rD[k];
      sLi[u] = rL[k];
    }
    if (u <= nb) {
      sE[u] = rE[k];
      sHi[u] = rH[k];
    }
  }
  __syncthreads();
  // this thread's split inside the block's slices
  const int64_t dl = (int64_t)threadIdx.x * kMergeP;
  int64_t lo = dl - nb > 0 ? dl - nb : 0, hi = dl < na ? dl : na;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (sD[mid] <= sE[dl - mid - 1]) lo = mid + 1; else hi = mid;
  }
  int64_t a = lo, b = dl - lo;
  for (int step = 0; step < kMergeP; ++step) {
    if (a < na && (b >= nb || sD[a] <= sE[b])) {
      const uint32_t id = sLi[a];
      const uint32_t r = id & kLow31;
      const uint32_t qv = (uint32_t)(kCap - (sD[a + 1] - sD[a]));
      // the donor: the first heavy not merged before this light
      const uint32_t dn = b0 + b < NH ? sHi[b] : id;
      et[r] = pack_entry(qv, id >> 31, dn & kLow31, dn >> 31);
      ++a;
    } else {
      const uint32_t id = sHi[b];
      const uint32_t r = id & kLow31;
      const uint64_t Eh = sE[b];
      const uint64_t Dn = sD[a];  // D of the next light, or Dt past the end
      if (Dn > Eh && b0 + b + 1 < NH) {
        const uint32_t nx = sHi[b + 1];
        et[r] = pack_entry((uint32_t)(Eh + kCap - Dn), id >> 31, nx & kLow31,
                           nx >> 31);
      } else {
        et[r] = pack_entry(0u, id >> 31, r, id >> 31);
      }
      ++b;
    }
  }
}

// scratch layout for a batch of `slots` slots and `tables` tables
static size_t alias_scratch_bytes(int64_t slots, int64_t tables) {
  return (size_t)slots * (8 + 4 + 8 + 4) + (size_t)(slots / kAliasBlk) *
         sizeof(Quad) + (size_t)tables * 24 +
         (size_t)(slots / kMergeBlk + tables) * 8 + 256;
}

// tables of 2^L >= 1024 slots from stored quanta, in batches of tables that
// fit the scratch
static hipError_t alias_large(const uint64_t* q, const double* tot, int64_t S,
                              int L, uint64_t* ent, void* scratch,
                              size_t scratch_bytes, hipStream_t st) {
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
    uint32_t* Li = (uint32_t*)p; p += slots * 4;
    uint32_t* Hi = (uint32_t*)p; p += slots * 4;
    Quad* bs = (Quad*)p; p += nblk * sizeof(Quad);
    uint64_t* NL = (uint64_t*)p; p += ns * 8;
    uint64_t* NH = (uint64_t*)p; p += ns * 8;
    uint64_t* Dt = (uint64_t*)p; p += ns * 8;
    int64_t* edges = (int64_t*)p;
    const uint64_t* qb = q + (s0 << L);
    k_alias_blocksum<<<(unsigned)nblk, 256, 0, st>>>(qb, bs);
    k_alias_blockscan<<<(unsigned)ns, 256, 0, st>>>(bs, ns, Np / kAliasBlk,
                                                    NL, NH, Dt);
    k_alias_scatter<<<(unsigned)nblk, 256, 0, st>>>(qb, bs, L, Ld, Li, He, Hi);
    const int64_t nedge = ns * (Np / kMergeBlk + 1);
    k_alias_edges<<<grid_for(nedge, 256), 256, 0, st>>>(Ld, He, NL, NH, ns, L,
                                                        edges);
    k_alias_merge<<<(unsigned)(slots / kMergeBlk), 256, 0, st>>>(
        Ld, Li, He, Hi, NL, NH, Dt, edges, tot, s0, L, ent);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

static hipError_t build_alias(const uint64_t* q, const double* tot, int64_t S,
                              int L, uint64_t* ent, void* scratch,
                              size_t scratch_bytes, hipStream_t st) {
  return alias_large(q, tot, S, L, ent, scratch, scratch_bytes, st);
}

// ---------------------------------------------------------------------------
// Column families of 2^L >= 1024 slots without stored prefixes or quanta.
// The prefixes are recomputed from X, which is cheaper than writing and
// reading them back:
//   run totals   per table and run of kRun items, the left-to-right sum;
//   offsets      E_c and T per table in the two-level order;
//   statistics   per table and run of kRun slots (slot runs = item runs,
//                padding after the items): light / heavy counts, deficit
//                and excess, from q_r = F_r - F_{r-1} walked in order;
//   block scan   exclusive offsets of those statistics per table;
//   lists        the same walk again, writing each light's exclusive
//                deficit prefix and slot id and each heavy's inclusive
//                excess prefix and slot id at their offsets;
//   merge        as for any large table.
// The prefix of the item before a run start is E_c itself (E_c = E_{c-1}
// + l of run c-1's last item is the same operation), so each run starts
// from F_{r-1} = floor(2^K E_c / T) (0 in the first run).
// ---------------------------------------------------------------------------
// loads of a column walk issued together (clamped to the run's last row,
// so they carry no branch)
constexpr int kColGroup = 32;

template <bool SCALE>
__global__ __launch_bounds__(64) void k_col_runtot(const float* X, int64_t d,
                                                   const double* scale,
                                                   int64_t S, int64_t N,
                                                   double* rtot) {
  const int64_t tiles = (S + 63) / 64;
  const int64_t c = blockIdx.x / tiles;
  const int64_t seg = (blockIdx.x % tiles) * 64 + threadIdx.x;
  const int64_t segc = seg < S ? seg : S - 1;
  const int64_t r0 = c * kRun;
  const int64_t r1 = N < r0 + kRun ? N : r0 + kRun;
  double l = 0.0;
  for (int64_t g0 = r0; g0 < r1; g0 += kColGroup) {
    float xv[kColGroup];
    double sv[kColGroup];
#pragma unroll
    for (int u = 0; u < kColGroup; ++u) {
      const int64_t r = g0 + u < r1 ? g0 + u : r1 - 1;
      xv[u] = X[r * d + segc];
      sv[u] = SCALE ? scale[r] : 1.0;
    }
    // no branch per item: the additions stay one dependent chain and the
    // rest interleaves
#pragma unroll
    for (int u = 0; u < kColGroup; ++u) {
      const int64_t r = g0 + u;
      const double w = SCALE ? fabs((double)xv[u]) * sv[u]
                             : fabs((double)xv[u]);
      const double lw = r == r0 ? w : l + w;
      l = r < r1 ? lw : l;
    }
  }
  if (seg < S) rtot[c * S + seg] = l;
}

// E_c (c < R) and T per table: E_0 = 0, E_{c+1} = E_c + rtot_c, T = E_R.
// One 256-thread block per table: the run totals are gathered into LDS in
// parallel, then one lane adds them left to right, 16 at a time through
// registers so that its LDS reads do not wait on its own writes.
constexpr int kOffChunk = 2048;
constexpr int kOffBatch = 16;

__global__ __launch_bounds__(256) void k_col_runoffsets(const double* rtot,
                                                        int64_t S, int64_t R,
                                                        double* E,
                                                        double* tot) {
  __shared__ double buf[kOffChunk];
  const int64_t seg = blockIdx.x;
  double e = 0.0;  // thread 0's running offset
  for (int64_t c0 = 0; c0 < R; c0 += kOffChunk) {
    const int nc = (int)(R - c0 < kOffChunk ? R - c0 : kOffChunk);
    // padded with zeros to whole batches: e + 0 = e exactly
    const int ncp = (nc + kOffBatch - 1) / kOffBatch * kOffBatch;
    for (int u = threadIdx.x; u < ncp; u += 256)
      buf[u] = u < nc ? rtot[(c0 + u) * S + seg] : 0.0;
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int u0 = 0; u0 < ncp; u0 += kOffBatch) {
        double x[kOffBatch];
#pragma unroll
        for (int j = 0; j < kOffBatch; ++j) x[j] = buf[u0 + j];
#pragma unroll
        for (int j = 0; j < kOffBatch; ++j) {
          const double ej = e;  // E_c
          e = e + x[j];
          x[j] = ej;
        }
#pragma unroll
        for (int j = 0; j < kOffBatch; ++j) buf[u0 + j] = x[j];
      }
    }
    __syncthreads();
    for (int u = threadIdx.x; u < nc; u += 256) E[(c0 + u) * S + seg] = buf[u];
    __syncthreads();
  }
  if (threadIdx.x == 0) tot[seg] = e;
}

// One wave per (slot run c, 64 consecutive tables of [s0, s0 + ns)), lane
// = table.  LISTS = false: the run's statistics into bs[t * B + c];
// LISTS = true: bs holds the exclusive offsets and the lists are written
// (positions relative to table t's base t << L).  Each group of 16 items
// passes through LDS as (list value with the heavy flag in bit 63, slot id
// with the sign in bit 31) per (item, table); then, four tables at a time
// (one per quarter-wave, lane = item), ballots give every entry its place
// and each table's lights and heavies of the group are stored as
// contiguous runs.  F64 selects the exact FP64 arithmetic of the
// statistics (L <= kF64MaxL; the lists are then written by k_col_lists).
// (Splitting each run over four waves, each first re-adding the run-local
// prefix before its quarter, was measured slower: the walks are bound by
// their instruction issue, not by the latency one wave sees.)
template <bool LISTS, bool SCALE, bool F64>
__global__ __launch_bounds__(64) void k_col_walk(
    const float* X, int64_t d, const double* scale, int64_t S, int64_t N,
    int L, const double* E, const double* tot, int64_t s0, int64_t ns,
    Quad* bs, uint64_t* Ld, uint32_t* Li, uint64_t* He, uint32_t* Hi) {
  // items per group: 32 for the statistics; 16 for the lists, so that the
  // LDS staging (12.5 KB) lets more waves share a CU
  constexpr int G = LISTS ? 16 : kColGroup;
  static_assert(G == 16 || !LISTS, "four tables per wave in the write-out");
  static_assert(!(LISTS && F64), "the F64 lists are k_col_lists");
  __shared__ uint64_t tv[LISTS ? G : 1][65];
  __shared__ uint32_t ti[LISTS ? G : 1][65];
  __shared__ uint64_t cnt0[LISTS ? 64 : 1][2];  // lights / heavies before
  const int64_t B = (int64_t(1) << L) / kRun;  // slot runs per table
  const int64_t tiles = (ns + 63) / 64;
  const int64_t lb = xcd_block();
  const int64_t c = lb / tiles;
  const int64_t t0 = (lb % tiles) * 64;
  const int lane = threadIdx.x;
  const int64_t t = t0 + lane;
  const bool mine = t < ns;
  const int64_t tc = mine ? t : ns - 1;
  const int64_t seg = s0 + tc;
  const double T = tot[seg];
  const bool live = T > 0.0;
  const double Tq = live ? T : 1.0;  // dead tables: no item is taken
  const int K = L + kCapBits;
  const int64_t r0 = c * kRun;
  const int64_t r1 = N < r0 + kRun ? N : r0 + kRun;  // items of this run
  const int64_t R = (N + kRun - 1) / kRun;
  const double Ec = live && c < R ? E[c * S + seg] : 0.0;
  // F of the item before the run: floor(2^K E_c / T), 0 in the first run
  const bool first = !(live && c > 0 && c < R);
  const double Fstart = first ? 0.0 : floor(ldexp(Ec / T, K));
  uint64_t Fp = (uint64_t)Fstart;
  double Fpd = Fstart;
  uint64_t nl = 0, nh = 0, da = 0, ea = 0;
  double dad = 0.0, ead = 0.0;
  if (LISTS) {
    const Quad o = bs[tc * B + c];
    nl = o.nl;
    nh = o.nh;
    da = o.sd;
    ea = o.se;
    dad = (double)o.sd;  // exact: below 2^52 on the F64 path
    ead = (double)o.se;
  }
  double l = 0.0;
  uint32_t nlr = 0;  // lights of this run so far (F64 statistics)
  for (int64_t g0 = r0; g0 < r0 + kRun; g0 += G) {
    float xv[G];
    double sv[G];
    if (g0 < r1) {
#pragma unroll
      for (int u = 0; u < G; ++u) {
        const int64_t r = g0 + u < r1 ? g0 + u : r1 - 1;
        xv[u] = X[r * d + seg];
        sv[u] = SCALE ? scale[r] : 1.0;
      }
    } else {  // padding slots only
#pragma unroll
      for (int u = 0; u < G; ++u) {
        xv[u] = 0.0f;
        sv[u] = 1.0;
      }
    }
    if (LISTS) {
      cnt0[lane][0] = nl;
      cnt0[lane][1] = nh;
    }
    if (F64) {
      // no branch per item: items past the run's end (and every item of a
      // dead table) weigh 0 and leave l, F and the sums unchanged apart
      // from a zero quantum
#pragma unroll
      for (int u = 0; u < G; ++u) {
        const int64_t r = g0 + u;
        const float x = live && r < r1 ? xv[u] : 0.0f;
        const double w = SCALE ? fabs((double)x) * sv[u] : fabs((double)x);
        l = l + w;
        const double F = floor(ldexp((Ec + l) / Tq, K));
        const double q = F - Fpd;
        Fpd = F;
        const bool light = q < kCapD;
        dad = dad + fmax(kCapD - q, 0.0);
        ead = ead + fmax(q - kCapD, 0.0);
        nlr += light ? 1u : 0u;
      }
    } else {
      // no branch per item: only the additions of l form a dependent
      // chain, so the divisions of consecutive items overlap
#pragma unroll
      for (int u = 0; u < G; ++u) {
        const int64_t r = g0 + u;
        const bool ok = live && r < r1;
        const double w = SCALE ? fabs((double)xv[u]) * sv[u]
                               : fabs((double)xv[u]);
        const double lw = r == r0 ? w : l + w;
        l = ok ? lw : l;
        const uint64_t F = (uint64_t)floor(ldexp((Ec + l) / Tq, K));
        const uint64_t q = ok ? F - Fp : 0ull;
        Fp = ok ? F : Fp;
        const uint32_t sg = ok ? sign_bit(xv[u]) : 0u;
        const bool light = q < kCap;
        const uint64_t ea2 = light ? ea : ea + (q - kCap);
        if (LISTS) tv[u][lane] = light ? da : (ea2 | (1ull << 63));
        da = light ? da + (kCap - q) : da;
        ea = ea2;
        nl += light ? 1 : 0;
        nh += light ? 0 : 1;
        if (LISTS) ti[u][lane] = (uint32_t)r | (sg << 31);
      }
    }
    if (LISTS) {
      __syncthreads();
      // write-out: quarter-wave h takes table j = p4 + h, lane & 15 = item
      const int h = lane >> 4, u = lane & 15;
      const uint64_t lt = (1ull << lane) - 1;
      const uint64_t half = 0xFFFFull << (16 * h);
      for (int p4 = 0; p4 < 64; p4 += 4) {
        const int j = p4 + h;
        const bool ok = t0 + j < ns;
        const uint64_t v = tv[u][j];
        const uint32_t id = ti[u][j];
        const bool heavy = (v >> 63) != 0;
        const uint64_t bh = __ballot(ok && heavy) & half;
        const uint64_t bl = __ballot(ok && !heavy) & half;
        const int64_t tb = (t0 + j) << L;
        if (ok) {
          if (heavy) {
            const int64_t pos = (int64_t)cnt0[j][1] + __popcll(bh & lt);
            He[tb + pos] = v & ~(1ull << 63);
            Hi[tb + pos] = id;
          } else {
            const int64_t pos = (int64_t)cnt0[j][0] + __popcll(bl & lt);
            Ld[tb + pos] = v;
            Li[tb + pos] = id;
          }
        }
      }
      __syncthreads();
    }
  }
  if (!LISTS && mine) {
    if (F64)
      bs[tc * B + c] = Quad{nlr, (uint64_t)(kRun - nlr), exact_u52(dad),
                            exact_u52(ead)};
    else
      bs[tc * B + c] = Quad{nl, nh, da, ea};
  }
}

constexpr int kListGroup = 32;  // items per write-out group

// The lists walk on the exact FP64 path (L <= kF64MaxL), one wave per (slot
// run c, 64 consecutive tables of [s0, s0 + ns)), lane = table: each lane
// knows its table's running light and heavy counts, so it gives each item
// its list position itself.  A group of G items then passes through LDS as
// (value with the heavy flag in bit 63, slot id with the sign in bit 31,
// position), and 64 / G tables at a time (G lanes each, lane = item) are
// stored, each table's lights and heavies of the group as contiguous runs.
// 32-item groups write 200 MB per C2 family where 16-item groups wrote
// 247 MB (157 MB of entries): longer runs leave fewer partly written
// lines.  (Packing id and position into one word, or 64-item groups, were
// not faster.)  Groups wholly inside the run's items load without
// clamping.
template <bool SCALE>
__global__ __launch_bounds__(64) void k_col_lists(
    const float* X, int64_t d, const double* scale, int64_t S, int64_t N,
    int L, const double* E, const double* tot, int64_t s0, int64_t ns,
    const Quad* bs, uint64_t* Ld, uint32_t* Li, uint64_t* He, uint32_t* Hi) {
  constexpr int G = kListGroup;
  constexpr int P = 64 / G;  // tables per write-out round
  __shared__ uint64_t tv[G][65];
  __shared__ uint32_t ti[G][65];
  __shared__ uint32_t tp[G][65];
  const int64_t B = (int64_t(1) << L) / kRun;  // slot runs per table
  const int64_t tiles = (ns + 63) / 64;
  const int64_t lb = xcd_block();
  const int64_t c = lb / tiles;
  const int64_t t0 = (lb % tiles) * 64;
  const int lane = threadIdx.x;
  const int64_t t = t0 + lane;
  const int64_t tc = t < ns ? t : ns - 1;
  const int64_t seg = s0 + tc;
  const double T = tot[seg];
  const bool live = T > 0.0;
  const double Tq = live ? T : 1.0;  // dead tables: no item is taken
  const int K = L + kCapBits;
  const int64_t r0 = c * kRun;
  const int64_t r1 = N < r0 + kRun ? N : r0 + kRun;  // items of this run
  const int64_t R = (N + kRun - 1) / kRun;
  const double Ec = live && c < R ? E[c * S + seg] : 0.0;
  const bool first = !(live && c > 0 && c < R);
  double Fp = first ? 0.0 : floor(ldexp(Ec / T, K));
  const Quad o = bs[tc * B + c];
  uint32_t nl = (uint32_t)o.nl, nh = (uint32_t)o.nh;  // below 2^L
  double da = (double)o.sd;  // exact: below 2^52
  double ea = (double)o.se;
  double l = 0.0;
  const float* xs = X + seg;
  for (int64_t g0 = r0; g0 < r0 + kRun; g0 += G) {
    float xv[G];
    double sv[G];
    if (g0 + G <= r1) {
      const float* xg = xs + g0 * d;
#pragma unroll
      for (int u = 0; u < G; ++u) {
        xv[u] = xg[(int64_t)u * d];
        sv[u] = SCALE ? scale[g0 + u] : 1.0;
      }
    } else if (g0 < r1) {
#pragma unroll
      for (int u = 0; u < G; ++u) {
        const int64_t r = g0 + u < r1 ? g0 + u : r1 - 1;
        xv[u] = xs[r * d];
        sv[u] = SCALE ? scale[r] : 1.0;
      }
    } else {  // padding slots only
#pragma unroll
      for (int u = 0; u < G; ++u) {
        xv[u] = 0.0f;
        sv[u] = 1.0;
      }
    }
    // items past the run's end (and every item of a dead table) weigh 0
    // and leave l, F and the sums unchanged apart from a zero quantum
#pragma unroll
    for (int u = 0; u < G; ++u) {
      const int64_t r = g0 + u;
      const float x = live && r < r1 ? xv[u] : 0.0f;
      const double w = SCALE ? fabs((double)x) * sv[u] : fabs((double)x);
      l = l + w;
      const double F = floor(ldexp((Ec + l) / Tq, K));
      const double q = F - Fp;
      Fp = F;
      const bool light = q < kCapD;
      const double dex = da;  // the light's exclusive deficit prefix
      da = da + fmax(kCapD - q, 0.0);
      ea = ea + fmax(q - kCapD, 0.0);
      tv[u][lane] = light ? exact_u52(dex) : (exact_u52(ea) | (1ull << 63));
      ti[u][lane] = (uint32_t)r | (sign_bit(x) << 31);
      tp[u][lane] = light ? nl : nh;
      nl += light ? 1u : 0u;
      nh += light ? 0u : 1u;
    }
    __syncthreads();
    // write-out: lane group h of G lanes takes table j = p + h, lane % G =
    // item
    const int h = lane / G, u = lane % G;
    for (int p = 0; p < 64; p += P) {
      const int j = p + h;
      const uint64_t v = tv[u][j];
      const uint32_t id = ti[u][j];
      const int64_t at = ((t0 + j) << L) + tp[u][j];
      if (t0 + j < ns) {
        if (v >> 63) {
          He[at] = v & ~(1ull << 63);
          Hi[at] = id;
        } else {
          Ld[at] = v;
          Li[at] = id;
        }
      }
    }
    __syncthreads();
  }
}

// scratch of col_tables: run totals and offsets (2 R S doubles), the run
// statistics (S B Quads), then the alias lists of a batch of tables
static size_t col_tables_fixed_bytes(int64_t S, int64_t N, int L) {
  const int64_t R = (N + kRun - 1) / kRun;
  const int64_t B = (int64_t(1) << L) / kRun;
  return (size_t)(2 * R * S) * 8 + (size_t)(S * B) * sizeof(Quad) + 256;
}

static hipError_t col_tables(const float* X, int64_t d, const double* scale,
                             int64_t S, int64_t N, int L, Family& f,
                             void* scratch, size_t scratch_bytes,
                             hipStream_t st, hipEvent_t tot_ready = nullptr) {
  const int64_t R = (N + kRun - 1) / kRun;
  const int64_t Np = int64_t(1) << L;
  const int64_t B = Np / kRun;
  const size_t fixed = col_tables_fixed_bytes(S, N, L);
  if (scratch_bytes < fixed) return hipErrorInvalidValue;
  char* p = (char*)scratch;
  double* rtot = (double*)p; p += (size_t)(R * S) * 8;
  double* E = (double*)p; p += (size_t)(R * S) * 8;
  Quad* bs = (Quad*)(((uintptr_t)p + 31) & ~(uintptr_t)31);
  p = (char*)(bs + S * B);
  const size_t left = scratch_bytes - (size_t)(p - (char*)scratch);
  // tables per batch of alias lists
  const size_t per_tab = alias_scratch_bytes(Np, 1);
  int64_t per = (int64_t)(left / per_tab);
  if (per < 1) return hipErrorOutOfMemory;
  const int64_t tiles = (S + 63) / 64;
  if (scale)
    k_col_runtot<true><<<(unsigned)(R * tiles), 64, 0, st>>>(X, d, scale, S,
                                                             N, rtot);
  else
    k_col_runtot<false><<<(unsigned)(R * tiles), 64, 0, st>>>(X, d, scale, S,
                                                              N, rtot);
  k_col_runoffsets<<<(unsigned)S, 256, 0, st>>>(rtot, S, R, E, f.tot);
  if (tot_ready) {  // the family's totals are final from here on
    const hipError_t e = hipEventRecord(tot_ready, st);
    if (e != hipSuccess) return e;
  }
  const bool f64 = L <= kF64MaxL;
  const unsigned sgrid = (unsigned)(B * tiles);
  if (scale && f64)
    k_col_walk<false, true, true><<<sgrid, 64, 0, st>>>(
        X, d, scale, S, N, L, E, f.tot, 0, S, bs, nullptr, nullptr, nullptr,
        nullptr);
  else if (scale)
    k_col_walk<false, true, false><<<sgrid, 64, 0, st>>>(
        X, d, scale, S, N, L, E, f.tot, 0, S, bs, nullptr, nullptr, nullptr,
        nullptr);
  else if (f64)
    k_col_walk<false, false, true><<<sgrid, 64, 0, st>>>(
        X, d, scale, S, N, L, E, f.tot, 0, S, bs, nullptr, nullptr, nullptr,
        nullptr);
  else
    k_col_walk<false, false, false><<<sgrid, 64, 0, st>>>(
        X, d, scale, S, N, L, E, f.tot, 0, S, bs, nullptr, nullptr, nullptr,
        nullptr);
  for (int64_t s0 = 0; s0 < S; s0 += per) {
    const int64_t ns = S - s0 < per ? S - s0 : per;
    const int64_t slots = ns * Np;
    char* a = p;
    uint64_t* Ld = (uint64_t*)a; a += slots * 8;
    uint64_t* He = (uint64_t*)a; a += slots * 8;
    uint32_t* Li = (uint32_t*)a; a += slots * 4;
    uint32_t* Hi = (uint32_t*)a; a += slots * 4;
    a += (slots / kAliasBlk) * sizeof(Quad);
    uint64_t* NL = (uint64_t*)a; a += ns * 8;
    uint64_t* NH = (uint64_t*)a; a += ns * 8;
    uint64_t* Dt = (uint64_t*)a; a += ns * 8;
    int64_t* edges = (int64_t*)a;
    Quad* bsb = bs + s0 * B;
    k_alias_blockscan<<<(unsigned)ns, 256, 0, st>>>(bsb, ns, B, NL, NH, Dt);
    const int64_t btiles = (ns + 63) / 64;
    const unsigned lgrid = (unsigned)(B * btiles);
    if (scale && f64)
      k_col_lists<true><<<lgrid, 64, 0, st>>>(
          X, d, scale, S, N, L, E, f.tot, s0, ns, bsb, Ld, Li, He, Hi);
    else if (scale)
      k_col_walk<true, true, false><<<lgrid, 64, 0, st>>>(
          X, d, scale, S, N, L, E, f.tot, s0, ns, bsb, Ld, Li, He, Hi);
    else if (f64)
      k_col_lists<false><<<lgrid, 64, 0, st>>>(
          X, d, scale, S, N, L, E, f.tot, s0, ns, bsb, Ld, Li, He, Hi);
    else
      k_col_walk<true, false, false><<<lgrid, 64, 0, st>>>(
          X, d, scale, S, N, L, E, f.tot, s0, ns, bsb, Ld, Li, He, Hi);
    const int64_t nedge = ns * (Np / kMergeBlk + 1);
    k_alias_edges<<<grid_for(nedge, 256), 256, 0, st>>>(Ld, He, NL, NH, ns, L,
                                                        edges);
    k_alias_merge<<<(unsigned)(slots / kMergeBlk), 256, 0, st>>>(
        Ld, Li, He, Hi, NL, NH, Dt, edges, f.tot, s0, L, f.ent);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// ---------------------------------------------------------------------------
// dense plan tables
// ---------------------------------------------------------------------------
// Binary inputs (Alg. 1): bit e of bits is 1 when entry e of B is 1;
// *flag = 0 when some entry is neither 0 nor 1 (the sampler then reads B
// itself).  Each wave reads 64 consecutive entries per step (coalesced) and
// writes their two 32-bit words from its ballots.
__global__ __launch_bounds__(256) void k_binary_bitmap(const float* B,
                                                       int64_t n,
                                                       uint32_t* bits,
                                                       int* flag) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  bool other = false;
  for (int64_t base = wave * 64; base < n; base += nwaves * 64) {
    const int64_t e = base + lane;
    const float v = e < n ? B[e] : 0.0f;
    const uint64_t one = __ballot(v == 1.0f);
    other |= v != 0.0f && v != 1.0f;
    if (lane < 2 && base + 32 * lane < n)
      bits[(base >> 5) + lane] = (uint32_t)(one >> (32 * lane));
  }
  if (__ballot(other) && lane == 0) *flag = 0;
}

// A == A^T for the squared variant (m x m): *flag = 1 on any difference.
// One workgroup per 64 x 64 tile pair (tile (bx, by) with bx <= by and its
// mirror), both staged in LDS so that every global read is coalesced.
__global__ __launch_bounds__(256) void k_check_symmetric(const float* A,
                                                         int64_t m,
                                                         int* flag) {
  __shared__ float t1[64][65];
  __shared__ float t2[64][65];
  const int64_t bx = blockIdx.x, by = blockIdx.y;
  if (bx > by) return;
  const int64_t r0 = by * 64, c0 = bx * 64;  // tile rows r0.., cols c0..
  for (int q = threadIdx.x; q < 64 * 64; q += 256) {
    const int r = q >> 6, c = q & 63;
    const int64_t i = r0 + r, k = c0 + c;
    t1[r][c] = (i < m && k < m) ? A[i * m + k] : 0.0f;
    const int64_t i2 = c0 + r, k2 = r0 + c;  // the mirror tile
    t2[r][c] = (i2 < m && k2 < m) ? A[i2 * m + k2] : 0.0f;
  }
  __syncthreads();
  bool diff = false;
  for (int q = threadIdx.x; q < 64 * 64; q += 256) {
    const int r = q >> 6, c = q & 63;
    if (t1[r][c] != t2[c][r]) diff = true;
  }
  if (diff) *flag = 1;
}

hipError_t launch_check_symmetric(const float* A, int64_t m, int* flag,
                                  hipStream_t st) {
  hipError_t e = launch_fill_u64((uint64_t*)flag, 1, 0ull, st);
  if (e != hipSuccess) return e;
  const unsigned g = (unsigned)((m + 63) / 64);
  k_check_symmetric<<<dim3(g, g), 256, 0, st>>>(A, m, flag);
  return hipGetLastError();
}

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
  if ((e = hipMalloc(&t.bad, 256)) != hipSuccess) return e;
  if ((e = hipMalloc(&t.bbits, 4 * (size_t)((n * d + 31) / 32))) !=
      hipSuccess)
    return e;
  if ((e = hipStreamCreateWithFlags(&t.side, hipStreamNonBlocking)) !=
          hipSuccess ||
      (e = hipStreamCreateWithFlags(&t.aux, hipStreamNonBlocking)) !=
          hipSuccess)
    return e;
  for (hipEvent_t* ev : {&t.fork, &t.join, &t.t1tot, &t.t2tot, &t.t0done,
                         &t.order_done, &t.sampled})
    if ((e = hipEventCreateWithFlags(ev, hipEventDisableTiming)) !=
        hipSuccess)
      return e;
  return hipSuccess;
}

void dense_tables_free(DenseTables& t) {
  family_free(t.T0);
  family_free(t.T1);
  family_free(t.T2);
  family_free(t.T3);
  if (t.om) (void)hipFree(t.om);
  if (t.bmax) (void)hipFree(t.bmax);
  if (t.bad) (void)hipFree(t.bad);
  if (t.bbits) (void)hipFree(t.bbits);
  t.bbits = nullptr;
  for (hipEvent_t* ev : {&t.fork, &t.join, &t.t1tot, &t.t2tot, &t.t0done,
                         &t.order_done, &t.sampled}) {
    if (*ev) (void)hipEventDestroy(*ev);
    *ev = nullptr;
  }
  if (t.side) (void)hipStreamDestroy(t.side);
  if (t.aux) (void)hipStreamDestroy(t.aux);
  t.om = nullptr;
  t.bmax = nullptr;
  t.bad = nullptr;
  t.side = t.aux = nullptr;
  t.t0_aux = 0;
}

static size_t run_doubles(int64_t S, int64_t N) {
  const int64_t R = (N + kRun - 1) / kRun;
  return (size_t)(2 * R * S);
}

hipError_t dense_tables_build(DenseTables& t, const float* A, const float* B,
                              bool check, DeviceBuffer& scratch_buf,
                              hipStream_t st) {
  const int64_t m = t.m, n = t.n, d = t.d;
  // scratch: for a row family (T3, T0) of 2^L > 512 slots its quanta, run
  // sums and alias lists; for a column family (T1, T2) of 2^L > 512 slots
  // its run data and statistics and alias lists.  Alias lists are batched
  // to at most 2^26 slots (at least one table).
  auto alias_for = [](const Family& f) {
    size_t sl = (size_t)(f.S << f.L);
    if (sl > ((size_t)1 << 26)) sl = (size_t)1 << 26;
    if (sl < ((size_t)1 << f.L)) sl = (size_t)1 << f.L;
    return alias_scratch_bytes((int64_t)sl, (int64_t)sl / kAliasBlk);
  };
  // main region: row families and T1; side region (B given): T2
  size_t need = 1024;
  for (const Family* f : {&t.T3, &t.T0})
    if (f->L > 9) {
      const size_t b = (size_t)(f->S << f->L) * 8 +
                       run_doubles(f->S, f->N) * 8 + alias_for(*f) + 1024;
      if (b > need) need = b;
    }
  if (t.T1.L > 9) {
    const size_t b = col_tables_fixed_bytes(t.T1.S, t.T1.N, t.T1.L) +
                     alias_for(t.T1) + 1024;
    if (b > need) need = b;
  }
  need = (need + 255) & ~(size_t)255;
  size_t need_side = 0;
  if (B && t.T2.L > 9)
    need_side = col_tables_fixed_bytes(t.T2.S, t.T2.N, t.T2.L) +
                alias_for(t.T2) + 1024;
  hipError_t e = dev_alloc(scratch_buf, need + need_side);
  if (e != hipSuccess) return e;
  // row-family layout of the main region
  char* p = (char*)scratch_buf.p;
  const size_t qslots = (size_t)(t.T3.S << t.T3.L) > (size_t)(t.T0.S << t.T0.L)
                            ? (size_t)(t.T3.S << t.T3.L)
                            : (size_t)(t.T0.S << t.T0.L);
  const size_t runs = run_doubles(t.T3.S, t.T3.N) > run_doubles(1, t.T0.N)
                          ? run_doubles(t.T3.S, t.T3.N)
                          : run_doubles(1, t.T0.N);
  uint64_t* q = (uint64_t*)p; p += qslots * 8;
  double* runbuf = (double*)p; p += runs * 8;
  void* abuf = p;
  const size_t used = (size_t)(p - (char*)scratch_buf.p);
  const size_t alias_bytes = need > used ? need - used : 0;
  void* side_scratch = (char*)scratch_buf.p + need;

  {
    FillBatch f{};
    f.p[0] = (uint64_t*)t.bmax;
    f.p[1] = (uint64_t*)t.bad;
    f.p[2] = (uint64_t*)(t.bad + 6);  // B binary until an entry says not
    f.n[0] = f.n[1] = f.n[2] = 1;
    f.v[2] = 1;
    f.count = 3;
    if ((e = launch_fill_multi(f, st)) != hipSuccess) return e;
  }
  if (check)
    k_scan_inputs<<<grid_for(m * d, 1024 * 16) > 256 ? 256
                        : grid_for(m * d, 1024 * 16), 1024, 0, st>>>(
        A, m * d, nullptr, t.bad);

  // the B side forks from here (after the clears above)
  // MAD_TABLES_ONE_STREAM=1 keeps the B side on the caller's stream (the
  // tables are the same; for timing the kernels apart)
  static const bool one_stream = [] {
    const char* v = getenv("MAD_TABLES_ONE_STREAM");
    return v && atoi(v) != 0;
  }();
  hipStream_t sd = one_stream ? st : t.side;
  if (B && !one_stream && (e = hipEventRecord(t.fork, st)) != hipSuccess)
    return e;
  // T0 on the aux stream (it needs no scratch when it has at most 512
  // slots), started by the T1 and T2 totals
  const bool t0_aux = B && !one_stream && t.T0.L <= 9;
  t.t0_aux = 0;
  // T3[i]: k' given i, weight |a_k'i|; totals na_i (the draw of k' in
  // Alg. 3)
  // (enqueued before the B side so that this stream has work at once)
  if (t.T3.L <= 9) {
    e = small_tables(WRowAbs{A, d}, m, d, t.T3.L, t.T3.tot, t.T3.ent, st);
  } else {
    e = uniform_quanta(WRowAbs{A, d}, m, d, t.T3.L, t.T3.tot, q, runbuf, st);
    if (e == hipSuccess)
      e = build_alias(q, t.T3.tot, m, t.T3.L, t.T3.ent, abuf,
                      alias_bytes, st);
  }
  if (e != hipSuccess) return e;
  // B side on the side stream: max |b| (and the finiteness check), then
  // T2[k]: j given k, weight |b_kj|; totals nb_k (the draw of j in
  // Alg. 3)
  if (B) {
    if (!one_stream && (e = hipStreamWaitEvent(sd, t.fork, 0)) != hipSuccess)
      return e;
    k_scan_inputs<<<grid_for(n * d, 1024 * 16) > 256 ? 256
                        : grid_for(n * d, 1024 * 16), 1024, 0, sd>>>(
        B, n * d, t.bmax, t.bad);
    {
      const int64_t waves = (n * d + 63) / 64;
      int64_t blocks = (waves + 3) / 4;
      if (blocks > 4096) blocks = 4096;
      k_binary_bitmap<<<(unsigned)blocks, 256, 0, sd>>>(B, n * d, t.bbits,
                                                        t.bad + 6);
    }
    if (t.T2.L <= 9) {
      e = small_tables(WColAbs{B, d, nullptr}, d, n, t.T2.L, t.T2.tot,
                       t.T2.ent, sd);
      if (e == hipSuccess && t0_aux) e = hipEventRecord(t.t2tot, sd);
    } else {
      e = col_tables(B, d, nullptr, d, n, t.T2.L, t.T2, side_scratch,
                     need_side, sd, t0_aux ? t.t2tot : nullptr);
    }
    const hipError_t ej =
        one_stream ? hipSuccess : hipEventRecord(t.join, sd);
    if (e == hipSuccess) e = ej;
    if (e != hipSuccess) return e;
  }

  // T1[k]: i given k, weight |a_ki| na_i; totals v_k
  if (e == hipSuccess) {
    if (t.T1.L <= 9) {
      e = small_tables(WColAbs{A, d, t.na}, d, m, t.T1.L, t.T1.tot, t.T1.ent,
                       st);
      if (e == hipSuccess && t0_aux) e = hipEventRecord(t.t1tot, st);
    } else {
      e = col_tables(A, d, t.na, d, m, t.T1.L, t.T1, scratch_buf.p, need, st,
                     t0_aux ? t.t1tot : nullptr);
    }
  }
  // T0: k with weight nb_k v_k; total ||W||_1 (the weights w_ki
  // of Alg. 3 and its draw of (k, i)).  On the aux stream it runs beside
  // the rest of T1 and T2, and the caller's stream waits for it.
  if (e == hipSuccess && t0_aux) {
    if ((e = hipStreamWaitEvent(t.aux, t.t1tot, 0)) != hipSuccess ||
        (e = hipStreamWaitEvent(t.aux, t.t2tot, 0)) != hipSuccess)
      return e;
    k_stage0_weights<<<grid_for(d, 256), 256, 0, t.aux>>>(t.nb, t.v, d,
                                                          t.om);
    if ((e = small_tables(WExplicit{t.om}, 1, d, t.T0.L, t.T0.tot, t.T0.ent,
                          t.aux)) != hipSuccess ||
        (e = hipEventRecord(t.t0done, t.aux)) != hipSuccess)
      return e;
    t.t0_aux = 1;
  }
  // the B side joins here; without B (MIPS) only the A side is built
  if (B && !one_stream) {
    const hipError_t ew = hipStreamWaitEvent(st, t.join, 0);
    if (e == hipSuccess) e = ew;
  }
  if (e == hipSuccess && t.t0_aux) e = hipStreamWaitEvent(st, t.t0done, 0);
  if (e != hipSuccess || !B || t.t0_aux) return e;
  if (e == hipSuccess) {
    k_stage0_weights<<<grid_for(d, 256), 256, 0, st>>>(t.nb, t.v, d, t.om);
    if (t.T0.L <= 9) {
      e = small_tables(WExplicit{t.om}, 1, d, t.T0.L, t.T0.tot, t.T0.ent, st);
    } else {
      e = uniform_quanta(WExplicit{t.om}, 1, d, t.T0.L, t.T0.tot, q, runbuf,
                         st);
      if (e == hipSuccess)
        e = build_alias(q, t.T0.tot, 1, t.T0.L, t.T0.ent, abuf,
                        alias_bytes, st);
    }
  }
  return e;
}

// ---------------------------------------------------------------------------
// MIPS stage-0 tables: one table per query over the d coordinates with
// weight |q_k| v_k (a one-vector B has ||B_k*||_1 = |q_k|, so this is
// nb_k v_k of the general plan).  Scratch is used only when 2^L > 512.
// ---------------------------------------------------------------------------
size_t query_tables_scratch_bytes(int64_t nq, int64_t d) {
  const int L = ceil_log2_host(d);
  if (L <= 9) return 256;  // small tables need no scratch
  const int64_t slots = nq << L;
  int64_t batch = slots < ((int64_t)1 << 26) ? slots : ((int64_t)1 << 26);
  if (batch < ((int64_t)1 << L)) batch = (int64_t)1 << L;
  return (size_t)slots * 8 + run_doubles(nq, d) * 8 +
         alias_scratch_bytes(batch, batch / kAliasBlk) + 1024;
}

hipError_t query_tables_build(const float* Q, int64_t nq, int64_t d,
                              const double* v, Family& T0q, void* scratch,
                              size_t scratch_bytes, hipStream_t st) {
  const WQuery w{Q, d, v};
  if (T0q.L <= 9) return small_tables(w, nq, d, T0q.L, T0q.tot, T0q.ent, st);
  char* p = (char*)scratch;
  uint64_t* q = (uint64_t*)p; p += (size_t)(nq << T0q.L) * 8;
  double* runbuf = (double*)p; p += run_doubles(nq, d) * 8;
  const size_t used = (size_t)(p - (char*)scratch);
  if (!scratch || scratch_bytes < used) return hipErrorInvalidValue;
  hipError_t e = uniform_quanta(w, nq, d, T0q.L, T0q.tot, q, runbuf, st);
  if (e != hipSuccess) return e;
  return build_alias(q, T0q.tot, nq, T0q.L, T0q.ent, p,
                     scratch_bytes - used, st);
}

size_t stage0_scratch_bytes(int64_t N) {
  return query_tables_scratch_bytes(1, N);
}

hipError_t stage0_table_build(const double* w, int64_t N, Family& T,
                              void* scratch, size_t scratch_bytes,
                              hipStream_t st) {
  const WExplicit wf{w};
  if (T.L <= 9) return small_tables(wf, 1, N, T.L, T.tot, T.ent, st);
  char* p = (char*)scratch;
  uint64_t* q = (uint64_t*)p; p += (size_t)8 << T.L;
  double* runbuf = (double*)p; p += run_doubles(1, N) * 8;
  const size_t used = (size_t)(p - (char*)scratch);
  if (!scratch || scratch_bytes < used) return hipErrorInvalidValue;
  hipError_t e = uniform_quanta(wf, 1, N, T.L, T.tot, q, runbuf, st);
  if (e != hipSuccess) return e;
  return build_alias(q, T.tot, 1, T.L, T.ent, p, scratch_bytes - used,
                     st);
}

hipError_t family_alloc_pub(Family& f, int64_t S, int64_t N) {
  return family_alloc(f, S, N);
}

void family_free_pub(Family& f) { family_free(f); }

}  // namespace mad
