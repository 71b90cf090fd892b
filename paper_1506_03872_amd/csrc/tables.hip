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

// max |x| (as float bits, atomically) and a flag for non-finite entries;
// float4 loads when X is 16-byte aligned
__global__ void k_scan_inputs(const float* X, int64_t n, float* amax,
                              int* bad) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  float mx = 0.0f;
  int nonfinite = 0;
  int64_t done = 0;
  if (((uintptr_t)X & 15) == 0) {
    const float4* X4 = (const float4*)X;
    const int64_t n4 = n / 4;
    for (int64_t e = tid; e < n4; e += stride) {
      const float4 v = X4[e];
      nonfinite |= !isfinite(v.x) | !isfinite(v.y) | !isfinite(v.z) |
                   !isfinite(v.w);
      mx = fmaxf(mx, fmaxf(fmaxf(fabsf(v.x), fabsf(v.y)),
                           fmaxf(fabsf(v.z), fabsf(v.w))));
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
  // one pair of atomics per block
  __shared__ float bmx[4];
  __shared__ int bnf[4];
  if ((threadIdx.x & 63) == 0) {
    bmx[threadIdx.x >> 6] = mx;
    bnf[threadIdx.x >> 6] = nonfinite;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    mx = fmaxf(fmaxf(bmx[0], bmx[1]), fmaxf(bmx[2], bmx[3]));
    nonfinite = bnf[0] | bnf[1] | bnf[2] | bnf[3];
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

// Column families (one table per coordinate k over the vectors): a wave
// handles one run of 64 consecutive tables, lane = table, so every load reads
// 64 consecutive floats of one vector.  Loads are issued kColGroup at a time
// (clamped to the last row, so they carry no branch and stay in flight
// together) ahead of the sequential adds, and quanta go out through an LDS
// transpose so each store writes 64 consecutive slots of one table.  The
// sign bit of each item is kept in bit 63 of its quantum (quanta are below
// 2^62) for the alias construction.
constexpr int kColGroup = 32;

// Column run walk: a wave handles one run of 64 consecutive tables, lane =
// table, and writes each item's run-local prefix l_r (FP64 bits, the item's
// sign bit in bit 63; l >= 0) through an LDS transpose into the
// table-major layout of the quanta.  The run total is l at the run's last
// item.  Loads are issued kColGroup at a time, clamped to the last row so
// they carry no branch and stay in flight together.
__global__ __launch_bounds__(64) void k_col_local(
    const float* X, int64_t d, const double* scale, int64_t S, int64_t N,
    int L, uint64_t* Lbuf) {
  __shared__ uint64_t buf[64][65];
  const int64_t tiles = (S + 63) / 64;
  const int64_t c = blockIdx.x / tiles;
  const int64_t seg0 = (blockIdx.x % tiles) * 64;
  const int lane = threadIdx.x;
  const int64_t seg = seg0 + lane;
  const int64_t segc = seg < S ? seg : S - 1;
  const int64_t r0 = c * kRun;
  const int64_t r1 = N < r0 + kRun ? N : r0 + kRun;
  double l = 0.0;
  for (int64_t g0 = r0; g0 < r1; g0 += 64) {
#pragma unroll
    for (int h = 0; h < 64; h += kColGroup) {
      float xv[kColGroup];
      double sv[kColGroup];
#pragma unroll
      for (int u = 0; u < kColGroup; ++u) {
        const int64_t r = g0 + h + u < r1 ? g0 + h + u : r1 - 1;
        xv[u] = X[r * d + segc];
        sv[u] = scale ? scale[r] : 1.0;
      }
#pragma unroll
      for (int u = 0; u < kColGroup; ++u) {
        const int64_t r = g0 + h + u;
        uint64_t bits = 0;
        if (r < r1) {
          const double w = scale ? fabs((double)xv[u]) * sv[u]
                                 : fabs((double)xv[u]);
          l = r == r0 ? w : l + w;
          bits = (uint64_t)__double_as_longlong(l) |
                 ((uint64_t)sign_bit(xv[u]) << 63);
        }
        buf[h + u][lane] = bits;
      }
    }
    __syncthreads();
    const int64_t r = g0 + lane;
    if (r < r1)
      for (int sl = 0; sl < 64 && seg0 + sl < S; ++sl)
        Lbuf[((seg0 + sl) << L) + r] = buf[lane][sl];
    __syncthreads();
  }
}

// run offsets from the stored run-local prefixes: E_0 = 0,
// E_{c+1} = E_c + l(last item of run c); total T = E_R.  One 64-thread
// block per table: the run totals are gathered in parallel into LDS, then
// one lane adds them left to right.
constexpr int kOffChunk = 2048;

__global__ __launch_bounds__(64) void k_col_offsets(const uint64_t* Lbuf,
                                                    int64_t S, int64_t N,
                                                    int L, double* E,
                                                    double* tot) {
  __shared__ double buf[kOffChunk];
  const int64_t seg = blockIdx.x;
  const int64_t R = (N + kRun - 1) / kRun;
  double e = 0.0;  // lane 0's running offset
  for (int64_t c0 = 0; c0 < R; c0 += kOffChunk) {
    const int64_t nc = R - c0 < kOffChunk ? R - c0 : kOffChunk;
    for (int64_t u = threadIdx.x; u < nc; u += 64) {
      const int64_t c = c0 + u;
      const int64_t last = (N < (c + 1) * kRun ? N : (c + 1) * kRun) - 1;
      const uint64_t raw = Lbuf[(seg << L) + last] & ~(1ull << 63);
      buf[u] = __longlong_as_double((long long)raw);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int64_t u = 0; u < nc; ++u) {
        const double sc = buf[u];
        buf[u] = e;  // E_c
        e = e + sc;
      }
    }
    __syncthreads();
    for (int64_t u = threadIdx.x; u < nc; u += 64) E[(c0 + u) * S + seg] = buf[u];
    __syncthreads();
  }
  if (threadIdx.x == 0) tot[seg] = e;
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
// one wave per table from stored quanta (2^L <= 64 * SPL <= 512 slots;
// 4 tables per block use at most 40 KB of LDS)
template <int SPL>
__global__ __launch_bounds__(256) void k_alias_wave(const uint64_t* q,
                                                    const double* tot,
                                                    int64_t S, int L,
                                                    uint64_t* ent) {
  extern __shared__ uint64_t smem64[];
  const int Np = 1 << L;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t seg = (int64_t)blockIdx.x * 4 + wv;
  const bool active = seg < S && tot[seg < S ? seg : 0] > 0.0;
  if (seg < S && !active)  // dead table: never sampled, entries zero
    for (int r = lane; r < Np; r += 64) ent[(seg << L) + r] = 0ull;
  uint64_t qv[SPL];
  uint32_t sg[SPL];
#pragma unroll
  for (int s = 0; s < SPL; ++s) {
    const int r = lane * SPL + s;
    const uint64_t raw = active && r < Np ? q[(seg << L) + r] : 0ull;
    qv[s] = raw & kQMask;
    sg[s] = (uint32_t)(raw >> 63);
  }
  wave_alias<SPL>(qv, sg, active, L, smem64 + (int64_t)wv * 2 * Np,
                  smem64 + (int64_t)wv * 2 * Np + Np,
                  (uint32_t*)(smem64 + 8 * Np) + (int64_t)wv * Np,
                  EmitPacked{ent + (seg << L)});
}


static hipError_t alias_small(const uint64_t* q, const double* tot, int64_t S,
                              int L, uint64_t* ent, hipStream_t st) {
  const int Np = 1 << L;
  const size_t lds = (size_t)4 * Np * 20;
  const unsigned blocks = grid_for(S, 4);
  if (Np <= 64)
    k_alias_wave<1><<<blocks, 256, lds, st>>>(q, tot, S, L, ent);
  else if (Np <= 128)
    k_alias_wave<2><<<blocks, 256, lds, st>>>(q, tot, S, L, ent);
  else if (Np <= 256)
    k_alias_wave<4><<<blocks, 256, lds, st>>>(q, tot, S, L, ent);
  else
    k_alias_wave<8><<<blocks, 256, lds, st>>>(q, tot, S, L, ent);
  return hipGetLastError();
}

// Small tables (N <= 2^L <= 512 items), one lane per table: the total in
// the two-level order, then the same prefix again with F_r = floor(2^K P_r
// / T) and q_r = F_r - F_{r-1} (the item's sign bit in bit 63); padding
// slots and dead tables get q = 0.  Every lane walks its own table, so the
// sequential FP64 chain keeps all lanes busy.  Two-level order inside one
// lane: l restarts at each run, E collects the run totals, P_r = E + l_r
// (E = 0 in the first run, where 0 + l_r = l_r exactly).  Loads go 8 at a
// time; every 8 slots the block's quanta pass through LDS so that each
// store writes 64 consecutive bytes of 8 tables.
template <class W>
__global__ __launch_bounds__(64) void k_lane_quanta(W w, int64_t S, int64_t N,
                                                    int L, double* tot,
                                                    uint64_t* q) {
  __shared__ uint64_t tq[64][9];
  const int lane = threadIdx.x;
  const int64_t seg0 = (int64_t)blockIdx.x * 64;
  const int64_t nseg = S - seg0 < 64 ? S - seg0 : 64;
  const int64_t seg = seg0 + (lane < nseg ? lane : nseg - 1);
  const bool mine = lane < nseg;
  const int64_t Np = int64_t(1) << L;
  double E = 0.0, l = 0.0;
  for (int64_t r0 = 0; r0 < N; r0 += 8) {
    double wv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) wv[u] = w(seg, r0 + u < N ? r0 + u : N - 1);
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t r = r0 + u;
      if (r < N) {
        if (r > 0 && r % kRun == 0) {
          E = E + l;
          l = 0.0;
        }
        l = l + wv[u];
      }
    }
  }
  const double T = E + l;
  if (mine) tot[seg] = T;
  const bool live = mine && T > 0.0;
  const int K = L + kCapBits;
  E = 0.0;
  l = 0.0;
  uint64_t Fp = 0;
  for (int64_t r0 = 0; r0 < Np; r0 += 8) {
    double wv[8];
    uint32_t sv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t rr = r0 + u < N ? r0 + u : N - 1;
      wv[u] = live ? w(seg, rr) : 0.0;
      sv[u] = live ? w.sgn(seg, rr) : 0u;
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t r = r0 + u;
      uint64_t qq = 0;
      if (live && r < N) {
        if (r > 0 && r % kRun == 0) {
          E = E + l;
          l = 0.0;
        }
        l = l + wv[u];
        const uint64_t F = (uint64_t)floor(ldexp((E + l) / T, K));
        qq = (F - Fp) | ((uint64_t)sv[u] << 63);
        Fp = F;
      }
      tq[lane][u] = qq;
    }
    __syncthreads();
    // lanes 8t .. 8t+7 write slots r0 .. r0+7 of table t (8 tables a pass)
    const int64_t nc = Np - r0 < 8 ? Np - r0 : 8;
    for (int t0 = 0; t0 < 64; t0 += 8) {
      const int sl = t0 + (lane >> 3), u = lane & 7;
      if (sl < nseg && u < nc) q[((seg0 + sl) << L) + r0 + u] = tq[sl][u];
    }
    __syncthreads();
  }
}

template <class W>
static hipError_t small_tables_q(W w, int64_t S, int64_t N, int L,
                                 double* tot, uint64_t* q, uint64_t* ent,
                                 hipStream_t st) {
  k_lane_quanta<W><<<grid_for(S, 64), 64, 0, st>>>(w, S, N, L, tot, q);
  return alias_small(q, tot, S, L, ent, st);
}

// large tables (2^L >= 1024 slots): blocks of 1024 slots (256 threads x 4)
// never straddle a table
constexpr int kAliasBlk = 1024;

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

// Quanta from stored prefixes, one thread per 4 consecutive slots:
// q_r = F_r - F_{r-1}, F_r = floor(2^K P_r / T) (F_{-1} = 0); padding and
// dead tables get q = 0.  Blocks cover 1024 slots; when bs is given (tables
// of >= 1024 slots) each block also writes its alias statistics.
__global__ __launch_bounds__(256) void k_q_from_prefix(
    const uint64_t* Lbuf, const double* E, const double* tot, int64_t S,
    int64_t N, int L, uint64_t* q, Quad* bs) {
  const int64_t total = S << L;
  const int64_t base = (int64_t)blockIdx.x * kAliasBlk + threadIdx.x * 4;
  const int64_t Np = int64_t(1) << L;
  const int K = L + kCapBits;
  Quad a{0, 0, 0, 0};
  uint64_t Fp = 0;  // F of the previous item of the same table
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const int64_t slot = base + s;
    if (slot >= total) break;
    const int64_t seg = slot >> L;
    const int64_t r = slot & (Np - 1);
    const double T = tot[seg];
    const bool live = T > 0.0;
    if (s == 0 || r == 0) {
      // the prefix of item r-1; at a run start it is exactly E_c
      Fp = 0;
      if (live && r > 0 && r - 1 < N) {
        const int64_t cp = (r - 1) / kRun;
        const uint64_t raw = Lbuf[slot - 1] & kQMask;
        const double Pp = E[cp * S + seg] +
                          __longlong_as_double((long long)raw);
        Fp = (uint64_t)floor(ldexp(Pp / T, K));
      }
    }
    uint64_t qq = 0;
    if (live && r < N) {
      const uint64_t raw = Lbuf[slot];
      const double Pv = E[(r / kRun) * S + seg] +
                        __longlong_as_double((long long)(raw & kQMask));
      const uint64_t F = (uint64_t)floor(ldexp(Pv / T, K));
      qq = (F - Fp) | (raw & ~kQMask);
      Fp = F;
    }
    q[slot] = qq;
    slot_stats(qq & kQMask, a);
  }
  if (bs) {
    Quad all = block_excl_scan(a);
    if (threadIdx.x == 0) bs[blockIdx.x] = all;
  }
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

// merge-path split of every block edge (kMergeBlk positions apart)
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

__global__ __launch_bounds__(256) void k_alias_merge(
    const uint64_t* Ld, const uint32_t* Li, const uint64_t* He,
    const uint32_t* Hi, const uint64_t* NLa, const uint64_t* NHa,
    const uint64_t* Dta, const int64_t* edges, const double* tot,
    int64_t seg0, int L, uint64_t* ent) {
  __shared__ uint64_t sD[kMergeBlk + 1], sE[kMergeBlk + 1];
  __shared__ uint32_t sLi[kMergeBlk + 1], sHi[kMergeBlk + 1];
  const int64_t Np = int64_t(1) << L;
  const int64_t blocks_per = Np / kMergeBlk;
  const int64_t segl = blockIdx.x / blocks_per;
  const int64_t bi = blockIdx.x % blocks_per;
  const int64_t seg = seg0 + segl;
  const int64_t d0 = bi * kMergeBlk;
  uint64_t* et = ent + (seg << L);
  if (!(tot[seg] > 0.0)) {  // dead table: never sampled, entries zero
    for (int u = threadIdx.x; u < kMergeBlk; u += 256) et[d0 + u] = 0ull;
    return;
  }
  const int64_t tb = segl << L;
  const int64_t NL = (int64_t)NLa[segl], NH = (int64_t)NHa[segl];
  const uint64_t Dt = Dta[segl];
  const uint64_t* D = Ld + tb;
  const uint64_t* E = He + tb;
  const int64_t* ed = edges + segl * (blocks_per + 1) + bi;
  const int64_t a0 = ed[0], b0 = d0 - ed[0];
  const int64_t na = ed[1] - a0, nb = (d0 + kMergeBlk - ed[1]) - b0;
  // slices, plus one element past each end (the next D bounds a light's
  // quantum; the next heavy id closes a heavy)
  for (int u = threadIdx.x; u <= na; u += 256) {
    sD[u] = a0 + u < NL ? D[a0 + u] : Dt;
    sLi[u] = a0 + u < NL ? Li[tb + a0 + u] : 0u;
  }
  for (int u = threadIdx.x; u <= nb; u += 256) {
    sE[u] = b0 + u < NH ? E[b0 + u] : ~0ull;
    sHi[u] = b0 + u < NH ? Hi[tb + b0 + u] : 0u;
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

// bsf: block statistics of the whole family (from k_q_from_prefix), or
// null to compute them here
static hipError_t alias_large(const uint64_t* q, const double* tot, int64_t S,
                              int L, uint64_t* ent, Quad* bsf, void* scratch,
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
    if (bsf) bs = bsf + (s0 << L) / kAliasBlk;
    else k_alias_blocksum<<<(unsigned)nblk, 256, 0, st>>>(qb, bs);
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
                              int L, uint64_t* ent, Quad* bsf, void* scratch,
                              size_t scratch_bytes, hipStream_t st) {
  if (L <= 9) return alias_small(q, tot, S, L, ent, st);
  return alias_large(q, tot, S, L, ent, bsf, scratch, scratch_bytes, st);
}

// Column families: one serial pass of run-local prefixes, the run offsets,
// then quanta (and, for tables of >= 1024 slots, the alias block
// statistics) in parallel.
static hipError_t col_quanta(const float* X, int64_t d, const double* scale,
                             int64_t S, int64_t N, int L, double* tot,
                             uint64_t* q, uint64_t* Lbuf, double* runbuf,
                             Quad* bsf, hipStream_t st) {
  const int64_t R = (N + kRun - 1) / kRun;
  const int64_t tiles = (S + 63) / 64;
  double* E = runbuf;  // R * S
  k_col_local<<<(unsigned)(R * tiles), 64, 0, st>>>(X, d, scale, S, N, L,
                                                    Lbuf);
  k_col_offsets<<<(unsigned)S, 64, 0, st>>>(Lbuf, S, N, L, E, tot);
  const int64_t total = S << L;
  k_q_from_prefix<<<grid_for(total, kAliasBlk), 256, 0, st>>>(
      Lbuf, E, tot, S, N, L, q, L >= 10 ? bsf : nullptr);
  return hipGetLastError();
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
  // scratch: quanta and prefixes of the largest family, run sums, block
  // statistics, alias lists (batched to at most 2^26 slots)
  size_t qslots = 0, runs = 0, blks = 0, alias_slots = 0;
  const Family* fams[4] = {&t.T0, &t.T1, &t.T2, &t.T3};
  for (const Family* f : fams) {
    const size_t sl = (size_t)(f->S << f->L);
    if (sl > qslots) qslots = sl;
    const size_t r = run_doubles(f->S, f->N);
    if (r > runs) runs = r;
    if (f->L > 9) {
      if (sl / kAliasBlk > blks) blks = sl / kAliasBlk;
      if (sl > alias_slots) alias_slots = sl;
    }
  }
  if (alias_slots > ((size_t)1 << 26)) alias_slots = (size_t)1 << 26;
  for (const Family* f : fams)  // at least one table per batch
    if (f->L > 9 && alias_slots < ((size_t)1 << f->L))
      alias_slots = (size_t)1 << f->L;
  const size_t alias_bytes =
      alias_slots ? alias_scratch_bytes((int64_t)alias_slots,
                                        (int64_t)alias_slots / kAliasBlk) : 0;
  const size_t total = 2 * qslots * 8 + runs * 8 + blks * sizeof(Quad) +
                       alias_bytes + 1024;
  hipError_t e = dev_alloc(scratch_buf, total);
  if (e != hipSuccess) return e;
  char* p = (char*)scratch_buf.p;
  uint64_t* q = (uint64_t*)p; p += qslots * 8;
  uint64_t* Pbuf = (uint64_t*)p; p += qslots * 8;
  double* runbuf = (double*)p; p += runs * 8;
  Quad* bsf = (Quad*)p; p += blks * sizeof(Quad);
  void* abuf = p;

  if ((e = launch_fill_u64((uint64_t*)t.bmax, 1, 0ull, st)) != hipSuccess ||
      (e = launch_fill_u64((uint64_t*)t.bad, 1, 0ull, st)) != hipSuccess)
    return e;
  if (check)
    k_scan_inputs<<<grid_for(m * d, 256 * 16) > 1024 ? 1024
                        : grid_for(m * d, 256 * 16), 256, 0, st>>>(
        A, m * d, nullptr, t.bad);
  if (B)
    k_scan_inputs<<<grid_for(n * d, 256 * 16) > 1024 ? 1024
                        : grid_for(n * d, 256 * 16), 256, 0, st>>>(
        B, n * d, t.bmax, t.bad);

  // T3[i]: k' given i, weight |a_k'i|; totals na_i (Alg. 2 line "ds3")
  if (t.T3.L <= 9) {
    e = small_tables_q(WRowAbs{A, d}, m, d, t.T3.L, t.T3.tot, q, t.T3.ent,
                       st);
  } else {
    e = uniform_quanta(WRowAbs{A, d}, m, d, t.T3.L, t.T3.tot, q, runbuf, st);
    if (e == hipSuccess)
      e = build_alias(q, t.T3.tot, m, t.T3.L, t.T3.ent, nullptr, abuf,
                      alias_bytes, st);
  }
  // T1[k]: i given k, weight |a_ki| na_i; totals v_k
  if (e == hipSuccess)
    e = col_quanta(A, d, t.na, d, m, t.T1.L, t.T1.tot, q, Pbuf, runbuf, bsf,
                   st);
  if (e == hipSuccess)
    e = build_alias(q, t.T1.tot, d, t.T1.L, t.T1.ent, bsf, abuf, alias_bytes,
                    st);
  // without B (MIPS) only the A side is built
  if (e != hipSuccess || !B) return e;
  // T2[k]: j given k, weight |b_kj|; totals nb_k (Alg. 2 line "ds2")
  if (e == hipSuccess)
    e = col_quanta(B, d, nullptr, d, n, t.T2.L, t.T2.tot, q, Pbuf, runbuf,
                   bsf, st);
  if (e == hipSuccess)
    e = build_alias(q, t.T2.tot, d, t.T2.L, t.T2.ent, bsf, abuf, alias_bytes,
                    st);
  // T0: k with weight nb_k v_k; total ||W||_1 (Alg. 2 lines "dw", "ds1")
  if (e == hipSuccess) {
    k_stage0_weights<<<grid_for(d, 256), 256, 0, st>>>(t.nb, t.v, d, t.om);
    if (t.T0.L <= 9) {
      e = small_tables_q(WExplicit{t.om}, 1, d, t.T0.L, t.T0.tot, q, t.T0.ent,
                         st);
    } else {
      e = uniform_quanta(WExplicit{t.om}, 1, d, t.T0.L, t.T0.tot, q, runbuf,
                         st);
      if (e == hipSuccess)
        e = build_alias(q, t.T0.tot, 1, t.T0.L, t.T0.ent, nullptr, abuf,
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
  if (L <= 9) return (size_t)(nq << L) * 8 + 256;
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
  if (T0q.L <= 9) {
    if (!scratch || scratch_bytes < (size_t)(nq << T0q.L) * 8)
      return hipErrorInvalidValue;
    return small_tables_q(w, nq, d, T0q.L, T0q.tot, (uint64_t*)scratch,
                          T0q.ent, st);
  }
  char* p = (char*)scratch;
  uint64_t* q = (uint64_t*)p; p += (size_t)(nq << T0q.L) * 8;
  double* runbuf = (double*)p; p += run_doubles(nq, d) * 8;
  const size_t used = (size_t)(p - (char*)scratch);
  if (!scratch || scratch_bytes < used) return hipErrorInvalidValue;
  hipError_t e = uniform_quanta(w, nq, d, T0q.L, T0q.tot, q, runbuf, st);
  if (e != hipSuccess) return e;
  return build_alias(q, T0q.tot, nq, T0q.L, T0q.ent, nullptr, p,
                     scratch_bytes - used, st);
}

size_t stage0_scratch_bytes(int64_t N) {
  return query_tables_scratch_bytes(1, N);
}

hipError_t stage0_table_build(const double* w, int64_t N, Family& T,
                              void* scratch, size_t scratch_bytes,
                              hipStream_t st) {
  const WExplicit wf{w};
  if (T.L <= 9) {
    if (!scratch || scratch_bytes < ((size_t)8 << T.L)) return hipErrorInvalidValue;
    return small_tables_q(wf, 1, N, T.L, T.tot, (uint64_t*)scratch, T.ent,
                          st);
  }
  char* p = (char*)scratch;
  uint64_t* q = (uint64_t*)p; p += (size_t)8 << T.L;
  double* runbuf = (double*)p; p += run_doubles(1, N) * 8;
  const size_t used = (size_t)(p - (char*)scratch);
  if (!scratch || scratch_bytes < used) return hipErrorInvalidValue;
  hipError_t e = uniform_quanta(wf, 1, N, T.L, T.tot, q, runbuf, st);
  if (e != hipSuccess) return e;
  return build_alias(q, T.tot, 1, T.L, T.ent, nullptr, p, scratch_bytes - used,
                     st);
}

hipError_t family_alloc_pub(Family& f, int64_t S, int64_t N) {
  return family_alloc(f, S, N);
}

void family_free_pub(Family& f) { family_free(f); }

}  // namespace mad
