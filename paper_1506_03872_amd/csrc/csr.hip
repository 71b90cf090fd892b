// csr.hip -- sparse inputs: vectors as compressed rows (coordinates
// strictly increasing within a vector), the setting of the paper's graph and
// rating experiments (Sec. 6).
//
// Preprocessing builds the same four stage distributions as the dense plan
// (the weights w_ki of Alg. 3 in the two-stage form), but over the non-zeros only:
//   T3[i]  over the entries of a_i            weight |a_k'i|
//   T1[k]  over the vectors i with an entry k weight |a_ki| na_i
//   T2[k]  over the vectors j with an entry k weight |b_kj|
//   T0     over the coordinates               weight ||B_k*||_1 v_k
// T1 and T2 need, per coordinate, its vectors in ascending order: a stable
// LSD radix sort of the entries by coordinate (4-bit digits) gives the
// transposes.  Tables have 2^ceil(log2 N) slots of 16-byte entries that
// carry the item ids, so a draw is one load (T1's and T2's entries are 32
// bytes: they also carry T3's meta word of each item i, and the coordinate
// signature of each vector j).  Tables of at most 512
// items are built one wave per table; larger ones one workgroup per table
// (two-level FP64 sums, integer quanta, then the alias lists and their
// merge, as in the dense builder).
//
// The sampler draws k, i, j, k' as the dense one does and reads the fourth
// edge b_k'j from an open-addressing table of B's entries keyed by
// j d + k' + 1 (0 when b_j stores no coordinate k').  The signature of b_j,
// one bit per coordinate hash, settles most absent k' without a probe.
#include <string.h>

#include <algorithm>
#include <vector>

#include "alias_common.hpp"
#include "mad_common.hpp"
#include "plan.hpp"

namespace mad {

static inline unsigned blocks_of(int64_t n, int per) {
  int64_t g = (n + per - 1) / per;
  return (unsigned)(g < 1 ? 1 : g);
}

// the signature bit of coordinate k: the top six bits of k times the
// golden-ratio constant (Fibonacci hashing).  A vector's signature ORs the
// bits of its coordinates, so a clear bit proves the coordinate absent.
__host__ __device__ __forceinline__ uint64_t coord_bit(uint64_t k) {
  return 1ull << ((k * 0x9E3779B97F4A7C15ull) >> 58);
}

static inline int ceil_log2_i(int64_t N) {
  int L = 0;
  while ((int64_t(1) << L) < N) ++L;
  return L;
}

// ---------------------------------------------------------------------------
// validation (one thread per vector): structure errors set bit 2 of *bad,
// non-finite values bit 1; amax (optional) receives max |value|
// ---------------------------------------------------------------------------
__global__ void k_csr_check(const int64_t* ptr, const int32_t* idx,
                            const float* val, int64_t rows, int64_t d,
                            int64_t nnz, float* amax, int* bad) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  float mx = 0.0f;
  int flag = 0;
  if (r < rows) {
    const int64_t p0 = ptr[r], p1 = ptr[r + 1];
    if (r == 0 && p0 != 0) flag |= 2;
    if (p0 < 0 || p1 < p0 || p1 > nnz) {
      flag |= 2;
    } else {
      int64_t prev = -1;
      for (int64_t e = p0; e < p1; ++e) {
        const int64_t k = idx[e];
        const float v = val[e];
        if (k <= prev || k >= d) flag |= 2;
        prev = k;
        if (!isfinite(v)) flag |= 1;
        mx = fmaxf(mx, fabsf(v));
      }
    }
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    mx = fmaxf(mx, __shfl_xor(mx, off, 64));
    flag |= __shfl_xor(flag, off, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    if (flag) atomicOr(bad, flag);
    else if (amax) atomicMax((unsigned int*)amax, __float_as_uint(mx));
  }
}

// row id of every entry (one wave per vector)
__global__ void k_row_ids(const int64_t* ptr, int64_t rows, uint32_t* rowid) {
  const int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int lane = threadIdx.x & 63;
  if (r >= rows) return;
  for (int64_t e = ptr[r] + lane; e < ptr[r + 1]; e += 64)
    rowid[e] = (uint32_t)r;
}

// ---------------------------------------------------------------------------
// exclusive prefix sums of u64 (tiles of 4096, recursive over tile sums)
// ---------------------------------------------------------------------------
constexpr int kScanThreads = 1024;
constexpr int kScanTile = kScanThreads * 4;

__global__ __launch_bounds__(kScanThreads) void k_scan_tiles(
    const uint64_t* in, uint64_t* out, int64_t n, uint64_t* tile_sums) {
  __shared__ uint64_t wsum[kScanThreads / 64];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)t * 4;
  uint64_t v[4], sum = 0;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    v[u] = base + u < n ? in[base + u] : 0ull;
    sum += v[u];
  }
  const uint64_t inc = wave_incl_scan(sum);
  if (lane == 63) wsum[wv] = inc;
  __syncthreads();
  uint64_t off = 0, all = 0;
  for (int w = 0; w < kScanThreads / 64; ++w) {
    off += w < wv ? wsum[w] : 0ull;
    all += wsum[w];
  }
  uint64_t run = off + inc - sum;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    if (base + u < n) out[base + u] = run;
    run += v[u];
  }
  if (t == 0) tile_sums[blockIdx.x] = all;
}

__global__ void k_scan_add(uint64_t* out, int64_t n, const uint64_t* offs) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) out[e] += offs[e / kScanTile];
}

static size_t scan_tmp_words(int64_t n) {
  size_t w = 0;
  while (n > 1) {
    n = (n + kScanTile - 1) / kScanTile;
    w += (size_t)n;
  }
  return w + 1;
}

// in may equal out; tmp holds scan_tmp_words(n) words
static hipError_t scan_u64(const uint64_t* in, uint64_t* out, int64_t n,
                           uint64_t* tmp, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int64_t nt = (n + kScanTile - 1) / kScanTile;
  k_scan_tiles<<<(unsigned)nt, kScanThreads, 0, st>>>(in, out, n, tmp);
  if (nt > 1) {
    hipError_t e = scan_u64(tmp, tmp, nt, tmp + nt, st);
    if (e != hipSuccess) return e;
    k_scan_add<<<blocks_of(n, 256), 256, 0, st>>>(out, n, tmp);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Stable LSD radix sort of (coordinate, payload) pairs by coordinate, 4-bit
// digits; the payload is (vector id << 32 | value bits), so the sorted
// payload is the transpose itself.  A tile of 4096 pairs is 256 threads x
// 16 consecutive pairs.  Per-thread digit counts are 16-bit fields of four
// u64, so one block scan of the four words gives every pair its rank in
// input order; the tile is reordered by digit in LDS and written out in
// runs of consecutive addresses.
// ---------------------------------------------------------------------------
constexpr int kRsThreads = 256;
constexpr int kRsPer = 16;
constexpr int kRsTile = kRsThreads * kRsPer;

struct Cnt16 {
  uint64_t c[4];
};

__device__ __forceinline__ void cnt_add(Cnt16& c, uint32_t dg) {
  const uint64_t inc = 1ull << (16 * (dg & 3));
  switch (dg >> 2) {
    case 0: c.c[0] += inc; break;
    case 1: c.c[1] += inc; break;
    case 2: c.c[2] += inc; break;
    default: c.c[3] += inc; break;
  }
}

__device__ __forceinline__ uint32_t cnt_get(const Cnt16& c, int dg) {
  uint64_t w;
  switch (dg >> 2) {
    case 0: w = c.c[0]; break;
    case 1: w = c.c[1]; break;
    case 2: w = c.c[2]; break;
    default: w = c.c[3]; break;
  }
  return (uint32_t)(w >> (16 * (dg & 3))) & 0xFFFFu;
}

// block exclusive scan of the packed counts (256 threads); returns totals
__device__ Cnt16 cnt_block_scan(Cnt16& v) {
  __shared__ uint64_t ws[4][4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  Cnt16 inc;
#pragma unroll
  for (int x = 0; x < 4; ++x) inc.c[x] = wave_incl_scan(v.c[x]);
  if (lane == 63)
    for (int x = 0; x < 4; ++x) ws[wv][x] = inc.c[x];
  __syncthreads();
  Cnt16 all;
#pragma unroll
  for (int x = 0; x < 4; ++x) {
    uint64_t off = 0, tot = 0;
    for (int w = 0; w < 4; ++w) {
      off += w < wv ? ws[w][x] : 0ull;
      tot += ws[w][x];
    }
    v.c[x] = off + inc.c[x] - v.c[x];
    all.c[x] = tot;
  }
  __syncthreads();
  return all;
}

__device__ __forceinline__ Cnt16 tile_counts(const uint32_t* key, int64_t n,
                                             int shift, int64_t base) {
  Cnt16 c{{0, 0, 0, 0}};
#pragma unroll
  for (int u = 0; u < kRsPer; ++u)
    if (base + u < n) cnt_add(c, (key[base + u] >> shift) & 15u);
  return c;
}

// exclusive prefix over the 16 digit fields of packed totals
__device__ __forceinline__ Cnt16 digit_excl(const Cnt16& all) {
  Cnt16 r{{0, 0, 0, 0}};
  uint64_t run = 0;
#pragma unroll
  for (int dg = 0; dg < 16; ++dg) {
    r.c[dg >> 2] |= run << (16 * (dg & 3));
    run += cnt_get(all, dg);
  }
  return r;
}

__global__ __launch_bounds__(kRsThreads) void k_rs_count(const uint32_t* key,
                                                         int64_t n, int shift,
                                                         uint64_t* counts,
                                                         int64_t ntiles) {
  const int64_t base =
      (int64_t)blockIdx.x * kRsTile + (int64_t)threadIdx.x * kRsPer;
  Cnt16 c = tile_counts(key, n, shift, base);
  const Cnt16 all = cnt_block_scan(c);
#pragma unroll
  for (int dg = 0; dg < 16; ++dg)
    if (threadIdx.x == dg)
      counts[(int64_t)dg * ntiles + blockIdx.x] = cnt_get(all, dg);
}

__global__ __launch_bounds__(kRsThreads) void k_rs_scatter(
    const uint32_t* kin, const uint64_t* vin, int64_t n, int shift,
    const uint64_t* offs, int64_t ntiles, uint32_t* kout, uint64_t* vout) {
  __shared__ uint32_t sk[kRsTile];
  __shared__ uint64_t sv[kRsTile];
  __shared__ uint64_t gbase[16];
  const int t = threadIdx.x;
  const int64_t tile0 = (int64_t)blockIdx.x * kRsTile;
  const int64_t base = tile0 + (int64_t)t * kRsPer;
  const int cnt_tile = n - tile0 < kRsTile ? (int)(n - tile0) : kRsTile;
  if (t < 16) gbase[t] = offs[(int64_t)t * ntiles + blockIdx.x];
  Cnt16 c = tile_counts(kin, n, shift, base);
  const Cnt16 all = cnt_block_scan(c);  // c := this thread's prefix
  const Cnt16 dstart = digit_excl(all);
  // local position of each pair: digit start + earlier pairs of the digit
  Cnt16 run;
#pragma unroll
  for (int x = 0; x < 4; ++x) run.c[x] = dstart.c[x] + c.c[x];
#pragma unroll
  for (int u = 0; u < kRsPer; ++u) {
    const int64_t e = base + u;
    if (e >= n) break;
    const uint32_t k = kin[e];
    const uint32_t dg = (k >> shift) & 15u;
    const uint32_t lp = cnt_get(run, (int)dg);
    cnt_add(run, dg);
    sk[lp] = k;
    sv[lp] = vin[e];
  }
  __syncthreads();
  for (int p = t; p < cnt_tile; p += kRsThreads) {
    const uint32_t k = sk[p];
    const int dg = (int)((k >> shift) & 15u);
    const int64_t g = (int64_t)gbase[dg] + (p - (int)cnt_get(dstart, dg));
    kout[g] = k;
    vout[g] = sv[p];
  }
}

// keys = coordinates, payload = (vector id << 32) | value bits
// key = coordinate, payload = (row, source position of the entry)
__global__ void k_sort_init(const int32_t* idx, const uint32_t* rowid,
                            int64_t n, uint32_t* key, uint64_t* pay) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) {
    key[e] = (uint32_t)idx[e];
    pay[e] = ((uint64_t)rowid[e] << 32) | (uint32_t)e;
  }
}

// tptr[k] = first sorted position with key >= k, for k in [0, d]
__global__ void k_lower_bound(const uint32_t* key, int64_t n, int64_t d,
                              int64_t* tptr) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k > d) return;
  int64_t lo = 0, hi = n;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if ((int64_t)key[mid] < k) lo = mid + 1; else hi = mid;
  }
  tptr[k] = lo;
}

__global__ void k_trans_split(const uint64_t* pay, int64_t n, uint32_t* trow,
                              uint32_t* tsrc) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p < n) {
    const uint64_t v = pay[p];
    trow[p] = (uint32_t)(v >> 32);
    tsrc[p] = (uint32_t)v;
  }
}

// transposed values from the vector-major ones: tval[p] = val[tsrc[p]]
__global__ void k_trans_gather(const uint32_t* tsrc, const float* val,
                               int64_t n, float* tval) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
       p += stride)
    tval[p] = val[tsrc[p]];
}

// max |v| over n values, into *amax (as float bits; values are finite)
__global__ __launch_bounds__(1024) void k_absmax(const float* v, int64_t n,
                                                 float* amax) {
  __shared__ float wm[16];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  float mx = 0.0f;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += stride)
    mx = fmaxf(mx, fabsf(v[e]));
  for (int off = 32; off > 0; off >>= 1)
    mx = fmaxf(mx, __shfl_xor(mx, off, 64));
  if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) mx = fmaxf(mx, wm[w]);
    atomicMax((unsigned int*)amax, __float_as_uint(mx));
  }
}

struct SortBufs {
  uint32_t* k0;
  uint32_t* k1;
  uint64_t* v0;
  uint64_t* v1;
  uint32_t* rowid;
  uint64_t* counts;  // 16 * tiles
  uint64_t* tmp;     // scan scratch
};

static size_t sort_bytes(int64_t nnz) {
  const int64_t tiles = (nnz + kRsTile - 1) / kRsTile;
  return (size_t)nnz * (4 + 4 + 8 + 8 + 4) + (size_t)(16 * tiles + 1) * 8 +
         scan_tmp_words(16 * tiles) * 8 + 8 * 256;
}

static SortBufs sort_carve(void* p, int64_t nnz) {
  const int64_t tiles = (nnz + kRsTile - 1) / kRsTile;
  char* c = (char*)p;
  SortBufs b;
  auto take = [&](size_t bytes) {
    char* r = c;
    c += (bytes + 255) & ~(size_t)255;
    return r;
  };
  b.k0 = (uint32_t*)take((size_t)nnz * 4);
  b.k1 = (uint32_t*)take((size_t)nnz * 4);
  b.v0 = (uint64_t*)take((size_t)nnz * 8);
  b.v1 = (uint64_t*)take((size_t)nnz * 8);
  b.rowid = (uint32_t*)take((size_t)nnz * 4);
  b.counts = (uint64_t*)take((size_t)(16 * tiles + 1) * 8);
  b.tmp = (uint64_t*)take(scan_tmp_words(16 * tiles) * 8);
  return b;
}

// the transpose of one input: tptr (d + 1), trow, tval (nnz)
static hipError_t csr_transpose(const int64_t* ptr, const int32_t* idx,
                                const float* val, int64_t rows, int64_t d,
                                int64_t nnz, int64_t* tptr, uint32_t* trow,
                                uint32_t* tsrc, float* tval, SortBufs b,
                                hipStream_t st) {
  if (nnz > 0) {
    k_row_ids<<<blocks_of(rows * 64, 256), 256, 0, st>>>(ptr, rows, b.rowid);
    k_sort_init<<<blocks_of(nnz, 256), 256, 0, st>>>(idx, b.rowid, nnz, b.k0,
                                                     b.v0);
    const int bits = ceil_log2_i(d);
    const int passes = bits > 0 ? (bits + 3) / 4 : 1;
    const int64_t tiles = (nnz + kRsTile - 1) / kRsTile;
    uint32_t *ka = b.k0, *kb = b.k1;
    uint64_t *va = b.v0, *vb = b.v1;
    for (int ps = 0; ps < passes; ++ps) {
      k_rs_count<<<(unsigned)tiles, kRsThreads, 0, st>>>(ka, nnz, 4 * ps,
                                                         b.counts, tiles);
      hipError_t e = scan_u64(b.counts, b.counts, 16 * tiles, b.tmp, st);
      if (e != hipSuccess) return e;
      k_rs_scatter<<<(unsigned)tiles, kRsThreads, 0, st>>>(
          ka, va, nnz, 4 * ps, b.counts, tiles, kb, vb);
      std::swap(ka, kb);
      std::swap(va, vb);
    }
    k_trans_split<<<blocks_of(nnz, 256), 256, 0, st>>>(va, nnz, trow, tsrc);
    k_trans_gather<<<blocks_of(nnz, 256 * 8) < 2048 ? blocks_of(nnz, 256 * 8)
                                                     : 2048,
                     256, 0, st>>>(tsrc, val, nnz, tval);
    k_lower_bound<<<blocks_of(d + 1, 256), 256, 0, st>>>(ka, nnz, d, tptr);
  } else {
    k_lower_bound<<<blocks_of(d + 1, 256), 256, 0, st>>>(nullptr, 0, d, tptr);
  }
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// weight / sign / item functors over item positions p
// ---------------------------------------------------------------------------
struct RowItems {  // T3: entries of a_i; item = coordinate
  const float* val;
  const int32_t* idx;
  __device__ double w(int64_t p) const { return fabs((double)val[p]); }
  __device__ uint32_t sgn(int64_t p) const { return sign_bit(val[p]); }
  __device__ uint32_t item(int64_t p) const { return (uint32_t)idx[p]; }
};

struct ColItems {  // T1 / T2: vectors with an entry at k; item = vector
  const float* tval;
  const uint32_t* trow;
  const double* scale;  // na for T1, null for T2
  // T1: the weights |a_ki| na_i computed once per build (k_col_scaled), so
  // that the passes over the table do not each gather na
  const double* wpre = nullptr;
  __device__ double w(int64_t p) const {
    if (wpre) return wpre[p];
    const double a = fabs((double)tval[p]);
    return scale ? a * scale[trow[p]] : a;
  }
  __device__ uint32_t sgn(int64_t p) const { return sign_bit(tval[p]); }
  __device__ uint32_t item(int64_t p) const { return trow[p]; }
};

template <class W>
struct EmitItems {
  void* et;  // the table's first entry
  int esz;   // 32: Ent32 with payloads, else Ent16
  W w;
  int64_t o;
  int64_t N;
  // payload per item position (pay[p] belongs to the item at position p,
  // so a table's payloads are as contiguous as its items), or null
  const uint64_t* pay;
  __device__ void operator()(int r, uint32_t thr, uint32_t ss, uint32_t al,
                             uint32_t sa) const {
    const uint64_t pw = pack_entry(thr, ss, al, sa);
    const uint32_t self = r < N ? w.item(o + r) : 0u;
    const uint32_t alias = w.item(o + (int64_t)al);
    if (esz == 32) {
      Ent32 e;
      e.w = pw;
      e.self = self;
      e.alias = alias;
      e.pself = pay && r < N ? pay[o + r] : 0ull;
      e.palias = pay ? pay[o + (int64_t)al] : 0ull;
      ((Ent32*)et)[r] = e;
    } else {
      ((Ent16*)et)[r] = Ent16{pw, self, alias};
    }
  }
};

// zero entries [r0, r1) of a table (dead tables: never sampled)
__device__ __forceinline__ void zero_entries(void* et, int esz, int64_t r0,
                                             int64_t r1, int64_t step) {
  for (int64_t r = r0; r < r1; r += step) {
    if (esz == 32)
      ((Ent32*)et)[r] = Ent32{0ull, 0u, 0u, 0ull, 0ull};
    else
      ((Ent16*)et)[r] = Ent16{0ull, 0u, 0u};
  }
}

__device__ __forceinline__ int spl_of(int L) {
  return L <= 6 ? 1 : (L == 7 ? 2 : (L == 8 ? 4 : 8));
}

static inline int spl_class_host(int L) {  // 0..3 for 1, 2, 4, 8 slots/lane
  return L <= 6 ? 0 : L - 6;
}

// ---------------------------------------------------------------------------
// tables of at most 512 items, one wave per table of one slots-per-lane
// class (every wave of the block runs every step: the block synchronises):
//   the table's weights go to LDS (sign bit in bit 63), coalesced;
//   lane c < R walks run c of kRun items left to right and overwrites them
//   with the run-local prefixes l_r, its total going to LDS;
//   E_c and T from the run totals in the two-level order (E_0 = 0, E_{c+1}
//   = E_c + run c's total, T = E_R), then per slot in parallel F_r =
//   floor(2^K (E_c + l_r) / T) and q_r = F_r - F_{r-1} (slots past the items
//   keep F = 2^K, so their quanta are zero);
//   wave_alias builds the table from the quanta in registers.
// (The quanta used to come from a kernel with one lane per table walking
// its items from global memory: about 0.3 ms per C3 family, spent in the
// walks of the longest tables.)
// ---------------------------------------------------------------------------
template <int SPL, class W>
__global__ __launch_bounds__(256) void k_ragged_alias(
    W w, const int64_t* off, const uint64_t* meta, const uint32_t* ids,
    int64_t count, double* tot, void* ent, int esz, const uint64_t* pay) {
  extern __shared__ uint64_t smem64[];
  __shared__ double rts[4][(512 + kRun - 1) / kRun];  // run totals per wave
  constexpr int NpMax = 64 * SPL;
  const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int64_t g = (int64_t)blockIdx.x * 4 + wv;
  const bool mine = g < count;
  const int64_t seg = ids[mine ? g : count - 1];
  const uint64_t mt = meta[seg];
  const int L = (int)(mt >> 56);
  const int64_t so = (int64_t)(mt & kSlotMask);
  const int64_t o = off[seg];
  const int N = mine ? (int)(off[seg + 1] - o) : 0;  // at most 512
  const int Np = 1 << L;
  const int K = L + kCapBits;
  uint64_t* Ld = smem64 + (int64_t)wv * 2 * NpMax;
  uint64_t* He = Ld + NpMax;
  uint32_t* Hi = (uint32_t*)(smem64 + 8 * NpMax) + (int64_t)wv * NpMax;
  for (int r = lane; r < N; r += 64)
    Ld[r] = (uint64_t)__double_as_longlong(w.w(o + r)) |
            ((uint64_t)w.sgn(o + r) << 63);
  __syncthreads();
  const int R = (N + kRun - 1) / kRun;
  if (lane < R) {
    const int r0 = lane * kRun, r1 = N < r0 + kRun ? N : r0 + kRun;
    double l = 0.0;
    for (int x0 = r0; x0 < r1; x0 += 8) {
      uint64_t x[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) x[u] = Ld[x0 + u < r1 ? x0 + u : r1 - 1];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int r = x0 + u;
        if (r < r1) {
          const double wr = __longlong_as_double((long long)(x[u] & kQMask));
          l = r == r0 ? wr : l + wr;
          Ld[r] = (uint64_t)__double_as_longlong(l) | (x[u] & ~kQMask);
        }
      }
    }
    rts[wv][lane] = l;
  }
  __syncthreads();
  double Ec[(512 + kRun - 1) / kRun] = {};
  double T = 0.0;
  for (int c = 0; c < R; ++c) {
    Ec[c] = T;
    T = T + rts[wv][c];
  }
  const bool live = mine && T > 0.0;
  if (mine && lane == 0) tot[seg] = T;
  char* et = (char*)ent + so * esz;
  if (mine && !live)  // dead table: never sampled, entries zero
    zero_entries(et, esz, lane, Np, 64);
  uint64_t F[SPL];
  uint32_t sg[SPL];
#pragma unroll
  for (int s = 0; s < SPL; ++s) {
    const int r = lane * SPL + s;
    F[s] = live ? (uint64_t)1 << K : 0ull;
    sg[s] = 0;
    if (live && r < N) {
      const uint64_t raw = Ld[r];
      const double lr = __longlong_as_double((long long)(raw & kQMask));
      F[s] = (uint64_t)floor(ldexp((Ec[r / kRun] + lr) / T, K));
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
  __syncthreads();  // the prefixes are read; wave_alias reuses Ld
  wave_alias<SPL, true>(qv, sg, live, L, Ld, He, Hi,
                        EmitItems<W>{et, esz, w, o, N, pay}, Fb);
}

// ---------------------------------------------------------------------------
// tables of more than 512 items: the large-table pipeline of the dense
// builder over the "big" slot region (tables back to back, each a multiple
// of 1024 slots), with a table lookup per 1024-slot block:
//   runs     one thread per run of 1024 items: run-local prefixes, totals
//   offsets  one workgroup per table: E_{c+1} = E_c + S_c left to right
//   quanta   one thread per 4 slots; 1024-slot block alias statistics
//   scan     one workgroup per table: exclusive scan of its block stats
//   scatter  light / heavy lists in slot order
//   edges    merge-path split at every 1024th merged position
//   merge    1024 merged positions per workgroup -> 16- or 32-byte entries
// ---------------------------------------------------------------------------
struct BigInfo {
  int64_t so;     // first slot (in the big region, a multiple of 1024)
  int64_t o;      // first item position
  int64_t N;      // items
  int64_t R;      // runs of kRun items
  int64_t run0;   // first global run id
  int64_t eoff;   // first run offset in E (R + 1 entries)
  int64_t edge0;  // first merge edge (2^L / 1024 + 1 per table)
  int32_t L;
  int32_t s;      // table id
};

constexpr int kBigBlk = 1024;  // slots per block of the big pipeline

struct BigScratch {
  uint64_t* Lb;   // run-local prefix bits (sign in bit 63), per slot
  uint64_t* q;    // quanta (sign in bit 63), per slot
  uint64_t* Ld;   // light deficit prefixes (exclusive)
  uint64_t* He;   // heavy excess prefixes (inclusive)
  uint32_t* Li;   // light slot ids (sign in bit 31)
  uint32_t* Hi;   // heavy slot ids (sign in bit 31)
  Quad* bs;       // per 1024-slot block statistics
  double* E;      // run offsets
  uint64_t* NL;   // per big table
  uint64_t* NH;
  uint64_t* Dt;
  int64_t* edges;
};

// block-wide exclusive scan of a Quad over 256 threads; returns the total
__device__ Quad quad_scan256(Quad& v) {
  __shared__ Quad wt[4];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  Quad inc{wave_incl_scan(v.nl), wave_incl_scan(v.nh), wave_incl_scan(v.sd),
           wave_incl_scan(v.se)};
  if (lane == 63) wt[wv] = inc;
  __syncthreads();
  Quad off{0, 0, 0, 0}, all{0, 0, 0, 0};
  for (int w = 0; w < 4; ++w) {
    const Quad x = wt[w];
    if (w < wv) {
      off.nl += x.nl; off.nh += x.nh; off.sd += x.sd; off.se += x.se;
    }
    all.nl += x.nl; all.nh += x.nh; all.sd += x.sd; all.se += x.se;
  }
  __syncthreads();
  v = Quad{off.nl + inc.nl - v.nl, off.nh + inc.nh - v.nh,
           off.sd + inc.sd - v.sd, off.se + inc.se - v.se};
  return all;
}

template <class W>
__global__ __launch_bounds__(256) void k_big_runs(W w, const BigInfo* big,
                                                  const uint32_t* runtab,
                                                  int64_t runs, BigScratch sc) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= runs) return;
  const BigInfo B = big[runtab[r]];
  const int64_t c = r - B.run0;
  const int64_t r0 = c * kRun;
  const int64_t r1 = r0 + kRun < B.N ? r0 + kRun : B.N;
  uint64_t* Lb = sc.Lb + B.so;
  double l = 0.0;
  for (int64_t x = r0; x < r1; x += 8) {
    double wv[8];
    uint32_t sv[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int64_t rr = x + u < r1 ? x + u : r1 - 1;
      wv[u] = w.w(B.o + rr);
      sv[u] = w.sgn(B.o + rr);
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      if (x + u < r1) {
        l = l + wv[u];
        Lb[x + u] = (uint64_t)__double_as_longlong(l) | ((uint64_t)sv[u] << 63);
      }
    }
  }
  sc.E[B.eoff + c + 1] = l;  // run total, turned into an offset next
}

// one workgroup per big table: the run offsets, left to right, through LDS
__global__ __launch_bounds__(256) void k_big_offsets(const BigInfo* big,
                                                     BigScratch sc,
                                                     double* tot) {
  __shared__ double buf[4096];
  __shared__ double carry;
  const BigInfo B = big[blockIdx.x];
  double* E = sc.E + B.eoff;
  if (threadIdx.x == 0) {
    carry = 0.0;
    E[0] = 0.0;
  }
  __syncthreads();
  for (int64_t c0 = 0; c0 < B.R; c0 += 4096) {
    const int64_t nc = B.R - c0 < 4096 ? B.R - c0 : 4096;
    for (int64_t u = threadIdx.x; u < nc; u += blockDim.x)
      buf[u] = E[c0 + u + 1];
    __syncthreads();
    if (threadIdx.x == 0) {
      double acc = carry;
      for (int64_t u = 0; u < nc; ++u) {
        acc = acc + buf[u];
        buf[u] = acc;
      }
      carry = acc;
    }
    __syncthreads();
    for (int64_t u = threadIdx.x; u < nc; u += blockDim.x)
      E[c0 + u + 1] = buf[u];
    __syncthreads();
  }
  if (threadIdx.x == 0) tot[B.s] = carry;
}

// quanta of 4 slots per thread, 1024 slots per block, block statistics
__global__ __launch_bounds__(256) void k_big_quanta(const BigInfo* big,
                                                    const uint32_t* btab,
                                                    const double* tot,
                                                    BigScratch sc) {
  const BigInfo B = big[btab[blockIdx.x]];
  const int64_t g0 = (int64_t)blockIdx.x * kBigBlk + threadIdx.x * 4;
  const int64_t r0 = g0 - B.so;  // table-relative slot
  const double T = tot[B.s];
  const bool live = T > 0.0;
  const int K = B.L + kCapBits;
  const double* E = sc.E + B.eoff;
  const uint64_t* Lb = sc.Lb + B.so;
  Quad a{0, 0, 0, 0};
  uint64_t Fp = 0;
  if (live && r0 > 0 && r0 - 1 < B.N) {
    const double Pp = E[(r0 - 1) / kRun] +
                      __longlong_as_double((long long)(Lb[r0 - 1] & kQMask));
    Fp = (uint64_t)floor(ldexp(Pp / T, K));
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int64_t r = r0 + u;
    uint64_t qq = 0;
    if (live && r < B.N) {
      const uint64_t raw = Lb[r];
      const double Pv = E[r / kRun] +
                        __longlong_as_double((long long)(raw & kQMask));
      const uint64_t F = (uint64_t)floor(ldexp(Pv / T, K));
      qq = (F - Fp) | (raw & ~kQMask);
      Fp = F;
    }
    sc.q[g0 + u] = qq;
    slot_stats(qq & kQMask, a);
  }
  const Quad all = quad_scan256(a);
  if (threadIdx.x == 0) sc.bs[blockIdx.x] = all;
}

// one workgroup per big table: exclusive scan of its block statistics
__global__ __launch_bounds__(256) void k_big_scan(const BigInfo* big,
                                                  BigScratch sc) {
  const BigInfo B = big[blockIdx.x];
  const int64_t b0 = B.so / kBigBlk;
  const int64_t nb = (int64_t(1) << B.L) / kBigBlk;
  Quad carry{0, 0, 0, 0};
  for (int64_t c0 = 0; c0 < nb; c0 += 256) {
    const int64_t i = c0 + threadIdx.x;
    Quad v = i < nb ? sc.bs[b0 + i] : Quad{0, 0, 0, 0};
    const Quad all = quad_scan256(v);
    if (i < nb)
      sc.bs[b0 + i] = Quad{carry.nl + v.nl, carry.nh + v.nh, carry.sd + v.sd,
                           carry.se + v.se};
    carry.nl += all.nl;
    carry.nh += all.nh;
    carry.sd += all.sd;
    carry.se += all.se;
  }
  if (threadIdx.x == 0) {
    sc.NL[blockIdx.x] = carry.nl;
    sc.NH[blockIdx.x] = carry.nh;
    sc.Dt[blockIdx.x] = carry.sd;
  }
}

// light / heavy lists in slot order (ids carry the sign in bit 31)
__global__ __launch_bounds__(256) void k_big_scatter(const BigInfo* big,
                                                     const uint32_t* btab,
                                                     BigScratch sc) {
  const BigInfo B = big[btab[blockIdx.x]];
  const int64_t g0 = (int64_t)blockIdx.x * kBigBlk + threadIdx.x * 4;
  uint64_t qv[4];
  uint32_t sg[4];
  Quad a{0, 0, 0, 0};
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const uint64_t raw = sc.q[g0 + u];
    qv[u] = raw & kQMask;
    sg[u] = (uint32_t)(raw >> 63);
    slot_stats(qv[u], a);
  }
  (void)quad_scan256(a);
  const Quad o = sc.bs[blockIdx.x];
  uint64_t lp = o.nl + a.nl, hp = o.nh + a.nh;
  uint64_t da = o.sd + a.sd, ea = o.se + a.se;
  uint64_t* Ld = sc.Ld + B.so;
  uint64_t* He = sc.He + B.so;
  uint32_t* Li = sc.Li + B.so;
  uint32_t* Hi = sc.Hi + B.so;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const uint32_t id = (uint32_t)(g0 + u - B.so) | (sg[u] << 31);
    if (qv[u] < kCap) {
      Ld[lp] = da;
      Li[lp] = id;
      da += kCap - qv[u];
      ++lp;
    } else {
      ea += qv[u] - kCap;
      He[hp] = ea;
      Hi[hp] = id;
      ++hp;
    }
  }
}

// merge-path split at every kBigBlk-th merged position of every big table
__global__ void k_big_edges(const BigInfo* big, int64_t nbig, int64_t nedges,
                            BigScratch sc) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= nedges) return;
  int64_t lo = 0, hi = nbig - 1;  // last table with edge0 <= e
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (big[mid].edge0 <= e) lo = mid; else hi = mid - 1;
  }
  const BigInfo B = big[lo];
  const int64_t d0 = (e - B.edge0) * kBigBlk;
  sc.edges[e] = merge_split(sc.Ld + B.so, (int64_t)sc.NL[lo], sc.He + B.so,
                            (int64_t)sc.NH[lo], d0);
}

constexpr int kBigMergeP = kBigBlk / 256;

template <class W>
__global__ __launch_bounds__(256) void k_big_merge(W w, const BigInfo* big,
                                                   const uint32_t* btab,
                                                   const double* tot,
                                                   BigScratch sc, void* ent,
                                                   int esz,
                                                   const uint64_t* pay) {
  __shared__ uint64_t sD[kBigBlk + 1], sE[kBigBlk + 1];
  __shared__ uint32_t sLi[kBigBlk + 1], sHi[kBigBlk + 1];
  const uint32_t bt = btab[blockIdx.x];
  const BigInfo B = big[bt];
  const int64_t bi = (int64_t)blockIdx.x - B.so / kBigBlk;
  const int64_t d0 = bi * kBigBlk;
  char* et = (char*)ent + B.so * esz;
  if (!(tot[B.s] > 0.0)) {  // dead table: never sampled, entries zero
    zero_entries(et, esz, d0 + threadIdx.x, d0 + kBigBlk, 256);
    return;
  }
  const int64_t NL = (int64_t)sc.NL[bt], NH = (int64_t)sc.NH[bt];
  const uint64_t Dt = sc.Dt[bt];
  const uint64_t* D = sc.Ld + B.so;
  const uint64_t* E = sc.He + B.so;
  const uint32_t* Li = sc.Li + B.so;
  const uint32_t* Hi = sc.Hi + B.so;
  const int64_t* ed = sc.edges + B.edge0 + bi;
  const int64_t a0 = ed[0], b0 = d0 - ed[0];
  const int64_t na = ed[1] - a0, nb = (d0 + kBigBlk - ed[1]) - b0;
  for (int u = threadIdx.x; u <= na; u += 256) {
    sD[u] = a0 + u < NL ? D[a0 + u] : Dt;
    sLi[u] = a0 + u < NL ? Li[a0 + u] : 0u;
  }
  for (int u = threadIdx.x; u <= nb; u += 256) {
    sE[u] = b0 + u < NH ? E[b0 + u] : ~0ull;
    sHi[u] = b0 + u < NH ? Hi[b0 + u] : 0u;
  }
  __syncthreads();
  const int64_t dl = (int64_t)threadIdx.x * kBigMergeP;
  int64_t lo = dl - nb > 0 ? dl - nb : 0, hi = dl < na ? dl : na;
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    if (sD[mid] <= sE[dl - mid - 1]) lo = mid + 1; else hi = mid;
  }
  int64_t a = lo, b = dl - lo;
  const EmitItems<W> emit{et, esz, w, B.o, B.N, pay};
  for (int step = 0; step < kBigMergeP; ++step) {
    if (a < na && (b >= nb || sD[a] <= sE[b])) {
      const uint32_t id = sLi[a];
      const uint32_t r = id & kLow31;
      const uint32_t qv = (uint32_t)(kCap - (sD[a + 1] - sD[a]));
      const uint32_t dn = b0 + b < NH ? sHi[b] : id;
      emit((int)r, qv, id >> 31, dn & kLow31, dn >> 31);
      ++a;
    } else {
      const uint32_t id = sHi[b];
      const uint32_t r = id & kLow31;
      const uint64_t Eh = sE[b];
      const uint64_t Dn = sD[a];  // D of the next light, or Dt past the end
      if (Dn > Eh && b0 + b + 1 < NH) {
        const uint32_t nx = sHi[b + 1];
        emit((int)r, (uint32_t)(Eh + kCap - Dn), id >> 31, nx & kLow31,
             nx >> 31);
      } else {
        emit((int)r, 0u, id >> 31, r, id >> 31);
      }
      ++b;
    }
  }
}

// ---------------------------------------------------------------------------
// host: layout of a family (slot offsets, big tables, small-table classes)
// ---------------------------------------------------------------------------
static void ragged_free(Ragged& R) {
  dev_free(R.lay);
  dev_free(R.ent_buf);
  dev_free(R.tot_buf);
  R = Ragged{};
}

static size_t al256(size_t b) { return (b + 255) & ~(size_t)255; }

static hipError_t ragged_layout(Ragged& R, const int64_t* off_dev, int64_t S,
                                int esz, hipStream_t st) {
  R.esz = esz;
  std::vector<int64_t> off((size_t)S + 1);
  hipError_t e = hipMemcpyAsync(off.data(), off_dev, off.size() * 8,
                                hipMemcpyDeviceToHost, st);
  if (e != hipSuccess || (e = hipStreamSynchronize(st)) != hipSuccess)
    return e;
  std::vector<uint64_t> meta((size_t)S);
  std::vector<BigInfo> big;
  std::vector<uint32_t> btab, runtab;
  std::vector<uint32_t> cls[4];
  int64_t bs = 0, runs = 0, eoff = 0, edges = 0;
  for (int64_t s = 0; s < S; ++s) {
    const int64_t N = off[(size_t)s + 1] - off[(size_t)s];
    if (N <= 512) continue;
    const int L = ceil_log2_i(N);
    BigInfo B;
    B.so = bs;
    B.o = off[(size_t)s];
    B.N = N;
    B.R = (N + kRun - 1) / kRun;
    B.run0 = runs;
    B.eoff = eoff;
    B.edge0 = edges;
    B.L = L;
    B.s = (int32_t)s;
    meta[(size_t)s] = (uint64_t)bs | ((uint64_t)L << 56);
    const int64_t Np = int64_t(1) << L;
    for (int64_t b = 0; b < Np / kBigBlk; ++b)
      btab.push_back((uint32_t)big.size());
    for (int64_t c = 0; c < B.R; ++c) runtab.push_back((uint32_t)big.size());
    big.push_back(B);
    bs += Np;
    runs += B.R;
    eoff += B.R + 1;
    edges += Np / kBigBlk + 1;
  }
  int64_t ss = bs;
  for (int64_t s = 0; s < S; ++s) {
    const int64_t N = off[(size_t)s + 1] - off[(size_t)s];
    if (N > 512) continue;
    const int L = ceil_log2_i(N);
    meta[(size_t)s] = (uint64_t)ss | ((uint64_t)L << 56);
    ss += int64_t(1) << L;
    cls[spl_class_host(L)].push_back((uint32_t)s);
  }
  R.S = S;
  R.off = off_dev;
  R.slots = ss;
  R.big_slots = bs;
  R.nbig = (int64_t)big.size();
  R.runs = runs;
  R.edges = edges;
  R.cls_off[0] = 0;
  for (int c = 0; c < 4; ++c)
    R.cls_off[c + 1] = R.cls_off[c] + (int64_t)cls[c].size();
  // one layout buffer: meta | big | btab | runtab | small ids
  const size_t b_meta = al256(8 * (size_t)(S > 0 ? S : 1));
  const size_t b_big = al256(sizeof(BigInfo) * (big.size() + 1));
  const size_t b_btab = al256(4 * (btab.size() + 1));
  const size_t b_run = al256(4 * (runtab.size() + 1));
  const size_t b_ids = al256(4 * (size_t)(R.cls_off[4] + 1));
  if ((e = dev_alloc(R.lay, b_meta + b_big + b_btab + b_run + b_ids)) !=
          hipSuccess ||
      (e = dev_alloc(R.ent_buf, (size_t)esz * (size_t)(ss > 0 ? ss : 1))) !=
          hipSuccess ||
      (e = dev_alloc(R.tot_buf, 8 * (size_t)(S > 0 ? S : 1))) != hipSuccess)
    return e;
  char* p = (char*)R.lay.p;
  R.meta = (uint64_t*)p;
  R.big = p + b_meta;
  R.btab = (uint32_t*)(p + b_meta + b_big);
  R.runtab = (uint32_t*)(p + b_meta + b_big + b_btab);
  R.small_ids = (uint32_t*)(p + b_meta + b_big + b_btab + b_run);
  R.ent = R.ent_buf.p;
  R.tot = (double*)R.tot_buf.p;
  std::vector<char> host(b_meta + b_big + b_btab + b_run + b_ids, 0);
  memcpy(host.data(), meta.data(), 8 * meta.size());
  memcpy(host.data() + b_meta, big.data(), sizeof(BigInfo) * big.size());
  memcpy(host.data() + b_meta + b_big, btab.data(), 4 * btab.size());
  memcpy(host.data() + b_meta + b_big + b_btab, runtab.data(),
         4 * runtab.size());
  char* ids = host.data() + b_meta + b_big + b_btab + b_run;
  for (int c = 0; c < 4; ++c)
    memcpy(ids + 4 * R.cls_off[c], cls[c].data(), 4 * cls[c].size());
  return hipMemcpyAsync(R.lay.p, host.data(), host.size(),
                        hipMemcpyHostToDevice, st) == hipSuccess
             ? hipStreamSynchronize(st)
             : hipErrorInvalidValue;
}

static size_t big_scratch_bytes(const Ragged& R) {
  const size_t n = (size_t)R.big_slots;
  return al256(n * 8) * 4 + al256(n * 4) * 2 +
         al256(sizeof(Quad) * (n / kBigBlk + 1)) +
         al256(8 * (size_t)(R.runs + R.nbig + 1)) +
         al256(8 * (size_t)(R.nbig + 1)) * 3 +
         al256(8 * (size_t)(R.edges + 1)) + 256;
}

static size_t ragged_scratch_bytes(const Ragged& R) {
  return al256(big_scratch_bytes(R));
}

static BigScratch big_carve(void* p, const Ragged& R) {
  char* c = (char*)p;
  auto take = [&](size_t bytes) {
    char* r = c;
    c += al256(bytes);
    return r;
  };
  BigScratch b;
  const size_t n = (size_t)R.big_slots;
  b.Lb = (uint64_t*)take(n * 8);
  b.q = (uint64_t*)take(n * 8);
  b.Ld = (uint64_t*)take(n * 8);
  b.He = (uint64_t*)take(n * 8);
  b.Li = (uint32_t*)take(n * 4);
  b.Hi = (uint32_t*)take(n * 4);
  b.bs = (Quad*)take(sizeof(Quad) * (n / kBigBlk + 1));
  b.E = (double*)take(8 * (size_t)(R.runs + R.nbig + 1));
  b.NL = (uint64_t*)take(8 * (size_t)(R.nbig + 1));
  b.NH = (uint64_t*)take(8 * (size_t)(R.nbig + 1));
  b.Dt = (uint64_t*)take(8 * (size_t)(R.nbig + 1));
  b.edges = (int64_t*)take(8 * (size_t)(R.edges + 1));
  return b;
}

template <class W>
static hipError_t ragged_build(const Ragged& R, W w, void* scratch,
                               hipStream_t st, const uint64_t* pay = nullptr) {
  if (R.S <= 0) return hipSuccess;
  const int64_t* c = R.cls_off;
  if (c[1] > c[0])
    k_ragged_alias<1, W><<<blocks_of(c[1] - c[0], 4), 256, 4 * 64 * 20, st>>>(
        w, R.off, R.meta, R.small_ids + c[0], c[1] - c[0], R.tot, R.ent,
        R.esz, pay);
  if (c[2] > c[1])
    k_ragged_alias<2, W><<<blocks_of(c[2] - c[1], 4), 256, 4 * 128 * 20, st>>>(
        w, R.off, R.meta, R.small_ids + c[1], c[2] - c[1], R.tot, R.ent,
        R.esz, pay);
  if (c[3] > c[2])
    k_ragged_alias<4, W><<<blocks_of(c[3] - c[2], 4), 256, 4 * 256 * 20, st>>>(
        w, R.off, R.meta, R.small_ids + c[2], c[3] - c[2], R.tot, R.ent,
        R.esz, pay);
  if (c[4] > c[3])
    k_ragged_alias<8, W><<<blocks_of(c[4] - c[3], 4), 256, 4 * 512 * 20, st>>>(
        w, R.off, R.meta, R.small_ids + c[3], c[4] - c[3], R.tot, R.ent,
        R.esz, pay);
  if (R.nbig > 0) {
    const BigScratch sc = big_carve(scratch, R);
    const BigInfo* big = (const BigInfo*)R.big;
    const unsigned nblk = (unsigned)(R.big_slots / kBigBlk);
    k_big_runs<W><<<blocks_of(R.runs, 256), 256, 0, st>>>(w, big, R.runtab,
                                                           R.runs, sc);
    k_big_offsets<<<(unsigned)R.nbig, 256, 0, st>>>(big, sc, R.tot);
    k_big_quanta<<<nblk, 256, 0, st>>>(big, R.btab, R.tot, sc);
    k_big_scan<<<(unsigned)R.nbig, 256, 0, st>>>(big, sc);
    k_big_scatter<<<nblk, 256, 0, st>>>(big, R.btab, sc);
    k_big_edges<<<blocks_of(R.edges, 256), 256, 0, st>>>(big, R.nbig,
                                                         R.edges, sc);
    k_big_merge<W><<<nblk, 256, 0, st>>>(w, big, R.btab, R.tot, sc, R.ent,
                                         R.esz, pay);
  }
  return hipGetLastError();
}

__global__ void k_stage0_csr(const double* nb, const double* v, int64_t d,
                             double* om) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < d) om[k] = nb[k] * v[k];
}

void csr_tables_free(CsrTables& t) {
  ragged_free(t.T1);
  ragged_free(t.T2);
  ragged_free(t.T3);
  family_free_pub(t.T0);
  void* ps[] = {t.at_ptr, t.at_row, t.at_val, t.at_src, t.bt_ptr, t.bt_row,
                t.bt_val, t.bt_src, t.at_w, t.om, t.bmax, t.bad, t.at_pay,
                t.bsig, t.bt_pay, t.bh};
  for (void* p : ps)
    if (p) (void)hipFree(p);
  t.at_ptr = t.bt_ptr = nullptr;
  t.at_row = t.bt_row = nullptr;
  t.at_val = t.bt_val = nullptr;
  t.at_src = t.bt_src = nullptr;
  t.at_w = nullptr;
  t.structured = false;
  t.om = nullptr;
  t.bmax = nullptr;
  t.bad = nullptr;
  t.at_pay = nullptr;
  t.bsig = nullptr;
  t.bt_pay = nullptr;
  t.bh = nullptr;
  t.bh_mask = 0;
  dev_free(t.work);
}

static hipError_t csr_tables_from_transposes(CsrTables& t, hipStream_t st);

// B's entries into the hash table: one thread per row j, each entry's key
// j d + k + 1 claimed by compare-and-swap at its first free slot from
// mix64(key) (linear probing; the table is at most half full), the slot
// then noting the entry's position e.  Keys are unique in a valid
// structure; a repeated one finds its own slot.
__global__ void k_bhash_insert(const int64_t* ptr, const int32_t* idx,
                               int64_t rows, int64_t d, BSlot* bh,
                               uint64_t mask) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= rows) return;
  for (int64_t e = ptr[j]; e < ptr[j + 1]; ++e) {
    const uint64_t key = (uint64_t)j * (uint64_t)d + (uint64_t)idx[e] + 1;
    uint64_t sl = mix64(key) & mask;
    while (true) {
      const unsigned long long prev = atomicCAS(
          (unsigned long long*)&bh[sl].key, 0ull, (unsigned long long)key);
      if (prev == 0ull || prev == key) break;
      sl = (sl + 1) & mask;
    }
    bh[sl].e = (uint32_t)e;
  }
}

// every build: each taken slot gathers its entry's value (the table is
// read in order and the values of B, a smaller array, at random)
__global__ void k_bhash_vals(const float* val, int64_t nslots, BSlot* bh) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
       s < nslots; s += stride) {
    const uint4 w = *(const uint4*)(bh + s);
    if (w.x | w.y) bh[s].val = val[w.w];
  }
}

// sig[j] = OR of coord_bit(k) over the coordinates k of vector j
__global__ void k_row_sig(const int64_t* ptr, const int32_t* idx,
                          int64_t rows, uint64_t* sig) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= rows) return;
  uint64_t s = 0;
  for (int64_t e = ptr[j]; e < ptr[j + 1]; ++e)
    s |= coord_bit((uint64_t)(uint32_t)idx[e]);
  sig[j] = s;
}

// out[p] = pay[item[p]]: the payload of the item at each transpose position
__global__ void k_gather_pay(const uint32_t* item, int64_t n,
                             const uint64_t* pay, uint64_t* out) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
       p += stride)
    out[p] = pay[item[p]];
}

hipError_t csr_tables_build(CsrTables& t, bool check, hipStream_t st) {
  hipError_t e;
  const int64_t m = t.m, n = t.n, d = t.d;
  // first build: fixed-size arrays
  if (!t.bad) {
    if ((e = hipMalloc(&t.bad, 256)) != hipSuccess ||
        (e = hipMalloc(&t.bmax, 256)) != hipSuccess ||
        (e = hipMalloc(&t.om, 8 * (size_t)d)) != hipSuccess ||
        (e = hipMalloc(&t.at_ptr, 8 * (size_t)(d + 1))) != hipSuccess ||
        (e = hipMalloc(&t.bt_ptr, 8 * (size_t)(d + 1))) != hipSuccess ||
        (e = hipMalloc(&t.at_row, 4 * (size_t)(t.nnzA + 1))) != hipSuccess ||
        (e = hipMalloc(&t.at_val, 4 * (size_t)(t.nnzA + 1))) != hipSuccess ||
        (e = hipMalloc(&t.bt_row, 4 * (size_t)(t.nnzB + 1))) != hipSuccess ||
        (e = hipMalloc(&t.bt_val, 4 * (size_t)(t.nnzB + 1))) != hipSuccess ||
        (e = hipMalloc(&t.at_src, 4 * (size_t)(t.nnzA + 1))) != hipSuccess ||
        (e = hipMalloc(&t.bt_src, 4 * (size_t)(t.nnzB + 1))) != hipSuccess ||
        (e = hipMalloc(&t.at_w, 8 * (size_t)(t.nnzA + 1))) != hipSuccess ||
        (e = hipMalloc(&t.at_pay, 8 * (size_t)(t.nnzA + 1))) != hipSuccess ||
        (e = hipMalloc(&t.bsig, 8 * (size_t)(n + 1))) != hipSuccess ||
        (e = hipMalloc(&t.bt_pay, 8 * (size_t)(t.nnzB + 1))) != hipSuccess ||
        (e = family_alloc_pub(t.T0, 1, d)) != hipSuccess)
      return e;
    int64_t cap = 1024;
    while (cap < 2 * t.nnzB) cap <<= 1;
    t.bh_mask = (uint64_t)(cap - 1);
    if ((e = hipMalloc(&t.bh, sizeof(BSlot) * (size_t)cap)) != hipSuccess)
      return e;
  }
  if (!check && t.structured) {
    // the caller vouches that the structure is the one of this plan's
    // first build: regather the transposed values, then the tables
    if ((e = launch_fill_u64((uint64_t*)t.bmax, 1, 0ull, st)) != hipSuccess)
      return e;
    const int64_t nzb = t.nnzB > 0 ? t.nnzB : 1;
    k_absmax<<<blocks_of(nzb, 1024 * 16) < 256 ? blocks_of(nzb, 1024 * 16)
                                               : 256,
               1024, 0, st>>>(t.in.b_val, t.nnzB, t.bmax);
    if (t.nnzA > 0)
      k_trans_gather<<<blocks_of(t.nnzA, 256 * 8) < 2048
                           ? blocks_of(t.nnzA, 256 * 8) : 2048,
                       256, 0, st>>>(t.at_src, t.in.a_val, t.nnzA, t.at_val);
    if (t.nnzB > 0)
      k_trans_gather<<<blocks_of(t.nnzB, 256 * 8) < 2048
                           ? blocks_of(t.nnzB, 256 * 8) : 2048,
                       256, 0, st>>>(t.bt_src, t.in.b_val, t.nnzB, t.bt_val);
    return csr_tables_from_transposes(t, st);
  }
  // validation: the structure on the first build of a plan and on every
  // checked build (every later index relies on it; without the check the
  // caller vouches that the arrays keep the structure they were validated
  // with), values when checked.  The scan also gives max |b|.
  if ((e = launch_fill_u64((uint64_t*)t.bad, 1, 0ull, st)) != hipSuccess ||
      (e = launch_fill_u64((uint64_t*)t.bmax, 1, 0ull, st)) != hipSuccess)
    return e;
  k_csr_check<<<blocks_of(m, 256), 256, 0, st>>>(
      t.in.a_ptr, t.in.a_idx, t.in.a_val, m, d, t.nnzA, nullptr, t.bad);
  k_csr_check<<<blocks_of(n, 256), 256, 0, st>>>(
      t.in.b_ptr, t.in.b_idx, t.in.b_val, n, d, t.nnzB, t.bmax, t.bad);
  if (check || !t.validated) {
    int bad = 0;
    if ((e = hipMemcpyAsync(&bad, t.bad, 4, hipMemcpyDeviceToHost, st)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
      return e;
    if ((bad & 2) || (check && (bad & 1))) return hipErrorInvalidValue;
    t.validated = true;
  }
  // B's entries into the hash table (structure only; the values follow in
  // every build)
  if ((e = launch_fill_u64((uint64_t*)t.bh, 2 * (int64_t)(t.bh_mask + 1),
                           0ull, st)) != hipSuccess)
    return e;
  if (n > 0)
    k_bhash_insert<<<blocks_of(n, 256), 256, 0, st>>>(
        t.in.b_ptr, t.in.b_idx, n, d, t.bh, t.bh_mask);
  // transposes
  const int64_t nz = t.nnzA > t.nnzB ? t.nnzA : t.nnzB;
  if ((e = dev_alloc(t.work, sort_bytes(nz))) != hipSuccess) return e;
  const SortBufs sb = sort_carve(t.work.p, nz);
  if ((e = csr_transpose(t.in.a_ptr, t.in.a_idx, t.in.a_val, m, d, t.nnzA,
                         t.at_ptr, t.at_row, t.at_src, t.at_val, sb,
                         st)) != hipSuccess ||
      (e = csr_transpose(t.in.b_ptr, t.in.b_idx, t.in.b_val, n, d, t.nnzB,
                         t.bt_ptr, t.bt_row, t.bt_src, t.bt_val, sb,
                         st)) != hipSuccess)
    return e;
  // layouts (host)
  // T1's entries carry T3's meta and T2's the signature of b_j (32 bytes);
  // T3's carry no payload
  if ((e = ragged_layout(t.T3, t.in.a_ptr, m, 16, st)) != hipSuccess ||
      (e = ragged_layout(t.T1, t.at_ptr, d, 32, st)) != hipSuccess ||
      (e = ragged_layout(t.T2, t.bt_ptr, d, 32, st)) != hipSuccess)
    return e;
  // the T1 and T2 payloads by transpose position (structure only)
  if (t.nnzA > 0)
    k_gather_pay<<<blocks_of(t.nnzA, 256 * 8) < 2048
                       ? blocks_of(t.nnzA, 256 * 8) : 2048,
                   256, 0, st>>>(t.at_row, t.nnzA, t.T3.meta, t.at_pay);
  if (n > 0)
    k_row_sig<<<blocks_of(n, 256), 256, 0, st>>>(t.in.b_ptr, t.in.b_idx, n,
                                                 t.bsig);
  if (t.nnzB > 0)
    k_gather_pay<<<blocks_of(t.nnzB, 256 * 8) < 2048
                       ? blocks_of(t.nnzB, 256 * 8) : 2048,
                   256, 0, st>>>(t.bt_row, t.nnzB, t.bsig, t.bt_pay);
  size_t need = ragged_scratch_bytes(t.T3);
  need = std::max(need, ragged_scratch_bytes(t.T1));
  need = std::max(need, ragged_scratch_bytes(t.T2));
  need = std::max(need, stage0_scratch_bytes(d));
  need = std::max(need, sort_bytes(nz));
  if ((e = dev_alloc(t.work, need)) != hipSuccess) return e;
  t.structured = true;
  return csr_tables_from_transposes(t, st);
}

// w[p] = |tval[p]| * scale[trow[p]]: the same product ColItems forms
__global__ void k_col_scaled(const float* tval, const uint32_t* trow,
                             const double* scale, int64_t n, double* w) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < n;
       p += stride)
    w[p] = fabs((double)tval[p]) * scale[trow[p]];
}

// the tables from the transposes and the layouts already in place
static hipError_t csr_tables_from_transposes(CsrTables& t, hipStream_t st) {
  // this build's values of B's entries into their hash slots
  if (t.nnzB > 0) {
    const int64_t nsl = (int64_t)t.bh_mask + 1;
    k_bhash_vals<<<blocks_of(nsl, 256 * 8) < 4096
                       ? blocks_of(nsl, 256 * 8) : 4096,
                   256, 0, st>>>(t.in.b_val, nsl, t.bh);
  }
  hipError_t e;
  const int64_t d = t.d;
  // T3 (totals na), T1 (weights |a_ki| na_i, totals v), T2 (totals nb), T0
  if ((e = ragged_build(t.T3, RowItems{t.in.a_val, t.in.a_idx}, t.work.p,
                        st)) != hipSuccess)
    return e;
  if (t.nnzA > 0)
    k_col_scaled<<<blocks_of(t.nnzA, 256 * 8) < 2048
                       ? blocks_of(t.nnzA, 256 * 8) : 2048,
                   256, 0, st>>>(t.at_val, t.at_row, t.T3.tot, t.nnzA,
                                 t.at_w);
  // T1's payload: T3's meta word of the drawn i; T2's: the signature of
  // the drawn j, which rules out most absent fourth edges before a probe
  if ((e = ragged_build(t.T1,
                        ColItems{t.at_val, t.at_row, t.T3.tot, t.at_w},
                        t.work.p, st, t.at_pay)) != hipSuccess ||
      (e = ragged_build(t.T2, ColItems{t.bt_val, t.bt_row, nullptr},
                        t.work.p, st, t.bt_pay)) != hipSuccess)
    return e;
  k_stage0_csr<<<blocks_of(d, 256), 256, 0, st>>>(t.T2.tot, t.T1.tot, d,
                                                  t.om);
  return stage0_table_build(t.om, d, t.T0, t.work.p, t.work.bytes, st);
}

// ---------------------------------------------------------------------------
// the sampler
// ---------------------------------------------------------------------------
constexpr int kT0LdsCsr = 4096;

struct CsrSampleArgs {
  const uint64_t* T0;
  int L0;
  const uint64_t* m1;
  const Ent32* e1;  // T1: with T3's meta of each item
  const uint64_t* m2;
  const Ent32* e2;  // T2: with the coordinate signature of each item
  const uint64_t* m3;
  const Ent16* e3;
  CsrView in;
  int64_t n;
  uint64_t seed, qid;
  int64_t l0, count;
  int gram;  // B = A: key of the pair with i < j, diagonal left out
  const BSlot* bh;      // B's entries by key j d + k + 1 (see CsrTables)
  uint64_t bh_mask;
  int64_t d;
  // squared variant (Sec. 3.2.3): the second pair of sample e, keyed by
  // (k, k') like the first, goes to pk2[e] / pv2[e] (pair form only)
  uint64_t* pk2;
  float* pv2;
};

__device__ __forceinline__ Drawn draw16(const Ent16& e, uint64_t U) {
  const uint32_t lo = (uint32_t)e.w, hi = (uint32_t)(e.w >> 32);
  const uint32_t coin = (uint32_t)U & kLow31;
  const bool self = coin < (lo & kLow31);
  return {self ? e.self : e.alias, (self ? lo : hi) >> 31};
}

__device__ __forceinline__ Drawn draw16(const Ent32& e, uint64_t U) {
  const uint32_t lo = (uint32_t)e.w, hi = (uint32_t)(e.w >> 32);
  const uint32_t coin = (uint32_t)U & kLow31;
  const bool self = coin < (lo & kLow31);
  return {self ? e.self : e.alias, (self ? lo : hi) >> 31};
}

// the drawn item's payload (the same coin as draw16)
__device__ __forceinline__ uint64_t draw_pay(const Ent32& e, uint64_t U) {
  const uint32_t coin = (uint32_t)U & kLow31;
  return coin < ((uint32_t)e.w & kLow31) ? e.pself : e.palias;
}

__device__ __forceinline__ uint64_t meta_slot(uint64_t mt, uint64_t U) {
  return (mt & kSlotMask) + slot_of(U, (int)(mt >> 56));
}

template <int U, bool DEBUG>
__global__ __launch_bounds__(256) void k_sample_csr(
    CsrSampleArgs a, const double* wtot, const float* bmax, int64_t s_for_F,
    int F_debug, uint64_t* hkeys, int64_t* hvals, uint64_t hmask,
    uint64_t* pkeys, float* pvals, SampleCounters* ctr, int32_t* ok,
    int32_t* oi,
    int32_t* oj, int32_t* okp, int64_t* oinc) {
  extern __shared__ uint64_t t0s[];
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
  const bool t0_lds = N0 <= kT0LdsCsr;
  if (t0_lds)
    for (int e = threadIdx.x; e < N0; e += blockDim.x) t0s[e] = a.T0[e];
  __syncthreads();
  const uint64_t* T0 = t0_lds ? t0s : a.T0;
  const int F = DEBUG ? F_debug : fix_exponent(*bmax, s_for_F);
  const int64_t nthreads = (int64_t)gridDim.x * blockDim.x;
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  unsigned long long nclosed = 0, ncreated = 0;
  for (int64_t base = tid; base < a.count; base += nthreads * U) {
    uint32_t k[U], i[U], j[U], kp[U], sg[U];
    uint64_t W1[U], W2[U], W3[U], mt1[U], mt2[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t e = base + (int64_t)u * nthreads;
      const uint64_t l = (uint64_t)(a.l0 + (e < a.count ? e : 0));
      const Philox4 r = philox4x64_10(l, a.qid, 0ull, 0ull, a.seed, 0ull);
      const uint32_t s0 = slot_of(r.w0, a.L0);
      k[u] = draw_entry(T0[s0], s0, r.w0).pos;
      W1[u] = r.w1;
      W2[u] = r.w2;
      W3[u] = r.w3;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      mt1[u] = a.m1[k[u]];
      mt2[u] = a.m2[k[u]];
    }
    Ent32 x1[U], x2[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      x1[u] = a.e1[meta_slot(mt1[u], W1[u])];
      x2[u] = a.e2[meta_slot(mt2[u], W2[u])];
    }
    // T3's meta of i comes with the drawn T1 entry, b_j's signature with
    // the drawn T2 entry (their payloads)
    uint64_t mt3[U], sj[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const Drawn di = draw16(x1[u], W1[u]);
      const Drawn dj = draw16(x2[u], W2[u]);
      i[u] = di.pos;
      j[u] = dj.pos;
      sg[u] = di.sgn ^ dj.sgn;
      mt3[u] = draw_pay(x1[u], W1[u]);
      sj[u] = draw_pay(x2[u], W2[u]);
    }
    Ent16 x3[U];
#pragma unroll
    for (int u = 0; u < U; ++u) x3[u] = a.e3[meta_slot(mt3[u], W3[u])];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const Drawn dk = draw16(x3[u], W3[u]);
      kp[u] = dk.pos;
      sg[u] ^= dk.sgn;
    }
    // dx: the fourth edge b_k'j from the table of B's entries (0 when b_j
    // stores no coordinate k', which a clear bit of b_j's signature already
    // proves); every sample's first probe is in flight at once, the rare
    // further probes follow
    float v[U];
    uint64_t hkey[U], hs[U];
    bool pend[U];
    bool anyp = false;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      hkey[u] = (uint64_t)j[u] * (uint64_t)a.d + (uint64_t)kp[u] + 1;
      hs[u] = mix64(hkey[u]) & a.bh_mask;
      v[u] = 0.0f;
      pend[u] = (sj[u] & coord_bit(kp[u])) != 0;
      anyp |= pend[u];
    }
    while (anyp) {
      uint4 hw[U];
#pragma unroll
      for (int u = 0; u < U; ++u)
        if (pend[u]) hw[u] = *(const uint4*)(a.bh + hs[u]);
      anyp = false;
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (!pend[u]) continue;
        const uint64_t kk = (uint64_t)hw[u].x | ((uint64_t)hw[u].y << 32);
        if (kk == hkey[u]) {
          v[u] = __uint_as_float(hw[u].z);
          pend[u] = false;
        } else if (kk == 0ull) {
          pend[u] = false;
        } else {
          hs[u] = (hs[u] + 1) & a.bh_mask;
          anyp = true;
        }
      }
    }
    int64_t inc[U];
    bool closed[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t e = base + (int64_t)u * nthreads;
      const bool live = e < a.count;
      closed[u] = live && v[u] != 0.0f;
      inc[u] = 0;
      if (closed[u]) {
        const int64_t mag = (int64_t)rint(ldexp((double)v[u], F));
        inc[u] = sg[u] ? -mag : mag;
      }
      if (DEBUG && live) {
        ok[e] = (int32_t)k[u];
        oi[e] = (int32_t)i[u];
        oj[e] = (int32_t)j[u];
        okp[e] = (int32_t)kp[u];
        oinc[e] = inc[u];
      }
    }
    if (!DEBUG) {
      uint64_t key[U], slot[U];
      bool pend[U], ins[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        uint64_t ii = i[u], jj = j[u];
        ins[u] = closed[u];
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
        nclosed += closed[u];
      }
      if (pkeys) {
        // pair form: the key and the signed fourth edge at the sample's
        // offset in this launch
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const int64_t e = base + (int64_t)u * nthreads;
          if (e < a.count) {
            __builtin_nontemporal_store(
                (unsigned long long)(ins[u] ? key[u] : kEmptyKey),
                (unsigned long long*)(pkeys + e));
            __builtin_nontemporal_store(sg[u] ? -v[u] : v[u], pvals + e);
            if (a.pk2) {  // Sec. 3.2.3: the same increment to x_kk'
              uint64_t kk = k[u], kq = kp[u];
              bool ins2 = closed[u] && kk != kq;  // diagonal left out
              if (kk > kq) {
                const uint64_t tmp = kk;
                kk = kq;
                kq = tmp;
              }
              __builtin_nontemporal_store(
                  (unsigned long long)(ins2 ? kk * (uint64_t)a.n + kq
                                            : kEmptyKey),
                  (unsigned long long*)(a.pk2 + e));
              __builtin_nontemporal_store(sg[u] ? -v[u] : v[u], a.pv2 + e);
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
        if (!pkeys && ins[u] && inc[u] != 0)
          atomicAdd((unsigned long long*)(hvals + slot[u]),
                    (unsigned long long)inc[u]);
    }
  }
  if (!DEBUG) {
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

// the squared variant needs A == A^T: the compressed rows of A must equal
// its transpose (per coordinate, the vectors in ascending order with their
// values) entry for entry; *flag = 1 on any difference
__global__ void k_check_csr_symmetric(const int64_t* ptr, const int32_t* idx,
                                      const float* val, const int64_t* tptr,
                                      const uint32_t* trow, const float* tval,
                                      int64_t rows, int64_t nnz, int* flag) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  bool diff = false;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
       e <= rows || e < nnz; e += stride) {
    if (e <= rows && ptr[e] != tptr[e]) diff = true;
    if (e < nnz && (idx[e] != (int32_t)trow[e] || val[e] != tval[e]))
      diff = true;
  }
  if (diff) *flag = 1;
}

hipError_t launch_check_csr_symmetric(const CsrTables& t, int* flag,
                                      hipStream_t st) {
  hipError_t e = launch_fill_u64((uint64_t*)flag, 1, 0ull, st);
  if (e != hipSuccess) return e;
  const int64_t work = (t.m + 1 > t.nnzA ? t.m + 1 : t.nnzA);
  int64_t blocks = (work + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  k_check_csr_symmetric<<<(unsigned)(blocks < 1 ? 1 : blocks), 256, 0, st>>>(
      t.in.a_ptr, t.in.a_idx, t.in.a_val, t.at_ptr, t.at_row, t.at_val, t.m,
      t.nnzA, flag);
  return hipGetLastError();
}

hipError_t csr_validate(const CsrView& in, int64_t m, int64_t n, int64_t d,
                        int64_t nnzA, int64_t nnzB, int* flag,
                        hipStream_t st) {
  hipError_t e = launch_fill_u64((uint64_t*)flag, 1, 0ull, st);
  if (e != hipSuccess) return e;
  k_csr_check<<<blocks_of(m, 256), 256, 0, st>>>(in.a_ptr, in.a_idx, in.a_val,
                                                  m, d, nnzA, nullptr, flag);
  k_csr_check<<<blocks_of(n, 256), 256, 0, st>>>(in.b_ptr, in.b_idx, in.b_val,
                                                  n, d, nnzB, nullptr, flag);
  int bad = 0;
  if ((e = hipMemcpyAsync(&bad, flag, 4, hipMemcpyDeviceToHost, st)) !=
          hipSuccess ||
      (e = hipStreamSynchronize(st)) != hipSuccess)
    return e;
  return bad ? hipErrorInvalidValue : hipSuccess;
}

static CsrSampleArgs csr_args(const CsrTables& t, uint64_t seed, uint64_t qid,
                              int64_t l0, int64_t count) {
  CsrSampleArgs a;
  a.T0 = t.T0.ent;
  a.L0 = t.T0.L;
  a.m1 = t.T1.meta;
  a.e1 = (const Ent32*)t.T1.ent;
  a.m2 = t.T2.meta;
  a.e2 = (const Ent32*)t.T2.ent;
  a.m3 = t.T3.meta;
  a.e3 = (const Ent16*)t.T3.ent;
  a.in = t.in;
  a.n = t.n;
  a.seed = seed;
  a.qid = qid;
  a.l0 = l0;
  a.count = count;
  a.gram = t.gram;
  a.bh = t.bh;
  a.bh_mask = t.bh_mask;
  a.d = t.d;
  a.pk2 = nullptr;
  a.pv2 = nullptr;
  return a;
}

// MAD_CSR_GRID caps the sampling grid and MAD_CSR_UNROLL (2, 4, 8, 16)
// sets the samples per thread in flight (the draws are chains of dependent
// random loads; with T2's 32-byte entries four per thread and a grid of up
// to 32768 blocks measured best, eight per thread holding half as many
// waves); neither changes the result
static unsigned csr_grid(int64_t count, int per_thread) {
  static const int64_t cap = [] {
    const char* e = getenv("MAD_CSR_GRID");
    const long v = e ? atol(e) : 32768;
    return (int64_t)(v >= 256 && v <= (1 << 20) ? v : 32768);
  }();
  int64_t blocks = (count + 256LL * per_thread - 1) / (256LL * per_thread);
  if (blocks > cap) blocks = cap;
  return (unsigned)(blocks < 1 ? 1 : blocks);
}

static int csr_unroll() {
  static const int u = [] {
    const char* e = getenv("MAD_CSR_UNROLL");
    const int v = e ? atoi(e) : 4;
    return v == 2 || v == 8 || v == 16 ? v : 4;
  }();
  return u;
}

static size_t csr_t0_lds(const CsrTables& t) {
  const int64_t N0 = int64_t(1) << t.T0.L;
  return N0 <= kT0LdsCsr ? (size_t)N0 * 8 : 0;
}

hipError_t launch_sample_csr(const CsrTables& t, uint64_t seed, uint64_t qid,
                             int64_t l0, int64_t count, int64_t s_for_F,
                             HashTable h, SampleCounters* ctr,
                             hipStream_t st) {
  if (count <= 0) return hipSuccess;
  CsrSampleArgs a = csr_args(t, seed, qid, l0, count);
  a.pk2 = h.pkeys2;
  a.pv2 = h.pvals2;
  switch (csr_unroll()) {
#define MAD_CSR_CASE(UU)                                                     \
  case UU:                                                                   \
    k_sample_csr<UU, false><<<csr_grid(count, UU), 256, csr_t0_lds(t), st>>>( \
        a, t.T0.tot, t.bmax, s_for_F, 0, h.keys, h.vals,                     \
        (uint64_t)h.cap - 1, h.pkeys, h.pvals, ctr, nullptr, nullptr,        \
        nullptr, nullptr, nullptr);                                          \
    break;
    MAD_CSR_CASE(2)
    MAD_CSR_CASE(8)
    MAD_CSR_CASE(16)
    default:
    MAD_CSR_CASE(4)
#undef MAD_CSR_CASE
  }
  return hipGetLastError();
}

hipError_t launch_sample_csr_debug(const CsrTables& t, uint64_t seed,
                                   uint64_t qid, int64_t l0, int64_t count,
                                   int F, int32_t* k, int32_t* i, int32_t* j,
                                   int32_t* kp, int64_t* inc, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  const CsrSampleArgs a = csr_args(t, seed, qid, l0, count);
  k_sample_csr<2, true><<<csr_grid(count, 2), 256, csr_t0_lds(t), st>>>(
      a, t.T0.tot, t.bmax, 0, F, nullptr, nullptr, 0, nullptr, nullptr, nullptr,
      k, i, j, kp, inc);
  return hipGetLastError();
}

}  // namespace mad
