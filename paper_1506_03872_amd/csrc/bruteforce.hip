// bruteforce.hip -- exhaustive t-MAD (Definition 1) with MFMA matrix cores:
// the products a_i . b_j of every pair, top t by |c|, without ever storing
// the m x n product (the exact baseline of Sec. 5.3 computes C in blocks and
// keeps a priority queue; here the GEMM epilogue filters against a bound).
//
//   pass A  GEMM over every 64th row of A; the epilogue histograms the lower
//           bounds |c^| - margin(i,j) of the computed values (2048 monotone
//           bins).  The lower edge tau of the bin holding the t-th largest
//           bound is <= the t-th largest |c| over all pairs.
//   pass B  GEMM over all pairs; the epilogue appends every pair with
//           |c^| + margin(i,j) >= tau.  That set holds every pair of the
//           exact top t.
//   final   fp32 dot products of the survivors (the same kernel the sampled
//           path uses) and an exact top-t selection on them.
//
// margin(i,j) bounds |c^ - c_fp32| for the MFMA arithmetic: inputs rounded to
// bf16 / fp8-e4m3 (relative error u, plus an absolute underflow term for
// fp8 after a per-vector power-of-two scale), fp32 accumulation over d
// terms (gamma_d), and the error of the fp32 re-rank itself (standard dot
// product error analysis, Higham, "Accuracy and Stability of Numerical
// Algorithms", 2nd ed., Sec. 3.1).
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include "../../include/mad.h"
#include "mad_common.hpp"
#include "plan.hpp"

namespace mad {

typedef float f16v __attribute__((ext_vector_type(16)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));
typedef int i8v __attribute__((ext_vector_type(8)));

enum Prec { kF32 = 0, kBF16 = 1, kFP8 = 2 };

// element bytes, k per MFMA, k per LDS chunk (a 128-byte row slice)
template <int P> struct PrecT;
template <> struct PrecT<kF32> {
  static constexpr int EB = 4, KS = 2, KC = 32;
};
template <> struct PrecT<kBF16> {
  static constexpr int EB = 2, KS = 16, KC = 64;
};
template <> struct PrecT<kFP8> {
  static constexpr int EB = 1, KS = 64, KC = 128;
};

constexpr int kBM = 128, kBN = 128;  // workgroup tile
constexpr int kRowBytes = 128;       // bytes of one row slice in LDS
constexpr int kLdsStride = kRowBytes + 16;

// ---------------------------------------------------------------------------
// preparation: padded low-precision copies (row stride Kp elements), the
// per-vector scale (fp8: a power of two), L2 and L1 norms of the fp32
// vector and the absolute rounding floor eta (in the vector's own units)
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint8_t to_fp8(float x) {
  // round to nearest even into e4m3; |x| < 2^7 after scaling
  const unsigned pk = __builtin_amdgcn_cvt_pk_fp8_f32(x, 0.0f, 0, false);
  return (uint8_t)(pk & 0xff);
}

__device__ __forceinline__ uint16_t to_bf16(float x) {
  // round to nearest even (inputs are finite)
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

template <int P>
__global__ __launch_bounds__(256) void k_prep(const float* X, int64_t rows,
                                              int64_t d, int64_t Kp,
                                              void* out, VecInfo* info) {
  const int lane = threadIdx.x & 63;
  const int64_t r = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  if (r >= rows) return;
  const float* x = X + r * d;
  double s2 = 0.0, s1 = 0.0;
  float mx = 0.0f;
  for (int64_t k = lane; k < d; k += 64) {
    const double v = x[k];
    s2 += v * v;
    s1 += fabs(v);
    mx = fmaxf(mx, fabsf(x[k]));
  }
  s2 = wave_sum(s2);
  s1 = wave_sum(s1);
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) mx = fmaxf(mx, __shfl_xor(mx, off, 64));
  float scale = 1.0f, eta = 0.0f;
  if (P == kFP8) {
    int e = 0;
    if (mx > 0.0f) (void)frexpf(mx, &e);  // mx < 2^e
    // scaled max < 2^7; 1 / scale stays a normal float (an E8M0 exponent)
    if (e < -119) e = -119;
    scale = ldexpf(1.0f, 7 - e);
    eta = ldexpf(1.0f, -10) / scale;      // half the e4m3 subnormal step
  } else if (P == kBF16) {
    eta = ldexpf(1.0f, -134);
  }
  if (lane == 0) {
    VecInfo vi;
    vi.n2 = (float)(sqrt(s2) * (1.0 + 1e-6));
    vi.n1 = (float)(s1 * (1.0 + 1e-6));
    vi.eta = eta;
    vi.inv_s = 1.0f / scale;
    info[r] = vi;
  }
  for (int64_t k = lane; k < Kp; k += 64) {
    const float v = k < d ? x[k] : 0.0f;
    if (P == kF32) ((float*)out)[r * Kp + k] = v;
    else if (P == kBF16) ((uint16_t*)out)[r * Kp + k] = to_bf16(v);
    else ((uint8_t*)out)[r * Kp + k] = to_fp8(v * scale);
  }
}

// ---------------------------------------------------------------------------
// the GEMM: a 128 x 128 tile per workgroup, 4 waves of 64 x 64, each wave
// 2 x 2 MFMA blocks of 32 x 32.  MFMA operand layout (32 x 32 x K): lane l
// supplies row (l mod 32) of A and column (l mod 32) of B for its k group
// (l / 32); accumulator register r of lane l is row 8(r/4) + 4(l/32) + r%4,
// column l mod 32 of the block.
// ---------------------------------------------------------------------------
struct GemmArgs {
  const void* A;  // rows of Kp elements
  const void* B;
  const VecInfo* ia;
  const VecInfo* ib;
  int64_t m_rows;  // rows of A used
  int64_t a_stride_rows;  // A row i of this pass is row i*stride of the copy
  int64_t m_key;   // row index multiplier for keys (= stride)
  int64_t n, Kp;
  float kappa;     // relative margin factor on ||a||_2 ||b||_2
  float onepu;     // 1 + u
  float d_f;       // d (for the eta * eta term)
  // pass A
  unsigned* hist;
  int screen;      // 1: no error margin (screening by the computed value)
  float mg_max;    // margin upper bound over all pairs (cheap pre-test)
  // pass B
  const unsigned* tau_bits;  // lower bound (float bits)
  float* cval;     // computed value of each survivor
  uint64_t* ckey;
  int64_t ccap;
  unsigned long long* ccount;
};

// the MFMA operands of one K step: rows (l mod 32) of the wave's two
// 32-row blocks of A and of B, K group l / 32
template <int P> struct Frag;
template <> struct Frag<kF32> { typedef float T; T a[2], b[2]; };
template <> struct Frag<kBF16> { typedef bf8v T; T a[2], b[2]; };
template <> struct Frag<kFP8> { typedef i8v T; T a[2], b[2]; };

template <int P>
__device__ __forceinline__ void frag_load(const char* la, const char* lb,
                                          int koff_bytes, int lane,
                                          Frag<P>& f) {
  const int r = lane & 31, g = lane >> 5;
  using PT = PrecT<P>;
  constexpr int gb = PT::KS / 2 * PT::EB;  // bytes of one K group
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    typedef typename Frag<P>::T T;
    f.a[u] = *(const T*)(la + (u * 32 + r) * kLdsStride + koff_bytes +
                         g * gb);
    f.b[u] = *(const T*)(lb + (u * 32 + r) * kLdsStride + koff_bytes +
                         g * gb);
  }
}

// ZERO: the accumulators start from zero (the tile's first K step)
template <int P, bool ZERO = false>
__device__ __forceinline__ void frag_mma(const Frag<P>& f, f16v (&acc)[2][2],
                                         const int (&sa)[2],
                                         const int (&sb)[2]) {
  const f16v zero = {};
#pragma unroll
  for (int bi = 0; bi < 2; ++bi)
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
      const f16v c = ZERO ? zero : acc[bi][bj];
      if constexpr (P == kF32)
        acc[bi][bj] = __builtin_amdgcn_mfma_f32_32x32x2f32(
            f.a[bi], f.b[bj], c, 0, 0, 0);
      else if constexpr (P == kBF16)
        acc[bi][bj] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
            f.a[bi], f.b[bj], c, 0, 0, 0);
      else
        acc[bi][bj] = __builtin_amdgcn_mfma_scale_f32_32x32x64_f8f6f4(
            f.a[bi], f.b[bj], c, 0, 0, 0, sa[bi], 0, sb[bj]);
    }
}

// monotone 11-bit digit of a non-negative float (exponent and the top 3
// mantissa bits); bin b holds the floats with bits in [b << 20, (b+1) << 20)
__device__ __forceinline__ int fbin32(uint32_t bits) {
  return (int)(bits >> 20) & 2047;
}

// E8M0 byte of a vector's power-of-two inverse scale (the MFMA multiplies
// the products of a lane's 32-element K block by 2^(byte - 127) per operand)
__device__ __forceinline__ int e8m0_of(float inv_s) {
  return (int)((__float_as_uint(inv_s) >> 23) & 0xff);
}

// Tiles of 128 x 128 in bands of 8 row-tiles; within a band the column
// tiles advance.  Workgroups are dispatched to the 8 XCDs round robin, so
// virtual block v = (blockIdx mod 8) G/8 + blockIdx / 8 gives each XCD a
// contiguous run of G/8 tiles per sweep: a column tile (a slice of B) is
// read by one XCD per band instead of by all eight.  K runs in stages of
// 128-byte row slices through two LDS buffers: the next stage (or the next
// tile's first) is loaded into registers while the current one computes.
__device__ __forceinline__ void gemm_coords(int64_t tile, int64_t tiles_m,
                                            int64_t tiles_n, int64_t& i0,
                                            int64_t& j0) {
  const int64_t band = tile / (8 * tiles_n);
  const int64_t within = tile % (8 * tiles_n);
  const int64_t band_rows = tiles_m - band * 8 < 8 ? tiles_m - band * 8 : 8;
  i0 = (band * 8 + within % band_rows) * kBM;
  j0 = (within / band_rows) * kBN;
}

// EARLY: the next stage's loads are issued ahead of the current stage's
// MFMAs (pays with at most four stages per tile; with longer K the loads
// issued after the MFMAs measured faster)
template <int P, bool HIST, bool EARLY>
__global__ __launch_bounds__(256) void k_gemm_topk(GemmArgs g) {
  using PT = PrecT<P>;
  __shared__ __attribute__((aligned(16))) char lds_a[2][kBM * kLdsStride];
  __shared__ __attribute__((aligned(16))) char lds_b[2][kBN * kLdsStride];
  __shared__ unsigned hist[HIST ? 2048 : 1];
  const int t = threadIdx.x, lane = t & 63, wv = t >> 6;
  const int wr = wv >> 1, wc = wv & 1;
  if (HIST) {
    for (int b = t; b < 2048; b += 256) hist[b] = 0;
    __syncthreads();
  }
  const int64_t tiles_m = (g.m_rows + kBM - 1) / kBM;
  const int64_t tiles_n = (g.n + kBN - 1) / kBN;
  const int64_t ntiles = tiles_m * tiles_n;
  const int64_t row_bytes = g.Kp * PT::EB;
  const int64_t nst = row_bytes / kRowBytes;  // Kp EB is a multiple of 128
  const char* Ab = (const char*)g.A;
  const char* Bb = (const char*)g.B;
  const float tau = HIST ? 0.0f : __uint_as_float(*g.tau_bits);
  const int64_t G = gridDim.x;  // a multiple of 8
  const int64_t v = (int64_t)(blockIdx.x & 7) * (G >> 3) + (blockIdx.x >> 3);
  // this thread's 4 x 16 bytes of each operand's stage: rows (t >> 3) +
  // 32 q, bytes (t & 7) 16 of the 128-byte slice
  const int seg = (t & 7) * 16;
// one 16-byte piece q of each operand's stage (rows (t >> 3) + 32 q), and
// its store to LDS; written out per q so that ra / rb stay in registers
#define MAD_BF_GLOAD1(Q, I0, J0, KB)                                         \
  {                                                                          \
    const int row = (t >> 3) + 32 * (Q);                                     \
    int64_t ia = (I0) + row;                                                 \
    ia = ia < g.m_rows ? ia : g.m_rows - 1;                                  \
    int64_t jb = (J0) + row;                                                 \
    jb = jb < g.n ? jb : g.n - 1;                                            \
    ra##Q = *(const uint4*)(Ab + ia * g.a_stride_rows * row_bytes + (KB) +   \
                            seg);                                            \
    rb##Q = *(const uint4*)(Bb + jb * row_bytes + (KB) + seg);               \
  }
#define MAD_BF_GLOAD(I0, J0, KB)                                             \
  MAD_BF_GLOAD1(0, I0, J0, KB) MAD_BF_GLOAD1(1, I0, J0, KB)                  \
  MAD_BF_GLOAD1(2, I0, J0, KB) MAD_BF_GLOAD1(3, I0, J0, KB)
#define MAD_BF_LSTORE1(Q, BUF)                                               \
  {                                                                          \
    const int row = (t >> 3) + 32 * (Q);                                     \
    *(uint4*)(lds_a[BUF] + row * kLdsStride + seg) = ra##Q;                  \
    *(uint4*)(lds_b[BUF] + row * kLdsStride + seg) = rb##Q;                  \
  }
#define MAD_BF_LSTORE(BUF)                                                   \
  MAD_BF_LSTORE1(0, BUF) MAD_BF_LSTORE1(1, BUF) MAD_BF_LSTORE1(2, BUF)       \
  MAD_BF_LSTORE1(3, BUF)
// full tiles (no row past the end): the 4 pieces of an operand are 32 rows
// apart, so one base pointer per tile serves every stage
#define MAD_BF_FULL(I0, J0) ((I0) + kBM <= g.m_rows && (J0) + kBN <= g.n)
#define MAD_BF_PA(I0) (Ab + ((I0) + trow) * g.a_stride_rows * row_bytes + seg)
#define MAD_BF_PB(J0) (Bb + ((J0) + trow) * row_bytes + seg)
#define MAD_BF_GLOADF(PA, PB, KB)                                            \
  {                                                                          \
    ra0 = *(const uint4*)((PA) + (KB));                                      \
    ra1 = *(const uint4*)((PA) + astep + (KB));                              \
    ra2 = *(const uint4*)((PA) + 2 * astep + (KB));                          \
    ra3 = *(const uint4*)((PA) + 3 * astep + (KB));                          \
    rb0 = *(const uint4*)((PB) + (KB));                                      \
    rb1 = *(const uint4*)((PB) + bstep + (KB));                              \
    rb2 = *(const uint4*)((PB) + 2 * bstep + (KB));                          \
    rb3 = *(const uint4*)((PB) + 3 * bstep + (KB));                          \
  }
  const int64_t trow = t >> 3;
  const int64_t astep = 32 * g.a_stride_rows * row_bytes;
  const int64_t bstep = 32 * row_bytes;
  uint4 ra0, ra1, ra2, ra3, rb0, rb1, rb2, rb3;
  int64_t tile = v;
  int64_t i0 = 0, j0 = 0;
  bool full = false;
  const char* pa = Ab;
  const char* pb = Bb;
  if (tile < ntiles) {
    gemm_coords(tile, tiles_m, tiles_n, i0, j0);
    full = MAD_BF_FULL(i0, j0);
    pa = MAD_BF_PA(i0);
    pb = MAD_BF_PB(j0);
    if (full) {
      MAD_BF_GLOADF(pa, pb, 0)
    } else {
      MAD_BF_GLOAD(i0, j0, 0)
    }
  }
  while (tile < ntiles) {
    const int64_t next = tile + G;
    int64_t ni0 = 0, nj0 = 0;
    if (next < ntiles) gemm_coords(next, tiles_m, tiles_n, ni0, nj0);
    const bool nfull = next < ntiles && MAD_BF_FULL(ni0, nj0);
    const char* npa = MAD_BF_PA(ni0);
    const char* npb = MAD_BF_PB(nj0);
    // fp8: the per-vector scales of the rows this lane feeds the MFMA
    int sa[2] = {127, 127}, sb[2] = {127, 127};
    if (P == kFP8) {
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        int64_t ia = i0 + wr * 64 + u * 32 + (lane & 31);
        ia = ia < g.m_rows ? ia : g.m_rows - 1;
        int64_t jb = j0 + wc * 64 + u * 32 + (lane & 31);
        jb = jb < g.n ? jb : g.n - 1;
        sa[u] = e8m0_of(g.ia[ia * g.a_stride_rows].inv_s);
        sb[u] = e8m0_of(g.ib[jb].inv_s);
      }
    }
    MAD_BF_LSTORE(0)
    __syncthreads();
    // the tile's first MFMAs start from a zero C operand (no per-tile
    // clearing of the 64 accumulators); a tile always has a stage (Kp >= 1)
    f16v acc[2][2];
    if (nst == 0) {
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
          for (int e = 0; e < 16; ++e) acc[bi][bj][e] = 0.0f;
    }
    int cur = 0;
    for (int64_t st = 0; st < nst; ++st) {
      // the next stage, else the next tile's first, else (last tile) a
      // harmless reload of this tile's first: unconditional loads keep
      // ra / rb in registers
      const bool more = st + 1 < nst;
      const bool nx = !more && next < ntiles;
      const int64_t li0 = nx ? ni0 : i0;
      const int64_t lj0 = nx ? nj0 : j0;
      const int64_t lkb = more ? (st + 1) * kRowBytes : 0;
      if (nx ? nfull : full) {
        const char* lpa = nx ? npa : pa;
        const char* lpb = nx ? npb : pb;
        MAD_BF_GLOADF(lpa, lpb, lkb)
      } else {
        MAD_BF_GLOAD(li0, lj0, lkb)
      }
      // keep the loads issued here, ahead of the MFMAs: without this the
      // compiler sinks them into the LDS store below, behind the stage's
      // MFMAs, and the stage then waits out a full memory latency
      if constexpr (EARLY) asm volatile("" ::: "memory");
      const char* la = lds_a[cur] + (wr * 64) * kLdsStride;
      const char* lb = lds_b[cur] + (wc * 64) * kLdsStride;
      // the next K step's operands are read from LDS while the current
      // step's MFMAs run
      constexpr int nks = PT::KC / PT::KS;
      Frag<P> fr[2];
      frag_load<P>(la, lb, 0, lane, fr[0]);
#pragma unroll
      for (int ks = 0; ks < nks; ++ks) {
        if (ks + 1 < nks)
          frag_load<P>(la, lb, (ks + 1) * PT::KS * PT::EB, lane,
                       fr[(ks + 1) & 1]);
        if (ks == 0 && st == 0)
          frag_mma<P, true>(fr[0], acc, sa, sb);
        else
          frag_mma<P>(fr[ks & 1], acc, sa, sb);
      }
      if (more) {
        MAD_BF_LSTORE(cur ^ 1)
      }
      __syncthreads();
      cur ^= 1;
    }
    // epilogue.  Pass B: |c| + margin >= tau only when |c| >= tau - mg_max,
    // which almost no pair meets; those few compute the exact margin.
    const int cl = lane & 31, rg = lane >> 5;
    // tau (1 - 2^-20) - mg_max absorbs the roundings of both comparisons
    const float pre = HIST ? 0.0f : fmaf(tau, 1.0f - 0x1p-20f, -g.mg_max);
    // pass B: one max over the lane's 64 values first; the per-element
    // work below runs only in waves where some lane passes
    bool any = true;
    if (!HIST) {
      float mx = 0.0f;
#pragma unroll
      for (int bi = 0; bi < 2; ++bi)
#pragma unroll
        for (int bj = 0; bj < 2; ++bj)
#pragma unroll
          for (int e = 0; e < 16; ++e) mx = fmaxf(mx, fabsf(acc[bi][bj][e]));
      any = mx >= pre;
    }
    if (any) {
#pragma unroll
    for (int bj = 0; bj < 2; ++bj) {
      const int64_t j = j0 + wc * 64 + bj * 32 + cl;
      const bool jok = j < g.n;
#pragma unroll
      for (int bi = 0; bi < 2; ++bi) {
#pragma unroll
        for (int e = 0; e < 16; ++e) {
          const int64_t i = i0 + wr * 64 + bi * 32 + 8 * (e >> 2) + 4 * rg +
                            (e & 3);
          const float c = acc[bi][bj][e];
          if (!HIST && !(fabsf(c) >= pre)) continue;
          if (!(jok && i < g.m_rows)) continue;
          const VecInfo va = g.ia[i * g.a_stride_rows];
          const VecInfo vb = g.ib[j];
          const float mg = g.screen ? 0.0f
                                    : g.kappa * va.n2 * vb.n2 +
                                      g.onepu * (va.eta * vb.n1 +
                                                 vb.eta * va.n1) +
                                      g.d_f * va.eta * vb.eta;
          if (HIST) {
            const float lo = fabsf(c) - mg;
            if (lo > 0.0f) atomicAdd(&hist[fbin32(__float_as_uint(lo))], 1u);
          } else if (fabsf(c) + mg >= tau) {
            const unsigned long long p = atomicAdd(g.ccount, 1ull);
            if ((int64_t)p < g.ccap) {
              g.ckey[p] = (uint64_t)(i * g.m_key) * (uint64_t)g.n + (uint64_t)j;
              g.cval[p] = c;
            }
          }
        }
      }
    }
    }
    tile = next;
    i0 = ni0;
    j0 = nj0;
    full = nfull;
    pa = npa;
    pb = npb;
  }
  if (HIST) {
    __syncthreads();
    for (int b = t; b < 2048; b += 256)
      if (hist[b]) atomicAdd(&g.hist[b], hist[b]);
  }
}
#undef MAD_BF_GLOAD1
#undef MAD_BF_GLOAD
#undef MAD_BF_FULL
#undef MAD_BF_PA
#undef MAD_BF_PB
#undef MAD_BF_GLOADF
#undef MAD_BF_LSTORE1
#undef MAD_BF_LSTORE

// maxima of n2, n1 and eta over the vectors (float bits, atomically)
__global__ void k_vecinfo_max(const VecInfo* v, int64_t rows, unsigned* mx) {
  float a = 0.0f, b = 0.0f, c = 0.0f;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < rows;
       r += stride) {
    a = fmaxf(a, v[r].n2);
    b = fmaxf(b, v[r].n1);
    c = fmaxf(c, v[r].eta);
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    a = fmaxf(a, __shfl_xor(a, off, 64));
    b = fmaxf(b, __shfl_xor(b, off, 64));
    c = fmaxf(c, __shfl_xor(c, off, 64));
  }
  if ((threadIdx.x & 63) == 0) {
    atomicMax(&mx[0], __float_as_uint(a));
    atomicMax(&mx[1], __float_as_uint(b));
    atomicMax(&mx[2], __float_as_uint(c));
  }
}

// lower edge (float bits) of the histogram bin holding the t-th largest
// bound, from the top; 0 when fewer than t bounds are positive
__global__ void k_bf_tau(const unsigned* hist, int64_t t, unsigned* tau_bits) {
  if (threadIdx.x != 0) return;
  unsigned long long acc = 0;
  int b = 2047;
  for (; b >= 0; --b) {
    acc += hist[b];
    if ((int64_t)acc >= t) break;
  }
  *tau_bits = b > 0 ? (unsigned)b << 20 : 0u;
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
struct BfWork {
  DeviceBuffer ac, bc, ia, ib, misc, keys, vals, sel, selbuf, fin;
  int64_t m = 0, n = 0, d = 0;
  int prec = -1;
  const float* A = nullptr;
  const float* B = nullptr;
};

static BfWork g_bf;  // process-wide cache of the conversion workspace

static double gamma_d(int64_t d) {
  const double u = ldexp(1.0, -24);
  return d * u / (1.0 - d * u);
}

template <int P>
static void launch_gemm(const GemmArgs& a, bool hist, hipStream_t st) {
  // persistent workgroups, two per CU (LDS), a multiple of 8 (one share
  // per XCD); MAD_BF_GRID overrides the count (the result is the same)
  const int64_t tiles = ((a.m_rows + kBM - 1) / kBM) * ((a.n + kBN - 1) / kBN);
  int64_t grid = tiles < 256 * 2 ? (tiles + 7) / 8 * 8 : 256 * 2;
  if (const char* ev = getenv("MAD_BF_GRID")) {
    const int64_t gv = atoll(ev) / 8 * 8;
    if (gv >= 8) grid = gv;
  }
  if (grid < 8) grid = 8;

  // early loads for tiles of at most four K stages (128-byte slices)
  const bool early = a.Kp * PrecT<P>::EB <= 4 * kRowBytes;
  if (hist) {
    if (early) k_gemm_topk<P, true, true><<<(unsigned)grid, 256, 0, st>>>(a);
    else k_gemm_topk<P, true, false><<<(unsigned)grid, 256, 0, st>>>(a);
  } else {
    if (early) k_gemm_topk<P, false, true><<<(unsigned)grid, 256, 0, st>>>(a);
    else k_gemm_topk<P, false, false><<<(unsigned)grid, 256, 0, st>>>(a);
  }
}

hipError_t lowp_prepare(const float* X, int64_t rows, int64_t d, int prec,
                        DeviceBuffer& data, DeviceBuffer& info, int64_t* Kp,
                        hipStream_t st) {
  const int KC = prec == kBF16 ? 64 : 128;
  const int EB = prec == kBF16 ? 2 : 1;
  if (prec != kBF16 && prec != kFP8) return hipErrorInvalidValue;
  const int64_t kp = (d + KC - 1) / KC * KC;
  hipError_t e;
  if ((e = dev_alloc(data, (size_t)rows * kp * EB)) != hipSuccess ||
      (e = dev_alloc(info, (size_t)rows * sizeof(VecInfo))) != hipSuccess)
    return e;
  const unsigned g = (unsigned)((rows + 3) / 4);
  if (prec == kBF16)
    k_prep<kBF16><<<g, 256, 0, st>>>(X, rows, d, kp, data.p,
                                      (VecInfo*)info.p);
  else
    k_prep<kFP8><<<g, 256, 0, st>>>(X, rows, d, kp, data.p,
                                     (VecInfo*)info.p);
  *Kp = kp;
  return hipGetLastError();
}

void lowp_consts(int prec, int64_t d, float* kappa, float* onepu) {
  const double u = prec == kF32 ? 0.0 : prec == kBF16 ? ldexp(1.0, -8)
                                                       : ldexp(1.0, -4);
  const double g = gamma_d(d);
  *kappa = (float)((2 * u + u * u + g * (1 + u) * (1 + u) + g) * (1 + 1e-5));
  *onepu = (float)((1 + u) * (1 + 1e-5));
}

hipError_t bruteforce_topk(const float* A, int64_t m, const float* B,
                           int64_t n, int64_t d, int prec, int64_t t,
                           int64_t cap_hint, void* out, int64_t* n_out,
                           BfStats* stats, hipStream_t st) {
  return bruteforce_run(A, m, B, n, d, prec, t, cap_hint, -1.0f, out, n_out,
                        nullptr, nullptr, stats, st);
}

hipError_t bruteforce_run(const float* A, int64_t m, const float* B,
                          int64_t n, int64_t d, int prec, int64_t t,
                          int64_t cap_hint, float tau_user, void* out,
                          int64_t* n_out, const uint64_t** cand_keys,
                          int64_t* cand_count, BfStats* stats,
                          hipStream_t st) {
  hipError_t e;
  int KC = prec == kF32 ? 32 : prec == kBF16 ? 64 : 128;
  int EB = prec == kF32 ? 4 : prec == kBF16 ? 2 : 1;
  const int64_t Kp = (d + KC - 1) / KC * KC;
  BfWork& w = g_bf;
  const bool fresh = w.m != m || w.n != n || w.d != d || w.prec != prec ||
                     w.A != A || w.B != B;
  if ((e = dev_alloc(w.ac, (size_t)m * Kp * EB)) != hipSuccess) return e;
  if ((e = dev_alloc(w.bc, (size_t)n * Kp * EB)) != hipSuccess) return e;
  if ((e = dev_alloc(w.ia, (size_t)m * sizeof(VecInfo))) != hipSuccess) return e;
  if ((e = dev_alloc(w.ib, (size_t)n * sizeof(VecInfo))) != hipSuccess) return e;
  if ((e = dev_alloc(w.misc, 2048 * 4 + 512)) != hipSuccess) return e;
  (void)fresh;
  w.m = m; w.n = n; w.d = d; w.prec = prec; w.A = A; w.B = B;
  hipEvent_t ev[4];
  for (auto& x : ev) (void)hipEventCreate(&x);
  (void)hipEventRecord(ev[0], st);
  // conversion is part of every call (the inputs may change between calls)
  const unsigned ga = (unsigned)((m + 3) / 4), gb = (unsigned)((n + 3) / 4);
  if (prec == kF32) {
    k_prep<kF32><<<ga, 256, 0, st>>>(A, m, d, Kp, w.ac.p, (VecInfo*)w.ia.p);
    k_prep<kF32><<<gb, 256, 0, st>>>(B, n, d, Kp, w.bc.p, (VecInfo*)w.ib.p);
  } else if (prec == kBF16) {
    k_prep<kBF16><<<ga, 256, 0, st>>>(A, m, d, Kp, w.ac.p, (VecInfo*)w.ia.p);
    k_prep<kBF16><<<gb, 256, 0, st>>>(B, n, d, Kp, w.bc.p, (VecInfo*)w.ib.p);
  } else {
    k_prep<kFP8><<<ga, 256, 0, st>>>(A, m, d, Kp, w.ac.p, (VecInfo*)w.ia.p);
    k_prep<kFP8><<<gb, 256, 0, st>>>(B, n, d, Kp, w.bc.p, (VecInfo*)w.ib.p);
  }
  unsigned* hist = (unsigned*)w.misc.p;
  unsigned* tau_bits = hist + 2048;
  unsigned long long* ccount = (unsigned long long*)(hist + 2048 + 16);
  unsigned* maxes = hist + 2048 + 32;  // n2, n1, eta of A then of B
  if ((e = launch_fill_u64((uint64_t*)hist, 1024 + 8 + 8 + 8, 0ull, st)) !=
      hipSuccess)
    return e;
  k_vecinfo_max<<<64, 256, 0, st>>>((const VecInfo*)w.ia.p, m, maxes);
  k_vecinfo_max<<<64, 256, 0, st>>>((const VecInfo*)w.ib.p, n, maxes + 4);
  // margin factor: input rounding (2u + u^2) plus gamma_d for the MFMA
  // accumulation and gamma_d for the fp32 re-rank
  const double u = prec == kF32 ? 0.0 : prec == kBF16 ? ldexp(1.0, -8)
                                                       : ldexp(1.0, -4);
  const double g = gamma_d(d);
  GemmArgs a;
  a.A = w.ac.p;
  a.B = w.bc.p;
  a.ia = (const VecInfo*)w.ia.p;
  a.ib = (const VecInfo*)w.ib.p;
  a.n = n;
  a.Kp = Kp;
  a.kappa = (float)((2 * u + u * u + g * (1 + u) * (1 + u) + g) * (1 + 1e-5));
  a.onepu = (float)((1 + u) * (1 + 1e-5));
  a.d_f = (float)d;
  a.hist = hist;
  a.tau_bits = tau_bits;
  // screening (t_screen > 0, low precision): threshold and filter on the
  // computed value, keep the t_screen largest, re-rank those in fp32
  const bool screen = prec != kF32 && cap_hint > 0;
  a.screen = screen ? 1 : 0;
  a.mg_max = 0.0f;
  // pass A over every stride-th row of A
  const int64_t stride = m >= 128 * 64 ? 64 : (m >= 128 * 8 ? 8 : 1);
  a.m_rows = (m + stride - 1) / stride;
  a.a_stride_rows = stride;
  a.m_key = stride;
  a.ckey = nullptr;
  a.ccap = 0;
  a.ccount = ccount;
  if (tau_user >= 0.0f) {
    // a threshold given by the caller (a lower bound it knows for the t-th
    // largest |c|): pass B keeps every pair that may reach it
    uint32_t tb;
    memcpy(&tb, &tau_user, 4);
    if ((e = launch_fill_u64((uint64_t*)tau_bits, 1, (uint64_t)tb, st)) !=
        hipSuccess)
      return e;
  } else {
    if (prec == kF32) launch_gemm<kF32>(a, true, st);
    else if (prec == kBF16) launch_gemm<kBF16>(a, true, st);
    else launch_gemm<kFP8>(a, true, st);
    // pass A's subset holds about 1/stride of the pairs
    const int64_t target =
        screen ? (cap_hint + stride - 1) / stride : t;
    k_bf_tau<<<1, 64, 0, st>>>(hist, target, tau_bits);
  }
  (void)hipEventRecord(ev[1], st);
  // the largest margin over all pairs, for pass B's pre-test
  {
    unsigned mxb[8];
    if ((e = hipMemcpyAsync(mxb, maxes, sizeof mxb, hipMemcpyDeviceToHost,
                            st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
      return e;
    float f[8];
    memcpy(f, mxb, sizeof f);
    const double mgm = screen ? 0.0
                              : (double)a.kappa * f[0] * f[4] +
                                    (double)a.onepu * (f[2] * f[5] + f[6] * f[1]) +
                                    (double)a.d_f * f[2] * f[6];
    a.mg_max = (float)(mgm * (1.0 + 1e-5));
  }
  // pass B over all pairs
  int64_t cap = screen ? 4 * cap_hint : (cap_hint > 0 ? cap_hint : (1 << 20));
  if (cap < 16 * t) cap = 16 * t;
  a.m_rows = m;
  a.a_stride_rows = 1;
  a.m_key = 1;
  unsigned long long count = 0;
  for (int attempt = 0; attempt < 4; ++attempt) {
    if ((e = dev_alloc(w.keys, (size_t)cap * 8)) != hipSuccess) break;
    if ((e = dev_alloc(w.vals, (size_t)cap * 4)) != hipSuccess) break;
    a.ckey = (uint64_t*)w.keys.p;
    a.cval = (float*)w.vals.p;
    a.ccap = cap;
    if ((e = launch_fill_u64((uint64_t*)ccount, 1, 0ull, st)) != hipSuccess)
      break;
    if (prec == kF32) launch_gemm<kF32>(a, false, st);
    else if (prec == kBF16) launch_gemm<kBF16>(a, false, st);
    else launch_gemm<kFP8>(a, false, st);
    if ((e = hipMemcpyAsync(&count, ccount, 8, hipMemcpyDeviceToHost, st)) !=
        hipSuccess) break;
    if ((e = hipStreamSynchronize(st)) != hipSuccess) break;
    if ((int64_t)count <= cap) break;
    if (count > (1ull << 28)) {  // the bound filters nothing useful
      e = hipErrorOutOfMemory;
      break;
    }
    cap = (int64_t)(count + count / 4 + 1024);  // rerun with room for all
  }
  (void)hipEventRecord(ev[2], st);
  int64_t nre = (int64_t)count;
  const uint64_t* rkeys = (const uint64_t*)w.keys.p;
  if (cand_keys) *cand_keys = rkeys;
  if (cand_count) *cand_count = nre;
  if (e == hipSuccess && screen && nre > cap_hint) {
    // the t_screen survivors with the largest computed |c|
    if ((e = dev_alloc(w.sel, (size_t)cap_hint * 8)) == hipSuccess)
      e = launch_select_keys_by_absval(rkeys, (const float*)w.vals.p, nre,
                                       cap_hint, w.selbuf,
                                       (uint64_t*)w.sel.p, st);
    rkeys = (const uint64_t*)w.sel.p;
    nre = cap_hint;
  }
  if (e == hipSuccess && out) {
    // final: fp32 re-rank and the exact top t of the re-ranked pairs
    e = launch_rerank_topk(rkeys, nre, A, B, n, d, t < nre ? t : nre, w.fin,
                           out, n_out, nullptr, st);
  }
  (void)hipEventRecord(ev[3], st);
  if (e == hipSuccess) e = hipEventSynchronize(ev[3]);
  if (e == hipSuccess && stats) {
    float f;
    (void)hipEventElapsedTime(&f, ev[0], ev[1]);
    stats->ms_screen = f;
    (void)hipEventElapsedTime(&f, ev[1], ev[2]);
    stats->ms_filter = f;
    (void)hipEventElapsedTime(&f, ev[2], ev[3]);
    stats->ms_rerank = f;
    stats->candidates = (int64_t)count;
    unsigned tb = 0;
    (void)hipMemcpy(&tb, tau_bits, 4, hipMemcpyDeviceToHost);
    float tf;
    memcpy(&tf, &tb, 4);
    stats->tau = tf;
    stats->row_stride = stride;
    stats->reranked = nre;
  }
  for (auto& x : ev) (void)hipEventDestroy(x);
  return e;
}

}  // namespace mad
