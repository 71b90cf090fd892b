// plan.hpp -- host-side plan and workspace structures of the library, and
// the launchers each kernel file exports.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

namespace mad {

// One family of equally sized alias tables (dense inputs): S tables of N
// items each, 2^L slots per table, entries at ent[s << L ...].
struct Family {
  int64_t S = 0;
  int64_t N = 0;
  int L = 0;
  uint64_t* ent = nullptr;  // S << L packed entries (device)
  double* tot = nullptr;    // S table totals (device)
};

struct DeviceBuffer {
  void* p = nullptr;
  size_t bytes = 0;
};

hipError_t dev_alloc(DeviceBuffer& b, size_t bytes);
void dev_free(DeviceBuffer& b);

// ---- tables.hip ----------------------------------------------------------
// Dense preprocessing: na (m), nb (d), v (d), om (d); families T0 (S=1,
// N=d), T1 (S=d, N=m), T2 (S=d, N=n), T3 (S=m, N=d); bmax = max |b|;
// bad != 0 when A or B holds NaN/Inf (only if check).
struct DenseTables {
  int64_t m = 0, n = 0, d = 0;
  Family T0, T1, T2, T3;
  double* na = nullptr;  // == T3.tot
  double* nb = nullptr;  // == T2.tot
  double* v = nullptr;   // == T1.tot
  double* om = nullptr;  // d
  float* bmax = nullptr; // 1
  int* bad = nullptr;    // 1 (block of 64 ints: bad[4] symmetry, bad[6]
                         // B binary)
  // binary inputs (Alg. 1): when every entry of B is 0 or 1 (bad[6] == 1),
  // bit j*d + k of bbits is b_jk and the sampler reads the fourth edge
  // from these n*d bits (an L2-sized array) instead of from B
  uint32_t* bbits = nullptr;
  int gram = 0;          // B = A, symmetrised scores (Sec. 3.2.2)
  int square = 0;        // B = A symmetric: x_kk' updated too (Sec. 3.2.3)
  // the B-side family T2 is built on a stream of its own, forked from and
  // joined back into the caller's stream
  hipStream_t side = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
  // T0 (of at most 512 slots) is built on `aux` as soon as the T1 and T2
  // totals exist (events t1tot, t2tot), beside the rest of T1 and T2; the
  // sampler's first order passes then run on `aux` too (order_done), once
  // the previous sampling launch is done with the order buffers (sampled).
  // t0_aux: the last build put T0 there.
  hipStream_t aux = nullptr;
  hipEvent_t t1tot = nullptr, t2tot = nullptr, t0done = nullptr;
  hipEvent_t order_done = nullptr, sampled = nullptr;
  int t0_aux = 0;
};

hipError_t dense_tables_alloc(DenseTables& t, int64_t m, int64_t n,
                              int64_t d);
void dense_tables_free(DenseTables& t);
hipError_t dense_tables_build(DenseTables& t, const float* A, const float* B,
                              bool check, DeviceBuffer& scratch,
                              hipStream_t st);
// *flag (device, 8-byte aligned) = 1 unless the m x m matrix A equals A^T
hipError_t launch_check_symmetric(const float* A, int64_t m, int* flag,
                                  hipStream_t st);

// MIPS: per-query stage-0 tables (S = nq tables over d coordinates, weight
// |q_k| v_k); scratch only when 2^ceil(log2 d) > 512
size_t query_tables_scratch_bytes(int64_t nq, int64_t d);
hipError_t query_tables_build(const float* Q, int64_t nq, int64_t d,
                              const double* v, Family& T0q, void* scratch,
                              size_t scratch_bytes, hipStream_t st);
hipError_t family_alloc_pub(Family& f, int64_t S, int64_t N);
void family_free_pub(Family& f);

// generic launchers reused by other files
hipError_t launch_fill_u64(uint64_t* p, int64_t n, uint64_t v, hipStream_t st);
constexpr int kFillMax = 4;
struct FillBatch {  // fill p[q][0 .. n[q]) with v[q], q < count
  uint64_t* p[kFillMax];
  int64_t n[kFillMax];
  uint64_t v[kFillMax];
  int count;
};
hipError_t launch_fill_multi(const FillBatch& f, hipStream_t st);

// ---- sampler.hip ---------------------------------------------------------
// The score table X.  Hash form: open addressing over `cap` slots (a power
// of two), EMPTY keys unused.  With `live` set only entries [0, *live) are
// read (EMPTY keys among them are unused).  With `pkeys` set the samplers
// write sample e's key at pkeys[e] (EMPTY for an open three-path) and its
// signed fourth edge at pvals[e] (increment rne(v 2^F)) instead of updating
// the table; X is then built by launch_accumulate.
struct HashTable {
  uint64_t* keys = nullptr;
  int64_t* vals = nullptr;
  int64_t cap = 0;
  const int64_t* live = nullptr;
  uint64_t* pkeys = nullptr;
  float* pvals = nullptr;
  // squared variant: sample e's second pair (key of (k, k')) at pkeys2[e]
  uint64_t* pkeys2 = nullptr;
  float* pvals2 = nullptr;
};

// sum of the increments rne(vals[e] 2^F) per key over n pairs (key EMPTY:
// skipped; F from *bmax and s_for_F as in the samplers, or F = s_for_F
// when bmax is null) into okey / oval:
// *o_len entries (one per non-EMPTY pair) holding the *o_count distinct
// keys and EMPTY elsewhere; work of accum_bytes(n) bytes; keys and vals are
// overwritten
size_t accum_bytes(int64_t n);
hipError_t launch_accumulate(uint64_t* keys, float* vals, int64_t n,
                             const float* bmax, int64_t s_for_F, void* work,
                             size_t work_bytes, uint64_t* okey, int64_t* oval,
                             int64_t* o_count, int64_t* o_len, hipStream_t st);
// the same when the pairs already come in G groups that no key spans
// (gstarts: device, G + 1 offsets): the groups are the first partition
// level, the hash partition of the other form is skipped
hipError_t launch_accumulate_grouped(uint64_t* keys, float* vals, int64_t n,
                                     const uint64_t* gstarts, int64_t G,
                                     const float* bmax, int64_t s_for_F,
                                     void* work, size_t work_bytes,
                                     uint64_t* okey, int64_t* oval,
                                     int64_t* o_count, int64_t* o_len,
                                     hipStream_t st);

struct SampleCounters {
  unsigned long long closed;    // closed three-paths (diamonds)
  unsigned long long distinct;  // keys inserted into X
  unsigned long long entries;   // pair form: entries of X written
  unsigned long long pad[5];
};

// Launch choices of the dense sampler (they never change a result):
// order 0 draws samples in index order, 1 in k order (samples counting-
// sorted by their stage-0 draw, in chunks of `chunk` samples, a power of
// two in [2^12, 2^28]), 2 in k order followed by the passes grouped by i
// and by j (the locality scheme of Sec. 5.2; pair form of X only).
struct SampleOptions {
  int order = 1;
  int64_t chunk = int64_t(1) << 28;
};
SampleOptions sample_options_default();
bool sample_options_valid(const SampleOptions& o);
// order_ws (order_bytes >= sample_order_bytes(t, count, o)) enables the
// ordered sampling launch; otherwise samples run in index order
size_t sample_order_bytes(const DenseTables& t, int64_t count,
                          const SampleOptions& o);
// Pairs left grouped by blocks of j (one chunk, not Gram): group g holds
// pairs [starts[g], starts[g+1]) of the pair arrays, starts (device) has
// G + 1 entries.  starts == nullptr when the pairs are not grouped.
struct PairGroups {
  const uint64_t* starts = nullptr;
  int64_t G = 0;
};
// main_start (optional) is recorded between the k-ordering passes and the
// sampling kernel(s); groups (optional) receives the grouping of the pairs
hipError_t launch_sample_dense(const DenseTables& t, const float* B,
                               uint64_t seed, uint64_t qid, int64_t l0,
                               int64_t count, int64_t s_for_F,
                               HashTable h, SampleCounters* ctr,
                               void* order_ws, size_t order_bytes,
                               const SampleOptions& o, PairGroups* groups,
                               hipEvent_t main_start, hipStream_t st);
hipError_t launch_sample_dense_debug(const DenseTables& t, const float* B,
                                     uint64_t seed, uint64_t qid, int64_t l0,
                                     int64_t count, int F, int32_t* k,
                                     int32_t* i, int32_t* j, int32_t* kp,
                                     int64_t* inc, hipStream_t st);

// ---- csr.hip -------------------------------------------------------------
// Alias entries of the sparse tables.  A 16-byte entry (T3) holds the
// packed word of a dense entry (threshold, alias position, two sign bits)
// and the item ids (vector or coordinate) of the slot's own item and of its
// alias.  A 32-byte entry (T1, T2) adds a payload per item that the sampler
// needs next and would otherwise load from another array: for T1 the meta
// word of T3[i] for its items i, for T2 the coordinate signature of b_j
// for its items j (see coord_bit in csr.hip).  Either sits in one cache
// line, so the payload costs no extra line per draw.
struct Ent16 {
  uint64_t w;
  uint32_t self;
  uint32_t alias;
};
struct Ent32 {
  uint64_t w;
  uint32_t self;
  uint32_t alias;
  uint64_t pself;
  uint64_t palias;
};

constexpr uint64_t kSlotMask = (1ull << 56) - 1;

// Tables of different sizes: table s covers item positions [off[s],
// off[s+1]) and 2^L_s slots from meta[s] & kSlotMask (L_s = meta[s] >> 56).
// Tables of more than 512 items ("big", 2^L >= 1024 slots) come first, in
// index order, then the others in index order.  The host plans the layout;
// device arrays are reused across rebuilds while they are large enough.
struct Ragged {
  int64_t S = 0;
  int64_t slots = 0, big_slots = 0, nbig = 0, runs = 0, edges = 0;
  int64_t cls_off[5] = {0, 0, 0, 0, 0};  // small tables by slots per lane
  const int64_t* off = nullptr;  // S + 1 (device)
  uint64_t* meta = nullptr;      // S (device)
  void* ent = nullptr;           // slots (device): Ent32 or Ent16
  int esz = 16;                  // bytes per entry (32: with payloads)
  double* tot = nullptr;         // S table totals (device)
  void* big = nullptr;           // per big table layout (device)
  uint32_t* btab = nullptr;      // big table of each 1024-slot block
  uint32_t* runtab = nullptr;    // big table of each 1024-item run
  uint32_t* small_ids = nullptr; // small tables grouped by class
  DeviceBuffer lay, ent_buf, tot_buf;
};

// sparse inputs as compressed rows of the vector-major arrays
struct CsrView {
  const int64_t* a_ptr;
  const int32_t* a_idx;
  const float* a_val;
  const int64_t* b_ptr;
  const int32_t* b_idx;
  const float* b_val;
};

// Sparse plan tables: T0 over coordinates (dense family), T1[k] over the
// vectors i with an entry at k (weight |a_ki| na_i), T2[k] over the j with
// an entry at k (weight |b_kj|), T3[i] over the coordinates of a_i (weight
// |a_k'i|).  The transposes list, per coordinate, its vectors in ascending
// order with their values.
// one slot of the table of B's stored entries (CsrTables::bh)
struct BSlot {
  uint64_t key;  // j d + k + 1 of entry b_jk; 0: empty
  float val;     // b_jk
  uint32_t e;    // the entry's position in B's compressed arrays
};

struct CsrTables {
  int64_t m = 0, n = 0, d = 0, nnzA = 0, nnzB = 0;
  CsrView in{};
  int64_t* at_ptr = nullptr;  // d + 1
  uint32_t* at_row = nullptr; // nnzA
  float* at_val = nullptr;    // nnzA
  int64_t* bt_ptr = nullptr;
  uint32_t* bt_row = nullptr;
  float* bt_val = nullptr;
  Ragged T1, T2, T3;
  Family T0;
  double* om = nullptr;   // d
  float* bmax = nullptr;  // 1
  int* bad = nullptr;     // 1: non-finite value, 2: malformed structure
  // the T1 payloads by transpose position: at_pay[p] = T3 meta of
  // at_row[p] (structure only)
  uint64_t* at_pay = nullptr;
  // the T2 payloads by transpose position: bt_pay[p] = bsig[bt_row[p]],
  // bsig[j] the OR of coord_bit(k) over b_j's coordinates (structure only)
  uint64_t* bsig = nullptr;   // n
  uint64_t* bt_pay = nullptr; // nnzB
  // B's stored entries in an open-addressing table of 16-byte slots keyed
  // by j d + k + 1, at most half full: the fourth edge b_jk' is one probe
  // of about one line instead of a search of b_j's coordinates and a load
  // of its value (and no probe when b_j's signature rules k' out).  The
  // keys and entry positions are structure; every build gathers the
  // values.
  BSlot* bh = nullptr;
  uint64_t bh_mask = 0;
  DeviceBuffer work;      // transposes' and tables' scratch
  int gram = 0;           // B = A, symmetrised scores (Sec. 3.2.2)
  int square = 0;         // B = A symmetric: x_kk' updated too (Sec. 3.2.3)
  bool validated = false; // the structure passed a check on this plan
  // the transposes' structure (pointers, rows, and the source position of
  // each entry) and the table layouts depend only on the sparsity
  // structure: built once, reused by unchecked refreshes, which regather
  // the values only
  bool structured = false;
  uint32_t* at_src = nullptr; // nnzA
  uint32_t* bt_src = nullptr; // nnzB
  double* at_w = nullptr;     // nnzA: T1 weights |a_ki| na_i of this build
};

// Allocates and builds every table (synchronises: the layout of the
// sparse tables is planned on the host).  Returns hipErrorInvalidValue when
// the inputs are malformed or hold NaN/Inf, with t.bad set.
hipError_t csr_tables_build(CsrTables& t, bool check, hipStream_t st);
// structure and finiteness of sparse inputs (flag: device, 8-byte aligned
// scratch); hipErrorInvalidValue when malformed or non-finite.  Synchronises.
hipError_t csr_validate(const CsrView& in, int64_t m, int64_t n, int64_t d,
                        int64_t nnzA, int64_t nnzB, int* flag,
                        hipStream_t st);
// *flag (device, 8-byte aligned) = 1 unless A's compressed rows equal its
// transpose (A == A^T); after csr_tables_build
hipError_t launch_check_csr_symmetric(const CsrTables& t, int* flag,
                                      hipStream_t st);
void csr_tables_free(CsrTables& t);
hipError_t launch_sample_csr(const CsrTables& t, uint64_t seed, uint64_t qid,
                             int64_t l0, int64_t count, int64_t s_for_F,
                             HashTable h, SampleCounters* ctr, hipStream_t st);
hipError_t launch_sample_csr_debug(const CsrTables& t, uint64_t seed,
                                   uint64_t qid, int64_t l0, int64_t count,
                                   int F, int32_t* k, int32_t* i, int32_t* j,
                                   int32_t* kp, int64_t* inc, hipStream_t st);
// stage-0 table over explicit weights (any size); scratch for 2^L > 512
size_t stage0_scratch_bytes(int64_t N);
hipError_t stage0_table_build(const double* w, int64_t N, Family& T,
                              void* scratch, size_t scratch_bytes,
                              hipStream_t st);

// ---- mips.hip ------------------------------------------------------------
// Per-query state of a MIPS batch.  The host fills everything but F and
// live; k_mips_query_info fills those from the query vector.
struct MipsQuery {
  int64_t s;       // sample budget s_q
  int64_t tp;      // candidate budget t'_q (>= t)
  int64_t hoff;    // first slot of the query's score table
  int64_t coff;    // first entry of its candidate list (capacity ccap)
  int64_t ccap;    // min(s_q, m) (>= 1)
  int64_t soff;    // first entry of its verified list (capacity scap)
  int64_t scap;    // min(ccap, t'_q)
  uint32_t hmask;  // table capacity - 1 (a power of two minus one)
  int F;           // fixed-point exponent (device)
  int live;        // 1: finite query (device)
  int pad;
};

// a contiguous range of one query's samples
struct MipsChunk {
  int32_t q;
  int32_t count;
  int64_t l0;
};

// per-query results of the postprocessing (device)
struct MipsQueryStats {
  int64_t n_pos;   // |Omega_s|: keys with x > 0
  int64_t n_cand;  // verified candidates
  int64_t n_fp32;  // candidates verified in fp32 (n_cand without screening)
  int64_t pad;
};

struct VecInfo;

struct MipsArgs {
  // database tables (A side of a dense plan) and the query stage-0 tables
  const uint64_t* T0q;
  const double* t0tot;
  const uint64_t* T1;
  const uint64_t* T3;
  int L0, L1, L3;
  const float* A;   // database, m x d
  const float* Q;   // queries, nq x d
  int64_t m, d, nq, t;
  uint64_t seed;
  const MipsQuery* qi;
  const int32_t* order;  // queries by descending budget
  const MipsChunk* chunks;
  int64_t nchunks;
  // score slots of the queries' tables: key i + 1 in the low kb bits, the
  // score x (fixed point) in the high 64 - kb bits; 0 is an empty slot
  uint64_t* hslot;
  int kb;
  uint64_t* cx;  // candidate scores
  uint32_t* ck;  // candidate keys (i)
  uint64_t* sx;  // verified: scores
  uint32_t* sk;  //           keys
  float* sc;     //           c
  uint64_t* sab; //           |c| bits
  SampleCounters* ctr;
  MipsQueryStats* qstats;
  void* out;       // nq x t mad_pair
  int64_t* n_out;  // nq
  // low-precision screening of the candidates (lp = 1 bf16, 2 fp8; 0 none):
  // rows of Kp elements of the database and of the queries, their VecInfo,
  // and the constants of the error bound
  int lp = 0;
  const void* Alp = nullptr;
  const VecInfo* ia = nullptr;
  const void* Qlp = nullptr;
  const VecInfo* iq = nullptr;
  int64_t Kp = 0;
  float kappa = 0.0f, onepu = 0.0f, d_f = 0.0f;
};

hipError_t launch_mips_query_info(const float* Q, int64_t nq, int64_t d,
                                  int kb, MipsQuery* qi, hipStream_t st);
hipError_t launch_sample_mips(const MipsArgs& a, int unroll, int grid,
                              hipStream_t st);
hipError_t launch_mips_post(const MipsArgs& a, hipStream_t st);
hipError_t launch_mips_dump(const MipsArgs& a, int64_t q, int64_t* keys,
                            int64_t* xfix, int64_t cap, int64_t* count,
                            hipStream_t st);
size_t mips_sample_lds_bytes(int L0, int64_t d);

// ---- select.hip ----------------------------------------------------------
struct SelectWork {
  uint64_t* x = nullptr;     // candidate primary keys
  uint64_t* key = nullptr;   // candidate secondary keys
  uint64_t* x2 = nullptr;    // selected primary
  uint64_t* key2 = nullptr;  // selected secondary
  float* c = nullptr;        // verified dot products
  int64_t cap = 0;           // capacity of x / key
  int64_t cap2 = 0;          // capacity of x2 / key2 / c
  void* state = nullptr;     // device select state
  unsigned int* hist = nullptr;
  int64_t* counts = nullptr; // device counters
  uint64_t* part = nullptr;  // per-block and / or slots of the two splits
  uint64_t* rx = nullptr;    // refined boundary list of candidate selection (x, key)
  uint64_t* rkey = nullptr;
  int64_t rcap = 0;          // its capacity
};

// SelectWork::counts slots
enum { kCountPos = 0, kCountDistinct = 1, kCountCand = 2, kCountFinal = 3 };
constexpr size_t kSelStateBytes = 512;
// and / or slots of the selection's two block splits: 4 words for each of
// at most kPartBlocks blocks per split
constexpr int kPartBlocks = 1024;
constexpr size_t kPartBytes = 2 * 4 * sizeof(uint64_t) * (size_t)kPartBlocks;
constexpr int kSelBins = 2048;

hipError_t launch_dump_scores(const HashTable& h, int64_t* keys,
                              int64_t* xfix, int64_t out_cap, int64_t* count,
                              hipStream_t st);

// Per-vector data of a low-precision copy: norms of the fp32 vector, the
// absolute rounding floor of one element and the inverse of the
// power-of-two scale applied before rounding.
struct VecInfo {
  float n2;     // ||x||_2, rounded up
  float n1;     // ||x||_1, rounded up
  float eta;    // absolute rounding floor of one element
  float inv_s;  // 1 / scale applied before rounding
};

// fp32 sum, added to acc, of the products of 16 bytes of two low-precision
// rows: 8 bf16 values (prec 1) or 16 fp8-e4m3 values (prec 2) each
__device__ __forceinline__ float lowp_dot16(const uint4 x, const uint4 y,
                                            int prec, float acc) {
  const uint32_t xa[4] = {x.x, x.y, x.z, x.w};
  const uint32_t ya[4] = {y.x, y.y, y.z, y.w};
  if (prec == 1) {  // bf16: 8 per load
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      acc = fmaf(__uint_as_float(xa[q] << 16), __uint_as_float(ya[q] << 16),
                 acc);
      acc = fmaf(__uint_as_float(xa[q] & 0xFFFF0000u),
                 __uint_as_float(ya[q] & 0xFFFF0000u), acc);
    }
  } else {  // fp8 e4m3: 16 per load
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      acc = fmaf(__builtin_amdgcn_cvt_f32_fp8((int)xa[q], 0),
                 __builtin_amdgcn_cvt_f32_fp8((int)ya[q], 0), acc);
      acc = fmaf(__builtin_amdgcn_cvt_f32_fp8((int)xa[q], 1),
                 __builtin_amdgcn_cvt_f32_fp8((int)ya[q], 1), acc);
      acc = fmaf(__builtin_amdgcn_cvt_f32_fp8((int)xa[q], 2),
                 __builtin_amdgcn_cvt_f32_fp8((int)ya[q], 2), acc);
      acc = fmaf(__builtin_amdgcn_cvt_f32_fp8((int)xa[q], 3),
                 __builtin_amdgcn_cvt_f32_fp8((int)ya[q], 3), acc);
    }
  }
  return acc;
}


// low-precision copies of A and B (rows of Kp elements) for the
// verification filter, with the margin constants of their error bound
struct LowpView {
  const void* A;
  const void* B;
  const VecInfo* ia;
  const VecInfo* ib;
  int64_t Kp;
  int prec;      // MAD_BF16 or MAD_FP8_E4M3
  float kappa;   // relative margin factor on ||a||_2 ||b||_2
  float onepu;   // 1 + u (absolute-floor terms)
  float d_f;     // d
};

// bruteforce.hip: the padded low-precision copy of X and its VecInfo
hipError_t lowp_prepare(const float* X, int64_t rows, int64_t d, int prec,
                        DeviceBuffer& data, DeviceBuffer& info, int64_t* Kp,
                        hipStream_t st);
void lowp_consts(int prec, int64_t d, float* kappa, float* onepu);
// c^ and its a-priori margin for given pair keys (select.hip)
hipError_t launch_lowp_screen_values(const uint64_t* keys, int64_t count,
                                     const LowpView& v, int64_t n,
                                     float* chat, float* margin,
                                     hipStream_t st);

// csr: sparse inputs for the verification (A, B unused), or null; lowp:
// low-precision filter of the candidates before the fp32 verification, or
// null
// x_shift: reported x = x_fix * 2^-(F + x_shift) (1 for symmetrised
// scores, which hold x_ij + x_ji)
// cleared: the caller has already run the fills of post_fills
void post_fills(SelectWork& w, FillBatch& f);
hipError_t launch_postprocess(const HashTable& h, const float* A,
                              const float* B, const CsrView* csr,
                              const LowpView* lowp, int64_t n, int64_t d,
                              int64_t t_prime, int64_t t, const float* bmax,
                              int64_t s, int x_shift, SelectWork& w,
                              void* out, int64_t* n_out, bool cleared,
                              hipStream_t st);

// fp32 re-rank of candidate keys (count known on the host) and the exact
// top t by |c| into mad_pair records; buf is grown as needed
// (csr: sparse inputs, the dot products then come from their compressed
// rows and A, B, d are unused)
hipError_t launch_rerank_topk(const uint64_t* keys, int64_t count,
                              const float* A, const float* B, int64_t n,
                              int64_t d, int64_t t, DeviceBuffer& buf,
                              void* out, int64_t* n_out, const CsrView* csr,
                              hipStream_t st);

// the k keys with the largest |v| (ties by key ascending) into out_keys
// (device, capacity k), unordered; count known on the host
hipError_t launch_select_keys_by_absval(const uint64_t* keys, const float* v,
                                        int64_t count, int64_t k,
                                        DeviceBuffer& buf, uint64_t* out_keys,
                                        hipStream_t st);

// ---- bruteforce.hip ------------------------------------------------------
struct BfStats {
  double ms_screen;   // conversion + pass A (threshold)
  double ms_filter;   // pass B (all pairs)
  double ms_rerank;   // fp32 re-rank and selection
  int64_t candidates; // pairs that passed the bound
  float tau;          // threshold of pass B
  int64_t row_stride; // rows of A used by pass A: every row_stride-th
  int64_t reranked;   // pairs re-ranked in fp32
};

hipError_t bruteforce_topk(const float* A, int64_t m, const float* B,
                           int64_t n, int64_t d, int prec, int64_t t,
                           int64_t cap_hint, void* out, int64_t* n_out,
                           BfStats* stats, hipStream_t st);
// the same with the pass-B threshold given (tau_user >= 0, pass A skipped)
// and the survivors of pass B returned (device keys i*n + j in a
// process-wide buffer valid until the next call, and their count); out may
// be null to skip the final selection
hipError_t bruteforce_run(const float* A, int64_t m, const float* B,
                          int64_t n, int64_t d, int prec, int64_t t,
                          int64_t cap_hint, float tau_user, void* out,
                          int64_t* n_out, const uint64_t** cand_keys,
                          int64_t* cand_count, BfStats* stats,
                          hipStream_t st);

// ---- exact_csr.hip ----------------------------------------------------
// exhaustive t-MAD of sparse inputs: the coordinates with the most wedges
// through the brute force (dense copies of their columns), the others'
// wedges listed and summed per pair; exact top t of the union of both
// parts' candidates (sparse dot products).  heavy_req > 0 fixes the number
// of heavy coordinates.  hipErrorNotSupported when more than 4096 heavy
// coordinates or 2^30 light wedges would be needed.  Synchronises.
struct BfCsrStats {
  double ms_split, ms_heavy, ms_light, ms_final;
  int64_t heavy, wedges, light_wedges;
  int64_t heavy_candidates, light_candidates, candidates;
  float tau;
};
hipError_t bruteforce_topk_csr(const CsrView& in, int64_t m, int64_t n,
                               int64_t d, int64_t nnzA, int64_t nnzB,
                               int prec, int64_t t, int64_t heavy_req,
                               void* out, int64_t* n_out, BfCsrStats* stats,
                               hipStream_t st);

}  // namespace mad
