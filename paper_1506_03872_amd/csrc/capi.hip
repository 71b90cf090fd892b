// capi.hip -- the C ABI (include/mad.h): argument checks, plan lifetime,
// workspace management and the launch sequence of Alg. 3 with Alg. 2.
#include <stdarg.h>
#include <stdlib.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/mad.h"
#include "mad_common.hpp"
#include "plan.hpp"

namespace {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  if (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation)
    return fail(MAD_ENOMEM, "%s: out of device memory", what);
  return fail(MAD_EHIP, "%s: %s", what, hipGetErrorString(e));
}

#define HIP_TRY(expr, what)                    \
  do {                                         \
    hipError_t e_ = (expr);                    \
    if (e_ != hipSuccess) return hip_fail(e_, what); \
  } while (0)

bool is_device_ptr(const void* p) {
  if (!p) return false;
  hipPointerAttribute_t at;
  if (hipPointerGetAttributes(&at, p) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  return at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeManaged;
}

int64_t next_pow2(int64_t v) {
  int64_t p = 1;
  while (p < v) p <<= 1;
  return p;
}

}  // namespace

// MIPS batch state: per-query layout, workspace, the captured launch graph
// and the tuned launch shape
struct MipsState {
  mad::Family T0q;  // stage-0 table per query (capacity nq_cap tables)
  int64_t nq_cap = 0;
  mad::DeviceBuffer qscratch, qinfo, order, chunks, hash, cx, ck, sx,
      sk, sc, sab, qstats, ctr;
  // layout of the prepared batch
  std::vector<int64_t> s, tp;
  int64_t nq = -1, t = -1;
  int64_t hslots = 0, nchunks = 0;
  int chunk_prepared = -1, slots_prepared = -1;
  // launch shape and score-table slots per possible key (result-invariant)
  int chunk = 4096, unroll = 4, grid = 2048, slots = 2;
  // file of the autotuner's choices ("" = none)
  std::string tune_cache;
  // captured graph and what it was captured for
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  const float* g_Q = nullptr;
  const void* g_out = nullptr;
  const void* g_nout = nullptr;
  uint64_t g_seed = 0;
  int g_chunk = -1, g_unroll = -1, g_grid = -1;
  int64_t g_layout = -1;
  // low-precision copies of the batch's queries (screened verification)
  mad::DeviceBuffer qlp, qlpi;
  int g_prec = -1;
  const void* g_qlp = nullptr;
  int64_t layout_version = 0;
  bool ran = false;
};

struct mad_plan {
  int kind = 0;  // 0 dense MAD, 1 MIPS database, 2 sparse (CSR) MAD
  const float* A = nullptr;
  const float* B = nullptr;
  int64_t m = 0, n = 0, d = 0;
  uint32_t flags = 0;
  mad::DenseTables dt;
  mad::CsrTables ct;
  mad::DeviceBuffer build;
  // low-precision copies for the verification filter (dense plans)
  int verify_prec = MAD_FP32;
  mad::DeviceBuffer lpA, lpB, lpIA, lpIB;
  mad::LowpView lv{};
  // workspace of mad_plan_topk
  mad::DeviceBuffer hk, hv, cx, ck, cx2, ck2, cc, cr, misc, ord, acc;
  mad::HashTable h;
  bool pairs = false;  // X built from per-sample pairs (else a hash table)
  // launch choices (result-invariant): how X is built and the sampler's
  // ordering; defaults from the environment, changed by mad_plan_set_option
  int opt_accum = -1;  // MAD_ACCUM_PAIRS or MAD_ACCUM_HASH (-1: default)
  mad::SampleOptions sopt;
  mad::HashTable h_run;  // X as the last run left it
  mad::SelectWork w;
  mad::SampleCounters* ctr = nullptr;
  int64_t ws_s = -1, ws_tp = -1, ws_t = -1;
  // last run
  int64_t last_s = -1;
  bool ran = false;
  // phase events (MAD_FLAG_TIMING): 0 tables start, 1 tables end, 2 clear
  // start, 3 sampling start, 7 sampling kernel start (after the k-order
  // passes), 4 sampling end, 6 score accumulation end, 5 postprocessing end
  hipEvent_t ev[8] = {nullptr, nullptr, nullptr, nullptr,
                      nullptr, nullptr, nullptr, nullptr};
  bool timed_tables = false, timed_topk = false;
  MipsState* mips = nullptr;
};

static void mips_free(MipsState* ms) {
  if (!ms) return;
  if (ms->exec) (void)hipGraphExecDestroy(ms->exec);
  if (ms->graph) (void)hipGraphDestroy(ms->graph);
  if (ms->cap_stream) (void)hipStreamDestroy(ms->cap_stream);
  mad::family_free_pub(ms->T0q);
  mad::DeviceBuffer* bufs[] = {&ms->qscratch, &ms->qinfo, &ms->order,
                               &ms->chunks, &ms->hash, &ms->cx,
                               &ms->ck, &ms->sx, &ms->sk, &ms->sc, &ms->sab,
                               &ms->qstats, &ms->ctr, &ms->qlp, &ms->qlpi};
  for (mad::DeviceBuffer* b : bufs) mad::dev_free(*b);
  delete ms;
}

static void record(mad_plan* p, int idx, hipStream_t st) {
  if (p->ev[idx]) (void)hipEventRecord(p->ev[idx], st);
}

// per-kind accessors: stage-0 totals (||W||_1), max |b|
static const double* plan_wtot(const mad_plan* p) {
  return p->kind == 2 ? p->ct.T0.tot : p->dt.T0.tot;
}

static const float* plan_bmax(const mad_plan* p) {
  return p->kind == 2 ? p->ct.bmax : p->dt.bmax;
}

static void plan_free_all(mad_plan* p) {
  mips_free(p->mips);
  p->mips = nullptr;
  mad::dense_tables_free(p->dt);
  mad::csr_tables_free(p->ct);
  mad::dev_free(p->build);
  mad::dev_free(p->hk);
  mad::dev_free(p->hv);
  mad::dev_free(p->cx);
  mad::dev_free(p->ck);
  mad::dev_free(p->cx2);
  mad::dev_free(p->ck2);
  mad::dev_free(p->cc);
  mad::dev_free(p->cr);
  mad::dev_free(p->misc);
  mad::dev_free(p->ord);
  mad::dev_free(p->acc);
  mad::dev_free(p->lpA);
  mad::dev_free(p->lpB);
  mad::dev_free(p->lpIA);
  mad::dev_free(p->lpIB);
  for (hipEvent_t& e : p->ev)
    if (e) {
      (void)hipEventDestroy(e);
      e = nullptr;
    }
}

static int check_bad_inputs(mad_plan* p, hipStream_t st) {
  if (p->flags & MAD_FLAG_NO_CHECK) return MAD_OK;
  int bad = 0;
  HIP_TRY(hipMemcpyAsync(&bad, p->dt.bad, sizeof(int), hipMemcpyDeviceToHost,
                         st), "reading the input check");
  HIP_TRY(hipStreamSynchronize(st), "input check");
  if (bad) return fail(MAD_EINVAL, "A or B holds NaN or Inf");
  return MAD_OK;
}

namespace {

// what a tuned choice depends on: the device, the database shape and the
// batch's budgets (their count, sum and largest), t and the verification
// precision
std::string tune_signature(mad_plan* p, int64_t nq, const int64_t* s,
                           const int64_t* tp, int64_t t) {
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return std::string();
  long long ssum = 0, smax = 0, tsum = 0;
  for (int64_t q = 0; q < nq; ++q) {
    ssum += s[q];
    smax = s[q] > smax ? s[q] : smax;
    tsum += tp[q];
  }
  char buf[512];
  snprintf(buf, sizeof buf,
           "%s m=%lld d=%lld nq=%lld s_sum=%lld s_max=%lld tp_sum=%lld "
           "t=%lld prec=%d",
           prop.gcnArchName, (long long)p->m, (long long)p->d, (long long)nq,
           ssum, smax, tsum, (long long)t, p->verify_prec);
  for (char* c = buf; *c; ++c)
    if (*c == '|' || *c == '\n') *c = '_';
  return std::string(buf);
}

struct TuneChoice {
  int chunk, unroll, grid, slots;
  double ms;
};

// the last line of the file for this signature: "<signature> | chunk
// unroll grid slots ms"; lines that do not parse are skipped
bool tune_lookup(const std::string& path, const std::string& sig,
                 TuneChoice* c) {
  FILE* f = fopen(path.c_str(), "r");
  if (!f) return false;
  char line[1024];
  bool found = false;
  while (fgets(line, sizeof line, f)) {
    char* bar = strstr(line, " | ");
    if (!bar) continue;
    if ((size_t)(bar - line) != sig.size() ||
        strncmp(line, sig.c_str(), sig.size()) != 0)
      continue;
    TuneChoice x;
    if (sscanf(bar + 3, "%d %d %d %d %lf", &x.chunk, &x.unroll, &x.grid,
               &x.slots, &x.ms) == 5) {
      *c = x;
      found = true;
    }
  }
  fclose(f);
  return found;
}

bool tune_append(const std::string& path, const std::string& sig,
                 const TuneChoice& c) {
  FILE* f = fopen(path.c_str(), "a");
  if (!f) return false;
  const int n = fprintf(f, "%s | %d %d %d %d %.4f\n", sig.c_str(), c.chunk,
                        c.unroll, c.grid, c.slots, c.ms);
  return fclose(f) == 0 && n > 0;
}

}  // namespace

extern "C" {

const char* mad_last_error(void) { return g_err.c_str(); }

int mad_plan_create_dense(const float* A, int64_t m, const float* B,
                          int64_t n, int64_t d, uint32_t flags, void* stream,
                          mad_plan** plan) {
  g_err.clear();
  if (!plan) return fail(MAD_EINVAL, "plan is NULL");
  *plan = nullptr;
  if (m < 1 || n < 1 || d < 1)
    return fail(MAD_EINVAL, "need m, n, d >= 1 (got %lld, %lld, %lld)",
                (long long)m, (long long)n, (long long)d);
  if (m >= (int64_t(1) << 31) || n >= (int64_t(1) << 31) ||
      d >= (int64_t(1) << 31))
    return fail(MAD_EINVAL, "m, n and d must be below 2^31");
  if (!is_device_ptr(A) || !is_device_ptr(B))
    return fail(MAD_EINVAL, "A and B must be device pointers");
  if ((flags & MAD_FLAG_GRAM) && (A != B || m != n))
    return fail(MAD_EINVAL, "MAD_FLAG_GRAM needs B == A (same pointer, n == m)");
  if ((flags & MAD_FLAG_SQUARE) && (A != B || m != n || m != d))
    return fail(MAD_EINVAL, "MAD_FLAG_SQUARE needs B == A (same pointer) and "
                "m == n == d");
  mad_plan* p = new (std::nothrow) mad_plan();
  if (!p) return fail(MAD_ENOMEM, "host allocation failed");
  p->kind = 0;
  p->A = A;
  p->B = B;
  p->m = m;
  p->n = n;
  p->d = d;
  p->flags = flags;
  p->sopt = mad::sample_options_default();
  hipError_t e = mad::dense_tables_alloc(p->dt, m, n, d);
  p->dt.square = (flags & MAD_FLAG_SQUARE) ? 1 : 0;
  p->dt.gram = ((flags & MAD_FLAG_GRAM) || p->dt.square) ? 1 : 0;
  if (e == hipSuccess && (flags & MAD_FLAG_TIMING))
    for (hipEvent_t& ev : p->ev)
      if ((e = hipEventCreate(&ev)) != hipSuccess) break;
  if (e != hipSuccess) {
    plan_free_all(p);
    delete p;
    return hip_fail(e, "allocating tables");
  }
  int rc = mad_plan_refresh(p, stream);
  if (rc != MAD_OK) {
    std::string keep = g_err;
    (void)hipDeviceSynchronize();
    plan_free_all(p);
    delete p;
    g_err = keep;
    return rc;
  }
  *plan = p;
  return MAD_OK;
}

int mad_plan_refresh(mad_plan* p, void* stream) {
  if (!p) return fail(MAD_EINVAL, "plan is NULL");
  hipStream_t st = (hipStream_t)stream;
  const bool check = !(p->flags & MAD_FLAG_NO_CHECK);
  record(p, 0, st);
  if (p->kind == 2) {
    hipError_t e = mad::csr_tables_build(p->ct, check, st);
    if (e == hipErrorInvalidValue) {
      int bad = 0;
      (void)hipMemcpy(&bad, p->ct.bad, sizeof bad, hipMemcpyDeviceToHost);
      if (bad & 2)
        return fail(MAD_EINVAL, "malformed CSR input (pointers not "
                    "non-decreasing, or coordinates not strictly increasing "
                    "within a vector and in [0, d))");
      return fail(MAD_EINVAL, "A or B holds NaN or Inf");
    }
    if (e != hipSuccess) return hip_fail(e, "building sparse tables");
    if (p->ct.square && check) {
      int sym = 0;
      HIP_TRY(mad::launch_check_csr_symmetric(p->ct, p->ct.bad + 4, st),
              "symmetry check");
      HIP_TRY(hipMemcpyAsync(&sym, p->ct.bad + 4, sizeof sym,
                             hipMemcpyDeviceToHost, st), "symmetry check");
      HIP_TRY(hipStreamSynchronize(st), "symmetry check");
      if (sym)
        return fail(MAD_EINVAL, "MAD_FLAG_SQUARE needs a symmetric A");
    }
    record(p, 1, st);
    p->timed_tables = p->ev[0] != nullptr;
    p->ran = false;
    return MAD_OK;
  }
  HIP_TRY(mad::dense_tables_build(p->dt, p->A, p->B, check, p->build, st),
          "building tables");
  if (p->verify_prec != MAD_FP32) {
    int64_t kp = 0;
    HIP_TRY(mad::lowp_prepare(p->A, p->m, p->d, p->verify_prec, p->lpA,
                              p->lpIA, &kp, st), "low-precision copies");
    if (p->B)
      HIP_TRY(mad::lowp_prepare(p->B, p->n, p->d, p->verify_prec, p->lpB,
                                p->lpIB, &kp, st), "low-precision copies");
  }
  record(p, 1, st);
  p->timed_tables = p->ev[0] != nullptr;
  p->ran = false;
  if (p->dt.square && check)
    HIP_TRY(mad::launch_check_symmetric(p->A, p->m, p->dt.bad + 4, st),
            "symmetry check");
  int rc = check_bad_inputs(p, st);
  if (rc != MAD_OK || !p->dt.square || !check) return rc;
  int sym = 0;
  HIP_TRY(hipMemcpy(&sym, p->dt.bad + 4, sizeof sym, hipMemcpyDeviceToHost),
          "symmetry check");
  if (sym) return fail(MAD_EINVAL, "MAD_FLAG_SQUARE needs a symmetric A");
  return MAD_OK;
}

void mad_plan_destroy(mad_plan* p) {
  if (!p) return;
  (void)hipDeviceSynchronize();
  plan_free_all(p);
  delete p;
}

// How X is built (result-invariant): from per-sample pairs by partitioned
// accumulation (default), or in an open-addressing hash table updated by the
// sampler with atomics (process default MAD_ACCUM=hash; per plan through
// mad_plan_set_option).
static int accum_default() {
  static const int v = [] {
    const char* e = getenv("MAD_ACCUM");
    return (e && strcmp(e, "hash") == 0) ? MAD_ACCUM_HASH : MAD_ACCUM_PAIRS;
  }();
  return v;
}

static bool plan_square(const mad_plan* p) {
  return p->kind == 2 ? p->ct.square != 0 : p->dt.square != 0;
}

// samples in s' updates of X: two per sample for the squared variant
static int64_t plan_updates(const mad_plan* p, int64_t s) {
  return plan_square(p) ? 2 * s : s;
}

static bool accum_pairs(const mad_plan* p) {
  if (plan_square(p)) return true;  // two pairs per sample: pair form only
  const int a = p->opt_accum < 0 ? accum_default() : p->opt_accum;
  return a == MAD_ACCUM_PAIRS;
}

// per-sample pairs: 8-byte keys, then 4-byte values (16-byte aligned end)
static size_t pair_bytes(int64_t s) {
  const size_t n = (size_t)(s > 1 ? s : 1);
  return 8 * n + (4 * n + 15) / 16 * 16;
}

static int ensure_workspace(mad_plan* p, int64_t s, int64_t tp, int64_t t) {
  if (s <= p->ws_s && tp <= p->ws_tp && t <= p->ws_t) return MAD_OK;
  const int64_t s2 = s > p->ws_s ? s : p->ws_s;
  const int64_t u2 = plan_updates(p, s2);  // updates of X (pairs)
  const int64_t tp2 = tp > p->ws_tp ? tp : p->ws_tp;
  const int64_t t2 = t > p->ws_t ? t : p->ws_t;
  const double mn = (double)p->m * (double)p->n;
  const int64_t pairs = (double)u2 < mn ? u2 : (int64_t)mn;
  const bool use_pairs = accum_pairs(p);
  // pair form: X is a table of s entries (each bin of pairs leaves its
  // distinct keys in its own range); hash form: a table of twice min(s, mn)
  // slots, rounded up to a power of two
  const int64_t hcap = use_pairs ? (u2 > 1 ? u2 : 1)
                                 : next_pow2(2 * (pairs > 512 ? pairs : 512));
  // candidates / boundary lists: candidate selection needs |Omega_s| <= pairs entries,
  // final selection needs 4 t (final set) + 4 t' (boundary of the candidates)
  int64_t ccap = pairs > 1 ? pairs : 1;
  if (ccap < 4 * t2 + 4 * tp2) ccap = 4 * t2 + 4 * tp2;
  const int64_t ccap2 = tp2 > 1 ? tp2 : 1;
  // candidate selection's refined boundary list (one digit's bin of a long boundary list)
  const int64_t rcap = ccap < (int64_t(1) << 21) ? ccap : (int64_t(1) << 21);
  // pair form: the pairs and the accumulation's partition are dead once X
  // is built, so the candidate selection's boundary lists (x, key) reuse
  // that region when it is large enough (16 bytes per sample less)
  const size_t acc_bytes = use_pairs ? pair_bytes(u2) + mad::accum_bytes(u2)
                                     : 0;
  const bool c_in_acc = use_pairs && 16 * (size_t)ccap <= acc_bytes;
  (void)hipDeviceSynchronize();
  if (c_in_acc) {
    mad::dev_free(p->cx);
    mad::dev_free(p->ck);
  }
  hipError_t e;
  if ((e = mad::dev_alloc(p->hk, 8 * (size_t)hcap)) != hipSuccess ||
      (e = mad::dev_alloc(p->hv, 8 * (size_t)hcap)) != hipSuccess ||
      (!c_in_acc &&
       (e = mad::dev_alloc(p->cx, 8 * (size_t)ccap)) != hipSuccess) ||
      (!c_in_acc &&
       (e = mad::dev_alloc(p->ck, 8 * (size_t)ccap)) != hipSuccess) ||
      (e = mad::dev_alloc(p->cx2, 8 * (size_t)ccap2)) != hipSuccess ||
      (e = mad::dev_alloc(p->ck2, 8 * (size_t)ccap2)) != hipSuccess ||
      (e = mad::dev_alloc(p->cc, 4 * (size_t)ccap2)) != hipSuccess ||
      (e = mad::dev_alloc(p->cr, 16 * (size_t)rcap + mad::kPartBytes)) !=
           hipSuccess ||
      (e = mad::dev_alloc(p->misc, mad::kSelStateBytes + 4 * mad::kSelBins +
                                       256 + 256)) != hipSuccess ||
      (p->kind == 0 &&
       (e = mad::dev_alloc(p->ord, mad::sample_order_bytes(p->dt, s2,
                                                           p->sopt))) !=
           hipSuccess) ||
      (use_pairs && (e = mad::dev_alloc(p->acc, acc_bytes)) != hipSuccess)) {
    p->ws_s = p->ws_tp = p->ws_t = -1;
    return hip_fail(e, "allocating workspace");
  }
  p->h.keys = (uint64_t*)p->hk.p;
  p->h.vals = (int64_t*)p->hv.p;
  p->h.cap = hcap;
  p->pairs = use_pairs;
  p->w.x = c_in_acc ? (uint64_t*)p->acc.p : (uint64_t*)p->cx.p;
  p->w.key = c_in_acc ? p->w.x + ccap : (uint64_t*)p->ck.p;
  p->w.x2 = (uint64_t*)p->cx2.p;
  p->w.key2 = (uint64_t*)p->ck2.p;
  p->w.c = (float*)p->cc.p;
  p->w.cap = ccap;
  p->w.cap2 = ccap2;
  p->w.rx = (uint64_t*)p->cr.p;
  p->w.rkey = p->w.rx + rcap;
  p->w.rcap = rcap;
  // the two splits' and / or slots (2 x 1024 blocks x 4 words) after it
  p->w.part = (uint64_t*)((char*)p->cr.p + 16 * (size_t)rcap);
  char* misc = (char*)p->misc.p;
  p->w.state = misc;
  p->w.hist = (unsigned*)(misc + mad::kSelStateBytes);
  p->w.counts = (int64_t*)(misc + mad::kSelStateBytes + 4 * mad::kSelBins);
  p->ctr = (mad::SampleCounters*)(misc + mad::kSelStateBytes +
                                  4 * mad::kSelBins + 256);
  p->ws_s = s2;
  p->ws_tp = tp2;
  p->ws_t = t2;
  return MAD_OK;
}

int mad_plan_topk(mad_plan* p, int64_t t, int64_t s, int64_t t_prime,
                  uint64_t seed, mad_pair* out, int64_t* n_out, void* stream) {
  g_err.clear();
  if (!p) return fail(MAD_EINVAL, "plan is NULL");
  if (p->kind == 1) return fail(MAD_EINVAL, "not a MAD plan (use mips_topk_batch)");
  if (!out || !n_out) return fail(MAD_EINVAL, "out and n_out are required");
  if (t < 1) return fail(MAD_EINVAL, "t must be >= 1");
  if (t_prime < t)
    return fail(MAD_EINVAL, "t' (%lld) must be >= t (%lld)",
                (long long)t_prime, (long long)t);
  if (s < 0) return fail(MAD_EINVAL, "s must be >= 0");
  if ((double)t > (double)p->m * (double)p->n)
    return fail(MAD_EINVAL, "t exceeds m*n");
  if (s >= (int64_t(1) << 40)) return fail(MAD_EINVAL, "s must be below 2^40");
  hipStream_t st = (hipStream_t)stream;
  // a t' above the number of pairs cannot be used
  const double mn = (double)p->m * (double)p->n;
  if ((double)t_prime > mn) t_prime = (int64_t)mn;
  int64_t tp_eff = t_prime < (s > 0 ? s : 1) ? t_prime : (s > 0 ? s : 1);
  if (tp_eff < t) tp_eff = t;
  int rc = ensure_workspace(p, s, tp_eff, t);
  if (rc != MAD_OK) return rc;
  record(p, 2, st);
  mad::HashTable h = p->h;
  const int64_t nu = plan_updates(p, s);  // pairs written: s or 2s
  if (p->pairs) {
    h.pkeys = (uint64_t*)p->acc.p;
    h.pvals = (float*)((char*)p->acc.p + 8 * (size_t)nu);
    h.cap = nu;
    if (plan_square(p)) {  // the (k, k') pairs in the second half
      h.pkeys2 = h.pkeys + s;
      h.pvals2 = h.pvals + s;
    }
  } else {
    HIP_TRY(mad::launch_fill_u64(h.keys, h.cap, mad::kEmptyKey, st),
            "clearing X");
    HIP_TRY(mad::launch_fill_u64((uint64_t*)h.vals, h.cap, 0ull, st),
            "clearing X");
  }
  {  // the sampler's counters and postprocessing's clears in one launch
    mad::FillBatch f{};
    f.p[0] = (uint64_t*)p->ctr;
    f.n[0] = 8;
    f.count = 1;
    mad::post_fills(p->w, f);
    HIP_TRY(mad::launch_fill_multi(f, st), "clearing counters");
  }
  record(p, 3, st);
  mad::PairGroups groups;
  if (p->kind == 2)
    HIP_TRY(mad::launch_sample_csr(p->ct, seed, 0, 0, s, s, h, p->ctr, st),
            "sampling");
  else
    HIP_TRY(mad::launch_sample_dense(p->dt, p->B, seed, 0, 0, s, s, h,
                                     p->ctr, p->ord.p, p->ord.bytes, p->sopt,
                                     &groups, p->ev[7], st),
            "sampling");
  record(p, 4, st);
  if (p->pairs) {
    const size_t pb = pair_bytes(nu);
    if (groups.starts)
      HIP_TRY(mad::launch_accumulate_grouped(
                  h.pkeys, h.pvals, s, groups.starts, groups.G, plan_bmax(p),
                  s, (char*)p->acc.p + pb, p->acc.bytes - pb, h.keys, h.vals,
                  (int64_t*)&p->ctr->distinct, (int64_t*)&p->ctr->entries, st),
              "accumulating X");
    else
      HIP_TRY(mad::launch_accumulate(h.pkeys, h.pvals, nu, plan_bmax(p), nu,
                                     (char*)p->acc.p + pb, p->acc.bytes - pb,
                                     h.keys, h.vals,
                                     (int64_t*)&p->ctr->distinct,
                                     (int64_t*)&p->ctr->entries, st),
              "accumulating X");
    h.live = (const int64_t*)&p->ctr->entries;
  }
  h.pkeys = nullptr;
  h.pvals = nullptr;
  p->h_run = h;
  record(p, 6, st);
  HIP_TRY(mad::launch_postprocess(h, p->A, p->B,
                                  p->kind == 2 ? &p->ct.in : nullptr,
                                  p->verify_prec != MAD_FP32 ? &p->lv : nullptr,
                                  p->n, p->d, tp_eff, t, plan_bmax(p), nu,
                                  plan_square(p)
                                      ? 2
                                      : (p->flags & MAD_FLAG_GRAM) ? 1 : 0,
                                  p->w,
                                  out, n_out, true, st),
          "postprocessing");
  record(p, 5, st);
  p->timed_topk = p->ev[0] != nullptr;
  p->last_s = s;
  p->ran = true;
  return MAD_OK;
}

int mad_plan_set_option(mad_plan* p, int option, int64_t value) {
  g_err.clear();
  if (!p) return fail(MAD_EINVAL, "plan is NULL");
  if (p->kind == 1) return fail(MAD_EINVAL, "not a MAD plan");
  switch (option) {
    case MAD_OPT_ACCUM:
      if (value != MAD_ACCUM_PAIRS && value != MAD_ACCUM_HASH)
        return fail(MAD_EINVAL, "MAD_OPT_ACCUM takes MAD_ACCUM_PAIRS or "
                    "MAD_ACCUM_HASH");
      if (value == MAD_ACCUM_HASH && plan_square(p))
        return fail(MAD_EUNSUPPORTED, "the squared variant builds X from "
                    "pairs only");
      if ((int)value != (p->opt_accum < 0 ? accum_default() : p->opt_accum))
        p->ws_s = p->ws_tp = p->ws_t = -1;  // workspace of the other form
      p->opt_accum = (int)value;
      return MAD_OK;
    case MAD_OPT_SAMPLER_ORDER: {
      if (p->kind != 0)
        return fail(MAD_EUNSUPPORTED, "sampler ordering is a dense-plan option");
      mad::SampleOptions o = p->sopt;
      o.order = (int)value;
      if (value < 0 || value > 2 || !mad::sample_options_valid(o))
        return fail(MAD_EINVAL, "MAD_OPT_SAMPLER_ORDER takes 0, 1 or 2");
      p->sopt = o;
      p->ws_s = p->ws_tp = p->ws_t = -1;
      return MAD_OK;
    }
    case MAD_OPT_ORDER_CHUNK: {
      if (p->kind != 0)
        return fail(MAD_EUNSUPPORTED, "sampler ordering is a dense-plan option");
      mad::SampleOptions o = p->sopt;
      o.chunk = value;
      if (!mad::sample_options_valid(o))
        return fail(MAD_EINVAL, "MAD_OPT_ORDER_CHUNK takes a power of two in "
                    "[2^12, 2^28]");
      p->sopt = o;
      p->ws_s = p->ws_tp = p->ws_t = -1;
      return MAD_OK;
    }
    default:
      return fail(MAD_EINVAL, "unknown option %d", option);
  }
}

int mad_plan_get_option(mad_plan* p, int option, int64_t* value) {
  if (!p || !value) return fail(MAD_EINVAL, "plan and value are required");
  if (p->kind == 1) return fail(MAD_EINVAL, "not a MAD plan");
  switch (option) {
    case MAD_OPT_ACCUM:
      *value = accum_pairs(p) ? MAD_ACCUM_PAIRS : MAD_ACCUM_HASH;
      return MAD_OK;
    case MAD_OPT_SAMPLER_ORDER:
      *value = p->kind == 0 ? p->sopt.order : 0;
      return MAD_OK;
    case MAD_OPT_ORDER_CHUNK:
      *value = p->kind == 0 ? p->sopt.chunk : 0;
      return MAD_OK;
    default:
      return fail(MAD_EINVAL, "unknown option %d", option);
  }
}

int mad_topk(const float* A, int64_t m, const float* B, int64_t n, int64_t d,
             int64_t t, int64_t s, int64_t t_prime, uint64_t seed,
             mad_pair* out, int64_t* n_out, void* stream) {
  mad_plan* p = nullptr;
  int rc = mad_plan_create_dense(A, m, B, n, d, MAD_FLAG_NONE, stream, &p);
  if (rc != MAD_OK) return rc;
  rc = mad_plan_topk(p, t, s, t_prime, seed, out, n_out, stream);
  if (rc == MAD_OK) {
    hipError_t e = hipStreamSynchronize((hipStream_t)stream);
    if (e != hipSuccess) rc = hip_fail(e, "mad_topk");
  }
  std::string keep = g_err;
  mad_plan_destroy(p);
  g_err = keep;
  return rc;
}

int mad_plan_stats(mad_plan* p, double* wnorm, int64_t* closed,
                   int64_t* distinct, int64_t* n_pos, int64_t* n_cand) {
  if (!p) return fail(MAD_EINVAL, "plan is NULL");
  if (p->kind == 1) return fail(MAD_EINVAL, "not a MAD plan (use mips_stats)");
  HIP_TRY(hipDeviceSynchronize(), "stats");
  if (wnorm)
    HIP_TRY(hipMemcpy(wnorm, plan_wtot(p), sizeof(double),
                      hipMemcpyDeviceToHost), "stats");
  int64_t cnt[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  mad::SampleCounters sc;
  memset(&sc, 0, sizeof sc);
  if (p->ran) {
    HIP_TRY(hipMemcpy(cnt, p->w.counts, sizeof cnt, hipMemcpyDeviceToHost),
            "stats");
    HIP_TRY(hipMemcpy(&sc, p->ctr, sizeof sc, hipMemcpyDeviceToHost),
            "stats");
  }
  if (closed) *closed = (int64_t)sc.closed;
  if (distinct) *distinct = (int64_t)sc.distinct;
  if (n_pos) *n_pos = cnt[mad::kCountPos];
  if (n_cand) *n_cand = p->verify_prec != MAD_FP32 ? cnt[7]
                                                   : cnt[mad::kCountCand];
  return MAD_OK;
}

int mad_plan_phase_ms(mad_plan* p, double* ms, int n) {
  if (!p || !ms) return fail(MAD_EINVAL, "plan and ms are required");
  if (!p->ev[0]) return fail(MAD_EINVAL, "plan was made without MAD_FLAG_TIMING");
  // MIPS plans record no accumulation event (their postprocessing is
  // 4..5); only dense plans record the sampling kernel's start
  const int post0 = p->kind == 1 ? 4 : 6;
  const int pairs[6][2] = {{0, 1}, {3, 4}, {post0, 5}, {2, 3}, {4, 6},
                           {7, 4}};
  const bool have[6] = {p->timed_tables, p->timed_topk, p->timed_topk,
                        p->timed_topk, p->timed_topk && p->kind != 1,
                        p->timed_topk && p->kind == 0};
  const hipEvent_t last = p->timed_topk ? p->ev[5] : p->ev[1];
  HIP_TRY(hipEventSynchronize(last), "phase timing");
  for (int q = 0; q < n && q < 6; ++q) {
    ms[q] = -1.0;
    if (!have[q]) continue;
    float f = 0.0f;
    HIP_TRY(hipEventElapsedTime(&f, p->ev[pairs[q][0]], p->ev[pairs[q][1]]),
            "phase timing");
    ms[q] = f;
  }
  return MAD_OK;
}

int mad_plan_set_verify_precision(mad_plan* p, int precision, void* stream) {
  g_err.clear();
  if (!p) return fail(MAD_EINVAL, "plan is NULL");
  if (precision != MAD_FP32 && precision != MAD_BF16 &&
      precision != MAD_FP8_E4M3)
    return fail(MAD_EINVAL, "unknown precision %d", precision);
  if (p->kind == 2 && precision != MAD_FP32)
    return fail(MAD_EUNSUPPORTED,
                "low-precision verification needs a dense or MIPS plan");
  p->verify_prec = precision;
  if (precision == MAD_FP32) return MAD_OK;
  hipStream_t st = (hipStream_t)stream;
  int64_t kp = 0;
  HIP_TRY(mad::lowp_prepare(p->A, p->m, p->d, precision, p->lpA, p->lpIA, &kp,
                            st), "low-precision copies");
  if (p->B)  // a MIPS plan's queries are converted per batch
    HIP_TRY(mad::lowp_prepare(p->B, p->n, p->d, precision, p->lpB, p->lpIB,
                              &kp, st), "low-precision copies");
  p->lv.A = p->lpA.p;
  p->lv.B = p->lpB.p;
  p->lv.ia = (const mad::VecInfo*)p->lpIA.p;
  p->lv.ib = (const mad::VecInfo*)p->lpIB.p;
  p->lv.Kp = kp;
  p->lv.prec = precision;
  p->lv.d_f = (float)p->d;
  mad::lowp_consts(precision, p->d, &p->lv.kappa, &p->lv.onepu);
  return MAD_OK;
}

int mad_plan_verify_stats(mad_plan* p, int64_t* n_cand, int64_t* n_reranked) {
  if (!p) return fail(MAD_EINVAL, "plan is NULL");
  if (p->kind == 1) {  // MIPS: totals over the queries of the last batch
    if (!p->mips->ran) return fail(MAD_EINVAL, "no batch has run");
    HIP_TRY(hipDeviceSynchronize(), "verify stats");
    std::vector<mad::MipsQueryStats> qs((size_t)p->mips->nq);
    HIP_TRY(hipMemcpy(qs.data(), p->mips->qstats.p, qs.size() * sizeof qs[0],
                      hipMemcpyDeviceToHost), "verify stats");
    int64_t nc = 0, nf = 0;
    for (const auto& x : qs) {
      nc += x.n_cand;
      nf += x.n_fp32;
    }
    if (n_cand) *n_cand = nc;
    if (n_reranked) *n_reranked = nf;
    return MAD_OK;
  }
  if (!p->ran) return fail(MAD_EINVAL, "no mad_plan_topk has run");
  HIP_TRY(hipDeviceSynchronize(), "verify stats");
  int64_t cnt[9];
  HIP_TRY(hipMemcpy(cnt, p->w.counts, sizeof cnt, hipMemcpyDeviceToHost),
          "verify stats");
  const bool lp = p->verify_prec != MAD_FP32;
  if (n_cand) *n_cand = lp ? cnt[7] : cnt[mad::kCountCand];
  if (n_reranked) *n_reranked = lp ? cnt[8] : cnt[mad::kCountCand];
  return MAD_OK;
}

int mad_debug_lowp_screen(mad_plan* p, const int64_t* keys, int64_t count,
                          float* chat, float* margin, void* stream) {
  g_err.clear();
  if (!p) return fail(MAD_EINVAL, "plan is NULL");
  if (p->kind != 0) return fail(MAD_EINVAL, "needs a dense MAD plan");
  if (p->verify_prec == MAD_FP32)
    return fail(MAD_EINVAL, "the plan verifies in fp32 (no screen)");
  if (count < 0) return fail(MAD_EINVAL, "count must be >= 0");
  if (count && (!keys || !chat || !margin))
    return fail(MAD_EINVAL, "keys, chat and margin are required");
  HIP_TRY(mad::launch_lowp_screen_values((const uint64_t*)keys, count, p->lv,
                                         p->n, chat, margin,
                                         (hipStream_t)stream),
          "screen values");
  return MAD_OK;
}

int mad_fix_exponent(mad_plan* p, int64_t s, int* F) {
  if (!p || !F) return fail(MAD_EINVAL, "plan and F are required");
  float bmax = 0.0f;
  HIP_TRY(hipDeviceSynchronize(), "fix exponent");
  HIP_TRY(hipMemcpy(&bmax, plan_bmax(p), sizeof(float), hipMemcpyDeviceToHost),
          "fix exponent");
  *F = mad::fix_exponent(bmax, plan_updates(p, s));
  return MAD_OK;
}

int mad_debug_table(mad_plan* p, int which, int64_t idx, uint32_t* thr,
                    uint32_t* alias, int32_t* item, int64_t cap,
                    int64_t* nslots) {
  if (!p) return fail(MAD_EINVAL, "plan is NULL");
  if (p->kind == 2 && which != 0) {
    const mad::Ragged* R = which == 1 ? &p->ct.T1
                         : which == 2 ? &p->ct.T2
                         : which == 3 ? &p->ct.T3 : nullptr;
    if (!R) return fail(MAD_EINVAL, "which must be 0..3");
    if (idx < 0 || idx >= R->S) return fail(MAD_EINVAL, "table index out of range");
    HIP_TRY(hipDeviceSynchronize(), "debug table");
    uint64_t mt = 0;
    HIP_TRY(hipMemcpy(&mt, R->meta + idx, 8, hipMemcpyDeviceToHost),
            "debug table");
    const int64_t Np = int64_t(1) << (mt >> 56);
    if (nslots) *nslots = Np;
    if (!thr && !alias && !item) return MAD_OK;
    if (cap < Np) return fail(MAD_EINVAL, "capacity %lld < %lld slots",
                              (long long)cap, (long long)Np);
    // entries of R->esz bytes, each starting with the packed word and the
    // two item ids
    std::vector<char> host((size_t)Np * (size_t)R->esz);
    HIP_TRY(hipMemcpy(host.data(),
                      (const char*)R->ent +
                          (int64_t)(mt & mad::kSlotMask) * R->esz,
                      host.size(), hipMemcpyDeviceToHost),
            "debug table");
    for (int64_t r = 0; r < Np; ++r) {
      mad::Ent16 x;
      memcpy(&x, host.data() + (size_t)r * (size_t)R->esz, sizeof x);
      if (thr) thr[r] = (uint32_t)x.w & mad::kLow31;
      if (alias) alias[r] = x.alias;
      if (item) item[r] = (int32_t)x.self;
    }
    return MAD_OK;
  }
  const mad::Family* f;
  switch (which) {
    case 0: f = p->kind == 2 ? &p->ct.T0 : &p->dt.T0; idx = 0; break;
    case 1: f = &p->dt.T1; break;
    case 2: f = &p->dt.T2; break;
    case 3: f = &p->dt.T3; break;
    default: return fail(MAD_EINVAL, "which must be 0..3");
  }
  if (idx < 0 || idx >= f->S) return fail(MAD_EINVAL, "table index out of range");
  const int64_t Np = int64_t(1) << f->L;
  if (nslots) *nslots = Np;
  if (!thr && !alias && !item) return MAD_OK;
  if (cap < Np) return fail(MAD_EINVAL, "capacity %lld < %lld slots",
                            (long long)cap, (long long)Np);
  uint64_t* host = new (std::nothrow) uint64_t[Np];
  if (!host) return fail(MAD_ENOMEM, "host allocation failed");
  HIP_TRY(hipDeviceSynchronize(), "debug table");
  hipError_t e = hipMemcpy(host, f->ent + (idx << f->L), 8 * (size_t)Np,
                           hipMemcpyDeviceToHost);
  if (e != hipSuccess) {
    delete[] host;
    return hip_fail(e, "debug table");
  }
  for (int64_t r = 0; r < Np; ++r) {
    const uint32_t lo = (uint32_t)host[r], hi = (uint32_t)(host[r] >> 32);
    if (thr) thr[r] = lo & mad::kLow31;
    if (alias) alias[r] = hi & mad::kLow31;
    if (item) item[r] = (int32_t)r;
  }
  delete[] host;
  return MAD_OK;
}

int mad_debug_norms(mad_plan* p, double* na, double* nb, double* v,
                    double* om) {
  if (!p) return fail(MAD_EINVAL, "plan is NULL");
  if (p->kind == 1 && (nb || om))
    return fail(MAD_EINVAL, "a MIPS plan has no nb or om");
  if (p->kind == 2) {
    HIP_TRY(hipDeviceSynchronize(), "debug norms");
    if (na) HIP_TRY(hipMemcpy(na, p->ct.T3.tot, 8 * (size_t)p->m,
                              hipMemcpyDeviceToHost), "debug norms");
    if (nb) HIP_TRY(hipMemcpy(nb, p->ct.T2.tot, 8 * (size_t)p->d,
                              hipMemcpyDeviceToHost), "debug norms");
    if (v) HIP_TRY(hipMemcpy(v, p->ct.T1.tot, 8 * (size_t)p->d,
                             hipMemcpyDeviceToHost), "debug norms");
    if (om) HIP_TRY(hipMemcpy(om, p->ct.om, 8 * (size_t)p->d,
                              hipMemcpyDeviceToHost), "debug norms");
    return MAD_OK;
  }
  HIP_TRY(hipDeviceSynchronize(), "debug norms");
  if (na) HIP_TRY(hipMemcpy(na, p->dt.na, 8 * (size_t)p->m,
                            hipMemcpyDeviceToHost), "debug norms");
  if (nb) HIP_TRY(hipMemcpy(nb, p->dt.nb, 8 * (size_t)p->d,
                            hipMemcpyDeviceToHost), "debug norms");
  if (v) HIP_TRY(hipMemcpy(v, p->dt.v, 8 * (size_t)p->d,
                           hipMemcpyDeviceToHost), "debug norms");
  if (om) HIP_TRY(hipMemcpy(om, p->dt.om, 8 * (size_t)p->d,
                            hipMemcpyDeviceToHost), "debug norms");
  return MAD_OK;
}

int mad_debug_samples(mad_plan* p, uint64_t seed, uint64_t qid, int64_t l0,
                      int64_t count, int F, int32_t* k, int32_t* i,
                      int32_t* j, int32_t* kp, int64_t* inc, void* stream) {
  if (!p) return fail(MAD_EINVAL, "plan is NULL");
  if (count < 0 || l0 < 0) return fail(MAD_EINVAL, "bad sample range");
  if (count && (!k || !i || !j || !kp || !inc))
    return fail(MAD_EINVAL, "output arrays are required");
  hipStream_t st = (hipStream_t)stream;
  if (p->kind == 2)
    HIP_TRY(mad::launch_sample_csr_debug(p->ct, seed, qid, l0, count, F, k, i,
                                         j, kp, inc, st),
            "debug samples");
  else
    HIP_TRY(mad::launch_sample_dense_debug(p->dt, p->B, seed, qid, l0, count,
                                           F, k, i, j, kp, inc, st),
            "debug samples");
  HIP_TRY(hipStreamSynchronize(st), "debug samples");
  return MAD_OK;
}

int mad_debug_accumulate(const uint64_t* keys, const float* vals, int64_t n,
                         int F, int64_t* out_keys, int64_t* out_x,
                         int64_t cap, int64_t* n_out, void* stream) {
  g_err.clear();
  if (!n_out) return fail(MAD_EINVAL, "n_out is required");
  if (n < 0) return fail(MAD_EINVAL, "n must be >= 0");
  if (n && (!is_device_ptr(keys) || !is_device_ptr(vals)))
    return fail(MAD_EINVAL, "keys and vals must be device pointers");
  if (cap && (!is_device_ptr(out_keys) || !is_device_ptr(out_x)))
    return fail(MAD_EINVAL, "outputs must be device pointers");
  hipStream_t st = (hipStream_t)stream;
  const int64_t nn = n > 1 ? n : 1;
  // the pairs are overwritten by the accumulation: work on copies
  mad::DeviceBuffer buf;
  const size_t pk = 8 * (size_t)nn, pv = (4 * (size_t)nn + 15) / 16 * 16;
  const size_t need = pk + pv + 16 * (size_t)nn + 64 + mad::accum_bytes(nn);
  HIP_TRY(mad::dev_alloc(buf, need), "debug accumulate");
  char* q = (char*)buf.p;
  uint64_t* k2 = (uint64_t*)q; q += pk;
  float* v2 = (float*)q; q += pv;
  uint64_t* okey = (uint64_t*)q; q += 8 * (size_t)nn;
  int64_t* oval = (int64_t*)q; q += 8 * (size_t)nn;
  int64_t* cnt = (int64_t*)q; q += 64;
  hipError_t e = hipSuccess;
  if (n) {
    e = hipMemcpyAsync(k2, keys, 8 * (size_t)n, hipMemcpyDeviceToDevice, st);
    if (e == hipSuccess)
      e = hipMemcpyAsync(v2, vals, 4 * (size_t)n, hipMemcpyDeviceToDevice, st);
  }
  if (e == hipSuccess)
    e = mad::launch_accumulate(k2, v2, n, nullptr, F, q,
                               need - (size_t)(q - (char*)buf.p), okey, oval,
                               cnt, cnt + 1, st);
  mad::HashTable h;
  h.keys = okey;
  h.vals = oval;
  h.cap = n;
  h.live = cnt + 1;
  if (e == hipSuccess)
    e = mad::launch_dump_scores(h, out_keys, out_x, out_keys ? cap : 0,
                                cnt + 2, st);
  int64_t got = 0;
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e == hipSuccess)
    e = hipMemcpy(&got, cnt + 2, 8, hipMemcpyDeviceToHost);
  mad::dev_free(buf);
  if (e != hipSuccess) return hip_fail(e, "debug accumulate");
  *n_out = got;
  if (out_keys && got > cap) return fail(MAD_EOVERFLOW, "capacity too small");
  return MAD_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free score accumulation.  Its workspace is a file-scope device
// array: every GPU holds its own copy until the process ends.  Host code
// never uses the array's name as an address: its device address is looked
// up once per device (hipGetSymbolAddress, with that device current) and
// only that address is passed to kernels and copies.  Calls that overlap on
// one GPU share the array and race; each call overwrites what it uses.
// ---------------------------------------------------------------------------
namespace {

constexpr int64_t kNoAllocMaxPairs = int64_t(1) << 18;
constexpr size_t kNoAllocScratchBytes = size_t(12) << 20;
constexpr int kNoAllocMaxDevices = 64;

__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kNoAllocMaxDevices] = {};

struct NoAllocLayout {
  uint64_t* k2;
  float* v2;
  uint64_t* okey;
  int64_t* oval;
  int64_t* cnt;
  char* work;
  size_t work_bytes;
  size_t total;
};

NoAllocLayout noalloc_layout(char* base, int64_t n) {
  const int64_t nn = n > 1 ? n : 1;
  NoAllocLayout L;
  char* q = base;
  L.k2 = (uint64_t*)q; q += (8 * (size_t)nn + 255) / 256 * 256;
  L.v2 = (float*)q; q += (4 * (size_t)nn + 255) / 256 * 256;
  L.okey = (uint64_t*)q; q += (8 * (size_t)nn + 255) / 256 * 256;
  L.oval = (int64_t*)q; q += (8 * (size_t)nn + 255) / 256 * 256;
  L.cnt = (int64_t*)q; q += 256;
  L.work = q;
  L.work_bytes = mad::accum_bytes(nn);
  L.total = (size_t)(q - base) + L.work_bytes;
  return L;
}

// the device address of this device's scratch array (looked up once)
int scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
  if (dev < 0 || dev >= kNoAllocMaxDevices)
    return fail(MAD_EUNSUPPORTED, "device %d beyond the scratch table", dev);
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol,
                      "looking up the scratch array");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return MAD_OK;
}

}  // namespace

int mad_accumulate_noalloc(const uint64_t* keys, const float* vals, int64_t n,
                           int F, int64_t* out_keys, int64_t* out_x,
                           int64_t* n_out, void* stream) {
  g_err.clear();
  if (n < 0) return fail(MAD_EINVAL, "n must be >= 0");
  if (n > kNoAllocMaxPairs)
    return fail(MAD_EINVAL, "n = %lld pairs exceeds the static workspace "
                "(at most %lld pairs)", (long long)n,
                (long long)kNoAllocMaxPairs);
  if (!n_out) return fail(MAD_EINVAL, "n_out is required");
  if (n && (!keys || !vals || !out_keys || !out_x))
    return fail(MAD_EINVAL, "keys, vals, out_keys and out_x are required");
  if (F < 0 || F > 62) return fail(MAD_EINVAL, "F must be in [0, 62]");
  void* base = nullptr;
  int rc = scratch_address(&base);
  if (rc != MAD_OK) return rc;
  const NoAllocLayout L = noalloc_layout((char*)base, n);
  if (L.total > kNoAllocScratchBytes)
    return fail(MAD_EOVERFLOW, "the static workspace is too small for %lld "
                "pairs", (long long)n);
  hipStream_t st = (hipStream_t)stream;
  if (n == 0) {
    HIP_TRY(mad::launch_fill_u64((uint64_t*)n_out, 1, 0ull, st),
            "accumulate (no allocation)");
    return MAD_OK;
  }
  // the accumulation overwrites its pairs: it works on copies
  HIP_TRY(hipMemcpyAsync(L.k2, keys, 8 * (size_t)n, hipMemcpyDeviceToDevice,
                         st), "accumulate (no allocation)");
  HIP_TRY(hipMemcpyAsync(L.v2, vals, 4 * (size_t)n, hipMemcpyDeviceToDevice,
                         st), "accumulate (no allocation)");
  HIP_TRY(mad::launch_accumulate(L.k2, L.v2, n, nullptr, F, L.work,
                                 L.work_bytes, L.okey, L.oval, L.cnt,
                                 L.cnt + 1, st),
          "accumulate (no allocation)");
  mad::HashTable h;
  h.keys = L.okey;
  h.vals = L.oval;
  h.cap = n;
  h.live = L.cnt + 1;
  HIP_TRY(mad::launch_dump_scores(h, out_keys, out_x, n, n_out, st),
          "accumulate (no allocation)");
  return MAD_OK;
}

int mad_debug_scores(mad_plan* p, int64_t* keys, int64_t* xfix, int64_t cap,
                     int64_t* n, int* F) {
  if (!p || !n) return fail(MAD_EINVAL, "plan and n are required");
  if (!p->ran) return fail(MAD_EINVAL, "no mad_plan_topk has run");
  int64_t* cnt = p->w.counts + 6;
  HIP_TRY(mad::launch_dump_scores(p->h_run, keys, xfix, keys ? cap : 0, cnt, 0),
          "debug scores");
  HIP_TRY(hipDeviceSynchronize(), "debug scores");
  int64_t total = 0;
  HIP_TRY(hipMemcpy(&total, cnt, 8, hipMemcpyDeviceToHost), "debug scores");
  *n = total;
  if (F) {
    int rc = mad_fix_exponent(p, p->last_s, F);
    if (rc != MAD_OK) return rc;
  }
  if (keys && total > cap) return fail(MAD_EOVERFLOW, "capacity too small");
  return MAD_OK;
}

int mad_debug_candidates(mad_plan* p, int64_t* keys, int64_t* xfix, float* c,
                         int64_t cap, int64_t* n) {
  if (!p || !n) return fail(MAD_EINVAL, "plan and n are required");
  if (!p->ran) return fail(MAD_EINVAL, "no mad_plan_topk has run");
  HIP_TRY(hipDeviceSynchronize(), "debug candidates");
  int64_t cnt[4];
  HIP_TRY(hipMemcpy(cnt, p->w.counts, sizeof cnt, hipMemcpyDeviceToHost),
          "debug candidates");
  const int64_t nc = cnt[mad::kCountCand];
  *n = nc;
  if (!keys && !xfix && !c) return MAD_OK;
  if (nc > cap) return fail(MAD_EOVERFLOW, "capacity too small");
  if (keys) HIP_TRY(hipMemcpy(keys, p->w.key2, 8 * (size_t)nc,
                              hipMemcpyDeviceToDevice), "debug candidates");
  if (xfix) HIP_TRY(hipMemcpy(xfix, p->w.x2, 8 * (size_t)nc,
                              hipMemcpyDeviceToDevice), "debug candidates");
  if (c) HIP_TRY(hipMemcpy(c, p->w.c, 4 * (size_t)nc,
                           hipMemcpyDeviceToDevice), "debug candidates");
  return MAD_OK;
}

int mad_bruteforce_topk(const float* A, int64_t m, const float* B, int64_t n,
                        int64_t d, int precision, int64_t t, int64_t t_screen,
                        mad_pair* out, int64_t* n_out, mad_bf_stats* stats,
                        void* stream) {
  g_err.clear();
  if (m < 1 || n < 1 || d < 1 || m >= (int64_t(1) << 31) ||
      n >= (int64_t(1) << 31))
    return fail(MAD_EINVAL, "need 1 <= m, n < 2^31 and d >= 1");
  if (t < 1 || (double)t > (double)m * (double)n)
    return fail(MAD_EINVAL, "need 1 <= t <= m*n");
  if (precision != MAD_FP32 && precision != MAD_BF16 &&
      precision != MAD_FP8_E4M3)
    return fail(MAD_EINVAL, "unknown precision %d", precision);
  if (!out || !n_out) return fail(MAD_EINVAL, "out and n_out are required");
  if (!is_device_ptr(A) || !is_device_ptr(B))
    return fail(MAD_EINVAL, "A and B must be device pointers");
  mad::BfStats bs;
  memset(&bs, 0, sizeof bs);
  hipError_t e = mad::bruteforce_topk(A, m, B, n, d, precision, t, t_screen,
                                      out, n_out, &bs, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "brute force");
  if (stats) {
    stats->ms_screen = bs.ms_screen;
    stats->ms_filter = bs.ms_filter;
    stats->ms_rerank = bs.ms_rerank;
    stats->candidates = bs.candidates;
    stats->tau = bs.tau;
    stats->row_stride = bs.row_stride;
    stats->reranked = bs.reranked;
  }
  return MAD_OK;
}

int mad_bruteforce_topk_csr(const int64_t* a_ptr, const int32_t* a_idx,
                            const float* a_val, int64_t m,
                            const int64_t* b_ptr, const int32_t* b_idx,
                            const float* b_val, int64_t n, int64_t d,
                            int precision, int64_t t, int64_t heavy,
                            mad_pair* out, int64_t* n_out,
                            mad_bf_csr_stats* stats, void* stream) {
  g_err.clear();
  if (m < 1 || n < 1 || d < 1 || m >= (int64_t(1) << 31) ||
      n >= (int64_t(1) << 31) || d >= (int64_t(1) << 31))
    return fail(MAD_EINVAL, "need 1 <= m, n, d < 2^31");
  if (t < 1 || (double)t > (double)m * (double)n)
    return fail(MAD_EINVAL, "need 1 <= t <= m*n");
  if (heavy < 0) return fail(MAD_EINVAL, "heavy must be >= 0");
  if (precision != MAD_FP32 && precision != MAD_BF16 &&
      precision != MAD_FP8_E4M3)
    return fail(MAD_EINVAL, "unknown precision %d", precision);
  if (!out || !n_out) return fail(MAD_EINVAL, "out and n_out are required");
  if (!is_device_ptr(a_ptr) || !is_device_ptr(b_ptr))
    return fail(MAD_EINVAL, "CSR pointer arrays must be device pointers");
  hipStream_t st = (hipStream_t)stream;
  int64_t nnzA = 0, nnzB = 0;
  HIP_TRY(hipMemcpy(&nnzA, a_ptr + m, 8, hipMemcpyDeviceToHost), "reading nnz");
  HIP_TRY(hipMemcpy(&nnzB, b_ptr + n, 8, hipMemcpyDeviceToHost), "reading nnz");
  if (nnzA < 0 || nnzB < 0 || nnzA >= (int64_t(1) << 31) ||
      nnzB >= (int64_t(1) << 31))
    return fail(MAD_EINVAL, "need 0 <= nnz < 2^31 (a_ptr[m], b_ptr[n])");
  if ((nnzA && (!is_device_ptr(a_idx) || !is_device_ptr(a_val))) ||
      (nnzB && (!is_device_ptr(b_idx) || !is_device_ptr(b_val))))
    return fail(MAD_EINVAL, "CSR arrays must be device pointers");
  const mad::CsrView in{a_ptr, a_idx, a_val, b_ptr, b_idx, b_val};
  static mad::DeviceBuffer flag;
  HIP_TRY(mad::dev_alloc(flag, 256), "brute force");
  hipError_t e = mad::csr_validate(in, m, n, d, nnzA, nnzB, (int*)flag.p, st);
  if (e == hipErrorInvalidValue)
    return fail(MAD_EINVAL, "malformed CSR input or non-finite values");
  if (e != hipSuccess) return hip_fail(e, "brute force");
  mad::BfCsrStats bs;
  memset(&bs, 0, sizeof bs);
  e = mad::bruteforce_topk_csr(in, m, n, d, nnzA, nnzB, precision, t, heavy,
                               out, n_out, &bs, st);
  if (e == hipErrorNotSupported)
    return fail(MAD_EUNSUPPORTED, "the split would need more than 4096 heavy "
                "coordinates or 2^30 light wedges");
  if (e != hipSuccess) return hip_fail(e, "sparse brute force");
  if (stats) {
    stats->ms_split = bs.ms_split;
    stats->ms_heavy = bs.ms_heavy;
    stats->ms_light = bs.ms_light;
    stats->ms_final = bs.ms_final;
    stats->heavy = bs.heavy;
    stats->wedges = bs.wedges;
    stats->light_wedges = bs.light_wedges;
    stats->heavy_candidates = bs.heavy_candidates;
    stats->light_candidates = bs.light_candidates;
    stats->candidates = bs.candidates;
    stats->tau = bs.tau;
  }
  return MAD_OK;
}

int mad_plan_create_csr(const int64_t* a_ptr, const int32_t* a_idx,
                        const float* a_val, int64_t m, const int64_t* b_ptr,
                        const int32_t* b_idx, const float* b_val, int64_t n,
                        int64_t d, uint32_t flags, void* stream,
                        mad_plan** plan) {
  g_err.clear();
  if (!plan) return fail(MAD_EINVAL, "plan is NULL");
  *plan = nullptr;
  if (m < 1 || n < 1 || d < 1 || m >= (int64_t(1) << 31) ||
      n >= (int64_t(1) << 31) || d >= (int64_t(1) << 31))
    return fail(MAD_EINVAL, "need 1 <= m, n, d < 2^31");
  if (!is_device_ptr(a_ptr) || !is_device_ptr(b_ptr))
    return fail(MAD_EINVAL, "CSR arrays must be device pointers");
  int64_t nnzA = 0, nnzB = 0;
  HIP_TRY(hipMemcpy(&nnzA, a_ptr + m, 8, hipMemcpyDeviceToHost), "reading nnz");
  HIP_TRY(hipMemcpy(&nnzB, b_ptr + n, 8, hipMemcpyDeviceToHost), "reading nnz");
  if (nnzA < 0 || nnzB < 0 || nnzA >= (int64_t(1) << 31) ||
      nnzB >= (int64_t(1) << 31))
    return fail(MAD_EINVAL, "need 0 <= nnz < 2^31 (a_ptr[m], b_ptr[n])");
  if ((nnzA && (!is_device_ptr(a_idx) || !is_device_ptr(a_val))) ||
      (nnzB && (!is_device_ptr(b_idx) || !is_device_ptr(b_val))))
    return fail(MAD_EINVAL, "CSR arrays must be device pointers");
  if ((flags & MAD_FLAG_GRAM) &&
      (a_ptr != b_ptr || a_idx != b_idx || a_val != b_val || m != n))
    return fail(MAD_EINVAL, "MAD_FLAG_GRAM needs B == A (same arrays, n == m)");
  if ((flags & MAD_FLAG_SQUARE) &&
      (a_ptr != b_ptr || a_idx != b_idx || a_val != b_val || m != n ||
       m != d))
    return fail(MAD_EINVAL, "MAD_FLAG_SQUARE needs B == A (same arrays) and "
                "m == n == d");
  mad_plan* p = new (std::nothrow) mad_plan();
  if (!p) return fail(MAD_ENOMEM, "host allocation failed");
  p->kind = 2;
  p->m = m;
  p->n = n;
  p->d = d;
  p->flags = flags;
  p->ct.m = m;
  p->ct.n = n;
  p->ct.d = d;
  p->ct.nnzA = nnzA;
  p->ct.nnzB = nnzB;
  p->ct.in = mad::CsrView{a_ptr, a_idx, a_val, b_ptr, b_idx, b_val};
  p->ct.square = (flags & MAD_FLAG_SQUARE) ? 1 : 0;
  p->ct.gram = ((flags & MAD_FLAG_GRAM) || p->ct.square) ? 1 : 0;
  hipError_t e = hipSuccess;
  if (flags & MAD_FLAG_TIMING)
    for (hipEvent_t& ev : p->ev)
      if ((e = hipEventCreate(&ev)) != hipSuccess) break;
  if (e != hipSuccess) {
    plan_free_all(p);
    delete p;
    return hip_fail(e, "creating events");
  }
  int rc = mad_plan_refresh(p, stream);
  if (rc != MAD_OK) {
    std::string keep = g_err;
    (void)hipDeviceSynchronize();
    plan_free_all(p);
    delete p;
    g_err = keep;
    return rc;
  }
  *plan = p;
  return MAD_OK;
}

// ---------------------------------------------------------------------------
// MIPS
// ---------------------------------------------------------------------------
int mips_plan_create(const float* A, int64_t m, int64_t d, uint32_t flags,
                     void* stream, mad_plan** plan) {
  g_err.clear();
  if (!plan) return fail(MAD_EINVAL, "plan is NULL");
  *plan = nullptr;
  if (m < 1 || d < 1)
    return fail(MAD_EINVAL, "need m, d >= 1 (got %lld, %lld)", (long long)m,
                (long long)d);
  if (m >= (int64_t(1) << 31) || d > 4096)
    return fail(m >= (int64_t(1) << 31) ? MAD_EINVAL : MAD_EUNSUPPORTED,
                "MIPS needs m < 2^31 and d <= 4096");
  if (!is_device_ptr(A)) return fail(MAD_EINVAL, "A must be a device pointer");
  mad_plan* p = new (std::nothrow) mad_plan();
  MipsState* ms = new (std::nothrow) MipsState();
  if (!p || !ms) {
    delete p;
    delete ms;
    return fail(MAD_ENOMEM, "host allocation failed");
  }
  p->kind = 1;
  p->A = A;
  p->B = nullptr;
  p->m = m;
  p->n = 1;
  p->d = d;
  p->flags = flags;
  p->mips = ms;
  hipError_t e = mad::dense_tables_alloc(p->dt, m, 1, d);
  if (e == hipSuccess && (flags & MAD_FLAG_TIMING))
    for (hipEvent_t& ev : p->ev)
      if ((e = hipEventCreate(&ev)) != hipSuccess) break;
  if (e == hipSuccess)
    e = hipStreamCreateWithFlags(&ms->cap_stream, hipStreamNonBlocking);
  if (e != hipSuccess) {
    plan_free_all(p);
    delete p;
    return hip_fail(e, "allocating tables");
  }
  int rc = mad_plan_refresh(p, stream);
  if (rc != MAD_OK) {
    std::string keep = g_err;
    (void)hipDeviceSynchronize();
    plan_free_all(p);
    delete p;
    g_err = keep;
    return rc;
  }
  *plan = p;
  return MAD_OK;
}

static void mips_drop_graph(MipsState* ms) {
  if (ms->exec) (void)hipGraphExecDestroy(ms->exec);
  if (ms->graph) (void)hipGraphDestroy(ms->graph);
  ms->exec = nullptr;
  ms->graph = nullptr;
}

// Host layout of a batch: per-query regions, the chunk list (queries by
// descending budget, chunks of ms->chunk samples) and the workspace.
static int mips_prepare(mad_plan* p, int64_t nq, const int64_t* s,
                        const int64_t* tp, int64_t t) {
  MipsState* ms = p->mips;
  const bool same = nq == ms->nq && t == ms->t &&
                    ms->chunk_prepared == ms->chunk &&
                    ms->slots_prepared == ms->slots &&
                    std::equal(s, s + nq, ms->s.begin()) &&
                    std::equal(tp, tp + nq, ms->tp.begin());
  if (same) return MAD_OK;
  const int64_t m = p->m;
  std::vector<mad::MipsQuery> qi((size_t)nq);
  std::vector<int32_t> order((size_t)nq);
  int64_t hs = 0, cs = 0, ss = 0;
  for (int64_t q = 0; q < nq; ++q) {
    mad::MipsQuery& x = qi[(size_t)q];
    memset(&x, 0, sizeof x);
    const int64_t sq = s[q];
    const int64_t pairs = sq < m ? sq : m;
    // a t' above the pairs or the samples cannot be used (as mad_plan_topk)
    int64_t tpe = tp[q] < m ? tp[q] : m;
    const int64_t sc1 = sq > 0 ? sq : 1;
    if (tpe > sc1) tpe = sc1;
    if (tpe < t) tpe = t;
    const int64_t hcap =
        next_pow2((int64_t)ms->slots * (pairs > 512 ? pairs : 512));
    x.s = sq;
    x.tp = tpe;
    x.hoff = hs;
    x.hmask = (uint32_t)(hcap - 1);
    x.coff = cs;
    x.ccap = pairs > 1 ? pairs : 1;
    x.soff = ss;
    x.scap = x.ccap < tpe ? x.ccap : tpe;
    hs += hcap;
    cs += x.ccap;
    ss += x.scap;
    order[(size_t)q] = (int32_t)q;
  }
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
    return s[a] > s[b];
  });
  std::vector<mad::MipsChunk> ch;
  for (int32_t q : order)
    for (int64_t l0 = 0; l0 < s[q]; l0 += ms->chunk) {
      mad::MipsChunk c;
      c.q = q;
      c.count = (int32_t)(s[q] - l0 < ms->chunk ? s[q] - l0 : ms->chunk);
      c.l0 = l0;
      ch.push_back(c);
    }
  (void)hipDeviceSynchronize();
  mips_drop_graph(ms);
  hipError_t e = hipSuccess;
  if (nq > ms->nq_cap) {
    mad::family_free_pub(ms->T0q);
    e = mad::family_alloc_pub(ms->T0q, nq, p->d);
    if (e != hipSuccess) return hip_fail(e, "allocating query tables");
    ms->nq_cap = nq;
  }
  ms->T0q.S = nq;
  const size_t qsb = mad::query_tables_scratch_bytes(nq, p->d);
  const size_t nqa = (size_t)(nq > 0 ? nq : 1);
  if ((e = mad::dev_alloc(ms->qscratch, qsb)) != hipSuccess ||
      (e = mad::dev_alloc(ms->qinfo, nqa * sizeof(mad::MipsQuery))) != hipSuccess ||
      (e = mad::dev_alloc(ms->order, nqa * 4)) != hipSuccess ||
      (e = mad::dev_alloc(ms->chunks, (ch.size() + 1) * sizeof(mad::MipsChunk))) != hipSuccess ||
      (e = mad::dev_alloc(ms->hash, (size_t)(hs + 1) * 8)) != hipSuccess ||
      (e = mad::dev_alloc(ms->cx, (size_t)(cs + 1) * 8)) != hipSuccess ||
      (e = mad::dev_alloc(ms->ck, (size_t)(cs + 1) * 4)) != hipSuccess ||
      (e = mad::dev_alloc(ms->sx, (size_t)(ss + 1) * 8)) != hipSuccess ||
      (e = mad::dev_alloc(ms->sk, (size_t)(ss + 1) * 4)) != hipSuccess ||
      (e = mad::dev_alloc(ms->sc, (size_t)(ss + 1) * 4)) != hipSuccess ||
      (e = mad::dev_alloc(ms->sab, (size_t)(ss + 1) * 8)) != hipSuccess ||
      (e = mad::dev_alloc(ms->qstats, nqa * sizeof(mad::MipsQueryStats))) != hipSuccess ||
      (e = mad::dev_alloc(ms->ctr, sizeof(mad::SampleCounters))) != hipSuccess) {
    ms->nq = -1;
    return hip_fail(e, "allocating the MIPS workspace");
  }
  if (nq > 0) {
    HIP_TRY(hipMemcpy(ms->qinfo.p, qi.data(), qi.size() * sizeof qi[0],
                      hipMemcpyHostToDevice), "uploading the batch layout");
    HIP_TRY(hipMemcpy(ms->order.p, order.data(), order.size() * 4,
                      hipMemcpyHostToDevice), "uploading the batch layout");
  }
  if (!ch.empty())
    HIP_TRY(hipMemcpy(ms->chunks.p, ch.data(), ch.size() * sizeof ch[0],
                      hipMemcpyHostToDevice), "uploading the batch layout");
  ms->s.assign(s, s + nq);
  ms->tp.assign(tp, tp + nq);
  ms->nq = nq;
  ms->t = t;
  ms->hslots = hs;
  ms->nchunks = (int64_t)ch.size();
  ms->chunk_prepared = ms->chunk;
  ms->slots_prepared = ms->slots;
  ++ms->layout_version;
  return MAD_OK;
}

// bits of a MIPS score slot's key field: i + 1 <= m < 2^kb
static int mips_key_bits(int64_t m) {
  int kb = 1;
  while ((int64_t(1) << kb) <= m) ++kb;
  return kb;
}

static mad::MipsArgs mips_args(mad_plan* p, const float* Q, uint64_t seed,
                               void* out, int64_t* n_out) {
  MipsState* ms = p->mips;
  mad::MipsArgs a;
  a.T0q = ms->T0q.ent;
  a.t0tot = ms->T0q.tot;
  a.T1 = p->dt.T1.ent;
  a.T3 = p->dt.T3.ent;
  a.L0 = ms->T0q.L;
  a.L1 = p->dt.T1.L;
  a.L3 = p->dt.T3.L;
  a.A = p->A;
  a.Q = Q;
  a.m = p->m;
  a.d = p->d;
  a.nq = ms->nq;
  a.t = ms->t;
  a.seed = seed;
  a.qi = (const mad::MipsQuery*)ms->qinfo.p;
  a.order = (const int32_t*)ms->order.p;
  a.chunks = (const mad::MipsChunk*)ms->chunks.p;
  a.nchunks = ms->nchunks;
  a.hslot = (uint64_t*)ms->hash.p;
  a.kb = mips_key_bits(p->m);
  a.cx = (uint64_t*)ms->cx.p;
  a.ck = (uint32_t*)ms->ck.p;
  a.sx = (uint64_t*)ms->sx.p;
  a.sk = (uint32_t*)ms->sk.p;
  a.sc = (float*)ms->sc.p;
  a.sab = (uint64_t*)ms->sab.p;
  a.ctr = (mad::SampleCounters*)ms->ctr.p;
  a.qstats = (mad::MipsQueryStats*)ms->qstats.p;
  a.out = out;
  a.n_out = n_out;
  if (p->verify_prec != MAD_FP32) {
    a.lp = p->verify_prec;
    a.Alp = p->lv.A;
    a.ia = p->lv.ia;
    a.Qlp = ms->qlp.p;
    a.iq = (const mad::VecInfo*)ms->qlpi.p;
    a.Kp = p->lv.Kp;
    a.kappa = p->lv.kappa;
    a.onepu = p->lv.onepu;
    a.d_f = p->lv.d_f;
  }
  return a;
}

// the launch sequence of one batch (captured into a graph, or run eagerly
// with phase events when the plan records timings)
static hipError_t mips_enqueue(mad_plan* p, const mad::MipsArgs& a,
                               hipStream_t st, bool events) {
  MipsState* ms = p->mips;
  hipError_t e;
  if (events) record(p, 0, st);
  if ((e = mad::launch_mips_query_info(a.Q, a.nq, a.d, a.kb,
                                       (mad::MipsQuery*)ms->qinfo.p, st)) !=
          hipSuccess ||
      (e = mad::query_tables_build(a.Q, a.nq, a.d, p->dt.v, ms->T0q,
                                   ms->qscratch.p, ms->qscratch.bytes, st)) !=
          hipSuccess)
    return e;
  if (a.lp) {  // the queries' low-precision rows (buffers sized already)
    int64_t kp = 0;
    if ((e = mad::lowp_prepare(a.Q, a.nq, a.d, a.lp, ms->qlp, ms->qlpi, &kp,
                               st)) != hipSuccess)
      return e;
  }
  if (events) {
    record(p, 1, st);
    record(p, 2, st);
  }
  if ((e = mad::launch_fill_u64((uint64_t*)ms->hash.p, ms->hslots, 0ull,
                                st)) != hipSuccess ||
      (e = mad::launch_fill_u64((uint64_t*)ms->ctr.p, 8, 0ull, st)) !=
          hipSuccess)
    return e;
  if (events) record(p, 3, st);
  if ((e = mad::launch_sample_mips(a, ms->unroll, ms->grid, st)) != hipSuccess)
    return e;
  if (events) record(p, 4, st);
  if ((e = mad::launch_mips_post(a, st)) != hipSuccess) return e;
  if (events) record(p, 5, st);
  return hipSuccess;
}

static int mips_check_batch(mad_plan* p, const float* Q, int64_t nq,
                            const int64_t* s, const int64_t* tp, int64_t t,
                            mad_pair* out, int64_t* n_out) {
  if (!p) return fail(MAD_EINVAL, "plan is NULL");
  if (p->kind != 1) return fail(MAD_EINVAL, "not a MIPS plan");
  if (nq < 0 || nq >= (int64_t(1) << 31))
    return fail(MAD_EINVAL, "need 0 <= nq < 2^31");
  if (t < 1 || t > 1024 || t > p->m)
    return fail(MAD_EINVAL, "need 1 <= t <= min(1024, m)");
  if (nq == 0) return MAD_OK;
  if (!s || !tp) return fail(MAD_EINVAL, "budgets are required");
  if (!is_device_ptr(Q) || !is_device_ptr(out) || !is_device_ptr(n_out))
    return fail(MAD_EINVAL, "Q, out and n_out must be device pointers");
  for (int64_t q = 0; q < nq; ++q) {
    if (s[q] < 0 || s[q] >= (int64_t(1) << 31))
      return fail(MAD_EINVAL, "query %lld: need 0 <= s < 2^31", (long long)q);
    if (tp[q] < t)
      return fail(MAD_EINVAL, "query %lld: t' (%lld) < t (%lld)",
                  (long long)q, (long long)tp[q], (long long)t);
  }
  return MAD_OK;
}

int mips_topk_batch(mad_plan* p, const float* Q, int64_t nq,
                    const int64_t* s_per_query, const int64_t* tprime_per_query,
                    int64_t t, uint64_t seed, mad_pair* out, int64_t* n_out,
                    void* stream) {
  g_err.clear();
  int rc = mips_check_batch(p, Q, nq, s_per_query, tprime_per_query, t, out,
                            n_out);
  if (rc != MAD_OK || nq == 0) return rc;
  MipsState* ms = p->mips;
  hipStream_t st = (hipStream_t)stream;
  if ((rc = mips_prepare(p, nq, s_per_query, tprime_per_query, t)) != MAD_OK)
    return rc;
  if (p->verify_prec != MAD_FP32) {  // outside any capture: no allocation there
    const int64_t kc = p->verify_prec == MAD_BF16 ? 64 : 128;
    const int64_t eb = p->verify_prec == MAD_BF16 ? 2 : 1;
    const int64_t kp = (p->d + kc - 1) / kc * kc;
    HIP_TRY(mad::dev_alloc(ms->qlp, (size_t)(nq * kp * eb)), "query copies");
    HIP_TRY(mad::dev_alloc(ms->qlpi, (size_t)nq * sizeof(mad::VecInfo)),
            "query copies");
  }
  const mad::MipsArgs a = mips_args(p, Q, seed, out, n_out);
  ms->ran = true;
  if (p->flags & MAD_FLAG_TIMING) {  // eager, with phase events
    HIP_TRY(mips_enqueue(p, a, st, true), "MIPS batch");
    p->timed_tables = p->timed_topk = true;
    return MAD_OK;
  }
  const bool fresh = ms->exec && ms->g_Q == Q && ms->g_out == out &&
                     ms->g_nout == n_out && ms->g_seed == seed &&
                     ms->g_chunk == ms->chunk && ms->g_unroll == ms->unroll &&
                     ms->g_grid == ms->grid &&
                     ms->g_layout == ms->layout_version &&
                     ms->g_prec == p->verify_prec && ms->g_qlp == ms->qlp.p;
  if (!fresh) {
    mips_drop_graph(ms);
    HIP_TRY(hipStreamBeginCapture(ms->cap_stream,
                                  hipStreamCaptureModeThreadLocal),
            "capturing the MIPS batch");
    hipError_t e = mips_enqueue(p, a, ms->cap_stream, false);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(ms->cap_stream, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      return hip_fail(e != hipSuccess ? e : e2, "capturing the MIPS batch");
    }
    ms->graph = g;
    e = hipGraphInstantiate(&ms->exec, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      mips_drop_graph(ms);
      return hip_fail(e, "instantiating the MIPS graph");
    }
    ms->g_Q = Q;
    ms->g_out = out;
    ms->g_nout = n_out;
    ms->g_seed = seed;
    ms->g_chunk = ms->chunk;
    ms->g_unroll = ms->unroll;
    ms->g_grid = ms->grid;
    ms->g_layout = ms->layout_version;
    ms->g_prec = p->verify_prec;
    ms->g_qlp = ms->qlp.p;
  }
  HIP_TRY(hipGraphLaunch(ms->exec, st), "launching the MIPS graph");
  return MAD_OK;
}

int mips_get_config(mad_plan* p, int* chunk, int* unroll, int* grid) {
  if (!p || p->kind != 1) return fail(MAD_EINVAL, "not a MIPS plan");
  if (chunk) *chunk = p->mips->chunk;
  if (unroll) *unroll = p->mips->unroll;
  if (grid) *grid = p->mips->grid;
  return MAD_OK;
}

int mips_set_config(mad_plan* p, int chunk, int unroll, int grid) {
  if (!p || p->kind != 1) return fail(MAD_EINVAL, "not a MIPS plan");
  if (chunk < 256 || chunk > (1 << 24) || (chunk & 255))
    return fail(MAD_EINVAL, "chunk must be a multiple of 256 in [256, 2^24]");
  if (unroll != 1 && unroll != 2 && unroll != 4 && unroll != 8)
    return fail(MAD_EINVAL, "unroll must be 1, 2, 4 or 8");
  if (grid < 1 || grid > (1 << 20)) return fail(MAD_EINVAL, "bad grid");
  p->mips->chunk = chunk;
  p->mips->unroll = unroll;
  p->mips->grid = grid;
  return MAD_OK;
}

int mips_get_table_factor(mad_plan* p, int* slots_per_key) {
  if (!p || p->kind != 1) return fail(MAD_EINVAL, "not a MIPS plan");
  if (slots_per_key) *slots_per_key = p->mips->slots;
  return MAD_OK;
}

int mips_set_table_factor(mad_plan* p, int slots_per_key) {
  if (!p || p->kind != 1) return fail(MAD_EINVAL, "not a MIPS plan");
  if (slots_per_key != 2 && slots_per_key != 4 && slots_per_key != 8)
    return fail(MAD_EINVAL, "slots per key must be 2, 4 or 8");
  p->mips->slots = slots_per_key;
  return MAD_OK;
}

int mips_autotune_cache(mad_plan* p, const char* path) {
  if (!p || p->kind != 1) return fail(MAD_EINVAL, "not a MIPS plan");
  p->mips->tune_cache = path ? path : "";
  return MAD_OK;
}

int mips_autotune(mad_plan* p, const float* Q, int64_t nq,
                  const int64_t* s_per_query, const int64_t* tprime_per_query,
                  int64_t t, uint64_t seed, mad_pair* out, int64_t* n_out,
                  int reps, void* stream, double* best_ms) {
  int rc = mips_check_batch(p, Q, nq, s_per_query, tprime_per_query, t, out,
                            n_out);
  if (rc != MAD_OK) return rc;
  if (nq == 0) return MAD_OK;
  if (p->flags & MAD_FLAG_TIMING)
    return fail(MAD_EINVAL, "autotune needs a plan without MAD_FLAG_TIMING");
  if (reps < 1) reps = 1;
  hipStream_t st = (hipStream_t)stream;
  MipsState* ms = p->mips;
  std::string sig;
  if (!ms->tune_cache.empty()) {
    sig = tune_signature(p, nq, s_per_query, tprime_per_query, t);
    if (sig.empty()) return fail(MAD_EHIP, "autotune: device properties");
    TuneChoice c;
    if (tune_lookup(ms->tune_cache, sig, &c) &&
        mips_set_config(p, c.chunk, c.unroll, c.grid) == MAD_OK &&
        mips_set_table_factor(p, c.slots) == MAD_OK) {
      if (best_ms) *best_ms = c.ms;
      return MAD_OK;
    }
  }
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0), "autotune");
  HIP_TRY(hipEventCreate(&e1), "autotune");
  static const int chunks[] = {1024, 4096, 16384, 65536};
  static const int unrolls[] = {2, 4, 8};
  static const int grids[] = {1024, 2048, 4096};
  static const int factors[] = {2, 4};
  double best = 1e300;
  int bc = ms->chunk, bu = ms->unroll, bg = ms->grid, bf = ms->slots;
  auto trial = [&](int c, int u, int g, int f) -> int {
    ms->chunk = c;
    ms->unroll = u;
    ms->grid = g;
    ms->slots = f;
    int r = mips_topk_batch(p, Q, nq, s_per_query, tprime_per_query, t, seed,
                            out, n_out, stream);  // warm (and capture)
    if (r != MAD_OK) return r;
    HIP_TRY(hipEventRecord(e0, st), "autotune");
    for (int k = 0; k < reps; ++k)
      if ((r = mips_topk_batch(p, Q, nq, s_per_query, tprime_per_query, t,
                               seed, out, n_out, stream)) != MAD_OK)
        return r;
    HIP_TRY(hipEventRecord(e1, st), "autotune");
    HIP_TRY(hipEventSynchronize(e1), "autotune");
    float ms_ = 0.0f;
    HIP_TRY(hipEventElapsedTime(&ms_, e0, e1), "autotune");
    const double per = ms_ / reps;
    if (per < best) {
      best = per;
      bc = c;
      bu = u;
      bg = g;
      bf = f;
    }
    return MAD_OK;
  };
  // chunk and unroll at the default grid and table factor, then the grid,
  // then the table factor
  const int f0 = ms->slots;
  for (int c : chunks)
    for (int u : unrolls)
      if ((rc = trial(c, u, 2048, f0)) != MAD_OK) break;
  if (rc == MAD_OK)
    for (int g : grids)
      if (g != 2048 && (rc = trial(bc, bu, g, f0)) != MAD_OK) break;
  if (rc == MAD_OK)
    for (int f : factors)
      if (f != f0 && (rc = trial(bc, bu, bg, f)) != MAD_OK) break;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  ms->chunk = bc;
  ms->unroll = bu;
  ms->grid = bg;
  ms->slots = bf;
  if (rc != MAD_OK) return rc;
  if (best_ms) *best_ms = best;
  if (!sig.empty() &&
      !tune_append(ms->tune_cache, sig, TuneChoice{bc, bu, bg, bf, best}))
    return fail(MAD_EINVAL, "autotune: cannot append to %s",
                ms->tune_cache.c_str());
  return MAD_OK;
}

int mips_stats(mad_plan* p, int64_t* n_pos, int64_t* n_cand, int64_t* closed,
               int64_t* distinct) {
  if (!p || p->kind != 1) return fail(MAD_EINVAL, "not a MIPS plan");
  MipsState* ms = p->mips;
  if (!ms->ran) return fail(MAD_EINVAL, "no batch has run");
  HIP_TRY(hipDeviceSynchronize(), "MIPS stats");
  if (n_pos || n_cand) {
    std::vector<mad::MipsQueryStats> qs((size_t)ms->nq);
    HIP_TRY(hipMemcpy(qs.data(), ms->qstats.p, qs.size() * sizeof qs[0],
                      hipMemcpyDeviceToHost), "MIPS stats");
    for (int64_t q = 0; q < ms->nq; ++q) {
      if (n_pos) n_pos[q] = qs[(size_t)q].n_pos;
      if (n_cand) n_cand[q] = qs[(size_t)q].n_cand;
    }
  }
  mad::SampleCounters sc;
  HIP_TRY(hipMemcpy(&sc, ms->ctr.p, sizeof sc, hipMemcpyDeviceToHost),
          "MIPS stats");
  if (closed) *closed = (int64_t)sc.closed;
  if (distinct) *distinct = (int64_t)sc.distinct;
  return MAD_OK;
}

int mips_debug_scores(mad_plan* p, int64_t q, int64_t* keys, int64_t* xfix,
                      int64_t cap, int64_t* n, int* F) {
  if (!p || p->kind != 1 || !n) return fail(MAD_EINVAL, "MIPS plan and n are required");
  MipsState* ms = p->mips;
  if (!ms->ran) return fail(MAD_EINVAL, "no batch has run");
  if (q < 0 || q >= ms->nq) return fail(MAD_EINVAL, "query out of range");
  HIP_TRY(hipDeviceSynchronize(), "MIPS debug scores");
  const mad::MipsArgs a = mips_args(p, nullptr, 0, nullptr, nullptr);
  int64_t* cnt = (int64_t*)ms->ctr.p + 4;
  HIP_TRY(mad::launch_mips_dump(a, q, keys, xfix, keys ? cap : 0, cnt, 0),
          "MIPS debug scores");
  HIP_TRY(hipDeviceSynchronize(), "MIPS debug scores");
  int64_t total = 0;
  HIP_TRY(hipMemcpy(&total, cnt, 8, hipMemcpyDeviceToHost), "MIPS debug scores");
  *n = total;
  if (F) {
    mad::MipsQuery qi;
    HIP_TRY(hipMemcpy(&qi, (const mad::MipsQuery*)ms->qinfo.p + q, sizeof qi,
                      hipMemcpyDeviceToHost), "MIPS debug scores");
    *F = qi.F;
  }
  if (keys && total > cap) return fail(MAD_EOVERFLOW, "capacity too small");
  return MAD_OK;
}

}  // extern "C"
