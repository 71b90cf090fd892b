// capi.hip -- the C ABI (include/mad.h): argument checks, plan lifetime,
// workspace management and the launch sequence of Alg. 2 + Alg. 3.
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <new>
#include <string>

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

struct mad_plan {
  int kind = 0;  // 0 dense
  const float* A = nullptr;
  const float* B = nullptr;
  int64_t m = 0, n = 0, d = 0;
  uint32_t flags = 0;
  mad::DenseTables dt;
  mad::DeviceBuffer build;
  // workspace of mad_plan_topk
  mad::DeviceBuffer hk, hv, cx, ck, cx2, ck2, cc, misc;
  mad::HashTable h;
  mad::SelectWork w;
  mad::SampleCounters* ctr = nullptr;
  int64_t ws_s = -1, ws_tp = -1, ws_t = -1;
  // last run
  int64_t last_s = -1;
  bool ran = false;
  // phase events (MAD_FLAG_TIMING): 0 tables start, 1 tables end, 2 clear
  // start, 3 sampler start, 4 sampler end, 5 postprocessing end
  hipEvent_t ev[6] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  bool timed_tables = false, timed_topk = false;
};

static void record(mad_plan* p, int idx, hipStream_t st) {
  if (p->ev[idx]) (void)hipEventRecord(p->ev[idx], st);
}

static void plan_free_all(mad_plan* p) {
  mad::dense_tables_free(p->dt);
  mad::dev_free(p->build);
  mad::dev_free(p->hk);
  mad::dev_free(p->hv);
  mad::dev_free(p->cx);
  mad::dev_free(p->ck);
  mad::dev_free(p->cx2);
  mad::dev_free(p->ck2);
  mad::dev_free(p->cc);
  mad::dev_free(p->misc);
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
  mad_plan* p = new (std::nothrow) mad_plan();
  if (!p) return fail(MAD_ENOMEM, "host allocation failed");
  p->kind = 0;
  p->A = A;
  p->B = B;
  p->m = m;
  p->n = n;
  p->d = d;
  p->flags = flags;
  hipError_t e = mad::dense_tables_alloc(p->dt, m, n, d);
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
  HIP_TRY(mad::dense_tables_build(p->dt, p->A, p->B, check, p->build, st),
          "building tables");
  record(p, 1, st);
  p->timed_tables = p->ev[0] != nullptr;
  p->ran = false;
  return check_bad_inputs(p, st);
}

void mad_plan_destroy(mad_plan* p) {
  if (!p) return;
  (void)hipDeviceSynchronize();
  plan_free_all(p);
  delete p;
}

static int ensure_workspace(mad_plan* p, int64_t s, int64_t tp, int64_t t) {
  if (s <= p->ws_s && tp <= p->ws_tp && t <= p->ws_t) return MAD_OK;
  const int64_t s2 = s > p->ws_s ? s : p->ws_s;
  const int64_t tp2 = tp > p->ws_tp ? tp : p->ws_tp;
  const int64_t t2 = t > p->ws_t ? t : p->ws_t;
  const double mn = (double)p->m * (double)p->n;
  const int64_t pairs = (double)s2 < mn ? s2 : (int64_t)mn;
  int64_t hcap = next_pow2(2 * (pairs > 512 ? pairs : 512));
  // candidates / boundary lists: post1 needs |Omega_s| <= pairs entries,
  // post3 needs 4 t (final set) + 4 t' (boundary of the candidates)
  int64_t ccap = pairs > 1 ? pairs : 1;
  if (ccap < 4 * t2 + 4 * tp2) ccap = 4 * t2 + 4 * tp2;
  const int64_t ccap2 = tp2 > 1 ? tp2 : 1;
  (void)hipDeviceSynchronize();
  hipError_t e;
  if ((e = mad::dev_alloc(p->hk, 8 * (size_t)hcap)) != hipSuccess ||
      (e = mad::dev_alloc(p->hv, 8 * (size_t)hcap)) != hipSuccess ||
      (e = mad::dev_alloc(p->cx, 8 * (size_t)ccap)) != hipSuccess ||
      (e = mad::dev_alloc(p->ck, 8 * (size_t)ccap)) != hipSuccess ||
      (e = mad::dev_alloc(p->cx2, 8 * (size_t)ccap2)) != hipSuccess ||
      (e = mad::dev_alloc(p->ck2, 8 * (size_t)ccap2)) != hipSuccess ||
      (e = mad::dev_alloc(p->cc, 4 * (size_t)ccap2)) != hipSuccess ||
      (e = mad::dev_alloc(p->misc, mad::kSelStateBytes + 4 * mad::kSelBins +
                                       256 + 256)) != hipSuccess) {
    p->ws_s = p->ws_tp = p->ws_t = -1;
    return hip_fail(e, "allocating workspace");
  }
  p->h.keys = (uint64_t*)p->hk.p;
  p->h.vals = (int64_t*)p->hv.p;
  p->h.cap = hcap;
  p->w.x = (uint64_t*)p->cx.p;
  p->w.key = (uint64_t*)p->ck.p;
  p->w.x2 = (uint64_t*)p->cx2.p;
  p->w.key2 = (uint64_t*)p->ck2.p;
  p->w.c = (float*)p->cc.p;
  p->w.cap = ccap;
  p->w.cap2 = ccap2;
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
  HIP_TRY(mad::launch_fill_u64(p->h.keys, p->h.cap, mad::kEmptyKey, st),
          "clearing X");
  HIP_TRY(mad::launch_fill_u64((uint64_t*)p->h.vals, p->h.cap, 0ull, st),
          "clearing X");
  HIP_TRY(mad::launch_fill_u64((uint64_t*)p->ctr, 8, 0ull, st),
          "clearing counters");
  record(p, 3, st);
  HIP_TRY(mad::launch_sample_dense(p->dt, p->B, seed, 0, 0, s, s, p->h,
                                   p->ctr, st),
          "sampling");
  record(p, 4, st);
  HIP_TRY(mad::launch_postprocess(p->h, p->A, p->B, p->n, p->d, tp_eff, t,
                                  p->dt.bmax, s, p->w, out, n_out, st),
          "postprocessing");
  record(p, 5, st);
  p->timed_topk = p->ev[0] != nullptr;
  p->last_s = s;
  p->ran = true;
  return MAD_OK;
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
  HIP_TRY(hipDeviceSynchronize(), "stats");
  if (wnorm)
    HIP_TRY(hipMemcpy(wnorm, p->dt.T0.tot, sizeof(double),
                      hipMemcpyDeviceToHost), "stats");
  int64_t cnt[4] = {0, 0, 0, 0};
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
  if (n_cand) *n_cand = cnt[mad::kCountCand];
  return MAD_OK;
}

int mad_plan_phase_ms(mad_plan* p, double* ms, int n) {
  if (!p || !ms) return fail(MAD_EINVAL, "plan and ms are required");
  if (!p->ev[0]) return fail(MAD_EINVAL, "plan was made without MAD_FLAG_TIMING");
  const int pairs[4][2] = {{0, 1}, {3, 4}, {4, 5}, {2, 3}};
  const bool have[4] = {p->timed_tables, p->timed_topk, p->timed_topk,
                        p->timed_topk};
  const hipEvent_t last = p->timed_topk ? p->ev[5] : p->ev[1];
  HIP_TRY(hipEventSynchronize(last), "phase timing");
  for (int q = 0; q < n && q < 4; ++q) {
    ms[q] = -1.0;
    if (!have[q]) continue;
    float f = 0.0f;
    HIP_TRY(hipEventElapsedTime(&f, p->ev[pairs[q][0]], p->ev[pairs[q][1]]),
            "phase timing");
    ms[q] = f;
  }
  return MAD_OK;
}

int mad_fix_exponent(mad_plan* p, int64_t s, int* F) {
  if (!p || !F) return fail(MAD_EINVAL, "plan and F are required");
  float bmax = 0.0f;
  HIP_TRY(hipDeviceSynchronize(), "fix exponent");
  HIP_TRY(hipMemcpy(&bmax, p->dt.bmax, sizeof(float), hipMemcpyDeviceToHost),
          "fix exponent");
  *F = mad::fix_exponent(bmax, s);
  return MAD_OK;
}

int mad_debug_table(mad_plan* p, int which, int64_t idx, uint32_t* thr,
                    uint32_t* alias, int32_t* item, int64_t cap,
                    int64_t* nslots) {
  if (!p) return fail(MAD_EINVAL, "plan is NULL");
  const mad::Family* f;
  switch (which) {
    case 0: f = &p->dt.T0; idx = 0; break;
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
  HIP_TRY(mad::launch_sample_dense_debug(p->dt, p->B, seed, qid, l0, count, F,
                                         k, i, j, kp, inc, st),
          "debug samples");
  HIP_TRY(hipStreamSynchronize(st), "debug samples");
  return MAD_OK;
}

int mad_debug_scores(mad_plan* p, int64_t* keys, int64_t* xfix, int64_t cap,
                     int64_t* n, int* F) {
  if (!p || !n) return fail(MAD_EINVAL, "plan and n are required");
  if (!p->ran) return fail(MAD_EINVAL, "no mad_plan_topk has run");
  int64_t* cnt = p->w.counts + 6;
  HIP_TRY(mad::launch_dump_scores(p->h, keys, xfix, keys ? cap : 0, cnt, 0),
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

int mad_plan_create_csr(const int64_t*, const int32_t*, const float*, int64_t,
                        const int64_t*, const int32_t*, const float*, int64_t,
                        int64_t, uint32_t, void*, mad_plan** plan) {
  if (plan) *plan = nullptr;
  return fail(MAD_EUNSUPPORTED, "sparse plans are not built yet");
}

}  // extern "C"
