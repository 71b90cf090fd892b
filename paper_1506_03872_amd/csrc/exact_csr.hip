// exact_csr.hip -- exhaustive t-MAD (Definition 1) for sparse inputs, the
// exact baseline of Sec. 5.3 for the sparse case.  The paper forms C one
// column at a time with a sparse product whose cost is the number of
// wedges (pairs of entries sharing a coordinate) and keeps a priority queue.
// On power-law inputs nearly all wedges meet at a few coordinates of huge
// degree, so here the coordinates are split in two:
//
//   heavy  the coordinates with the most wedges (deg_A(k) deg_B(k)); their
//          columns are copied into dense m x H and n x H matrices and every
//          pair's heavy part c^H_ij goes through the MFMA brute force;
//   light  the rest; their wedges (i, j, a_ik b_jk) are listed and summed
//          per pair, giving c^L_ij for the pairs P_L that share one.
//
// c_ij = c^H_ij outside P_L and c^H_ij + c^L_ij on it.  With tau_lb a
// lower bound on the t-th largest |c| (the exact values of the heavy part's
// own top-t candidates), the exact top t lies in
//   {pairs with |c^H| >= tau_lb}          (the certified brute-force filter)
//   {pairs of P_L whose bound |c^L| + ||a_i^H|| ||b_j^H|| >= tau_lb}
// whose union is re-ranked with sparse dot products of the candidates.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>
#include <numeric>
#include <vector>

#include "mad_common.hpp"
#include "plan.hpp"

namespace mad {

constexpr int64_t kMaxLightWedges = int64_t(1) << 30;
constexpr int64_t kMaxHeavy = 4096;
constexpr int kWedgeSteps = 32;  // wedges per lane of the listing kernel

__global__ void k_coord_degrees(const int32_t* idx, int64_t nnz,
                                uint32_t* deg) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz;
       e += stride)
    atomicAdd(&deg[idx[e]], 1u);
}

// one thread per vector: its heavy entries into column pos[k] of a dense
// row (zero-filled before), and the L2 norms of its heavy and of its light
// entries, rounded up
__global__ void k_split_rows(const int64_t* ptr, const int32_t* idx,
                             const float* val, int64_t rows,
                             const int32_t* pos, int64_t H, float* dense,
                             float* nh, float* nl) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  double sh = 0.0, sl = 0.0;
  for (int64_t e = ptr[r]; e < ptr[r + 1]; ++e) {
    const float v = val[e];
    const int32_t p = pos[idx[e]];
    if (p >= 0) {
      dense[r * H + p] = v;
      sh += (double)v * v;
    } else {
      sl += (double)v * v;
    }
  }
  nh[r] = (float)(sqrt(sh) * (1.0 + 1e-6));
  nl[r] = (float)(sqrt(sl) * (1.0 + 1e-6));
}

// the light coordinates' lists of vectors (any order inside a list)
__global__ void k_light_lists(const int64_t* ptr, const int32_t* idx,
                              const float* val, int64_t rows,
                              const int32_t* pos, const int64_t* tptr,
                              uint32_t* cur, uint32_t* trow, float* tval) {
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= rows) return;
  for (int64_t e = ptr[r]; e < ptr[r + 1]; ++e) {
    const int32_t k = idx[e];
    if (pos[k] >= 0) continue;
    const int64_t p = tptr[k] + atomicAdd(&cur[k], 1u);
    trow[p] = (uint32_t)r;
    tval[p] = val[e];
  }
}

// every light wedge: wedge w of light coordinate lk[q] (wpre[q] <= w <
// wpre[q+1]) pairs entry w' / deg_B of A's list with entry w' % deg_B of
// B's list, w' = w - wpre[q]; key i*n + j, value a_ik b_jk (fp32).  A wave
// takes 64 * kWedgeSteps consecutive wedges, lane l every 64th from l.
__global__ __launch_bounds__(256) void k_light_wedges(
    const int32_t* lk, const int64_t* wpre, int64_t nl, int64_t W,
    const int64_t* taptr, const uint32_t* tarow, const float* taval,
    const int64_t* tbptr, const uint32_t* tbrow, const float* tbval,
    int64_t n, uint64_t* keys, float* vals) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t nwaves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  for (int64_t w0 = wave * 64 * kWedgeSteps; w0 < W;
       w0 += nwaves * 64 * kWedgeSteps) {
    int64_t w = w0 + lane;
    if (w >= W) continue;
    // the list holding wedge w: last q with wpre[q] <= w
    int64_t lo = 0, hi = nl;  // wpre[lo] <= w < wpre[hi]
    while (hi - lo > 1) {
      const int64_t mid = (lo + hi) >> 1;
      if (wpre[mid] <= w) lo = mid; else hi = mid;
    }
    int64_t q = lo;
    for (int s = 0; s < kWedgeSteps && w < W; ++s, w += 64) {
      while (wpre[q + 1] <= w) ++q;
      const int32_t k = lk[q];
      const int64_t db = tbptr[k + 1] - tbptr[k];
      const int64_t loc = w - wpre[q];
      const int64_t ia = loc / db, jb = loc - ia * db;
      const int64_t pa = taptr[k] + ia, pb = tbptr[k] + jb;
      keys[w] = (uint64_t)tarow[pa] * (uint64_t)n + tbrow[pb];
      vals[w] = taval[pa] * tbval[pb];
    }
  }
}

// pairs of P_L that may reach tau: |c^L| (with its rounding) plus the bound
// ||a_i^H|| ||b_j^H|| on the heavy part
__global__ void k_light_prune(const uint64_t* okey, const int64_t* oval,
                              const int64_t* len, int F, double wslack,
                              int64_t n, const float* nha, const float* nla,
                              const float* nhb, const float* nlb, float tau,
                              uint64_t* out, unsigned long long* cnt,
                              int64_t cap) {
  const int64_t L = *len;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < L;
       e += stride) {
    const uint64_t key = okey[e];
    if (key == kEmptyKey) continue;
    const int64_t i = (int64_t)(key / (uint64_t)n);
    const int64_t j = (int64_t)(key - (uint64_t)i * (uint64_t)n);
    const double x = fabs(ldexp((double)oval[e], -F));
    // fp32 products err by at most 2^-24 of sum |a_ik b_jk| <= ||a^L||
    // ||b^L||, the fixed-point sum by 2^-F per wedge (wslack = W 2^-F
    // bounds them all), the heavy part by ||a^H|| ||b^H||
    const double ub = x + 1e-5 * (double)nla[i] * nlb[j] + wslack +
                      (double)nha[i] * nhb[j] * (1.0 + 1e-5);
    if (ub >= (double)tau) {
      const unsigned long long p = atomicAdd(cnt, 1ull);
      if ((int64_t)p < cap) out[p] = key;
    }
  }
}

static unsigned grid_of(int64_t n, int per, unsigned cap) {
  int64_t g = (n + per - 1) / per;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (unsigned)g;
}

struct ExactWork {
  DeviceBuffer deg, pos, ah, bh, norms, lk, wpre, tptr, cur, tlist, pairs,
      acc, tab, cand, fin, misc;
};
static ExactWork g_ex;

hipError_t bruteforce_topk_csr(const CsrView& in, int64_t m, int64_t n,
                               int64_t d, int64_t nnzA, int64_t nnzB,
                               int prec, int64_t t, int64_t heavy_req,
                               void* out, int64_t* n_out, BfCsrStats* stats,
                               hipStream_t st) {
  hipError_t e;
  ExactWork& w = g_ex;
  struct Events {  // destroyed on every return
    hipEvent_t ev[5] = {};
    Events() {
      for (auto& x : ev) (void)hipEventCreate(&x);
    }
    ~Events() {
      for (auto& x : ev)
        if (x) (void)hipEventDestroy(x);
    }
  } evs;
  hipEvent_t* ev = evs.ev;
  (void)hipEventRecord(ev[0], st);
  // ---- coordinate degrees and the heavy / light split (host) -------------
  if ((e = dev_alloc(w.deg, 8 * (size_t)d + 256)) != hipSuccess) return e;
  uint32_t* dA = (uint32_t*)w.deg.p;
  uint32_t* dB = dA + d;
  if ((e = launch_fill_u64((uint64_t*)dA, d, 0ull, st)) != hipSuccess)
    return e;
  k_coord_degrees<<<grid_of(nnzA, 256 * 16, 4096), 256, 0, st>>>(in.a_idx,
                                                                 nnzA, dA);
  k_coord_degrees<<<grid_of(nnzB, 256 * 16, 4096), 256, 0, st>>>(in.b_idx,
                                                                 nnzB, dB);
  std::vector<uint32_t> hd(2 * (size_t)d);
  if ((e = hipMemcpyAsync(hd.data(), dA, 8 * (size_t)d,
                          hipMemcpyDeviceToHost, st)) != hipSuccess ||
      (e = hipStreamSynchronize(st)) != hipSuccess)
    return e;
  std::vector<double> wk((size_t)d);
  double total = 0.0;
  for (int64_t k = 0; k < d; ++k) {
    wk[k] = (double)hd[k] * (double)hd[d + k];
    total += wk[k];
  }
  std::vector<int32_t> order((size_t)d);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(),
                   [&](int32_t x, int32_t y) { return wk[x] > wk[y]; });
  int64_t live = 0;
  while (live < d && wk[order[live]] > 0.0) ++live;
  if (live == 0) {  // no coordinate is shared: every c_ij is 0
    if (stats) memset(stats, 0, sizeof *stats);
    return launch_fill_u64((uint64_t*)n_out, 1, 0ull, st);
  }
  int64_t H;
  if (heavy_req > 0) {
    H = heavy_req < live ? heavy_req : live;
  } else {
    // the fewest heavy coordinates (a multiple of 64) that leave at most
    // kMaxLightWedges light wedges
    H = 0;
    double light = total;
    while (H < live && (light > (double)kMaxLightWedges || H % 64 != 0)) {
      light -= wk[order[H]];
      ++H;
    }
  }
  if (H < 1 && live > 0) H = 1;
  if (H > kMaxHeavy) return hipErrorNotSupported;
  std::vector<int32_t> pos((size_t)d, -1);
  for (int64_t h = 0; h < H; ++h) pos[order[h]] = (int32_t)h;
  // light lists: pointer of each coordinate's list, the light coordinates
  // with wedges, and their wedge prefix
  std::vector<int64_t> taptr((size_t)d + 1, 0), tbptr((size_t)d + 1, 0);
  std::vector<int32_t> lk;
  std::vector<int64_t> wpre(1, 0);
  for (int64_t k = 0; k < d; ++k) {
    const bool light = pos[k] < 0;
    taptr[k + 1] = taptr[k] + (light ? hd[k] : 0);
    tbptr[k + 1] = tbptr[k] + (light ? hd[d + k] : 0);
    if (light && wk[k] > 0.0) {
      lk.push_back((int32_t)k);
      wpre.push_back(wpre.back() + (int64_t)hd[k] * (int64_t)hd[d + k]);
    }
  }
  const int64_t W = wpre.back();
  const int64_t nl = (int64_t)lk.size();
  if (W > kMaxLightWedges) return hipErrorNotSupported;
  // ---- device copies of the split -----------------------------------------
  const int64_t Hc = H > 0 ? H : 1;
  if ((e = dev_alloc(w.pos, 4 * (size_t)d)) != hipSuccess ||
      (e = dev_alloc(w.ah, 4 * (size_t)m * Hc)) != hipSuccess ||
      (e = dev_alloc(w.bh, 4 * (size_t)n * Hc)) != hipSuccess ||
      (e = dev_alloc(w.norms, 8 * (size_t)(m + n) + 256)) != hipSuccess ||
      (e = dev_alloc(w.tptr, 16 * (size_t)(d + 1))) != hipSuccess ||
      (e = dev_alloc(w.cur, 8 * (size_t)d + 256)) != hipSuccess ||
      (e = dev_alloc(w.lk, 4 * (size_t)(nl + 1))) != hipSuccess ||
      (e = dev_alloc(w.wpre, 8 * (size_t)(nl + 2))) != hipSuccess ||
      (e = dev_alloc(w.tlist, 8 * (size_t)(taptr[d] + tbptr[d] + 2))) !=
          hipSuccess ||
      (e = dev_alloc(w.misc, 4096)) != hipSuccess)
    return e;
  int32_t* dpos = (int32_t*)w.pos.p;
  float* nha = (float*)w.norms.p;
  float* nla = nha + m;
  float* nhb = nla + m;
  float* nlb = nhb + n;
  int64_t* dtaptr = (int64_t*)w.tptr.p;
  int64_t* dtbptr = dtaptr + d + 1;
  uint32_t* curA = (uint32_t*)w.cur.p;
  uint32_t* curB = curA + d;
  uint32_t* tarow = (uint32_t*)w.tlist.p;
  float* taval = (float*)(tarow + taptr[d]);
  uint32_t* tbrow = (uint32_t*)(taval + taptr[d]);
  float* tbval = (float*)(tbrow + tbptr[d]);
  wpre.push_back(wpre.back());  // sentinel: wpre[nl + 1] = W
  if ((e = hipMemcpyAsync(dpos, pos.data(), 4 * (size_t)d,
                          hipMemcpyHostToDevice, st)) != hipSuccess ||
      (e = hipMemcpyAsync(dtaptr, taptr.data(), 8 * (size_t)(d + 1),
                          hipMemcpyHostToDevice, st)) != hipSuccess ||
      (e = hipMemcpyAsync(dtbptr, tbptr.data(), 8 * (size_t)(d + 1),
                          hipMemcpyHostToDevice, st)) != hipSuccess ||
      (nl > 0 &&
       (e = hipMemcpyAsync(w.lk.p, lk.data(), 4 * (size_t)nl,
                           hipMemcpyHostToDevice, st)) != hipSuccess) ||
      (e = hipMemcpyAsync(w.wpre.p, wpre.data(), 8 * (size_t)(nl + 2),
                          hipMemcpyHostToDevice, st)) != hipSuccess)
    return e;
  if ((e = launch_fill_u64((uint64_t*)w.ah.p, ((int64_t)m * Hc + 1) / 2, 0ull,
                           st)) != hipSuccess ||
      (e = launch_fill_u64((uint64_t*)w.bh.p, ((int64_t)n * Hc + 1) / 2, 0ull,
                           st)) != hipSuccess ||
      (e = launch_fill_u64((uint64_t*)curA, d, 0ull, st)) != hipSuccess)
    return e;
  k_split_rows<<<grid_of(m, 256, 1u << 30), 256, 0, st>>>(
      in.a_ptr, in.a_idx, in.a_val, m, dpos, Hc, (float*)w.ah.p, nha, nla);
  k_split_rows<<<grid_of(n, 256, 1u << 30), 256, 0, st>>>(
      in.b_ptr, in.b_idx, in.b_val, n, dpos, Hc, (float*)w.bh.p, nhb, nlb);
  k_light_lists<<<grid_of(m, 256, 1u << 30), 256, 0, st>>>(
      in.a_ptr, in.a_idx, in.a_val, m, dpos, dtaptr, curA, tarow, taval);
  k_light_lists<<<grid_of(n, 256, 1u << 30), 256, 0, st>>>(
      in.b_ptr, in.b_idx, in.b_val, n, dpos, dtbptr, curB, tbrow, tbval);
  (void)hipEventRecord(ev[1], st);
  // ---- heavy part: certified brute force, then tau_lb ---------------------
  // tau_lb = the t-th largest exact |c| among the candidates of the heavy
  // part's own top t (each is a real pair, so t of them reach it)
  const uint64_t* ck = nullptr;
  int64_t cc = 0;
  BfStats bs;
  memset(&bs, 0, sizeof bs);
  const float* AH = (const float*)w.ah.p;
  const float* BH = (const float*)w.bh.p;
  if ((e = bruteforce_run(AH, m, BH, n, Hc, prec, t, 0, -1.0f, nullptr,
                          nullptr, &ck, &cc, &bs, st)) != hipSuccess)
    return e;
  int64_t* dn = (int64_t*)w.misc.p;
  std::vector<char> tmp((size_t)t * 24);
  if ((e = dev_alloc(w.cand, 24 * (size_t)(t > 1 ? t : 1))) != hipSuccess)
    return e;
  float tau_lb = 0.0f;
  if (cc > 0) {
    if ((e = launch_rerank_topk(ck, cc, nullptr, nullptr, n, 0,
                                t < cc ? t : cc, w.fin, w.cand.p, dn, &in,
                                st)) != hipSuccess)
      return e;
    int64_t got = 0;
    if ((e = hipMemcpyAsync(&got, dn, 8, hipMemcpyDeviceToHost, st)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
      return e;
    if (got >= t) {
      if ((e = hipMemcpy(tmp.data(), w.cand.p, 24 * (size_t)t,
                         hipMemcpyDeviceToHost)) != hipSuccess)
        return e;
      float c;
      memcpy(&c, tmp.data() + 24 * (size_t)(t - 1) + 16, 4);
      tau_lb = fabsf(c);
    }
  }
  // pass B again only when tau_lb is below the threshold it ran with
  const float tau_use = tau_lb * (1.0f - 1e-5f);
  if (tau_use < bs.tau) {
    const float tu = tau_use > 0.0f ? tau_use : 1e-30f;
    if ((e = bruteforce_run(AH, m, BH, n, Hc, prec, t, 0, tu, nullptr,
                            nullptr, &ck, &cc, &bs, st)) != hipSuccess)
      return e;
  }
  const int64_t heavy_cand = cc;
  (void)hipEventRecord(ev[2], st);
  // ---- light part: its wedges summed per pair, then the bound ------------
  int64_t light_cand = 0;
  const size_t pk = 8 * (size_t)(W > 1 ? W : 1);
  const size_t pv = (4 * (size_t)(W > 1 ? W : 1) + 255) / 256 * 256;
  // candidates: heavy survivors, then light survivors (cap: W or 2^27)
  const int64_t lcap = W < (int64_t(1) << 27) ? W : (int64_t(1) << 27);
  const int64_t ccap = heavy_cand + lcap + 1;
  if ((e = dev_alloc(w.tab, 8 * (size_t)ccap + (4 * (size_t)ccap + 255) /
                                                   256 * 256 +
                                16 * (size_t)ccap + 256 +
                                accum_bytes(ccap))) != hipSuccess)
    return e;
  uint64_t* ukeys = (uint64_t*)w.tab.p;
  float* uvals = (float*)((char*)w.tab.p + 8 * (size_t)ccap);
  char* tail = (char*)uvals + (4 * (size_t)ccap + 255) / 256 * 256;
  uint64_t* dkeys = (uint64_t*)tail;
  int64_t* dx = (int64_t*)(dkeys + ccap);
  int64_t* dcnt = (int64_t*)(dx + ccap);
  char* uwork = (char*)(dcnt + 32);
  if (heavy_cand > 0 &&
      (e = hipMemcpyAsync(ukeys, ck, 8 * (size_t)heavy_cand,
                          hipMemcpyDeviceToDevice, st)) != hipSuccess)
    return e;
  if (W > 0) {
    if ((e = dev_alloc(w.pairs, pk + pv)) != hipSuccess ||
        (e = dev_alloc(w.acc, 16 * (size_t)W + 256 + accum_bytes(W))) !=
            hipSuccess)
      return e;
    uint64_t* lkeys = (uint64_t*)w.pairs.p;
    float* lvals = (float*)((char*)w.pairs.p + pk);
    const int64_t per_wave = 64 * kWedgeSteps;
    k_light_wedges<<<grid_of((W + per_wave - 1) / per_wave, 4, 1u << 20), 256,
                     0, st>>>((const int32_t*)w.lk.p,
                              (const int64_t*)w.wpre.p, nl, W, dtaptr, tarow,
                              taval, dtbptr, tbrow, tbval, n, lkeys, lvals);
    // fixed point: |products| < 2^(ea + eb), at most W of them per pair
    float amax = 0.0f, bmax = 0.0f;
    {  // max |a|, |b| on the host from the lists (light entries only)
      std::vector<float> va((size_t)taptr[d]), vb((size_t)tbptr[d]);
      if ((taptr[d] &&
           (e = hipMemcpyAsync(va.data(), taval, 4 * (size_t)taptr[d],
                               hipMemcpyDeviceToHost, st)) != hipSuccess) ||
          (tbptr[d] &&
           (e = hipMemcpyAsync(vb.data(), tbval, 4 * (size_t)tbptr[d],
                               hipMemcpyDeviceToHost, st)) != hipSuccess) ||
          (e = hipStreamSynchronize(st)) != hipSuccess)
        return e;
      for (float v : va) amax = fmaxf(amax, fabsf(v));
      for (float v : vb) bmax = fmaxf(bmax, fabsf(v));
    }
    int ea = 0, eb = 0, lw = 0;
    (void)frexpf(amax, &ea);
    (void)frexpf(bmax, &eb);
    while ((int64_t(1) << lw) < W) ++lw;
    const int F = 62 - ea - eb - lw;
    uint64_t* okey = (uint64_t*)w.acc.p;
    int64_t* oval = (int64_t*)(okey + W);
    int64_t* lcnt = (int64_t*)(oval + W);
    char* awork = (char*)(lcnt + 32);
    if ((e = launch_accumulate(lkeys, lvals, W, nullptr, F, awork,
                               accum_bytes(W), okey, oval, lcnt, lcnt + 1,
                               st)) != hipSuccess)
      return e;
    unsigned long long* ucnt = (unsigned long long*)(lcnt + 2);
    if ((e = launch_fill_u64((uint64_t*)ucnt, 1, 0ull, st)) != hipSuccess)
      return e;
    k_light_prune<<<grid_of(W, 256 * 8, 8192), 256, 0, st>>>(
        okey, oval, lcnt + 1, F, ldexp((double)W, -F), n, nha, nla, nhb,
        nlb, tau_use,
        ukeys + heavy_cand, ucnt, lcap);
    unsigned long long got = 0;
    if ((e = hipMemcpyAsync(&got, ucnt, 8, hipMemcpyDeviceToHost, st)) !=
            hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
      return e;
    if ((int64_t)got > lcap) return hipErrorOutOfMemory;
    light_cand = (int64_t)got;
  }
  (void)hipEventRecord(ev[3], st);
  // ---- union without repeats, exact dot products, top t --------------------
  const int64_t nu = heavy_cand + light_cand;
  int64_t distinct = 0;
  if (nu > 0) {
    if ((e = launch_fill_u64((uint64_t*)uvals, (nu + 1) / 2, 0ull, st)) !=
        hipSuccess)
      return e;
    if ((e = launch_accumulate(ukeys, uvals, nu, nullptr, 0, uwork,
                               accum_bytes(ccap), dkeys, dx, dcnt, dcnt + 1,
                               st)) != hipSuccess)
      return e;
    HashTable hsel;
    hsel.keys = dkeys;
    hsel.vals = dx;
    hsel.cap = nu;
    hsel.live = dcnt + 1;
    // the distinct keys to the front of ukeys
    if ((e = launch_dump_scores(hsel, (int64_t*)ukeys, (int64_t*)uwork, nu,
                                dcnt + 2, st)) != hipSuccess)
      return e;
    if ((e = hipMemcpyAsync(&distinct, dcnt + 2, 8, hipMemcpyDeviceToHost,
                            st)) != hipSuccess ||
        (e = hipStreamSynchronize(st)) != hipSuccess)
      return e;
  }
  if (distinct > 0) {
    if ((e = launch_rerank_topk(ukeys, distinct, nullptr, nullptr, n, 0,
                                t < distinct ? t : distinct, w.fin, out, n_out,
                                &in, st)) != hipSuccess)
      return e;
  } else {
    if ((e = launch_fill_u64((uint64_t*)n_out, 1, 0ull, st)) != hipSuccess)
      return e;
  }
  (void)hipEventRecord(ev[4], st);
  if ((e = hipEventSynchronize(ev[4])) != hipSuccess) return e;
  if (stats) {
    float f;
    (void)hipEventElapsedTime(&f, ev[0], ev[1]);
    stats->ms_split = f;
    (void)hipEventElapsedTime(&f, ev[1], ev[2]);
    stats->ms_heavy = f;
    (void)hipEventElapsedTime(&f, ev[2], ev[3]);
    stats->ms_light = f;
    (void)hipEventElapsedTime(&f, ev[3], ev[4]);
    stats->ms_final = f;
    stats->heavy = H;
    stats->wedges = (int64_t)total;
    stats->light_wedges = W;
    stats->heavy_candidates = heavy_cand;
    stats->light_candidates = light_cand;
    stats->candidates = distinct;
    stats->tau = tau_use;
  }
  return hipSuccess;
}

}  // namespace mad
