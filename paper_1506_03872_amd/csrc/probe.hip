// probe.hip -- measurement kernels for the ceilings the sampler and the
// score table run against: random 8- and 4-byte loads, random 64-bit atomic
// adds and compare-and-swaps, a compare-and-swap followed by an add (one
// score-table insert of a new key), and a streaming copy.  Addresses come
// from mix64 of the operation index, uniformly over the buffer.
#include "../../include/mad.h"
#include "mad_common.hpp"
#include "plan.hpp"

namespace mad {

template <int KIND>
__global__ __launch_bounds__(256) void k_probe(uint64_t* buf, int64_t nwords,
                                               int64_t nops, uint64_t seed,
                                               uint64_t* sink) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const uint64_t mask = (uint64_t)nwords - 1;  // nwords is a power of two
  uint64_t acc = 0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nops;
       e += 4 * stride) {
    uint64_t h[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) h[u] = mix64((uint64_t)(e + u * stride) ^ seed);
    bool live[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) live[u] = e + u * stride < nops;
    if (KIND == 0) {  // random 8-byte loads
      uint64_t v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) v[u] = live[u] ? buf[h[u] & mask] : 0;
#pragma unroll
      for (int u = 0; u < 4; ++u) acc += v[u];
    } else if (KIND == 1) {  // random 4-byte loads
      const uint32_t* b32 = (const uint32_t*)buf;
      uint32_t v[4];
#pragma unroll
      for (int u = 0; u < 4; ++u)
        v[u] = live[u] ? b32[h[u] & (2 * mask + 1)] : 0;
#pragma unroll
      for (int u = 0; u < 4; ++u) acc += v[u];
    } else if (KIND == 2) {  // random 64-bit atomic add, no return
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (live[u])
          atomicAdd((unsigned long long*)&buf[h[u] & mask], 1ull);
    } else if (KIND == 3) {  // random 64-bit compare-and-swap, returned
#pragma unroll
      for (int u = 0; u < 4; ++u)
        if (live[u])
          acc += atomicCAS((unsigned long long*)&buf[h[u] & mask], 0ull,
                           (unsigned long long)h[u]);
    } else if (KIND == 4) {  // CAS on a 16-byte entry's key, then add
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (!live[u]) continue;
        const uint64_t slot = (h[u] & mask) & ~1ull;
        const uint64_t prev = atomicCAS((unsigned long long*)&buf[slot],
                                        0ull, (unsigned long long)h[u]);
        atomicAdd((unsigned long long*)&buf[slot + 1], prev + 1);
      }
    } else {  // streaming copy of the first half onto the second half
      const int64_t half = nwords / 2;
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        const int64_t w = e + u * stride;
        if (live[u] && w < half) buf[half + w] = buf[w];
      }
    }
  }
  if (acc == 0x5DEECE66Dull) *sink = acc;  // keeps the loads alive
}

}  // namespace mad

extern "C" int mad_probe_memory(int kind, void* buf, int64_t nwords,
                                int64_t nops, uint64_t seed, void* stream) {
  if (!buf || nwords < 2 || (nwords & (nwords - 1)) || nops < 0 || kind < 0 ||
      kind > 5)
    return MAD_EINVAL;
  if (kind == 5 && nops > nwords / 2) return MAD_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  uint64_t* b = (uint64_t*)buf;
  uint64_t* sink = b;  // written only in the (practically impossible) case
  const unsigned grid = 256 * 32;
  switch (kind) {
    case 0: mad::k_probe<0><<<grid, 256, 0, st>>>(b, nwords, nops, seed, sink); break;
    case 1: mad::k_probe<1><<<grid, 256, 0, st>>>(b, nwords, nops, seed, sink); break;
    case 2: mad::k_probe<2><<<grid, 256, 0, st>>>(b, nwords, nops, seed, sink); break;
    case 3: mad::k_probe<3><<<grid, 256, 0, st>>>(b, nwords, nops, seed, sink); break;
    case 4: mad::k_probe<4><<<grid, 256, 0, st>>>(b, nwords, nops, seed, sink); break;
    default: mad::k_probe<5><<<grid, 256, 0, st>>>(b, nwords, nops, seed, sink); break;
  }
  return hipGetLastError() == hipSuccess ? MAD_OK : MAD_EHIP;
}
