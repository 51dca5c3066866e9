// batch.h -- work queue of the persistent batch kernels.
//
// Workgroups take runs of tiles_per_ticket global tiles from an atomic
// ticket.  The ticket for the next run is requested when the current run
// starts, so the atomic's latency overlaps the run's work; the item that
// owns a tile is found by a 64-ary search only when a tile leaves the item
// of the previous one.  Tickets are still handed out in increasing order, and
// the smallest tile taken but not finished is always being processed (its
// holder has no smaller unfinished tile), so look-back waits always end.
#pragma once
#include "kernels.h"

namespace apax {

// Item owning global tile u: the largest i with starts[i] <= u, found by a
// 64-ary search (one ballot per round) on one wave.
__device__ __forceinline__ uint32_t find_item(const int64_t* starts, uint32_t n, int64_t u) {
  uint32_t lo = 0, hi = n;
  const int lane = lane_id();
  while (hi - lo > 1) {
    uint32_t step = (hi - lo + 63) / 64;
    uint32_t idx = lo + (uint32_t)lane * step;
    bool ok = idx < hi && starts[idx] <= u;
    uint64_t m = __ballot(ok);
    int k = 63 - __clzll((long long)m);
    lo = lo + (uint32_t)k * step;
    uint32_t h2 = lo + step;
    hi = h2 < hi ? h2 : hi;
  }
  return lo;
}

// Runs body(item, tile) for every tile this workgroup takes; body is called
// by all threads and may synchronize the workgroup.
template <typename Body>
__device__ __forceinline__ void batch_loop(const BatchArgs& B, Body&& body) {
  __shared__ uint32_t s_u, s_item;
  if (threadIdx.x == 0) s_u = atomicAdd(B.ticket, B.tiles_per_ticket);
  __syncthreads();
  uint32_t it = 0;
  int64_t it_lo = 0, it_hi = 0;  // tiles [it_lo, it_hi) belong to item it (uniform)
  for (;;) {
    const int64_t u0 = (int64_t)s_u;
    __syncthreads();
    if (u0 >= B.total_tiles) break;
    uint32_t nxt = 0;
    if (threadIdx.x == 0) nxt = atomicAdd(B.ticket, B.tiles_per_ticket);
    const int64_t u1 = u0 + B.tiles_per_ticket < B.total_tiles ? u0 + B.tiles_per_ticket : B.total_tiles;
    for (int64_t u = u0; u < u1; u++) {
      if (u < it_lo || u >= it_hi) {
        if (threadIdx.x < 64) {
          const uint32_t f = find_item(B.starts, B.n, u);
          if (threadIdx.x == 0) s_item = f;
        }
        __syncthreads();
        it = __builtin_amdgcn_readfirstlane(s_item);
        it_lo = B.starts[it];
        it_hi = it + 1 < B.n ? B.starts[it + 1] : B.total_tiles;
        __syncthreads();
      }
      body(it, u);
      __syncthreads();
    }
    if (threadIdx.x == 0) s_u = nxt;
    __syncthreads();
  }
}

}  // namespace apax
