// batch_dec.hip -- persistent batch decoder: the decode counterpart of
// batch_enc.hip (same work queue and item search; tiles are independent).
#include "decode_tile.h"

namespace apax {

// Item owning global tile u: the largest i with starts[i] <= u, found by a
// 64-ary search (one ballot per round) on wave 0.
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

template <int LPB, int NDIM, int WP>
__global__ __launch_bounds__(WP * 64) void k_decode_batch(BatchArgs B) {
  extern __shared__ __align__(16) uint32_t lds[];
  __shared__ DecShared<WP> sm;
  __shared__ uint32_t s_u, s_item;
  const BatchDec* items = (const BatchDec*)B.items;
  for (;;) {
    if (threadIdx.x == 0) s_u = atomicAdd(B.ticket, B.tiles_per_ticket);
    __syncthreads();
    const int64_t u0 = (int64_t)s_u;
    __syncthreads();
    if (u0 >= B.total_tiles) break;
    const int64_t u1 = u0 + B.tiles_per_ticket < B.total_tiles ? u0 + B.tiles_per_ticket : B.total_tiles;
    for (int64_t u = u0; u < u1; u++) {
      if (threadIdx.x < 64) {
        uint32_t it = find_item(B.starts, B.n, u);
        if (threadIdx.x == 0) s_item = it;
      }
      __syncthreads();
      const uint32_t it = __builtin_amdgcn_readfirstlane(s_item);
      const BatchDec& D = items[it];
      const int64_t t = u - D.tile_start;
      switch (D.dtype) {
        case DT_I8: decode_tile<int8_t, LPB, NDIM, WP>(D.a, t, sm, lds); break;
        case DT_I16: decode_tile<int16_t, LPB, NDIM, WP>(D.a, t, sm, lds); break;
        case DT_I32: decode_tile<int32_t, LPB, NDIM, WP>(D.a, t, sm, lds); break;
        case DT_F32: decode_tile<float, LPB, NDIM, WP>(D.a, t, sm, lds); break;
        default: decode_tile<double, LPB, NDIM, WP>(D.a, t, sm, lds); break;
      }
      __syncthreads();
    }
  }
}

template <int LPB, int NDIM>
static hipError_t launch_wp(int wp, const BatchArgs& B, int grid, size_t lds, hipStream_t s) {
  if (wp == 2) hipLaunchKernelGGL((k_decode_batch<LPB, NDIM, 2>), dim3(grid), dim3(128), lds, s, B);
  else if (wp == 8) hipLaunchKernelGGL((k_decode_batch<LPB, NDIM, 8>), dim3(grid), dim3(512), lds, s, B);
  else hipLaunchKernelGGL((k_decode_batch<LPB, NDIM, 4>), dim3(grid), dim3(256), lds, s, B);
  return hipGetLastError();
}

template <int LPB>
static hipError_t launch_nd(int ndim, int wp, const BatchArgs& B, int grid, size_t lds, hipStream_t s) {
  if (ndim == 1) return launch_wp<LPB, 1>(wp, B, grid, lds, s);
  if (ndim == 2) return launch_wp<LPB, 2>(wp, B, grid, lds, s);
  return launch_wp<LPB, 3>(wp, B, grid, lds, s);
}

hipError_t launch_decode_batch(int lpb, int ndim, int wp, const BatchArgs& B, int grid, size_t lds,
                               hipStream_t s) {
  if (lpb == 16) return launch_nd<16>(ndim, wp, B, grid, lds, s);
  if (lpb == 32) return launch_nd<32>(ndim, wp, B, grid, lds, s);
  return launch_nd<64>(ndim, wp, B, grid, lds, s);
}

}  // namespace apax
