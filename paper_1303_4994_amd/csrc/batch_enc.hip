// batch_enc.hip -- persistent batch encoder: thousands of arrays of mixed
// dtypes and sizes in one launch per (LPB, NDIM) class.  Workgroups take
// runs of tiles from an atomic ticket; every tile belongs to one item and is
// encoded exactly as the single-array kernel would (same tile body), so the
// output is byte-identical to separate calls.  Tickets are handed out in
// increasing order, so each item's tiles start in order and its look-back
// only waits on tiles already taken by running workgroups.
#include "encode_tile.h"

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
__global__ __launch_bounds__(WP * 64) void k_encode_batch(BatchArgs B) {
  extern __shared__ __align__(16) uint32_t lds[];
  __shared__ EncShared<WP> sm;
  __shared__ uint32_t s_u, s_item;
  const BatchEnc* items = (const BatchEnc*)B.items;
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
      const BatchEnc& E = items[it];
      const int64_t t = u - E.tile_start;
      switch (E.dtype) {
        case DT_I8: encode_tile<int8_t, LPB, NDIM, WP>(E.a, t, sm, lds); break;
        case DT_I16: encode_tile<int16_t, LPB, NDIM, WP>(E.a, t, sm, lds); break;
        case DT_I32: encode_tile<int32_t, LPB, NDIM, WP>(E.a, t, sm, lds); break;
        case DT_F32: encode_tile<float, LPB, NDIM, WP>(E.a, t, sm, lds); break;
        default: encode_tile<double, LPB, NDIM, WP>(E.a, t, sm, lds); break;
      }
      __syncthreads();
    }
  }
}

__global__ void k_batch_reset(uint32_t* ticket, uint64_t* tile_state, int64_t n) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) *ticket = 0;
  for (; i < n; i += (int64_t)gridDim.x * blockDim.x) tile_state[i] = 0;
}

hipError_t launch_batch_reset(uint32_t* ticket, uint64_t* tile_state, int64_t n, hipStream_t s) {
  int64_t nb = (n + 255) / 256;
  unsigned grid = (unsigned)(nb > 1024 ? 1024 : (nb < 1 ? 1 : nb));
  hipLaunchKernelGGL(k_batch_reset, dim3(grid), dim3(256), 0, s, ticket, tile_state, n);
  return hipGetLastError();
}

template <int LPB, int NDIM>
static hipError_t launch_wp(int wp, const BatchArgs& B, int grid, size_t lds, hipStream_t s) {
  if (wp == 2) hipLaunchKernelGGL((k_encode_batch<LPB, NDIM, 2>), dim3(grid), dim3(128), lds, s, B);
  else if (wp == 8) hipLaunchKernelGGL((k_encode_batch<LPB, NDIM, 8>), dim3(grid), dim3(512), lds, s, B);
  else hipLaunchKernelGGL((k_encode_batch<LPB, NDIM, 4>), dim3(grid), dim3(256), lds, s, B);
  return hipGetLastError();
}

template <int LPB>
static hipError_t launch_nd(int ndim, int wp, const BatchArgs& B, int grid, size_t lds, hipStream_t s) {
  if (ndim == 1) return launch_wp<LPB, 1>(wp, B, grid, lds, s);
  if (ndim == 2) return launch_wp<LPB, 2>(wp, B, grid, lds, s);
  return launch_wp<LPB, 3>(wp, B, grid, lds, s);
}

hipError_t launch_encode_batch(int lpb, int ndim, int wp, const BatchArgs& B, int grid, size_t lds,
                               hipStream_t s) {
  if (lpb == 16) return launch_nd<16>(ndim, wp, B, grid, lds, s);
  if (lpb == 32) return launch_nd<32>(ndim, wp, B, grid, lds, s);
  return launch_nd<64>(ndim, wp, B, grid, lds, s);
}

}  // namespace apax
