// batch_enc.hip -- persistent batch encoder: thousands of arrays of mixed
// dtypes and sizes in one launch per (LPB, NDIM) class.  Workgroups take
// runs of up to RUN consecutive global tiles from an atomic ticket (a run may
// span items); every tile is encoded exactly as the single-array kernel
// would (same analyse / place / store phases), so the output is
// byte-identical to separate calls.
#include "batch.h"
#include "encode_tile.h"

namespace apax {

template <int LPB, int NDIM, int WP>
__global__ __launch_bounds__(WP * 64) void k_encode_batch(BatchArgs B) {
  constexpr int BPW = 64 / LPB;
  extern __shared__ __align__(16) uint32_t lds[];
  __shared__ EncShared<WP> sm;
  __shared__ uint32_t s_u, s_item;
  const BatchEnc* items = (const BatchEnc*)B.items;
  const int per = (int)(B.tiles_per_ticket < (uint32_t)RUN ? B.tiles_per_ticket : (uint32_t)RUN);
  uint32_t it = 0;
  int64_t it_lo = 0, it_hi = 0;  // tiles [it_lo, it_hi) belong to item it (uniform)
  for (;;) {
    if (threadIdx.x == 0) s_u = atomicAdd(B.ticket, (uint32_t)per);
    __syncthreads();
    const int64_t u0 = (int64_t)s_u;
    __syncthreads();
    if (u0 >= B.total_tiles) break;
    const int n = B.total_tiles - u0 < per ? (int)(B.total_tiles - u0) : per;
    // phase 1: analyse and assemble every tile of the run, publish its count
#pragma unroll 1
    for (int r = 0; r < n; r++) {
      const int64_t u = u0 + r;
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
      if (threadIdx.x == 0) sm.item[r] = it;
      const BatchEnc& E = items[it];
      const int64_t t = u - E.tile_start;
      switch (E.dtype) {
        case DT_I8: encode_analyze<int8_t, LPB, NDIM, WP>(E.a, t, r, B.ldsw, sm, lds); break;
        case DT_I16: encode_analyze<int16_t, LPB, NDIM, WP>(E.a, t, r, B.ldsw, sm, lds); break;
        case DT_I32: encode_analyze<int32_t, LPB, NDIM, WP>(E.a, t, r, B.ldsw, sm, lds); break;
        case DT_F32: encode_analyze<float, LPB, NDIM, WP>(E.a, t, r, B.ldsw, sm, lds); break;
        default: encode_analyze<double, LPB, NDIM, WP>(E.a, t, r, B.ldsw, sm, lds); break;
      }
    }
    // phase 2 (wave 0, run order): offsets; consecutive tiles of one item chain
    if ((threadIdx.x >> 6) == 0) {
      uint64_t base = 0;
#pragma unroll 1
      for (int r = 0; r < n; r++) {
        const uint32_t ir = sm.item[r];
        const BatchEnc& E = items[ir];
        const bool chain = r > 0 && sm.item[r - 1] == ir;
        if (chain) base += sm.agg[r - 1];
        encode_place<WP, BPW>(E.a, E.a.hdr, u0 + r - E.tile_start, r, sm, chain, base);
      }
    }
    __syncthreads();
    // phase 3: stores
#pragma unroll 1
    for (int r = 0; r < n; r++) {
      const BatchEnc& E = items[sm.item[r]];
      encode_store<LPB, WP>(E.a, u0 + r - E.tile_start, r, B.ldsw, sm, lds);
    }
    __syncthreads();
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
