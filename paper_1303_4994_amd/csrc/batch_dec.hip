// batch_dec.hip -- persistent batch decoder: the decode counterpart of
// batch_enc.hip (same work queue and item search; tiles are independent).
#include "batch.h"
#include "decode_tile.h"

namespace apax {

template <int LPB, int NDIM, int WP>
__global__ __launch_bounds__(WP * 64) void k_decode_batch(BatchArgs B) {
  extern __shared__ __align__(16) uint32_t lds[];
  __shared__ DecShared<WP> sm;
  const BatchDec* items = (const BatchDec*)B.items;
  batch_loop(B, [&](uint32_t it, int64_t u) {
    const BatchDec& D = items[it];
    const int64_t t = u - D.tile_start;
    switch (D.dtype) {
      case DT_I8: decode_tile<int8_t, LPB, NDIM, WP>(D.a, t, sm, lds); break;
      case DT_I16: decode_tile<int16_t, LPB, NDIM, WP>(D.a, t, sm, lds); break;
      case DT_I32: decode_tile<int32_t, LPB, NDIM, WP>(D.a, t, sm, lds); break;
      case DT_F32: decode_tile<float, LPB, NDIM, WP>(D.a, t, sm, lds); break;
      default: decode_tile<double, LPB, NDIM, WP>(D.a, t, sm, lds); break;
    }
  });
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
