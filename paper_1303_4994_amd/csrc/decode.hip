// decode.hip -- single-array APAX decoder kernel for gfx950 (one workgroup
// per tile; the tile body is in decode_tile.h).
#include "decode_tile.h"

namespace apax {

template <typename T, int LPB, int NDIM, int WP>
__global__ __launch_bounds__(WP * 64) void k_decode(DecArgs A) {
  extern __shared__ __align__(16) uint32_t lds[];
  __shared__ DecShared<WP> sm;
  decode_tile<T, LPB, NDIM, WP>(A, (int64_t)blockIdx.x, sm, lds);
}

template <typename T, int LPB, int NDIM>
static hipError_t launch_t(const DecArgs& A, hipStream_t s) {
  constexpr int BPW = 64 / LPB;
  size_t lds = (size_t)WPG * BPW * A.g.ldsw * 4;
  hipLaunchKernelGGL((k_decode<T, LPB, NDIM, WPG>), dim3((unsigned)A.ntiles), dim3(WPG * 64), lds, s, A);
  return hipGetLastError();
}

template <typename T, int NDIM>
static hipError_t launch_lpb(const DecArgs& A, hipStream_t s) {
  if (A.g.G <= 16) return launch_t<T, 16, NDIM>(A, s);
  if (A.g.G <= 32) return launch_t<T, 32, NDIM>(A, s);
  return launch_t<T, 64, NDIM>(A, s);
}

template <typename T>
static hipError_t launch_nd(const DecArgs& A, int ndim, hipStream_t s) {
  if (ndim == 1) return launch_lpb<T, 1>(A, s);
  if (ndim == 2) return launch_lpb<T, 2>(A, s);
  return launch_lpb<T, 3>(A, s);
}

hipError_t launch_decode(int dtype, int ndim, DecArgs& A, hipStream_t s) {
  A.ntiles = encode_tiles(A.g);
  if (A.ntiles == 0) return hipSuccess;
  switch (dtype) {
    case DT_I8: return launch_nd<int8_t>(A, ndim, s);
    case DT_I16: return launch_nd<int16_t>(A, ndim, s);
    case DT_I32: return launch_nd<int32_t>(A, ndim, s);
    case DT_F32: return launch_nd<float>(A, ndim, s);
    default: return launch_nd<double>(A, ndim, s);
  }
}

}  // namespace apax
