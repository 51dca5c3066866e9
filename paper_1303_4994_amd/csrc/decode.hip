// decode.hip -- single-array APAX decoder kernel for gfx950 (one workgroup
// per tile; the tile body is in decode_tile.h).
#include "block.h"
#include "decode_tile.h"

namespace apax {

template <typename T, int LPB, int NDIM, int WP>
__global__ __launch_bounds__(WP * 64) void k_decode(DecArgs A) {
  extern __shared__ __align__(16) uint32_t lds[];
  __shared__ DecShared<WP> sm;
  decode_tile<T, LPB, NDIM, WP>(A, (int64_t)blockIdx.x, sm, lds);
}

// Decode-on-read consumer: the dot product of the decoded array with w, one
// workgroup per tile, binary64 lane partials summed in a fixed order into
// one partial per tile (k_dot_reduce adds those in tile order).
template <typename T, int LPB, int NDIM, int WP>
__global__ __launch_bounds__(WP * 64) void k_decode_dot(DecArgs A, const T* w, double* partial) {
  extern __shared__ __align__(16) uint32_t lds[];
  __shared__ DecShared<WP> sm;
  __shared__ double s_sum[WP];
  double dot = 0.0;
  decode_tile<T, LPB, NDIM, WP, true>(A, (int64_t)blockIdx.x, sm, lds, w, &dot);
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) dot += __shfl_down(dot, o, 64);
  if ((threadIdx.x & 63) == 0) s_sum[threadIdx.x >> 6] = dot;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = s_sum[0];
    for (int i = 1; i < WP; i++) t += s_sum[i];
    partial[blockIdx.x] = t;
  }
}

// The same consumer on an uncompressed array: dot(x, w), 4 samples per
// thread per step, one partial per workgroup.
template <typename T>
__global__ __launch_bounds__(256) void k_dot_plain(const T* __restrict__ x, const T* __restrict__ w, int64_t n,
                                                 double* partial) {
  __shared__ double s_sum[4];
  double dot = 0.0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x * 4;
#pragma unroll 4
  for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 4; i < n; i += stride) {
    const int nv = n - i >= 4 ? 4 : (int)(n - i);
    T xv[4], wv[4];
    load4<T>(x, i, nv, xv);  // 4 * sizeof(T)-byte vector loads where aligned
    load4<T>(w, i, nv, wv);
#pragma unroll
    for (int k = 0; k < 4; k++) dot += (double)xv[k] * (double)wv[k];
  }
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) dot += __shfl_down(dot, o, 64);
  if ((threadIdx.x & 63) == 0) s_sum[threadIdx.x >> 6] = dot;
  __syncthreads();
  if (threadIdx.x == 0) partial[blockIdx.x] = s_sum[0] + s_sum[1] + s_sum[2] + s_sum[3];
}

// Sum of n partials in index order (one workgroup: contiguous chunks per
// thread, then the chunk sums in order by thread 0).
__global__ __launch_bounds__(256) void k_dot_reduce(const double* partial, int64_t n, double* out) {
  __shared__ double s_c[256];
  const int64_t per = (n + 255) / 256;
  const int64_t lo = threadIdx.x * per, hi = lo + per < n ? lo + per : n;
  double t = 0.0;
  for (int64_t i = lo; i < hi; i++) t += partial[i];
  s_c[threadIdx.x] = t;
  __syncthreads();
  if (threadIdx.x == 0) {
    double r = 0.0;
    for (int i = 0; i < 256; i++) r += s_c[i];
    *out = r;
  }
}

void launch_dot_reduce(const double* partial, int64_t n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_dot_reduce, dim3(1), dim3(256), 0, s, partial, n, out);
}

template <typename T, int LPB, int NDIM>
static hipError_t launch_dot_t(const DecArgs& A, const void* w, double* partial, hipStream_t s) {
  constexpr int BPW = 64 / LPB;
  size_t lds = (size_t)WPG * BPW * A.g.ldsw * 4;
  hipLaunchKernelGGL((k_decode_dot<T, LPB, NDIM, WPG>), dim3((unsigned)A.ntiles), dim3(WPG * 64), lds, s, A,
                     (const T*)w, partial);
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_dot_nd(const DecArgs& A, int ndim, const void* w, double* partial, hipStream_t s) {
  const int G = A.g.G;
#define APAX_DOT_LPB(ND)                                                   \
  if (G <= 16) return launch_dot_t<T, 16, ND>(A, w, partial, s);          \
  if (G <= 32) return launch_dot_t<T, 32, ND>(A, w, partial, s);          \
  return launch_dot_t<T, 64, ND>(A, w, partial, s);
  if (ndim == 1) { APAX_DOT_LPB(1) }
  if (ndim == 2) { APAX_DOT_LPB(2) }
  APAX_DOT_LPB(3)
#undef APAX_DOT_LPB
}

hipError_t launch_decode_dot(int dtype, int ndim, DecArgs& A, const void* w, double* partial, double* out,
                             hipStream_t s) {
  A.ntiles = encode_tiles(A.g);
  if (A.ntiles == 0) return hipSuccess;
  hipError_t e;
  switch (dtype) {
    case DT_I8: e = launch_dot_nd<int8_t>(A, ndim, w, partial, s); break;
    case DT_I16: e = launch_dot_nd<int16_t>(A, ndim, w, partial, s); break;
    case DT_I32: e = launch_dot_nd<int32_t>(A, ndim, w, partial, s); break;
    case DT_F32: e = launch_dot_nd<float>(A, ndim, w, partial, s); break;
    default: e = launch_dot_nd<double>(A, ndim, w, partial, s); break;
  }
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_dot_reduce, dim3(1), dim3(256), 0, s, (const double*)partial, A.ntiles, out);
  return hipGetLastError();
}

hipError_t launch_dot_plain(int dtype, const void* x, const void* w, int64_t n, double* partial, int nwg,
                            double* out, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  switch (dtype) {
    case DT_I8: hipLaunchKernelGGL(k_dot_plain<int8_t>, dim3(nwg), dim3(256), 0, s, (const int8_t*)x, (const int8_t*)w, n, partial); break;
    case DT_I16: hipLaunchKernelGGL(k_dot_plain<int16_t>, dim3(nwg), dim3(256), 0, s, (const int16_t*)x, (const int16_t*)w, n, partial); break;
    case DT_I32: hipLaunchKernelGGL(k_dot_plain<int32_t>, dim3(nwg), dim3(256), 0, s, (const int32_t*)x, (const int32_t*)w, n, partial); break;
    case DT_F32: hipLaunchKernelGGL(k_dot_plain<float>, dim3(nwg), dim3(256), 0, s, (const float*)x, (const float*)w, n, partial); break;
    default: hipLaunchKernelGGL(k_dot_plain<double>, dim3(nwg), dim3(256), 0, s, (const double*)x, (const double*)w, n, partial); break;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_dot_reduce, dim3(1), dim3(256), 0, s, (const double*)partial, (int64_t)nwg, out);
  return hipGetLastError();
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
