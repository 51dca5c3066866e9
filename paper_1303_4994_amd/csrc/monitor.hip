// monitor.hip -- the signal monitor's autocorrelation (Sec. 6): of the array
// in memory order, binary64, R[k] = sum over n >= k of x[n] x[n - k] for the
// lags k = 0..16 that decide which nearby samples are correlated.
//
// A workgroup step covers 4096 samples: 256 lanes stage them, with the 16
// before them, as binary64 in LDS (one pad word per 16, so that the per-lane
// windows below are read without bank conflicts); each lane then holds a
// window of 32 consecutive samples in registers and accumulates the 17 lag
// products of its own 16, while the loads of its next step are in flight.
// Samples outside 0..n-1 read as zero, which keeps every sum to the pairs
// inside the array.  Workgroups grid-stride over the steps and write one
// partial per lag; a fixed-order reduction sums them.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "codec.h"
#include "monitor.h"

namespace apax {

constexpr int ACF_SPAN = ACF_LAGS + ACF_TILE;  // staged samples per step

__device__ __forceinline__ int acf_slot(int i) { return i + (i >> 4); }

template <typename T>
struct AcfStage {
  T v[ACF_TILE / 256];  // samples st * 4096 + t + 256 m
  T h;                  // lanes 0..15: sample st * 4096 - 16 + t
  __device__ __forceinline__ void load(const T* x, int64_t n, int64_t st, int t) {
    const int64_t base = st * ACF_TILE;
#pragma unroll
    for (int m = 0; m < ACF_TILE / 256; m++) {
      const int64_t g = base + t + 256 * m;
      v[m] = g < n ? x[g] : T(0);
    }
    h = (t < ACF_LAGS && base - ACF_LAGS + t >= 0) ? x[base - ACF_LAGS + t] : T(0);
  }
};

template <typename T>
__global__ __launch_bounds__(256) void k_acf(AcfArgs A) {
  __shared__ double s_t[ACF_SPAN + ACF_SPAN / 16 + 1];
  __shared__ double s_p[ACF_LAGS + 1][8];
  const T* x = (const T*)A.x;
  const int t = threadIdx.x;
  const int64_t steps = (A.n + ACF_TILE - 1) / ACF_TILE;
  double acc[ACF_LAGS + 1];
#pragma unroll
  for (int k = 0; k <= ACF_LAGS; k++) acc[k] = 0.0;

  // every load of a step is issued before any is used, and the next step's
  // loads are in flight while this step computes
  AcfStage<T> nx;
  if ((int64_t)blockIdx.x < steps) nx.load(x, A.n, blockIdx.x, t);
  for (int64_t st = blockIdx.x; st < steps; st += gridDim.x) {
#pragma unroll
    for (int m = 0; m < ACF_TILE / 256; m++) s_t[acf_slot(ACF_LAGS + t + 256 * m)] = (double)nx.v[m];
    if (t < ACF_LAGS) s_t[acf_slot(t)] = (double)nx.h;
    __syncthreads();
    if (st + gridDim.x < steps) nx.load(x, A.n, st + gridDim.x, t);
    double w[2 * ACF_LAGS];  // staged indexes 16 t .. 16 t + 31
#pragma unroll
    for (int j = 0; j < 2 * ACF_LAGS; j++) w[j] = s_t[acf_slot(16 * t + j)];
#pragma unroll
    for (int u = 0; u < 16; u++) {
      const double xn = w[ACF_LAGS + u];  // sample st * 4096 + 16 t + u
#pragma unroll
      for (int k = 0; k <= ACF_LAGS; k++) acc[k] = fma(xn, w[ACF_LAGS + u - k], acc[k]);
    }
    __syncthreads();  // the window is read before the next step stages
  }
  // workgroup sum per lag through LDS: lag k's 256 values in s_t[k * 256 ..],
  // eight runs of 32 summed by eight lanes, then the eight in order
#pragma unroll
  for (int k = 0; k <= ACF_LAGS; k++) s_t[k * 256 + t] = acc[k];
  __syncthreads();
  if (t < (ACF_LAGS + 1) * 8) {
    const int k = t >> 3, r = t & 7;
    double v = 0.0;
    for (int i = 0; i < 32; i++) v += s_t[k * 256 + r * 32 + i];
    s_p[k][r] = v;
  }
  __syncthreads();
  if (t <= ACF_LAGS) {
    double v = s_p[t][0];
    for (int r = 1; r < 8; r++) v += s_p[t][r];
    A.partial[(int64_t)blockIdx.x * (ACF_LAGS + 1) + t] = v;
  }
  if (blockIdx.x == 0 && t < 2 * ACF_LAGS) {  // the samples the sums' end terms need
    double v = 0.0;
    if (A.n >= 2 * ACF_LAGS) v = (double)x[t < ACF_LAGS ? t : A.n - 2 * ACF_LAGS + t];
    A.ends[t] = v;
  }
}

// out[k] = sum of the workgroup partials of lag k: one workgroup per lag,
// strided per-lane sums, then a fixed tree through LDS.
__global__ __launch_bounds__(256) void k_acf_reduce(const double* partial, int nwg, double* out) {
  __shared__ double s[256];
  const int k = blockIdx.x, t = threadIdx.x;
  double v = 0.0;
  for (int w = t; w < nwg; w += 256) v += partial[(int64_t)w * (ACF_LAGS + 1) + k];
  s[t] = v;
  __syncthreads();
  for (int h = 128; h >= 1; h >>= 1) {
    if (t < h) s[t] += s[t + h];
    __syncthreads();
  }
  if (t == 0) out[k] = s[0];
}

// Residual energy of the stride filter the monitor selected: sum over
// n >= k of (x[n] - sg x[n - k])^2, binary64, summed directly (a difference
// of lag sums would cancel when the filter removes most of the energy).
// Grid-stride per lane, then one partial per workgroup (slot 0 of the lag
// sums' record layout, so k_acf_reduce sums them).
template <typename T>
__global__ __launch_bounds__(256) void k_resid(const T* __restrict__ x, int64_t n, int k, double sg,
                                               double* partial) {
  __shared__ double s[256];
  const int t = threadIdx.x;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + t + k; i < n; i += (int64_t)gridDim.x * 256) {
    const double d = (double)x[i] - sg * (double)x[i - k];
    acc += d * d;
  }
  s[t] = acc;
  __syncthreads();
  for (int h = 128; h >= 1; h >>= 1) {
    if (t < h) s[t] += s[t + h];
    __syncthreads();
  }
  if (t == 0) partial[(int64_t)blockIdx.x * (ACF_LAGS + 1)] = s[0];
}

hipError_t launch_resid(int dtype, const void* x, int64_t n, int k, int sg, double* partial, double* out,
                        hipStream_t s) {
  if (n <= k) return hipSuccess;
  int64_t nwg = (n + ACF_TILE - 1) / ACF_TILE;
  if (nwg > ACF_MAX_WGS) nwg = ACF_MAX_WGS;
  const dim3 grid((unsigned)nwg), block(256);
  const double sd = (double)sg;
  switch (dtype) {
    case DT_I8: hipLaunchKernelGGL(k_resid<int8_t>, grid, block, 0, s, (const int8_t*)x, n, k, sd, partial); break;
    case DT_I16: hipLaunchKernelGGL(k_resid<int16_t>, grid, block, 0, s, (const int16_t*)x, n, k, sd, partial); break;
    case DT_I32: hipLaunchKernelGGL(k_resid<int32_t>, grid, block, 0, s, (const int32_t*)x, n, k, sd, partial); break;
    case DT_F32: hipLaunchKernelGGL(k_resid<float>, grid, block, 0, s, (const float*)x, n, k, sd, partial); break;
    default: hipLaunchKernelGGL(k_resid<double>, grid, block, 0, s, (const double*)x, n, k, sd, partial); break;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_acf_reduce, dim3(1), dim3(256), 0, s, (const double*)partial, (int)nwg, out);
  return hipGetLastError();
}

hipError_t launch_acf(int dtype, AcfArgs& A, hipStream_t s) {
  if (A.n <= 0) return hipSuccess;
  int64_t nwg = (A.n + ACF_TILE - 1) / ACF_TILE;
  if (nwg > ACF_MAX_WGS) nwg = ACF_MAX_WGS;
  const dim3 grid((unsigned)nwg), block(256);
  switch (dtype) {
    case DT_I8: hipLaunchKernelGGL(k_acf<int8_t>, grid, block, 0, s, A); break;
    case DT_I16: hipLaunchKernelGGL(k_acf<int16_t>, grid, block, 0, s, A); break;
    case DT_I32: hipLaunchKernelGGL(k_acf<int32_t>, grid, block, 0, s, A); break;
    case DT_F32: hipLaunchKernelGGL(k_acf<float>, grid, block, 0, s, A); break;
    default: hipLaunchKernelGGL(k_acf<double>, grid, block, 0, s, A); break;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_acf_reduce, dim3(ACF_LAGS + 1), dim3(256), 0, s, (const double*)A.partial, (int)nwg, A.out);
  return hipGetLastError();
}

}  // namespace apax
