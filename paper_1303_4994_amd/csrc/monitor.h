// monitor.h -- launch interface of the signal monitor's lag sums (Sec. 6):
// R[k] = sum_{n >= k} x[n] x[n - k], k = 0..16, of an array in memory order.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace apax {

constexpr int ACF_LAGS = 16;
constexpr int ACF_TILE = 4096;     // samples per workgroup step
constexpr int ACF_MAX_WGS = 1024;
struct AcfArgs {
  const void* x;
  int64_t n;
  double* partial;  // [workgroup][ACF_LAGS + 1]
  double* out;      // [ACF_LAGS + 1]
  double* ends;     // [32]: x[0..15] and x[n - 16..n - 1] (n >= 32; zeros otherwise)
};
hipError_t launch_acf(int dtype, AcfArgs& A, hipStream_t s);
// *out = sum_{n >= k} (x[n] - sg x[n - k])^2 (partial: AcfArgs::partial's region)
hipError_t launch_resid(int dtype, const void* x, int64_t n, int k, int sg, double* partial, double* out,
                        hipStream_t s);

}  // namespace apax
