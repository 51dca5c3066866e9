// spectra.h -- launch interface of the Welch power spectra (Sec. 4 Windows
// 3-4 and the signal monitor of Sec. 6).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace apax {

// Welch spectra of x, y, x - y (1024-sample segments, hop 512)
constexpr int PSD_MAX_WGS = 512;  // two workgroups per CU (64 KB of LDS each)
struct PsdArgs {
  const void* x;
  const void* y;
  const double* window;   // 1024 Hann weights
  const void* twiddle;    // 1024 complex e^(-2 pi i k / 1024)
  double* partial;        // [workgroup][3][512]
  double* out;            // [3][512] sums over segments
  int64_t segments;
  int32_t nsig;           // 3: x, y and d; 1: x only
  int32_t pad;
};
hipError_t launch_psd(int dtype, PsdArgs& A, hipStream_t s);
// window (1024 doubles) then twiddles (1024 complex doubles) into t
hipError_t launch_psd_tables(double* t, hipStream_t s);

}  // namespace apax
