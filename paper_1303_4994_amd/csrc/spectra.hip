// spectra.hip -- Welch power spectra of x, y and d = x - y for the spectral
// metrics of Sec. 4 (Windows 3-4), or of x alone for the signal monitor of
// Sec. 6: segments of 1024 samples of the array in memory order, hop 512,
// periodic Hann window, one-sided bins 1..512.
//
// One launch per signal, one wave per pair of segments: for x, y or d
// (binary64, d formed per sample), the two windowed segments form one complex
// sequence,
// transformed by a radix-4 Stockham FFT (five stages, in place in the wave's
// LDS buffer: every lane reads its 16 inputs before any lane writes); the two
// real spectra follow from Z_f and Z_(1024-f).  Each lane accumulates the
// power of its 8 bins over the wave's segments; workgroups write partial
// spectra, one fixed-order reduction kernel sums them (deterministic).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "codec.h"
#include "spectra.h"

namespace apax {

constexpr int PSD_N = 1024;
constexpr int PSD_WAVES = 4;

struct C64 {
  double re, im;
};
__device__ __forceinline__ C64 cadd(C64 a, C64 b) { return {a.re + b.re, a.im + b.im}; }
__device__ __forceinline__ C64 csub(C64 a, C64 b) { return {a.re - b.re, a.im - b.im}; }
__device__ __forceinline__ C64 cmul(C64 a, C64 b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}

__device__ __forceinline__ void wave_sync_lds() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Radix-4 Stockham FFT of 1024 points by one wave, in place in z (LDS).
// v: this lane's stage-0 inputs, v[m] = input[lane + 64 m]; the result is
// left in z in natural order.
__device__ __forceinline__ void fft1024(C64 (&v)[16], C64* z, const C64* tw, int lane) {
#pragma unroll
  for (int ns = 1; ns < PSD_N; ns *= 4) {  // five stages, unrolled: ns, step are constants
    if (ns > 1) {
#pragma unroll
      for (int q = 0; q < 4; q++)
#pragma unroll
        for (int r = 0; r < 4; r++) v[q + 4 * r] = z[lane + 64 * q + 256 * r];
      wave_sync_lds();  // every lane has read before any lane writes
    }
    const int step = PSD_N / (ns * 4);
#pragma unroll
    for (int q = 0; q < 4; q++) {
      const int j = lane + 64 * q;
      const int k = j % ns;
      C64 a0 = v[q], a1 = v[q + 4], a2 = v[q + 8], a3 = v[q + 12];
      if (ns > 1) {
        a1 = cmul(a1, tw[(k * step) & (PSD_N - 1)]);
        a2 = cmul(a2, tw[(2 * k * step) & (PSD_N - 1)]);
        a3 = cmul(a3, tw[(3 * k * step) & (PSD_N - 1)]);
      }
      const C64 b0 = cadd(a0, a2), b1 = csub(a0, a2), b2 = cadd(a1, a3);
      const C64 d13 = csub(a1, a3);
      const C64 b3 = {d13.im, -d13.re};  // (a1 - a3) * (-i)
      const int o = (j / ns) * ns * 4 + k;
      z[o] = cadd(b0, b2);
      z[o + ns] = cadd(b1, b3);
      z[o + 2 * ns] = csub(b0, b2);
      z[o + 3 * ns] = csub(b1, b3);
    }
    wave_sync_lds();
  }
}

// Sample s of signal `which` (0 x, 1 y, 2 d = x - y) as binary64.
template <typename T>
__device__ __forceinline__ double sig(const T* x, const T* y, int which, int64_t i) {
  if (which == 0) return (double)x[i];
  if (which == 1) return (double)y[i];
  return (double)x[i] - (double)y[i];
}

// A wave takes segment pairs (2p, 2p + 1).  Each signal gets its own FFT,
// the pair's two segments as real and imaginary parts: packing two real
// transforms costs an error relative to the larger of the two, so only
// segments of the same signal (alike in size) share one.
// One launch per signal SIG (0 x, 1 y, 2 d), which writes row SIG of the
// workgroup partials: three signals in one wave would hold three spectra of
// sums and halve the waves a SIMD can run.
template <typename T, int SIG>
__global__ __launch_bounds__(PSD_WAVES * 64) void k_psd(PsdArgs A) {
  __shared__ C64 s_z[PSD_WAVES][PSD_N];
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const T* x = (const T*)A.x;
  const T* y = (const T*)A.y;
  const C64* tw = (const C64*)A.twiddle;  // e^(-2 pi i k / 1024)
  const double* win = A.window;           // sin^2(pi i / 1024)
  C64* z = s_z[wave];
  double acc[8];
#pragma unroll
  for (int m = 0; m < 8; m++) acc[m] = 0.0;

  const int64_t pairs = (A.segments + 1) / 2;
  const int64_t wid = (int64_t)blockIdx.x * PSD_WAVES + wave;
  const int64_t nw = (int64_t)gridDim.x * PSD_WAVES;
  for (int64_t pr = wid; pr < pairs; pr += nw) {
    const int64_t b0 = pr * PSD_N;            // segment 2p starts at 2p * 512
    const bool second = 2 * pr + 1 < A.segments;
    {
      constexpr int which = SIG;
      C64 v[16];
#pragma unroll
      for (int m = 0; m < 16; m++) {
        const int i = lane + 64 * m;
        const double w = win[i];
        v[m] = {sig(x, y, which, b0 + i) * w, second ? sig(x, y, which, b0 + PSD_N / 2 + i) * w : 0.0};
      }
      fft1024(v, z, tw, lane);
      // bins f = 1 + lane + 64 m: A = (Z_f + conj Z_(N-f)) / 2, B = (Z_f - conj Z_(N-f)) / 2i
#pragma unroll
      for (int m = 0; m < 8; m++) {
        const int f = 1 + lane + 64 * m;
        const C64 zf = z[f], zn = z[(PSD_N - f) & (PSD_N - 1)];
        const double ar = 0.5 * (zf.re + zn.re), ai = 0.5 * (zf.im - zn.im);
        const double br = 0.5 * (zf.im + zn.im), bi = -0.5 * (zf.re - zn.re);
        double p = ar * ar + ai * ai;
        if (second) p += br * br + bi * bi;
        acc[m] += p;
      }
      wave_sync_lds();  // the bins are read before the next transform writes
    }
  }
  // workgroup partial: the waves in order, through LDS
  __syncthreads();
  double* red = reinterpret_cast<double*>(&s_z[0][0]);  // [wave][512]
#pragma unroll
  for (int m = 0; m < 8; m++) red[wave * 512 + lane + 64 * m] = acc[m];
  __syncthreads();
  for (int t = threadIdx.x; t < 512; t += blockDim.x) {
    double sum = red[t];
    for (int w = 1; w < PSD_WAVES; w++) sum += red[w * 512 + t];
    A.partial[(int64_t)blockIdx.x * 3 * 512 + SIG * 512 + t] = sum;
  }
}

// Sum of the workgroup partials, out[s][f - 1], in a fixed order: a
// workgroup takes 64 of the 1536 columns; its four waves sum four
// consecutive runs of rows (eight loads in flight), then the runs in order.
__global__ __launch_bounds__(256) void k_psd_reduce(const double* partial, int nwg, double* out) {
  __shared__ double s_run[4][64];
  const int c = blockIdx.x * 64 + (threadIdx.x & 63);
  const int g = threadIdx.x >> 6;
  const int per = (nwg + 3) / 4;
  const int lo = g * per, hi = lo + per < nwg ? lo + per : nwg;
  double sum = 0.0;
  int w = lo;
  for (; w + 8 <= hi; w += 8) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; u++) v[u] = partial[(int64_t)(w + u) * 3 * 512 + c];
#pragma unroll
    for (int u = 0; u < 8; u++) sum += v[u];
  }
  for (; w < hi; w++) sum += partial[(int64_t)w * 3 * 512 + c];
  s_run[g][threadIdx.x & 63] = sum;
  __syncthreads();
  if (g == 0) {
    const int l = threadIdx.x;
    out[c] = ((s_run[0][l] + s_run[1][l]) + s_run[2][l]) + s_run[3][l];
  }
}

// The Hann window sin^2(pi i / 1024) and the twiddles e^(-2 pi i k / 1024),
// binary64, with the argument reduction of sinpi/cospi (exact multiples of pi).
__global__ __launch_bounds__(256) void k_psd_tables(double* t) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= PSD_N) return;
  const double sn = sinpi(i / (double)PSD_N);
  t[i] = sn * sn;
  double s2, c2;
  sincospi(2.0 * i / (double)PSD_N, &s2, &c2);
  t[PSD_N + 2 * i] = c2;
  t[PSD_N + 2 * i + 1] = -s2;
}

hipError_t launch_psd_tables(double* t, hipStream_t s) {
  hipLaunchKernelGGL(k_psd_tables, dim3(PSD_N / 256), dim3(256), 0, s, t);
  return hipGetLastError();
}

hipError_t launch_psd(int dtype, PsdArgs& A, hipStream_t s) {
  if (A.segments <= 0) return hipSuccess;
  if (A.nsig < 1 || A.nsig > 3) return hipErrorInvalidValue;
  int64_t nwg = ((A.segments + 1) / 2 + PSD_WAVES - 1) / PSD_WAVES;
  if (nwg > PSD_MAX_WGS) nwg = PSD_MAX_WGS;
  const dim3 grid((unsigned)nwg), block(PSD_WAVES * 64);
  for (int sg = 0; sg < A.nsig; sg++) {
    switch (dtype * 4 + sg) {
#define PSD_CASE(DT, TY)                                                                  \
  case DT * 4 + 0: hipLaunchKernelGGL((k_psd<TY, 0>), grid, block, 0, s, A); break;      \
  case DT * 4 + 1: hipLaunchKernelGGL((k_psd<TY, 1>), grid, block, 0, s, A); break;      \
  case DT * 4 + 2: hipLaunchKernelGGL((k_psd<TY, 2>), grid, block, 0, s, A); break;
      PSD_CASE(DT_I8, int8_t)
      PSD_CASE(DT_I16, int16_t)
      PSD_CASE(DT_I32, int32_t)
      PSD_CASE(DT_F32, float)
      PSD_CASE(DT_F64, double)
#undef PSD_CASE
      default: return hipErrorInvalidValue;
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  // only the rows of the signals computed (row r: columns r * 512 ..)
  hipLaunchKernelGGL(k_psd_reduce, dim3(A.nsig * 512 / 64), dim3(256), 0, s, (const double*)A.partial, (int)nwg, A.out);
  return hipGetLastError();
}

}  // namespace apax
