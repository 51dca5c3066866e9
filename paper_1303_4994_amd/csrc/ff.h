// ff.h -- FP32 float-float arithmetic for the profiler's sums: a value is
// an unevaluated pair hi + lo (|lo| <= ulp(hi)/2), added with TwoSum (Knuth)
// and renormalised with Fast2Sum (Dekker); wave totals of several such
// values by recursive halving.
#pragma once
#include "codec.h"

namespace apax {

struct FF {
  float hi, lo;
};

__device__ __forceinline__ FF fast2sum(float a, float b) {
  float s = a + b;
  float e = b - (s - a);
  return {s, e};
}

__device__ __forceinline__ FF ff_add(FF a, FF b) {
  float s = a.hi + b.hi;
  float bb = s - a.hi;
  float e = (a.hi - (s - bb)) + (b.hi - bb);
  e += a.lo + b.lo;
  return fast2sum(s, e);
}

__device__ __forceinline__ FF ff_of(double t) {
  float hi = (float)t;
  float lo = (float)(t - (double)hi);
  return {hi, lo};
}

__device__ __forceinline__ FF ff_shfl_xor(FF a, int o) {
  return {__shfl_xor(a.hi, o, 64), __shfl_xor(a.lo, o, 64)};
}

// Totals over the 64 lanes of a wave of the N float-float values v[] (N <= 8,
// padded to P = 2^k): recursive halving -- at level k a lane keeps half of
// its values, adds its partner's (lane ^ 2^k) copies of that half, and
// hands over the other half -- so the first levels take P/2, P/4, ...
// additions instead of N each; a butterfly over the remaining levels
// follows.  Lane l then holds the total of value bitrev(l mod P) (returned).
template <int N>
__device__ __forceinline__ FF wave_totals(const FF (&v)[N], int lane) {
  constexpr int P = N <= 1 ? 1 : (N <= 2 ? 2 : (N <= 4 ? 4 : 8));
  FF w[P];
#pragma unroll
  for (int i = 0; i < P; i++) w[i] = i < N ? v[i] : FF{0.f, 0.f};
  int lvl = 0;
#pragma unroll
  for (int m = P; m > 1; m >>= 1, lvl++) {
    const int h = m >> 1;
    const bool up = (lane >> lvl) & 1;
#pragma unroll
    for (int j = 0; j < h; j++) {
      const FF keep = up ? w[j + h] : w[j];
      const FF give = up ? w[j] : w[j + h];
      w[j] = ff_add(keep, ff_shfl_xor(give, 1 << lvl));
    }
  }
#pragma unroll
  for (int o = P; o < 64; o <<= 1) w[0] = ff_add(w[0], ff_shfl_xor(w[0], o));
  return w[0];
}

// index of the value whose total lane l holds after wave_totals<N>
template <int N>
__device__ __forceinline__ int wave_totals_index(int lane) {
  constexpr int P = N <= 1 ? 1 : (N <= 2 ? 2 : (N <= 4 ? 4 : 8));
  int idx = 0;
#pragma unroll
  for (int k = 0, h = P >> 1; h >= 1; k++, h >>= 1) idx += ((lane >> k) & 1) * h;
  return idx;
}

}  // namespace apax
