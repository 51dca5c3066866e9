// totals.h -- wave totals of the profiler's binary64 partial sums.
#pragma once
#include "codec.h"

namespace apax {

// Totals over the 64 lanes of a wave of the N values v[] (N <= 8, padded to
// P = 2^k): recursive halving -- at level k a lane keeps half of its values,
// adds its partner's (lane ^ 2^k) copies of that half, and hands over the
// other half -- so the first levels take P/2, P/4, ... additions instead of N
// each; a butterfly over the remaining levels follows.  Lane l then holds the
// total of value bitrev(l mod P) (returned).  Every lane adds in the same
// fixed order, so the totals are deterministic.
template <int N>
__device__ __forceinline__ double wave_totals(const double (&v)[N], int lane) {
  constexpr int P = N <= 1 ? 1 : (N <= 2 ? 2 : (N <= 4 ? 4 : 8));
  double w[P];
#pragma unroll
  for (int i = 0; i < P; i++) w[i] = i < N ? v[i] : 0.0;
  int lvl = 0;
#pragma unroll
  for (int m = P; m > 1; m >>= 1, lvl++) {
    const int h = m >> 1;
    const bool up = (lane >> lvl) & 1;
#pragma unroll
    for (int j = 0; j < h; j++) {
      const double keep = up ? w[j + h] : w[j];
      const double give = up ? w[j] : w[j + h];
      w[j] = keep + __shfl_xor(give, 1 << lvl, 64);
    }
  }
#pragma unroll
  for (int o = P; o < 64; o <<= 1) w[0] += __shfl_xor(w[0], o, 64);
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
