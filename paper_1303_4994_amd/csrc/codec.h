// codec.h -- device building blocks of the APAX codec for gfx950 (wave64).
//
// One 64-lane wavefront works on 64/LPB blocks at once ("segments" of LPB
// lanes); lane gi of a segment owns group gi (4 consecutive samples along x,
// Sec. 6 "groups of N = 4") of its block, so a block of B <= 256 samples is
// held in registers as one value per group and lane.  Cross-lane data moves
// with ds_bpermute shuffles inside a segment, per-block decisions are made on
// 64-bit ballot masks with scalar bit arithmetic (JEE token counts), and
// block sizes / bit offsets come from segmented wave reductions and scans.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace apax {

enum { DT_I8 = 1, DT_I16 = 2, DT_I32 = 3, DT_F32 = 4, DT_F64 = 5 };
enum { M_LOSSLESS = 0, M_RATE = 1, M_QUALITY = 2, M_ADAPT = 3 };
enum : uint32_t { ST_NONFINITE = 1u, ST_CORRUPT = 2u, ST_INTERNAL = 4u, ST_NOPROFILE = 8u };

template <typename T> struct Traits;
template <> struct Traits<int8_t> { static constexpr int W = 8, H = 32; static constexpr bool isint = true; };
template <> struct Traits<int16_t> { static constexpr int W = 16, H = 32; static constexpr bool isint = true; };
template <> struct Traits<int32_t> { static constexpr int W = 32, H = 32; static constexpr bool isint = true; };
template <> struct Traits<float> { static constexpr int W = 32, H = 48; static constexpr bool isint = false; };
template <> struct Traits<double> { static constexpr int W = 32, H = 48; static constexpr bool isint = false; };

// Geometry of one array, passed by value to every kernel.
struct Geo {
  int64_t n[3];     // extent z, y, x (leading 1s below 3-d)
  int64_t nbx, nby; // bricks along x, y
  int64_t nblocks;
  int32_t b[3];     // brick z, y, x
  int32_t B, G;     // samples / groups per block
  int32_t rowq;     // groups per brick row = b[2] / 4
  int32_t plane;    // groups per brick plane = b[1] * rowq
  int32_t mode;
  uint32_t mask;    // effective stream mask
  int32_t budget;   // fixed-rate words per block (0 otherwise)
  int32_t code;     // gain code (fixed-rate start / fixed-quality)
  int32_t cmin, cmax;
  int32_t maxw;     // words of the largest variable-size block (verbatim)
  int32_t ldsw;     // LDS words of one block buffer: worst BFPE encoding + 2
  // n / d = (n * m) >> sh for n < 2^31 (divisors nbx, nby, rowq, plane)
  uint32_t nbx_m, nby_m, rowq_m, plane_m;
  int32_t nbx_s, nby_s, rowq_s, plane_s;
  // whole bricks: element strides of one brick step along z and y (x: b[2]),
  // number of bricks that lie wholly inside the array per axis, and whether
  // a brick's lane offsets fit 31 bits with every row 4-sample aligned
  int64_t sz, sy;
  int32_t fbx, fby, fbz;
  int32_t dense_ok;
  // adaptive rate: target words per block, the controller's window of
  // requested codes [alo, alo + awd)
  int32_t target, alo, awd;
  // filter stream (1-d): stride (0: none) and sign (1: x[n] + x[n-k])
  int32_t fk, fneg;
  // groups of 4 per exponent: 1, or 2 for groups of 8 samples
  int32_t gq, pad_;
};

// Division of a numerator below 2^31 by a divisor known on the host
// (Granlund-Montgomery: m = ceil(2^(31+l) / d), l = ceil(log2 d)).
__device__ __forceinline__ uint32_t fdiv(uint32_t n, uint32_t m, int sh) {
  return (uint32_t)(((uint64_t)n * m) >> sh);
}

// ------------------------------------------------------------ gain grid
// Attenuator values (Sec. 6): g(c) = (16 + f) 2^(k-4), c = 16k + f.  An
// arithmetic shift is floor division by 16 for negative codes as well.
__device__ __forceinline__ double gain_of(int c) {
  return ldexp((double)(16 + (c & 15)), (c >> 4) - 4);
}

// Code bracket of a block (Sec. 6 attenuator, reading R18): c_floor = the
// largest code with fl64(M g(c)) <= 1/2 (every sample quantizes to 0),
// c_cap = the largest with fl64(M g(c)) <= 2^31 - 1 (no quantized sample
// leaves 32 bits; integer dtypes: 0), both clamped to [cmin, cmax].
// Exact integer arithmetic on M = m 2^e (m an integer below 2^53): with
// v = m (16 + f), M g(c) = v 2^(e + k - 4), so fl64(M g) <= 1/2 reads
// fl64(v) <= 2^(3 - e - k).  ROUND: v is rounded to 53 bits (binary64 M);
// otherwise it is exact (m below 2^24 or an integer below 2^31).
//  * The smallest t with 16 m <= 2^t is t0 = bitlen(m) + 3 (m a power of two)
//    or + 4; k0 = 3 - e - t0 is the top octave that fits at f = 0, and no
//    code of octave k0 + 1 fits (2^(t0-1) < 16 m, also after rounding since
//    16 m - 2^(t0-1) >= 16 exceeds half an ulp for t0 <= 57).
//  * f = the largest f <= 15 with fl64(m (16 + f)) <= 2^t0, i.e.
//    m (16 + f) <= 2^t0 + 2^(t0-53) when rounding (the tie rounds to even
//    2^t0), found by a 4-step binary search.
//  * g(c + 512) = 2^32 g(c) exactly, so c_cap is c_floor + 512 when
//    fl64(M g(c_floor)) <= 1/2 - 2^-32 and c_floor + 511 otherwise (the code
//    below c_floor is at most 31/32 of its gain, far below that bound).
template <bool ROUND>
__host__ __device__ __forceinline__ void bracket_me(uint64_t m, int e, int cmin, int cmax, bool isint, int& cf,
                                                    int& cc) {
  if (m == 0) {
    cf = cmax;
    cc = isint ? 0 : cmax;
    return;
  }
  const int b = 64 - __builtin_clzll(m);
  const bool p2 = (m & (m - 1)) == 0;
  const int t0 = b + (p2 ? 3 : 4);
  const uint64_t X = (1ull << t0) + ((ROUND && t0 >= 53) ? (1ull << (t0 - 53)) : 0ull);
  uint64_t v = m << 4;
  int f = 0;
#pragma unroll
  for (int s = 3; s >= 0; s--) {
    const uint64_t cand = v + (m << s);
    if (cand <= X) {
      v = cand;
      f += 1 << s;
    }
  }
  const int craw = 16 * (3 - e - t0) + f;
  cf = craw < cmin ? cmin : (craw > cmax ? cmax : craw);
  if (isint) {
    cc = 0;
    return;
  }
  // fl64(v) <= 2^t0 - 2^(t0-31): integer bound, plus half an ulp when rounding
  uint64_t Y;
  if (t0 >= 54) Y = (1ull << t0) - (1ull << (t0 - 31)) + (ROUND ? (1ull << (t0 - 54)) : 0ull);
  else if (t0 >= 31) Y = (1ull << t0) - (1ull << (t0 - 31));
  else Y = (1ull << t0) - 1ull;
  const int ccraw = craw + (v <= Y ? 512 : 511);
  cc = ccraw > cmax ? cmax : (ccraw < cf ? cf : ccraw);
}

__device__ __forceinline__ int clampc(int c, int lo, int hi) { return c < lo ? lo : (c > hi ? hi : c); }

// Quantizer: a = rint(fl64(x) * g), round half to even, binary64.
__device__ __forceinline__ int32_t quant(double x, double g) {
  return (int32_t)__builtin_rint(x * g);
}

// Dequantizer: y = ldexp(fl64(a * R[f]), -k), R[f] = fl64(16 / (16 + f)).
// The 16 correctly rounded quotients are folded at compile time.
__device__ __forceinline__ double inv_mantissa(int c) {
  constexpr double R[16] = {16.0 / 16, 16.0 / 17, 16.0 / 18, 16.0 / 19, 16.0 / 20, 16.0 / 21,
                            16.0 / 22, 16.0 / 23, 16.0 / 24, 16.0 / 25, 16.0 / 26, 16.0 / 27,
                            16.0 / 28, 16.0 / 29, 16.0 / 30, 16.0 / 31};
  return R[c & 15];
}
__device__ __forceinline__ double dequant(int32_t a, int c) {
  return ldexp((double)a * inv_mantissa(c), -(c >> 4));
}
// the same with the code's factors hoisted (R = inv_mantissa(c), e = -(c >> 4))
__device__ __forceinline__ double dequant_rk(int32_t a, double R, int e) {
  return ldexp((double)a * R, e);
}

template <typename T>
__device__ __forceinline__ T to_out(double y) {
  if constexpr (!Traits<T>::isint) {
    return (T)y;  // binary64 -> binary32 cast rounds to nearest even
  } else {
    double r = __builtin_rint(y);
    constexpr double lo = Traits<T>::W == 8 ? -128.0 : (Traits<T>::W == 16 ? -32768.0 : -2147483648.0);
    constexpr double hi = Traits<T>::W == 8 ? 127.0 : (Traits<T>::W == 16 ? 32767.0 : 2147483647.0);
    r = r < lo ? lo : (r > hi ? hi : r);
    return (T)(int32_t)r;
  }
}

// Adaptive rate (Sec. 6 feedback loop): the controller's next state for a
// block of n words at state w: one step towards the target T, inside the
// window of wd states.
__device__ __forceinline__ uint8_t adapt_next(int w, int n, int T, int wd) {
  int s = w + (n < T ? 1 : (n > T ? -1 : 0));
  s = s < 0 ? 0 : (s > wd - 1 ? wd - 1 : s);
  return (uint8_t)s;
}

// Values D positions back in a block held 4 samples per lane (lane gi of a
// segment holds positions 4 gi .. 4 gi + 3): o[m] = v at position 4 gi + m - D
// of the same block, 0 before the block's start.  D is wave-uniform; every
// lane of the wave must take part (lane shuffles).
__device__ __forceinline__ void back_by(const uint32_t v[4], int gi, int D, uint32_t o[4]) {
#pragma unroll
  for (int m = 0; m < 4; m++) {
    const int dl = (D - m + 3) >> 2;  // lanes back
    const int r = (m - D) & 3;        // sample of the source lane
    const uint32_t sv = r == 0 ? v[0] : (r == 1 ? v[1] : (r == 2 ? v[2] : v[3]));
    const uint32_t pv = (uint32_t)__shfl_up((int)sv, (unsigned)(dl < 64 ? dl : 63), 64);
    o[m] = gi >= dl ? pv : 0u;
  }
}

// Inverse of the filter stream over a block of n samples (4 per lane):
// a[p] = v[p] + s a[p - k], as log-step sums over multiples of k (the first
// step carries the sign, the later ones its square).
__device__ __forceinline__ void unfilter(uint32_t r[4], int gi, int k, int neg, int n) {
  bool first = true;
  for (int D = k; D < n; D <<= 1) {
    uint32_t o[4];
    back_by(r, gi, D, o);
#pragma unroll
    for (int m = 0; m < 4; m++) r[m] = (first && neg) ? r[m] - o[m] : r[m] + o[m];
    first = false;
  }
}

// ------------------------------------------------------------ W-bit wrap
template <int W>
__device__ __forceinline__ int32_t wrapw(uint32_t v) {
  if constexpr (W == 32) return (int32_t)v;
  else return ((int32_t)(v << (32 - W))) >> (32 - W);
}

// Exponent of a group (minimal two's-complement width, Sec. 6 BFPE): the
// widest sample is the largest or the smallest; u = max(mx, ~mn) >= 0 is one
// bit narrower than the group, except that u = 0 stands for both {0} and a
// group holding -1, told apart by mn's low bit.  eps saturates at 31;
// width(31) is 32 bits when W = 32.
template <int W>
__device__ __forceinline__ void group_eps(const int32_t v[4], int& eps, int& pw) {
  const int32_t mx = max(max(v[0], v[1]), max(v[2], v[3]));
  const int32_t mn = min(min(v[0], v[1]), min(v[2], v[3]));
  const uint32_t u = (uint32_t)max(mx, ~mn);
  const uint32_t t = (u << 1) | ((uint32_t)mn & 1u);
  const int w = 32 - __clz((int)t);
  eps = w > 31 ? 31 : w;
  pw = (W == 32 && w >= 31) ? 32 : w;
}

// ------------------------------------------------------------ wave helpers
__device__ __forceinline__ int lane_id() { return __lane_id(); }

// DPP lane moves (wave64, GFX9 controls): lane l receives lane l-1 / l+1
// (0 at the wave edge).  Segment edges are masked by the callers.
__device__ __forceinline__ uint32_t shr1(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x138, 0xf, 0xf, true);
}
__device__ __forceinline__ uint32_t shl1(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x130, 0xf, 0xf, true);
}
template <int K>
__device__ __forceinline__ uint32_t row_shr(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x110 + K, 0xf, 0xf, true);
}
__device__ __forceinline__ uint32_t bcast15(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);
}
__device__ __forceinline__ uint32_t bcast31(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);
}

// Keep a value computed where it is: the compiler may otherwise move a DPP
// lane move that only feeds one arm of a select into that arm, where lanes
// outside it are disabled and read as zero.
__device__ __forceinline__ uint32_t pin(uint32_t v) {
  asm volatile("" : "+v"(v));
  return v;
}

// inclusive scan (sum mod 2^32) inside segments of LPB lanes
template <int LPB>
__device__ __forceinline__ uint32_t seg_scan_add(uint32_t v) {
  v += row_shr<1>(v);
  v += row_shr<2>(v);
  v += row_shr<4>(v);
  v += row_shr<8>(v);
  if constexpr (LPB >= 32) v += bcast15(v);
  if constexpr (LPB == 64) v += bcast31(v);
  return v;
}
template <int LPB>
__device__ __forceinline__ uint32_t seg_scan_max(uint32_t v) {
  v = max(v, row_shr<1>(v));
  v = max(v, row_shr<2>(v));
  v = max(v, row_shr<4>(v));
  v = max(v, row_shr<8>(v));
  if constexpr (LPB >= 32) v = max(v, bcast15(v));
  if constexpr (LPB == 64) v = max(v, bcast31(v));
  return v;
}
// value of the last lane of this lane's segment (after an inclusive scan)
template <int LPB>
__device__ __forceinline__ uint32_t seg_last(uint32_t v, int seg) {
  if constexpr (LPB == 64) {
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
  } else if constexpr (LPB == 32) {
    uint32_t a = (uint32_t)__builtin_amdgcn_readlane((int)v, 31);
    uint32_t b = (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
    return seg ? b : a;
  } else {
    uint32_t a = (uint32_t)__builtin_amdgcn_readlane((int)v, 15);
    uint32_t b = (uint32_t)__builtin_amdgcn_readlane((int)v, 31);
    uint32_t c = (uint32_t)__builtin_amdgcn_readlane((int)v, 47);
    uint32_t d = (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
    return seg == 0 ? a : (seg == 1 ? b : (seg == 2 ? c : d));
  }
}
// per-segment popcount of a wave mask, as a value of this lane's segment
template <int LPB>
__device__ __forceinline__ int seg_popc(uint64_t m, int seg) {
  if constexpr (LPB == 64) {
    return __popcll(m);
  } else if constexpr (LPB == 32) {
    int a = __popc((uint32_t)m), b = __popc((uint32_t)(m >> 32));
    return seg ? b : a;
  } else {
    int a = __popc((uint32_t)m & 0xFFFFu), b = __popc((uint32_t)(m >> 16) & 0xFFFFu);
    int c = __popc((uint32_t)(m >> 32) & 0xFFFFu), d = __popc((uint32_t)(m >> 48));
    return seg == 0 ? a : (seg == 1 ? b : (seg == 2 ? c : d));
  }
}
// x when sel, else 0, without a select over memory
__device__ __forceinline__ uint32_t pick(bool sel, uint32_t x) { return x & (0u - (uint32_t)sel); }

template <int LPB>
__device__ __forceinline__ uint64_t seg_bits(int seg) {
  if constexpr (LPB == 64) return ~0ull;
  else return ((1ull << LPB) - 1ull) << (LPB * seg);
}

// value from lane (gi - d) of the same segment (caller masks gi < d)
template <int LPB>
__device__ __forceinline__ int32_t up(int32_t v, int d) { return __shfl_up(v, (unsigned)d, LPB); }
template <int LPB>
__device__ __forceinline__ int32_t dn(int32_t v, int d) { return __shfl_down(v, (unsigned)d, LPB); }

template <int LPB>
__device__ __forceinline__ int32_t seg_sum(int32_t v) {
#pragma unroll
  for (int o = 1; o < LPB; o <<= 1) v += __shfl_xor(v, o, LPB);
  return v;
}
template <int LPB>
__device__ __forceinline__ uint32_t seg_max_u(uint32_t v) {
#pragma unroll
  for (int o = 1; o < LPB; o <<= 1) {
    uint32_t t = (uint32_t)__shfl_xor((int)v, o, LPB);
    v = t > v ? t : v;
  }
  return v;
}
template <int LPB>
__device__ __forceinline__ int32_t seg_excl_scan(int32_t v, int gi) {
  int32_t inc = v;
#pragma unroll
  for (int o = 1; o < LPB; o <<= 1) {
    int32_t t = __shfl_up(inc, (unsigned)o, LPB);
    if (gi >= o) inc += t;
  }
  return inc - v;
}

// number of set bits of m below this lane, inside this lane's segment
template <int LPB>
__device__ __forceinline__ int below_in_seg(uint64_t m, int seg) {
  int all = __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0));
  if constexpr (LPB == 64) return all;
  else return all - __popcll(m & ((1ull << (LPB * seg)) - 1ull));
}

// JEE (Sec. 6), greedy parse as bit arithmetic.  m: positions whose exponent
// difference is in [-1, 1] (bit 0 of every segment clear, so runs never
// cross segments).  Inside a maximal run starting at p the greedy parse emits
// tokens at p, p+2, ... (pairs, plus a single at the end of an odd run).
// Adding the run-start bit of every run that starts on an even position
// clears exactly those runs; what survives are the odd-start runs.
__device__ __forceinline__ uint64_t jee_token_starts(uint64_t m) {
  const uint64_t E = 0x5555555555555555ull;
  uint64_t st = m & ~(m << 1);
  uint64_t rodd = (m + (st & E)) & m;
  uint64_t reven = m & ~rodd;
  return (reven & E) | (rodd & ~E);
}

}  // namespace apax
