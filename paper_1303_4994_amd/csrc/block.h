// block.h -- per-block analysis shared by the encode and profile kernels.
//
// A wavefront holds 64/LPB blocks; lane gi of segment seg owns group gi of
// block j.  For a given gain code it quantizes its 4 samples, forms every
// candidate derivative stream (Sec. 5 / Sec. 6 redundancy remover), the group
// exponent of each stream, and the block size of each stream: header + JEE
// tokens (bit arithmetic on ballots) + BFPE payload (segmented wave sum).
#pragma once
#include "codec.h"

namespace apax {

template <int LPB>
struct LaneMap {
  int lane, seg, gi;
  int z, y, xq;
  bool hx, hy, hz;
};

template <int LPB>
__device__ __forceinline__ LaneMap<LPB> lane_map(const Geo& g) {
  LaneMap<LPB> L;
  L.lane = lane_id();
  L.seg = L.lane / LPB;
  L.gi = L.lane % LPB;
  int gi = L.gi < g.G ? L.gi : 0;
  L.z = gi / g.plane;
  int r = gi - L.z * g.plane;
  L.y = r / g.rowq;
  L.xq = r - L.y * g.rowq;
  L.hx = L.xq > 0;
  L.hy = L.y > 0;
  L.hz = L.z > 0;
  return L;
}

// Linear index of sample 0 of the lane's group and the number of valid
// samples (0..4) in it; -1 if the group lies past the array edge.
template <int NDIM, int LPB>
__device__ __forceinline__ int64_t group_index(const Geo& g, const LaneMap<LPB>& L, int64_t j,
                                               int& nvalid) {
  int64_t X, Y = 0, Z = 0;
  if constexpr (NDIM == 1) {
    X = j * (int64_t)g.b[2] + 4 * L.xq;
  } else {
    uint32_t jj = (uint32_t)j;
    uint32_t nbx = (uint32_t)g.nbx, nby = (uint32_t)g.nby;
    uint32_t t = jj / nbx;
    uint32_t bxI = jj - t * nbx;
    uint32_t bzI = t / nby;
    uint32_t byI = t - bzI * nby;
    X = (int64_t)bxI * g.b[2] + 4 * L.xq;
    Y = (int64_t)byI * g.b[1] + L.y;
    Z = (int64_t)bzI * g.b[0] + L.z;
  }
  if (X >= g.n[2] || Y >= g.n[1] || Z >= g.n[0]) {
    nvalid = 0;
    return -1;
  }
  int64_t rem = g.n[2] - X;
  nvalid = rem >= 4 ? 4 : (int)rem;
  return (Z * g.n[1] + Y) * g.n[2] + X;
}

template <typename T>
__device__ __forceinline__ void load4(const T* __restrict__ x, int64_t idx, int nvalid, T v[4]) {
  v[0] = v[1] = v[2] = v[3] = (T)0;
  if (nvalid <= 0) return;
  const T* p = x + idx;
  bool aligned = (((uintptr_t)p) & (4 * sizeof(T) - 1)) == 0;
  if (nvalid == 4 && aligned) {
    if constexpr (sizeof(T) == 4) {
      uint4 u = *reinterpret_cast<const uint4*>(p);
      uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
      for (int k = 0; k < 4; k++) v[k] = __builtin_bit_cast(T, w[k]);
    } else if constexpr (sizeof(T) == 8) {
      const uint4* q = reinterpret_cast<const uint4*>(p);
      uint4 u0 = q[0], u1 = q[1];
      v[0] = __builtin_bit_cast(T, ((uint64_t)u0.y << 32) | u0.x);
      v[1] = __builtin_bit_cast(T, ((uint64_t)u0.w << 32) | u0.z);
      v[2] = __builtin_bit_cast(T, ((uint64_t)u1.y << 32) | u1.x);
      v[3] = __builtin_bit_cast(T, ((uint64_t)u1.w << 32) | u1.z);
    } else if constexpr (sizeof(T) == 2) {
      uint2 u = *reinterpret_cast<const uint2*>(p);
      v[0] = (T)(int16_t)(u.x & 0xFFFF);
      v[1] = (T)(int16_t)(u.x >> 16);
      v[2] = (T)(int16_t)(u.y & 0xFFFF);
      v[3] = (T)(int16_t)(u.y >> 16);
    } else {
      uint32_t u = *reinterpret_cast<const uint32_t*>(p);
#pragma unroll
      for (int k = 0; k < 4; k++) v[k] = (T)(int8_t)((u >> (8 * k)) & 0xFF);
    }
  } else {
#pragma unroll
    for (int k = 0; k < 4; k++)
      if (k < nvalid) v[k] = p[k];
  }
}

// Per-lane state of a block held by a wave segment.
template <typename T, int LPB, int NDIM>
struct Blk {
  static constexpr int W = Traits<T>::W;
  static constexpr int H = Traits<T>::H;
  static constexpr bool ISINT = Traits<T>::isint;
  static constexpr uint32_t NDMASK = NDIM == 1 ? 0x07u : (NDIM == 2 ? 0x2Fu : 0x7Fu);

  LaneMap<LPB> L;
  int64_t j;
  bool act;      // this lane owns a real group of a real block
  bool blk_ok;   // this lane's block exists
  int nvalid;
  double xd[4];  // samples (0 past the edge)
  double M;      // block max |x| (segment-uniform)
  int cf, cc;    // code bracket (segment-uniform)
  bool nonfinite;
  uint64_t vpos; // ballot: lanes with a JEE position (1 <= gi < G)

  __device__ __forceinline__ void init(const Geo& g, int64_t j_) {
    L = lane_map<LPB>(g);
    j = j_;
    blk_ok = j < g.nblocks;
    act = blk_ok && L.gi < g.G;
    vpos = __ballot(act && L.gi >= 1);
  }

  __device__ __forceinline__ int64_t load(const T* __restrict__ x, const Geo& g) {
    T v[4];
    int64_t idx = -1;
    nvalid = 0;
    if (act) idx = group_index<NDIM, LPB>(g, L, j, nvalid);
    load4<T>(x, idx, nvalid, v);
    double m = 0.0;
    bool nf = false;
#pragma unroll
    for (int k = 0; k < 4; k++) {
      xd[k] = (double)v[k];
      if constexpr (!ISINT) nf |= !__builtin_isfinite(xd[k]);
      double ax = __builtin_fabs(xd[k]);
      m = ax > m ? ax : m;  // NaN never wins
    }
#pragma unroll
    for (int o = 1; o < LPB; o <<= 1) {
      double t = __shfl_xor(m, o, LPB);
      m = t > m ? t : m;
    }
    M = m;
    nonfinite = nf;
    bracket<T>(M, g.cmin, g.cmax, cf, cc);
    return idx;
  }

  __device__ __forceinline__ bool valid(int k) const { return k < nvalid; }

  // quantized samples at code c (lossless: the integers themselves)
  __device__ __forceinline__ void quantize(int c, bool lossless, int32_t a[4]) const {
    double gv = gain_of(c);
#pragma unroll
    for (int k = 0; k < 4; k++) {
      int32_t q = lossless ? (int32_t)xd[k] : quant(xd[k], gv);
      a[k] = valid(k) ? q : 0;
    }
  }

  // candidate streams 0..6 (only those of NDIM are formed)
  __device__ __forceinline__ void streams(const Geo& g, const int32_t a[4], int32_t v[7][4]) const {
    uint32_t A[4] = {(uint32_t)a[0], (uint32_t)a[1], (uint32_t)a[2], (uint32_t)a[3]};
    uint32_t p3 = (uint32_t)up<LPB>(a[3], 1), p2 = (uint32_t)up<LPB>(a[2], 1);
    if (!L.hx) { p3 = 0; p2 = 0; }
    uint32_t d[4] = {A[0] - p3, A[1] - A[0], A[2] - A[1], A[3] - A[2]};
    uint32_t dp = p3 - p2;
    uint32_t s[7][4];
#pragma unroll
    for (int k = 0; k < 4; k++) { s[0][k] = A[k]; s[1][k] = d[k]; }
    s[2][0] = d[0] - dp;
    s[2][1] = d[1] - d[0];
    s[2][2] = d[2] - d[1];
    s[2][3] = d[3] - d[2];
#pragma unroll
    for (int k = 0; k < 4; k++) { s[3][k] = 0; s[4][k] = 0; s[5][k] = 0; s[6][k] = 0; }
    if constexpr (NDIM >= 2) {
      uint32_t f[4];
#pragma unroll
      for (int k = 0; k < 4; k++) {
        uint32_t q = (uint32_t)up<LPB>(a[k], g.rowq);
        f[k] = A[k] - (L.hy ? q : 0u);
      }
      uint32_t fp = (uint32_t)up<LPB>((int32_t)f[3], 1);
      if (!L.hx) fp = 0;
#pragma unroll
      for (int k = 0; k < 4; k++) s[3][k] = f[k];
      s[5][0] = f[0] - fp;
      s[5][1] = f[1] - f[0];
      s[5][2] = f[2] - f[1];
      s[5][3] = f[3] - f[2];
    }
    if constexpr (NDIM == 3) {
      uint32_t h[4], u[4];
#pragma unroll
      for (int k = 0; k < 4; k++) {
        uint32_t r = (uint32_t)up<LPB>(a[k], g.plane);
        h[k] = A[k] - (L.hz ? r : 0u);
      }
#pragma unroll
      for (int k = 0; k < 4; k++) {
        uint32_t q = (uint32_t)up<LPB>((int32_t)h[k], g.rowq);
        u[k] = h[k] - (L.hy ? q : 0u);
      }
      uint32_t upv = (uint32_t)up<LPB>((int32_t)u[3], 1);
      if (!L.hx) upv = 0;
#pragma unroll
      for (int k = 0; k < 4; k++) s[4][k] = h[k];
      s[6][0] = u[0] - upv;
      s[6][1] = u[1] - u[0];
      s[6][2] = u[2] - u[1];
      s[6][3] = u[3] - u[2];
    }
#pragma unroll
    for (int t = 0; t < 7; t++)
#pragma unroll
      for (int k = 0; k < 4; k++) v[t][k] = valid(k) ? wrapw<W>(s[t][k]) : 0;
  }

  // JEE token nibbles of one stream for this lane's block (segment-uniform)
  __device__ __forceinline__ int token_nibbles(int eps, int G) const {
    int em1 = up<LPB>(eps, 1);
    int d = eps - em1;
    bool pos = act && L.gi >= 1;
    uint64_t m1 = __ballot(pos && (uint32_t)(d + 1) <= 2u);
    uint64_t m2 = __ballot(pos && (uint32_t)(d + 2) <= 4u);
    uint64_t Tm = jee_token_starts(m1);
    uint64_t starts = Tm | (~m1 & vpos);
    uint64_t ab = ~m2 & vpos;
    uint64_t sb = seg_bits<LPB>(L.seg);
    return __popcll(starts & sb) + __popcll(ab & sb);
  }

  // sizes (bits) of every allowed stream at the current quantization; keeps
  // the stream values, exponents and payload widths
  __device__ __forceinline__ void sizes(const Geo& g, uint32_t mask, const int32_t a[4],
                                        int32_t v[7][4], int eps[7], int pw[7], int32_t sz[8]) const {
    streams(g, a, v);
#pragma unroll
    for (int t = 0; t < 7; t++) {
      sz[t] = 0x7FFFFFFF;
      eps[t] = 0;
      pw[t] = 0;
      if (!((NDMASK >> t) & 1)) continue;
      group_eps<W>(v[t], eps[t], pw[t]);
      if (!act) { eps[t] = 0; pw[t] = 0; }
      if (!((mask >> t) & 1)) continue;  // mask is wave-uniform
      int nib = token_nibbles(eps[t], g.G);
      int pay = seg_sum<LPB>(4 * pw[t]);
      sz[t] = H + 4 * nib + pay;
    }
    sz[7] = ((mask >> 7) & 1) ? H + g.B * W : 0x7FFFFFFF;
  }

  // lowest-id stream of minimal size among mask
  __device__ __forceinline__ static int argmin(const int32_t sz[8], uint32_t mask, int32_t& best) {
    int bs = 0;
    best = 0x7FFFFFFF;
#pragma unroll
    for (int t = 0; t < 8; t++)
      if (((mask >> t) & 1) && sz[t] < best) { best = sz[t]; bs = t; }
    return bs;
  }

  // Fixed-rate per-block gain search (cap and descend; reading of the
  // adaptive loop, Sec. 6).  Returns the code; st receives the stream chosen
  // at the start code, kept for the whole search.
  __device__ int rate_search(const Geo& g, uint32_t mask, int cp, int& st) const {
    int32_t a[4], v[7][4], sz[8];
    int eps[7], pw[7];
    const int32_t budget_bits = 32 * g.budget;
    uint32_t m7 = mask & 0x7Fu;
    int c = clampc(cp, cf, cc);
    quantize(c, false, a);
    sizes(g, m7, a, v, eps, pw, sz);
    int32_t best;
    st = argmin(sz, m7, best);
    bool need = act && best > budget_bits;
    if (!__ballot(need)) return c;
    int hi = c, lo = c;
    // descend by octaves (never below c_floor, where everything is 0)
    bool done = !need;
    int guard = 0;
    while (__ballot(!done)) {
      if (++guard > 4096) break;  // unreachable: c_floor always fits a valid budget
      int ct = done ? c : (c - 16 < cf ? cf : c - 16);
      quantize(ct, false, a);
      sizes(g, m7, a, v, eps, pw, sz);
      int32_t s_of = sel8(sz, st);
      if (!done) {
        if (s_of <= budget_bits) { done = true; lo = ct; }
        else { hi = ct; }
        c = ct;
      }
    }
    if (!need) { lo = c; hi = c; }
    // bisection between the last fitting (lo) and last failing (hi) code
    while (__ballot(hi - lo > 1)) {
      bool on = hi - lo > 1;
      int mid = lo + ((hi - lo) >> 1);
      quantize(on ? mid : lo, false, a);
      sizes(g, m7, a, v, eps, pw, sz);
      int32_t s_of = sel8(sz, st);
      if (on) {
        if (s_of <= budget_bits) lo = mid;
        else hi = mid;
      }
    }
    return lo;
  }

  __device__ __forceinline__ static int32_t sel8(const int32_t sz[8], int s) {
    int32_t r = sz[0];
#pragma unroll
    for (int t = 1; t < 8; t++) r = s == t ? sz[t] : r;
    return r;
  }
};

}  // namespace apax
