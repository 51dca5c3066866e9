// block.h -- per-block analysis shared by the encode and profile kernels.
//
// A wavefront holds 64/LPB blocks; lane gi of segment seg owns group gi of
// block j.  For a given gain code it quantizes its 4 samples, forms every
// candidate derivative stream (Sec. 5 / Sec. 6 redundancy remover), the group
// exponent of each stream, and the block size of each stream: header + JEE
// tokens (bit arithmetic on ballots, scalar unit) + BFPE payload (DPP
// segmented scans, two streams packed per 32-bit lane value).  x-neighbours
// move with DPP wave shifts; y/z-neighbours through a per-wave LDS exchange.
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
  L.z = (int)fdiv((uint32_t)gi, g.plane_m, g.plane_s);
  int r = gi - L.z * g.plane;
  L.y = (int)fdiv((uint32_t)r, g.rowq_m, g.rowq_s);
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
  if constexpr (LPB == 64) {  // one block per wave: block coordinates on the scalar unit
    j = ((int64_t)__builtin_amdgcn_readfirstlane((int)(j >> 32)) << 32) |
        (uint32_t)__builtin_amdgcn_readfirstlane((int)j);
  }
  if constexpr (NDIM == 1) {
    X = j * (int64_t)g.b[2] + 4 * L.xq;
  } else {
    uint32_t jj = (uint32_t)j;
    uint32_t nbx = (uint32_t)g.nbx, nby = (uint32_t)g.nby;
    uint32_t t = fdiv(jj, g.nbx_m, g.nbx_s);
    uint32_t bxI = jj - t * nbx;
    uint32_t bzI = fdiv(t, g.nby_m, g.nby_s);
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

// Costs of the candidate streams of one evaluation (segment-uniform values).
struct Costs {
  int32_t sz[8];   // bits per stream (0x7FFFFFFF if not allowed)
};

// Per-lane state of a block held by a wave segment.
template <typename T, int LPB, int NDIM>
struct Blk {
  static constexpr int W = Traits<T>::W;
  static constexpr int H = Traits<T>::H;
  static constexpr bool ISINT = Traits<T>::isint;
  static constexpr uint32_t NDMASK = NDIM == 1 ? 0x07u : (NDIM == 2 ? 0x2Fu : 0x7Fu);
  static constexpr int BIG = 0x7FFFFFFF;

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
  uint4* xch;    // per-wave LDS exchange (64 entries), used for NDIM >= 2

  __device__ __forceinline__ void init(const Geo& g, int64_t j_, uint4* xch_) {
    L = lane_map<LPB>(g);
    j = j_;
    blk_ok = j < g.nblocks;
    act = blk_ok && L.gi < g.G;
    vpos = __ballot(act && L.gi >= 1);
    xch = xch_;
  }

  // BRACKET = false skips the block max and code bracket (callers that get
  // the block's code from elsewhere)
  template <bool BRACKET = true>
  __device__ __forceinline__ void load(const T* __restrict__ x, const Geo& g) {
    T v[4];
    fetch(x, g, v);
    take<BRACKET>(g, v);
  }

  // load() in two halves: fetch() issues the loads of this lane's samples
  // into v[] (other work can run while they are in flight), take() finishes
  // with the values
  __device__ __forceinline__ void fetch(const T* __restrict__ x, const Geo& g, T v[4]) {
    int64_t idx = -1;
    nvalid = 0;
    if (act) idx = group_index<NDIM, LPB>(g, L, j, nvalid);
    load4<T>(x, idx, nvalid, v);
  }

  template <bool BRACKET = true>
  __device__ __forceinline__ void take(const Geo& g, const T v[4]) {
    bool nf = false;
#pragma unroll
    for (int k = 0; k < 4; k++) {
      xd[k] = (double)v[k];
      if constexpr (!ISINT) nf |= !__builtin_isfinite(xd[k]);
    }
    nonfinite = nf;
    if constexpr (!BRACKET) {
      M = 0.0;
      cf = cc = 0;
      return;
    }
    // block max |x|: reduce the magnitude bit patterns (monotone in value)
    if constexpr (sizeof(T) <= 4) {
      uint32_t key = 0;
#pragma unroll
      for (int k = 0; k < 4; k++) {
        uint32_t kk;
        if constexpr (ISINT) {
          int32_t iv = (int32_t)v[k];
          kk = iv < 0 ? (uint32_t)(-(int64_t)iv) : (uint32_t)iv;
        } else {
          kk = __builtin_bit_cast(uint32_t, (float)v[k]) & 0x7FFFFFFFu;
          if (kk > 0x7F800000u) kk = 0;  // NaN never wins
        }
        key = kk > key ? kk : key;
      }
      key = seg_last<LPB>(seg_scan_max<LPB>(key), L.seg);
      if constexpr (ISINT) M = (double)key;
      else M = (double)__builtin_bit_cast(float, key);
    } else {
      uint64_t key = 0;
#pragma unroll
      for (int k = 0; k < 4; k++) {
        uint64_t kk = __builtin_bit_cast(uint64_t, xd[k]) & 0x7FFFFFFFFFFFFFFFull;
        if (kk > 0x7FF0000000000000ull) kk = 0;
        key = kk > key ? kk : key;
      }
      uint32_t hi = seg_last<LPB>(seg_scan_max<LPB>((uint32_t)(key >> 32)), L.seg);
      uint32_t lo = (uint32_t)(key >> 32) == hi ? (uint32_t)key : 0u;
      lo = seg_last<LPB>(seg_scan_max<LPB>(lo), L.seg);
      M = __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
    }
    bracket<T>(M, g.cmin, g.cmax, cf, cc);
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

  // candidate streams 0..6 (only those of NDIM in `need` are formed; `need`
  // is wave-uniform), mod 2^W, 0 past the edge
  __device__ __forceinline__ void streams(const Geo& g, const int32_t a[4], int32_t v[7][4],
                                          uint32_t need = 0x7Fu) const {
    uint32_t A[4] = {(uint32_t)a[0], (uint32_t)a[1], (uint32_t)a[2], (uint32_t)a[3]};
    uint32_t p3 = shr1(A[3]), p2 = shr1(A[2]);
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
    if (NDIM >= 2 && (need & 0x78u)) {
      const int lane = L.lane;
      xch[lane] = make_uint4(A[0], A[1], A[2], A[3]);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      uint4 q = xch[L.hy ? lane - g.rowq : lane];
      uint32_t Q[4] = {q.x, q.y, q.z, q.w};
      uint32_t f[4];
#pragma unroll
      for (int k = 0; k < 4; k++) f[k] = A[k] - (L.hy ? Q[k] : 0u);
      uint32_t fp = shr1(f[3]);
      if (!L.hx) fp = 0;
#pragma unroll
      for (int k = 0; k < 4; k++) s[3][k] = f[k];
      s[5][0] = f[0] - fp;
      s[5][1] = f[1] - f[0];
      s[5][2] = f[2] - f[1];
      s[5][3] = f[3] - f[2];
      if constexpr (NDIM == 3) {
        uint4 r = xch[L.hz ? lane - g.plane : lane];
        uint4 rq = xch[(L.hz && L.hy) ? lane - g.plane - g.rowq : lane];
        uint32_t Rr[4] = {r.x, r.y, r.z, r.w}, RQ[4] = {rq.x, rq.y, rq.z, rq.w};
        uint32_t h[4], u[4];
#pragma unroll
        for (int k = 0; k < 4; k++) {
          h[k] = A[k] - (L.hz ? Rr[k] : 0u);
          // dz dy a = a - a(y-1) - a(z-1) + a(y-1, z-1)
          u[k] = h[k] - (L.hy ? Q[k] : 0u) + ((L.hz && L.hy) ? RQ[k] : 0u);
        }
        uint32_t upv = shr1(u[3]);
        if (!L.hx) upv = 0;
#pragma unroll
        for (int k = 0; k < 4; k++) s[4][k] = h[k];
        s[6][0] = u[0] - upv;
        s[6][1] = u[1] - u[0];
        s[6][2] = u[2] - u[1];
        s[6][3] = u[3] - u[2];
      }
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
    }
#pragma unroll
    for (int t = 0; t < 7; t++) {
      if (!((NDMASK & need) >> t & 1)) {
#pragma unroll
        for (int k = 0; k < 4; k++) v[t][k] = 0;
        continue;
      }
#pragma unroll
      for (int k = 0; k < 4; k++) v[t][k] = valid(k) ? wrapw<W>(s[t][k]) : 0;
    }
  }

  // JEE token nibbles of one stream for each segment's block (value of this lane's segment)
  __device__ __forceinline__ int token_nibbles(int eps) const {
    int em1 = (int)shr1((uint32_t)eps);
    int d = eps - em1;
    bool pos = act && L.gi >= 1;
    uint64_t m1 = __ballot(pos && (uint32_t)(d + 1) <= 2u);
    uint64_t m2 = __ballot(pos && (uint32_t)(d + 2) <= 4u);
    uint64_t Tm = jee_token_starts(m1);
    uint64_t starts = Tm | (~m1 & vpos);
    uint64_t ab = ~m2 & vpos;
    return seg_popc<LPB>(starts, L.seg) + seg_popc<LPB>(ab, L.seg);
  }

  // sizes (bits) of every allowed stream; also the stream values, exponents
  // and payload widths (zero for lanes without a group)
  __device__ __forceinline__ void sizes(const Geo& g, uint32_t mask, const int32_t a[4],
                                        int32_t v[7][4], int eps[7], int pw[7], Costs& C) const {
    streams(g, a, v, mask);
#pragma unroll
    for (int t = 0; t < 7; t++) {
      eps[t] = 0;
      pw[t] = 0;
      if ((NDMASK & mask) >> t & 1) {  // mask is wave-uniform
        group_eps<W>(v[t], eps[t], pw[t]);
        if (!act) { eps[t] = 0; pw[t] = 0; }
      }
    }
    // payload: two streams per 32-bit scan (each segment total <= 64 * 32)
    uint32_t pay[8];
#pragma unroll
    for (int t = 0; t < 7; t += 2) {
      uint32_t pk = (uint32_t)pw[t] | (t + 1 < 7 ? ((uint32_t)pw[t + 1] << 16) : 0u);
      bool need = (((NDMASK & mask) >> t) & 1) || (t + 1 < 7 && (((NDMASK & mask) >> (t + 1)) & 1));
      uint32_t tot = 0;
      if (need) tot = seg_last<LPB>(seg_scan_add<LPB>(pk), L.seg);
      pay[t] = tot & 0xFFFFu;
      pay[t + 1] = tot >> 16;
    }
#pragma unroll
    for (int t = 0; t < 7; t++) {
      C.sz[t] = BIG;
      if (!(((NDMASK & mask) >> t) & 1)) continue;  // mask is wave-uniform
      C.sz[t] = H + 4 * token_nibbles(eps[t]) + 4 * (int)pay[t];
    }
    C.sz[7] = ((mask >> 7) & 1) ? H + g.B * W : BIG;
  }

  // size of one stream st (segment-uniform) at the given values; `only`:
  // streams() formed stream st alone (the others are zero)
  __device__ __forceinline__ int size_of(int st, const int32_t v[7][4], bool only = false) const {
    int32_t vv[4];
    if (only) {
#pragma unroll
      for (int k = 0; k < 4; k++) {
        uint32_t r = 0;
#pragma unroll
        for (int t = 0; t < 7; t++)
          if ((NDMASK >> t) & 1) r |= (uint32_t)v[t][k];
        vv[k] = (int32_t)r;
      }
    } else {
      select_stream(st, v, vv);
    }
    int e, p;
    group_eps<W>(vv, e, p);
    if (!act) { e = 0; p = 0; }
    uint32_t tot = seg_last<LPB>(seg_scan_add<LPB>((uint32_t)p), L.seg);
    return H + 4 * token_nibbles(e) + 4 * (int)tot;
  }

  __device__ __forceinline__ static void select_stream(int st, const int32_t v[7][4], int32_t vv[4]) {
    if constexpr (LPB == 64) {  // st is wave-uniform: conditional moves on a scalar condition
      const int su = __builtin_amdgcn_readfirstlane(st);
#pragma unroll
      for (int k = 0; k < 4; k++) {
        int32_t r = 0;
#pragma unroll
        for (int t = 0; t < 7; t++)
          if ((NDMASK >> t) & 1) r = su == t ? v[t][k] : r;
        vv[k] = r;
      }
      return;
    }
#pragma unroll
    for (int k = 0; k < 4; k++) {
      uint32_t r = 0;
#pragma unroll
      for (int t = 0; t < 7; t++)
        if ((NDMASK >> t) & 1) r |= pick(st == t, (uint32_t)v[t][k]);
      vv[k] = (int32_t)r;
    }
  }

  __device__ __forceinline__ static int pick_int(int st, const int x[7]) {
    if constexpr (LPB == 64) {
      const int su = __builtin_amdgcn_readfirstlane(st);
      int r = 0;
#pragma unroll
      for (int t = 0; t < 7; t++)
        if ((NDMASK >> t) & 1) r = su == t ? x[t] : r;
      return r;
    }
    uint32_t r = 0;
#pragma unroll
    for (int t = 0; t < 7; t++)
      if ((NDMASK >> t) & 1) r |= pick(st == t, (uint32_t)x[t]);
    return (int)r;
  }

  // lowest-id stream of minimal size among mask
  __device__ __forceinline__ static int argmin(const Costs& C, uint32_t mask, int32_t& best) {
    int bs = 0;
    best = BIG;
#pragma unroll
    for (int t = 0; t < 8; t++)
      if (((mask >> t) & 1) && C.sz[t] < best) { best = C.sz[t]; bs = t; }
    return bs;
  }

  __device__ __forceinline__ static int32_t size_sel(const Costs& C, int st) {
    uint32_t r = 0;
#pragma unroll
    for (int t = 0; t < 8; t++) r |= pick(st == t, (uint32_t)C.sz[t]);
    return (int32_t)r;
  }

  // streams a probe of stream st needs: st alone when one block fills the
  // wave (st is then wave-uniform), else every allowed stream
  __device__ __forceinline__ static uint32_t need_mask(int st, uint32_t mask) {
    if constexpr (LPB == 64) return 1u << __builtin_amdgcn_readfirstlane(st);
    else return mask | 1u;
  }

  // Fixed-rate per-block gain search (cap and descend; reading of the
  // adaptive loop, Sec. 6), from an evaluation at the start code c0 that
  // chose stream st.  Returns the final code (c0 when the block fits there).
  // Probes need only the chosen stream's size.
  __device__ int rate_search(const Geo& g, uint32_t mask, int c0, int st, bool need) const {
    int32_t a[4], v[7][4];
    const int32_t budget_bits = 32 * g.budget;
    int c = c0, hi = c0, lo = c0;
    bool done = !need;
    int guard = 0;
    while (__ballot(!done)) {
      if (++guard > 4096) break;  // unreachable: c_floor always fits a valid budget
      int ct = done ? c : (c - 16 < cf ? cf : c - 16);
      quantize(ct, false, a);
      streams(g, a, v, need_mask(st, mask));
      int s_of = size_of(st, v, LPB == 64);
      if (!done) {
        if (s_of <= budget_bits) { done = true; lo = ct; }
        else { hi = ct; }
        c = ct;
      }
    }
    if (!need) { lo = c0; hi = c0; }
    // bisection between the last fitting (lo) and last failing (hi) code
    while (__ballot(hi - lo > 1)) {
      bool on = hi - lo > 1;
      int mid = lo + ((hi - lo) >> 1);
      quantize(on ? mid : lo, false, a);
      streams(g, a, v, need_mask(st, mask));
      int s_of = size_of(st, v, LPB == 64);
      if (on) {
        if (s_of <= budget_bits) lo = mid;
        else hi = mid;
      }
    }
    return lo;
  }
};

}  // namespace apax
