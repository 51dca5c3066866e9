// block.h -- per-block analysis shared by the encode and profile kernels.
//
// A wavefront holds 64/LPB blocks; lane gi of segment seg owns group gi of
// block j.  For a given gain code it quantizes its 4 samples, forms every
// candidate derivative stream (Sec. 5 / Sec. 6 redundancy remover), the group
// exponent of each stream, and the block size of each stream: header + JEE
// tokens (bit arithmetic on ballots, scalar unit) + BFPE payload (DPP
// segmented sums, two streams packed per 32-bit lane value).  x-neighbours
// move with DPP wave shifts; y/z-neighbours through a per-wave LDS exchange.
//
// Cost notes (the kernels are bound by vector instruction issue):
//  * the block bracket is integer arithmetic on the bits of the block max,
//    so with one block per wave it runs on the scalar unit;
//  * a wave whose lanes all own 4 samples of a real block ("dense": every
//    block except those at the array edge) skips the validity masks;
//  * x-differences take the predecessor's value through a DPP add of its
//    negation (the sending lane zeroes it at a brick-row end), so no masking
//    is needed on the receiving side; y/z predecessors outside the brick read
//    a zero entry of the exchange;
//  * with one block per wave the chosen stream is wave-uniform and is formed
//    alone (a scalar branch) instead of being selected out of all of them.
#pragma once
#include "codec.h"

namespace apax {

constexpr int XCH = 65;  // LDS exchange entries per wave: one per lane, then a zero entry

template <int LPB>
struct LaneMap {
  int lane, seg, gi;
  int z, y, xq;
  bool hx, hy, hz;
  uint32_t sxm;     // all ones when this lane's x-successor continues its brick row
  int ry, rz, ryz;  // exchange entries of the y-, z- and yz-predecessors (XCH - 1 when absent)
};

template <int LPB>
__device__ __forceinline__ LaneMap<LPB> lane_map(const Geo& g) {
  LaneMap<LPB> L;
  L.lane = lane_id();
  L.seg = L.lane / LPB;
  L.gi = L.lane % LPB;
  const bool own = L.gi < g.G;
  int gi = own ? L.gi : 0;
  L.z = (int)fdiv((uint32_t)gi, g.plane_m, g.plane_s);
  int r = gi - L.z * g.plane;
  L.y = (int)fdiv((uint32_t)r, g.rowq_m, g.rowq_s);
  L.xq = r - L.y * g.rowq;
  L.hx = L.xq > 0;
  L.hy = L.y > 0;
  L.hz = L.z > 0;
  L.sxm = (own && L.gi + 1 < LPB && L.xq < g.rowq - 1) ? ~0u : 0u;
  L.ry = L.hy ? L.lane - g.rowq : XCH - 1;
  L.rz = L.hz ? L.lane - g.plane : XCH - 1;
  L.ryz = (L.hz && L.hy) ? L.lane - g.plane - g.rowq : XCH - 1;
  return L;
}

// Brick coordinates of block j (bricks in row-major order).
__device__ __forceinline__ void brick_of(const Geo& g, int64_t j, int64_t& bz, int64_t& by, int64_t& bx) {
  uint32_t jj = (uint32_t)j;
  uint32_t nbx = (uint32_t)g.nbx, nby = (uint32_t)g.nby;
  uint32_t t = fdiv(jj, g.nbx_m, g.nbx_s);
  bx = jj - t * nbx;
  bz = fdiv(t, g.nby_m, g.nby_s);
  by = t - (uint32_t)bz * nby;
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
    int64_t bz, by, bx;
    brick_of(g, j, bz, by, bx);
    X = bx * g.b[2] + 4 * L.xq;
    Y = by * g.b[1] + L.y;
    Z = bz * g.b[0] + L.z;
  }
  if (X >= g.n[2] || Y >= g.n[1] || Z >= g.n[0]) {
    nvalid = 0;
    return -1;
  }
  int64_t rem = g.n[2] - X;
  nvalid = rem >= 4 ? 4 : (int)rem;
  return (Z * g.n[1] + Y) * g.n[2] + X;
}

// Block j of a one-block-per-wave layout lies wholly inside the array, every
// lane owns a group (G = 64), and its lane offsets fit 31 bits with rows
// 4-sample aligned (g.dense_ok, set on the host): then sample 0 of block j is
// at `base` and the lane's group at base + off (elements).
template <int NDIM, int LPB>
__device__ __forceinline__ bool dense_block(const Geo& g, const LaneMap<LPB>& L, int64_t j, int64_t& base,
                                            uint32_t& off) {
  if constexpr (LPB != 64) {
    return false;
  } else {
    const uint32_t jj = (uint32_t)__builtin_amdgcn_readfirstlane((int)j);  // j < 2^31
    if (!g.dense_ok || g.G != 64 || (int64_t)jj >= g.nblocks) return false;
    if constexpr (NDIM == 1) {
      if ((int64_t)jj >= (int64_t)g.fbx) return false;
      base = (int64_t)jj * g.b[2];
    } else {
      const uint32_t t = fdiv(jj, g.nbx_m, g.nbx_s);
      const uint32_t bx = jj - t * (uint32_t)g.nbx;
      const uint32_t bz = fdiv(t, g.nby_m, g.nby_s);
      const uint32_t by = t - bz * (uint32_t)g.nby;
      if (bx >= (uint32_t)g.fbx || by >= (uint32_t)g.fby || bz >= (uint32_t)g.fbz) return false;
      base = (int64_t)bz * g.sz + (int64_t)by * g.sy + (int64_t)bx * g.b[2];
    }
    off = ((uint32_t)L.z * (uint32_t)g.n[1] + (uint32_t)L.y) * (uint32_t)g.n[2] + 4u * (uint32_t)L.xq;
    return true;
  }
}

template <typename T>
__device__ __forceinline__ void load4_full(const T* __restrict__ p, T v[4]) {
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
}

template <typename T>
__device__ __forceinline__ void load4(const T* __restrict__ x, int64_t idx, int nvalid, T v[4]) {
  v[0] = v[1] = v[2] = v[3] = (T)0;
  if (nvalid <= 0) return;
  const T* p = x + idx;
  bool aligned = (((uintptr_t)p) & (4 * sizeof(T) - 1)) == 0;
  if (nvalid == 4 && aligned) {
    load4_full<T>(p, v);
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
  // 1-d: stream 3 is the filter stream (allowed by the mask only when the
  // array has one)
  static constexpr uint32_t NDMASK = NDIM == 1 ? 0x0Fu : (NDIM == 2 ? 0x2Fu : 0x7Fu);
  static constexpr int BIG = 0x7FFFFFFF;

  LaneMap<LPB> L;
  int64_t j;
  bool act;      // this lane owns a real group of a real block
  bool blk_ok;   // this lane's block exists
  bool dense;    // wave-uniform: every lane of the wave owns 4 valid samples
  int nvalid;
  double xd[4];  // float dtypes: samples as binary64 (0 past the edge)
  int32_t xi[4]; // integer dtypes: the samples
  int cf, cc;    // code bracket (segment-uniform)
  bool nonfinite;  // segment-uniform: the block holds NaN or Inf
  uint64_t vpos; // ballot: lanes with a JEE position (1 <= gi < G)
  uint4* xch;    // per-wave LDS exchange (XCH entries), used for NDIM >= 2

  __device__ __forceinline__ void init(const Geo& g, int64_t j_, uint4* xch_) {
    L = lane_map<LPB>(g);
    j = j_;
    blk_ok = j < g.nblocks;
    act = blk_ok && L.gi < g.G;
    vpos = __ballot(act && L.gi >= 1);
    xch = xch_;
    if (NDIM >= 2 && xch_ && L.lane == 0) xch_[XCH - 1] = make_uint4(0u, 0u, 0u, 0u);
  }

  // sample k as binary64
  __device__ __forceinline__ double xv(int k) const {
    if constexpr (ISINT) return (double)xi[k];
    else return xd[k];
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
    int64_t base;
    uint32_t off;
    // dense: a whole block per wave, every group 4 aligned samples (x 16-byte
    // aligned for the vector loads); wave-uniform
    const bool aligned = (((uintptr_t)x) & (4 * sizeof(T) - 1)) == 0;
    if (aligned && dense_block<NDIM, LPB>(g, L, j, base, off)) {
      dense = true;
      nvalid = 4;
      load4_full<T>(x + base + off, v);
      return;
    }
    int64_t idx = -1;
    nvalid = 0;
    if (act) idx = group_index<NDIM, LPB>(g, L, j, nvalid);
    load4<T>(x, idx, nvalid, v);
    dense = __ballot(act && nvalid == 4) == ~0ull;
  }

  template <bool BRACKET = true>
  __device__ __forceinline__ void take(const Geo& g, const T v[4]) {
#pragma unroll
    for (int k = 0; k < 4; k++) {
      if constexpr (ISINT) xi[k] = (int32_t)v[k];
      else xd[k] = (double)v[k];
    }
    nonfinite = false;
    cf = cc = 0;
    if constexpr (!BRACKET) return;
    // block max |x| as a magnitude key (monotone in |x|; NaN and Inf above
    // every finite value)
    if constexpr (sizeof(T) <= 4) {
      uint32_t key;
      if constexpr (ISINT) {
        const int32_t mx = max(max(xi[0], xi[1]), max(xi[2], xi[3]));
        const int32_t mn = min(min(xi[0], xi[1]), min(xi[2], xi[3]));
        key = max((uint32_t)max(mx, 0), 0u - (uint32_t)min(mn, 0));
      } else {
        uint32_t k4[4];
#pragma unroll
        for (int k = 0; k < 4; k++) k4[k] = __builtin_bit_cast(uint32_t, (float)v[k]) & 0x7FFFFFFFu;
        key = max(max(k4[0], k4[1]), max(k4[2], k4[3]));
      }
      key = seg_last<LPB>(seg_scan_max<LPB>(key), L.seg);
      uint64_t m;
      int e;
      if constexpr (ISINT) {
        m = key;
        e = 0;
      } else {
        nonfinite = key >= 0x7F800000u;
        const uint32_t E = key >> 23;
        m = (uint64_t)((key & 0x7FFFFFu) | (E ? 0x800000u : 0u));
        e = E ? (int)E - 150 : -149;
      }
      bracket_me<false>(m, e, g.cmin, g.cmax, ISINT, cf, cc);
    } else {
      uint64_t k4[4];
#pragma unroll
      for (int k = 0; k < 4; k++) k4[k] = __builtin_bit_cast(uint64_t, xd[k]) & 0x7FFFFFFFFFFFFFFFull;
      const uint64_t key = max(max(k4[0], k4[1]), max(k4[2], k4[3]));
      const uint32_t hi = seg_last<LPB>(seg_scan_max<LPB>((uint32_t)(key >> 32)), L.seg);
      uint32_t lo = (uint32_t)(key >> 32) == hi ? (uint32_t)key : 0u;
      lo = seg_last<LPB>(seg_scan_max<LPB>(lo), L.seg);
      nonfinite = hi >= 0x7FF00000u;
      const uint32_t E = hi >> 20;
      const uint64_t m = ((uint64_t)(hi & 0xFFFFFu) << 32 | lo) | (E ? (1ull << 52) : 0ull);
      const int e = E ? (int)E - 1075 : -1074;
      bracket_me<true>(m, e, g.cmin, g.cmax, false, cf, cc);
    }
  }

  __device__ __forceinline__ bool valid(int k) const { return k < nvalid; }

  // quantized samples at code c (lossless: the integers themselves); samples
  // past the edge are 0 and quantize to 0
  __device__ __forceinline__ void quantize(int c, bool lossless, int32_t a[4]) const {
    if constexpr (ISINT) {
      if (lossless) {
#pragma unroll
        for (int k = 0; k < 4; k++) a[k] = xi[k];
        return;
      }
    }
    const double gv = gain_of(c);
#pragma unroll
    for (int k = 0; k < 4; k++) a[k] = quant(xv(k), gv);
  }

  // x difference of a 4-sample run per lane: sample 0's predecessor is the
  // previous lane's sample 3, sent negated (zero where this lane's brick row
  // does not continue) and added by a DPP lane shift
  __device__ __forceinline__ void xdiff(const uint32_t s[4], uint32_t o[4]) const {
    uint32_t n3 = 0u - s[3];
    if constexpr (!(NDIM == 1 && LPB == 64)) n3 &= L.sxm;
    o[0] = s[0] + shr1(n3);
    o[1] = s[1] - s[0];
    o[2] = s[2] - s[1];
    o[3] = s[3] - s[2];
  }

  // the filter stream x[n] - s x[n-k] of the 1-d block (Sec. 5 / Sec. 6)
  __device__ __forceinline__ void filt(const Geo& g, const uint32_t s_[4], uint32_t o[4]) const {
    uint32_t pv[4];
    back_by(s_, L.gi, g.fk, pv);
#pragma unroll
    for (int k = 0; k < 4; k++) o[k] = g.fneg ? s_[k] + pv[k] : s_[k] - pv[k];
  }

  // the y (and z) predecessors through the wave's LDS exchange
  __device__ __forceinline__ void exchange(const uint32_t A[4], uint32_t Q[4], uint32_t R[4], uint32_t RQ[4],
                                           bool needz) const {
    xch[L.lane] = make_uint4(A[0], A[1], A[2], A[3]);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    const uint4 q = xch[L.ry];
    Q[0] = q.x; Q[1] = q.y; Q[2] = q.z; Q[3] = q.w;
    if (NDIM == 3 && needz) {
      const uint4 r = xch[L.rz], rq = xch[L.ryz];
      R[0] = r.x; R[1] = r.y; R[2] = r.z; R[3] = r.w;
      RQ[0] = rq.x; RQ[1] = rq.y; RQ[2] = rq.z; RQ[3] = rq.w;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
  }

  // wrap to W bits; zero samples past the edge (DENSE: the wave has none)
  template <bool DENSE>
  __device__ __forceinline__ void finish(const uint32_t s[4], int32_t v[4]) const {
#pragma unroll
    for (int k = 0; k < 4; k++) v[k] = wrapw<W>(s[k]);
    if constexpr (!DENSE) {
#pragma unroll
      for (int k = 0; k < 4; k++) v[k] = valid(k) ? v[k] : 0;
    }
  }

  // candidate streams 0..6 (only those of NDIM in `need` are formed; `need`
  // is wave-uniform), mod 2^W, 0 past the edge
  __device__ __forceinline__ void streams(const Geo& g, const int32_t a[4], int32_t v[7][4],
                                          uint32_t need = 0x7Fu) const {
    if (dense) streams_t<true>(g, a, v, need);
    else streams_t<false>(g, a, v, need);
  }
  template <bool DENSE>
  __device__ __forceinline__ void streams_t(const Geo& g, const int32_t a[4], int32_t v[7][4],
                                            uint32_t need) const {
    const uint32_t nd = (uint32_t)__builtin_amdgcn_readfirstlane((int)(NDMASK & need));  // wave-uniform
    uint32_t A[4] = {(uint32_t)a[0], (uint32_t)a[1], (uint32_t)a[2], (uint32_t)a[3]};
    uint32_t s[4];
#pragma unroll
    for (int t = 0; t < 7; t++)
#pragma unroll
      for (int k = 0; k < 4; k++) v[t][k] = 0;
    if (nd & 1u) finish<DENSE>(A, v[0]);
    if (nd & 6u) {
      uint32_t d[4];
      xdiff(A, d);
      if (nd & 2u) finish<DENSE>(d, v[1]);
      if (nd & 4u) {
        xdiff(d, s);
        finish<DENSE>(s, v[2]);
      }
    }
    if constexpr (NDIM == 1) {
      if (nd & 8u) {
        uint32_t F[4];
        filt(g, A, F);
        finish<DENSE>(F, v[3]);
      }
    }
    if (NDIM >= 2 && (nd & 0x78u)) {
      uint32_t Q[4], R[4], RQ[4];
      exchange(A, Q, R, RQ, (nd & 0x50u) != 0);
      uint32_t f[4];
#pragma unroll
      for (int k = 0; k < 4; k++) f[k] = A[k] - Q[k];
      if (nd & 8u) finish<DENSE>(f, v[3]);
      if (nd & 0x20u) {
        xdiff(f, s);
        finish<DENSE>(s, v[5]);
      }
      if (NDIM == 3 && (nd & 0x50u)) {
        uint32_t h[4], u[4];
#pragma unroll
        for (int k = 0; k < 4; k++) {
          h[k] = A[k] - R[k];
          // dz dy a = a - a(y-1) - a(z-1) + a(y-1, z-1)
          u[k] = f[k] - R[k] + RQ[k];
        }
        if (nd & 0x10u) finish<DENSE>(h, v[4]);
        if (nd & 0x40u) {
          xdiff(u, s);
          finish<DENSE>(s, v[6]);
        }
      }
    }
  }

  // stream st alone (st wave-uniform: one block per wave), mod 2^W, 0 past the edge
  __device__ __forceinline__ void stream_one(const Geo& g, int st, const int32_t a[4], int32_t vv[4]) const {
    const int su = __builtin_amdgcn_readfirstlane(st);
    int32_t v[7][4];
    switch (su) {
      case 0: streams(g, a, v, 1u); break;
      case 1: streams(g, a, v, 2u); break;
      case 2: streams(g, a, v, 4u); break;
      case 3: streams(g, a, v, 8u); break;
      case 4: streams(g, a, v, 0x10u); break;
      case 5: streams(g, a, v, 0x20u); break;
      default: streams(g, a, v, 0x40u); break;
    }
#pragma unroll
    for (int k = 0; k < 4; k++) {
      int32_t r = v[0][k];
#pragma unroll
      for (int t = 1; t < 7; t++)
        if ((NDMASK >> t) & 1) r |= v[t][k];
      vv[k] = r;
    }
  }

  // exponent and payload width of a lane's group; zero for lanes without one
  template <bool DENSE = false>
  __device__ __forceinline__ void eps_of(const int32_t v[4], int& e, int& p) const {
    group_eps<W>(v, e, p);
    if (!DENSE && !act) {
      e = 0;
      p = 0;
    }
  }

  // JEE token nibbles of one stream for each segment's block (value of this lane's segment)
  __device__ __forceinline__ int token_nibbles(int eps) const {
    uint64_t m1, m2;
    jee_masks(eps, m1, m2);
    uint64_t Tm = jee_token_starts(m1);
    uint64_t starts = Tm | (~m1 & vpos);
    uint64_t ab = ~m2 & vpos;
    return seg_popc<LPB>(starts, L.seg) + seg_popc<LPB>(ab, L.seg);
  }

  // positions whose exponent difference lies in [-1, 1] (m1) and [-2, 2] (m2)
  __device__ __forceinline__ void jee_masks(int eps, uint64_t& m1, uint64_t& m2) const {
    const uint32_t e = (uint32_t)eps, em1 = shr1(e);
    const uint32_t ad = max(e, em1) - min(e, em1);  // |eps - eps_prev| (v_sad_u32)
    m1 = __ballot(ad <= 1u) & vpos;
    m2 = __ballot(ad <= 2u) & vpos;
  }

  // sizes (bits) of every allowed stream (mask wave-uniform).  Each stream is
  // costed as soon as it is formed -- exponents, JEE token count, payload
  // width -- so no stream's values outlive its own costing.
  __device__ __forceinline__ void costs(const Geo& g, uint32_t mask, const int32_t a[4], Costs& C) const {
    if (dense) costs_t<true>(g, mask, a, C);
    else costs_t<false>(g, mask, a, C);
  }
  template <bool DENSE>
  __device__ __forceinline__ void costs_t(const Geo& g, uint32_t mask, const int32_t a[4], Costs& C) const {
    const uint32_t nd = (uint32_t)__builtin_amdgcn_readfirstlane((int)(NDMASK & mask));  // wave-uniform
    const uint32_t A[4] = {(uint32_t)a[0], (uint32_t)a[1], (uint32_t)a[2], (uint32_t)a[3]};
    uint32_t pk[4] = {0u, 0u, 0u, 0u};  // payload widths, streams 2i and 2i+1 in the halves of pk[i]
    int tk[7] = {0, 0, 0, 0, 0, 0, 0};
    auto cost1 = [&](int t, const uint32_t s[4]) {
      int32_t v[4];
      finish<DENSE>(s, v);
      int e, p;
      eps_of<DENSE>(v, e, p);
      tk[t] = token_nibbles(e);
      pk[t >> 1] |= (uint32_t)p << (16 * (t & 1));
    };
    if (nd & 1u) cost1(0, A);
    if (nd & 6u) {
      uint32_t d[4];
      xdiff(A, d);
      if (nd & 2u) cost1(1, d);
      if (nd & 4u) {
        uint32_t s2[4];
        xdiff(d, s2);
        cost1(2, s2);
      }
    }
    if constexpr (NDIM == 1) {
      if (nd & 8u) {
        uint32_t F[4];
        filt(g, A, F);
        cost1(3, F);
      }
    }
    if (NDIM >= 2 && (nd & 0x78u)) {
      uint32_t Q[4], R[4], RQ[4], f[4];
      exchange(A, Q, R, RQ, (nd & 0x50u) != 0);
#pragma unroll
      for (int k = 0; k < 4; k++) f[k] = A[k] - Q[k];
      if (nd & 8u) cost1(3, f);
      if (nd & 0x20u) {
        uint32_t s5[4];
        xdiff(f, s5);
        cost1(5, s5);
      }
      if (NDIM == 3 && (nd & 0x50u)) {
        uint32_t h[4], u[4];
#pragma unroll
        for (int k = 0; k < 4; k++) {
          h[k] = A[k] - R[k];
          u[k] = f[k] - R[k] + RQ[k];  // dz dy a = a - a(y-1) - a(z-1) + a(y-1, z-1)
        }
        if (nd & 0x10u) cost1(4, h);
        if (nd & 0x40u) {
          uint32_t s6[4];
          xdiff(u, s6);
          cost1(6, s6);
        }
      }
    }
    // payload bits: two streams per 32-bit sum (each segment total <= 64 * 32)
    uint32_t pay[8];
#pragma unroll
    for (int i = 0; i < 4; i++) {
      uint32_t tot = 0;
      if (nd & (3u << (2 * i))) tot = seg_last<LPB>(seg_scan_add<LPB>(pk[i]), L.seg);
      pay[2 * i] = tot & 0xFFFFu;
      pay[2 * i + 1] = tot >> 16;
    }
#pragma unroll
    for (int t = 0; t < 7; t++) C.sz[t] = ((nd >> t) & 1) ? H + 4 * tk[t] + 4 * (int)pay[t] : BIG;
    C.sz[7] = ((mask >> 7) & 1) ? H + g.B * W : BIG;
  }

  // The cheapest stream of `mask` and its size (`best`), exactly as costs()
  // + argmin() (ties: the lowest id), by branch and bound: streams are
  // formed most-likely-smallest first, two at a time, their payload sizes
  // summed in one scan per pair, and a stream's JEE token count is taken
  // only where its payload plus the minimum token bits (half a nibble per
  // position) could still beat or tie, with a lower id, the best so far in
  // some block of the wave.
  __device__ __forceinline__ int best_stream(const Geo& g, uint32_t mask, const int32_t a[4], int32_t& best) const {
    return dense ? best_stream_t<true>(g, mask, a, best) : best_stream_t<false>(g, mask, a, best);
  }
  template <bool DENSE>
  __device__ __forceinline__ int best_stream_t(const Geo& g, uint32_t mask, const int32_t a[4], int32_t& best) const {
    const uint32_t nd = (uint32_t)__builtin_amdgcn_readfirstlane((int)(NDMASK & mask));  // wave-uniform
    const uint32_t A[4] = {(uint32_t)a[0], (uint32_t)a[1], (uint32_t)a[2], (uint32_t)a[3]};
    const int tmin = 4 * (g.G / 2);
    int bs = 7;
    best = ((mask >> 7) & 1) ? H + g.B * W : BIG;
    // one stream's exponent and payload width per lane
    auto prep = [&](const uint32_t s[4], int& e, int& p) {
      int32_t v[4];
      finish<DENSE>(s, v);
      eps_of<DENSE>(v, e, p);
    };
    // a stream whose payload bits `tot` are known: its tokens, if it can win
    auto judge = [&](int t, int e, uint32_t tot) {
      const int lb = H + tmin + 4 * (int)tot;
      if (__ballot(blk_ok && (lb < best || (lb == best && t < bs))) == 0) return;
      const int sz = H + 4 * token_nibbles(e) + 4 * (int)tot;
      if (sz < best || (sz == best && t < bs)) {
        best = sz;
        bs = t;
      }
    };
    // two streams (ta, tb; tb < 0: none) with one scan of their packed
    // payload widths (each segment total <= 64 * 128 < 2^16)
    auto pair = [&](int ta, const uint32_t sa[4], int tb, const uint32_t sb[4]) {
      int ea, pa, eb = 0, pb = 0;
      prep(sa, ea, pa);
      if (tb >= 0) prep(sb, eb, pb);
      const uint32_t tot = seg_last<LPB>(seg_scan_add<LPB>((uint32_t)pa | ((uint32_t)pb << 16)), L.seg);
      judge(ta, ea, tot & 0xFFFFu);
      if (tb >= 0) judge(tb, eb, tot >> 16);
    };
    uint32_t d[4];
    if (nd & 6u) xdiff(A, d);
    if (NDIM >= 2 && (nd & 0x78u)) {
      uint32_t Q[4], R[4], RQ[4], f[4];
      exchange(A, Q, R, RQ, (nd & 0x50u) != 0);
#pragma unroll
      for (int k = 0; k < 4; k++) f[k] = A[k] - Q[k];
      if (NDIM == 3 && (nd & 0x50u)) {
        uint32_t h[4], u[4], s6[4];
#pragma unroll
        for (int k = 0; k < 4; k++) {
          h[k] = A[k] - R[k];
          u[k] = f[k] - R[k] + RQ[k];  // dz dy a
        }
        xdiff(u, s6);
        if ((nd & 0x40u) && (nd & 0x10u)) pair(6, s6, 4, h);
        else if (nd & 0x40u) pair(6, s6, -1, s6);
        else pair(4, h, -1, h);
      }
      uint32_t s5[4];
      xdiff(f, s5);
      if ((nd & 0x20u) && (nd & 8u)) pair(5, s5, 3, f);
      else if (nd & 0x20u) pair(5, s5, -1, s5);
      else if (nd & 8u) pair(3, f, -1, f);
    }
    if (nd & 6u) {
      uint32_t s2[4];
      xdiff(d, s2);
      if ((nd & 2u) && (nd & 4u)) pair(1, d, 2, s2);
      else if (nd & 2u) pair(1, d, -1, d);
      else pair(2, s2, -1, s2);
    }
    if constexpr (NDIM == 1) {
      if (nd & 8u) {
        uint32_t F[4];
        filt(g, A, F);
        if (nd & 1u) pair(3, F, 0, A);
        else pair(3, F, -1, F);
      } else if (nd & 1u) {
        pair(0, A, -1, A);
      }
    } else {
      if (nd & 1u) pair(0, A, -1, A);
    }
    return bs;
  }

  // Fixed-rate fit test (this lane's block): whether some stream of `mask`
  // codes the block in at most `lim` bits, i.e. min over the mask <= lim.
  // The streams are tried most-likely-smallest first (the verbatim size
  // needs no work; then the highest-order derivatives of the brick's
  // dimension) and the test stops once every block of the wave fits.
  __device__ __forceinline__ bool fits(const Geo& g, uint32_t mask, const int32_t a[4], int lim) const {
    return dense ? fits_t<true>(g, mask, a, lim) : fits_t<false>(g, mask, a, lim);
  }
  template <bool DENSE>
  __device__ __forceinline__ bool fits_t(const Geo& g, uint32_t mask, const int32_t a[4], int lim) const {
    const uint32_t nd = (uint32_t)__builtin_amdgcn_readfirstlane((int)(NDMASK & mask));  // wave-uniform
    const uint32_t A[4] = {(uint32_t)a[0], (uint32_t)a[1], (uint32_t)a[2], (uint32_t)a[3]};
    bool fit = ((mask >> 7) & 1) && H + g.B * W <= lim;
    // true once every lane's block fits (wave-uniform)
    auto done = [&]() { return __ballot(blk_ok && !fit) == 0; };
    // every JEE position takes at least half a nibble (a pair token covers
    // two), so H + 4 ceil((G - 1) / 2) + payload bounds a stream's size from
    // below: where that bound exceeds lim in every block of the wave, the
    // token count is not needed
    const int tmin = 4 * (g.G / 2);
    auto try1 = [&](const uint32_t s[4]) {
      int32_t v[4];
      finish<DENSE>(s, v);
      int e, p;
      eps_of<DENSE>(v, e, p);
      const uint32_t tot = seg_last<LPB>(seg_scan_add<LPB>((uint32_t)p), L.seg);
      const int lb = H + tmin + 4 * (int)tot;
      if (__ballot(blk_ok && !fit && lb <= lim) == 0) return false;  // no block of the wave can fit with it
      const int tk = token_nibbles(e);
      fit = fit || H + 4 * tk + 4 * (int)tot <= lim;
      return done();
    };
    if (done()) return fit;
    uint32_t d[4];
    if (nd & 6u) xdiff(A, d);
    if (NDIM >= 2 && (nd & 0x78u)) {
      uint32_t Q[4], R[4], RQ[4], f[4];
      exchange(A, Q, R, RQ, (nd & 0x50u) != 0);
#pragma unroll
      for (int k = 0; k < 4; k++) f[k] = A[k] - Q[k];
      if (NDIM == 3 && (nd & 0x50u)) {
        uint32_t h[4], u[4];
#pragma unroll
        for (int k = 0; k < 4; k++) {
          h[k] = A[k] - R[k];
          u[k] = f[k] - R[k] + RQ[k];  // dz dy a
        }
        if (nd & 0x40u) {
          uint32_t s6[4];
          xdiff(u, s6);
          if (try1(s6)) return fit;
        }
        if ((nd & 0x10u) && try1(h)) return fit;
      }
      if (nd & 0x20u) {
        uint32_t s5[4];
        xdiff(f, s5);
        if (try1(s5)) return fit;
      }
      if ((nd & 8u) && try1(f)) return fit;
    }
    if ((nd & 2u) && try1(d)) return fit;
    if (nd & 4u) {
      uint32_t s2[4];
      xdiff(d, s2);
      if (try1(s2)) return fit;
    }
    if constexpr (NDIM == 1) {
      if (nd & 8u) {
        uint32_t F[4];
        filt(g, A, F);
        if (try1(F)) return fit;
      }
    }
    if (nd & 1u) try1(A);
    return fit;
  }

  // size of one stream from its values (segment-uniform)
  __device__ __forceinline__ int size_vals(const int32_t vv[4], int& e, int& p) const {
    eps_of(vv, e, p);
    uint32_t tot = seg_last<LPB>(seg_scan_add<LPB>((uint32_t)p), L.seg);
    return H + 4 * token_nibbles(e) + 4 * (int)tot;
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
    return size_vals(vv, e, p);
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

  // size of stream st at code c (fixed rate probes), and its values
  __device__ __forceinline__ int probe(const Geo& g, uint32_t mask, int c, int st, int32_t vv[4]) const {
    int32_t a[4];
    quantize(c, false, a);
    if constexpr (LPB == 64) {
      stream_one(g, st, a, vv);
    } else {
      int32_t v[7][4];
      streams(g, a, v, mask | 1u);
      select_stream(st, v, vv);
    }
    int e, p;
    return size_vals(vv, e, p);
  }

  // Fixed-rate per-block gain search (cap and descend; reading of the
  // adaptive loop, Sec. 6), from an evaluation at the start code c0 that
  // chose stream st.  Returns the final code (c0 when the block fits there).
  // Probes need only the chosen stream's size.
  __device__ int rate_search(const Geo& g, uint32_t mask, int c0, int st, bool need) const {
    int32_t vv[4];
    const int32_t budget_bits = 32 * g.budget;
    int c = c0, hi = c0, lo = c0;
    bool done = !need;
    int guard = 0;
    while (__ballot(!done)) {
      if (++guard > 4096) break;  // unreachable: c_floor always fits a valid budget
      int ct = done ? c : (c - 16 < cf ? cf : c - 16);
      int s_of = probe(g, mask, ct, st, vv);
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
      int s_of = probe(g, mask, on ? mid : lo, st, vv);
      if (on) {
        if (s_of <= budget_bits) lo = mid;
        else hi = mid;
      }
    }
    return lo;
  }
};

}  // namespace apax
