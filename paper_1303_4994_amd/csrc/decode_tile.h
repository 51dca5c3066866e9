// decode_tile.h -- one tile of the APAX decoder, shared by the single-array
// kernel and the persistent batch kernel.
//
// Same lane layout as the encoder: one wave segment per block, lane gi owns
// group gi.  Per block: offset from the block-length index (superblock offset
// + segmented sum of up to 63 lengths), block words staged in LDS, header
// checked, JEE tokens parsed in parallel -- a nibble is the low half of an
// 8-bit token exactly when it follows an escape nibble that itself starts a
// token, and inside a run of escape-valued nibbles starts alternate, so the
// token starts follow from the same run-parity bit arithmetic as on encode;
// token coverage prefix sums place each exponent difference at its group,
// a segmented scan rebuilds the exponents, an exclusive scan of payload
// widths gives every group's bit offset, values are extracted with 64-bit
// funnel shifts, running sums along x/y/z undo the derivative stream, and
// the dequantizer restores the samples.
#pragma once
#include "block.h"
#include "kernels.h"

namespace apax {

// token-start mask of a nibble sequence (lo = first 64 nibbles, hi = next
// 64); esc marks nibbles with value >= 14.  Returns the "low half" mask.
__device__ __forceinline__ void low_half_mask(uint64_t elo, uint64_t ehi, uint64_t& llo,
                                              uint64_t& lhi) {
  const uint64_t EV = 0x5555555555555555ull;
  // run starts st = M & ~(M << 1) (128-bit shift)
  uint64_t shl_lo = elo << 1, shl_hi = (ehi << 1) | (elo >> 63);
  uint64_t st_lo = elo & ~shl_lo, st_hi = ehi & ~shl_hi;
  uint64_t t_lo = st_lo & EV, t_hi = st_hi & EV;
  // M + t, 128-bit
  uint64_t s_lo = elo + t_lo;
  uint64_t carry = s_lo < elo ? 1ull : 0ull;
  uint64_t s_hi = ehi + t_hi + carry;
  uint64_t rodd_lo = s_lo & elo, rodd_hi = s_hi & ehi;
  uint64_t rev_lo = elo & ~rodd_lo, rev_hi = ehi & ~rodd_hi;
  uint64_t se_lo = (rev_lo & EV) | (rodd_lo & ~EV);
  uint64_t se_hi = (rev_hi & EV) | (rodd_hi & ~EV);
  llo = se_lo << 1;
  lhi = (se_hi << 1) | (se_lo >> 63);
}

template <int LPB>
__device__ __forceinline__ int32_t seg_shfl(int32_t v, int src) {
  return __shfl(v, src, LPB);
}

template <typename T>
__device__ __forceinline__ void store4_full(T* __restrict__ p, const T v[4]) {
  if constexpr (sizeof(T) == 4) {
    uint4 u;
    u.x = __builtin_bit_cast(uint32_t, v[0]);
    u.y = __builtin_bit_cast(uint32_t, v[1]);
    u.z = __builtin_bit_cast(uint32_t, v[2]);
    u.w = __builtin_bit_cast(uint32_t, v[3]);
    *reinterpret_cast<uint4*>(p) = u;
  } else if constexpr (sizeof(T) == 8) {
    uint64_t w[4];
#pragma unroll
    for (int k = 0; k < 4; k++) w[k] = __builtin_bit_cast(uint64_t, v[k]);
    uint4 u0, u1;
    u0.x = (uint32_t)w[0]; u0.y = (uint32_t)(w[0] >> 32); u0.z = (uint32_t)w[1]; u0.w = (uint32_t)(w[1] >> 32);
    u1.x = (uint32_t)w[2]; u1.y = (uint32_t)(w[2] >> 32); u1.z = (uint32_t)w[3]; u1.w = (uint32_t)(w[3] >> 32);
    uint4* q = reinterpret_cast<uint4*>(p);
    q[0] = u0;
    q[1] = u1;
  } else if constexpr (sizeof(T) == 2) {
    uint2 u;
    u.x = (uint32_t)(uint16_t)v[0] | ((uint32_t)(uint16_t)v[1] << 16);
    u.y = (uint32_t)(uint16_t)v[2] | ((uint32_t)(uint16_t)v[3] << 16);
    *reinterpret_cast<uint2*>(p) = u;
  } else {
    uint32_t u = 0;
#pragma unroll
    for (int k = 0; k < 4; k++) u |= (uint32_t)(uint8_t)v[k] << (8 * k);
    *reinterpret_cast<uint32_t*>(p) = u;
  }
}

template <typename T>
__device__ __forceinline__ void store4(T* __restrict__ y, int64_t idx, int nvalid, const T v[4]) {
  if (nvalid <= 0) return;
  T* p = y + idx;
  bool aligned = (((uintptr_t)p) & (4 * sizeof(T) - 1)) == 0;
  if (nvalid == 4 && aligned) {
    if constexpr (sizeof(T) == 4) {
      uint4 u;
      u.x = __builtin_bit_cast(uint32_t, v[0]);
      u.y = __builtin_bit_cast(uint32_t, v[1]);
      u.z = __builtin_bit_cast(uint32_t, v[2]);
      u.w = __builtin_bit_cast(uint32_t, v[3]);
      *reinterpret_cast<uint4*>(p) = u;
    } else if constexpr (sizeof(T) == 8) {
      uint64_t w[4];
#pragma unroll
      for (int k = 0; k < 4; k++) w[k] = __builtin_bit_cast(uint64_t, v[k]);
      uint4 u0, u1;
      u0.x = (uint32_t)w[0]; u0.y = (uint32_t)(w[0] >> 32); u0.z = (uint32_t)w[1]; u0.w = (uint32_t)(w[1] >> 32);
      u1.x = (uint32_t)w[2]; u1.y = (uint32_t)(w[2] >> 32); u1.z = (uint32_t)w[3]; u1.w = (uint32_t)(w[3] >> 32);
      uint4* q = reinterpret_cast<uint4*>(p);
      q[0] = u0;
      q[1] = u1;
    } else if constexpr (sizeof(T) == 2) {
      uint2 u;
      u.x = (uint32_t)(uint16_t)v[0] | ((uint32_t)(uint16_t)v[1] << 16);
      u.y = (uint32_t)(uint16_t)v[2] | ((uint32_t)(uint16_t)v[3] << 16);
      *reinterpret_cast<uint2*>(p) = u;
    } else {
      uint32_t u = 0;
#pragma unroll
      for (int k = 0; k < 4; k++) u |= (uint32_t)(uint8_t)v[k] << (8 * k);
      *reinterpret_cast<uint32_t*>(p) = u;
    }
  } else {
#pragma unroll
    for (int k = 0; k < 4; k++)
      if (k < nvalid) p[k] = v[k];
  }
}

template <int LPB>
__device__ __forceinline__ void sum_x(uint32_t r[4], int xq, int rowq) {
  r[1] += r[0];
  r[2] += r[1];
  r[3] += r[2];
  uint32_t t = r[3], inc = t;
#pragma unroll
  for (int o = 1; o < LPB; o <<= 1) {
    uint32_t u = (uint32_t)up<LPB>((int32_t)inc, o);
    if (o < rowq && xq >= o) inc += u;
  }
  uint32_t ex = inc - t;
#pragma unroll
  for (int k = 0; k < 4; k++) r[k] += ex;
}

template <int LPB>
__device__ __forceinline__ void sum_axis(uint32_t r[4], int coord, int extent, int lanestep) {
#pragma unroll
  for (int o = 1; o < LPB; o <<= 1) {
#pragma unroll
    for (int k = 0; k < 4; k++) {
      uint32_t u = (uint32_t)up<LPB>((int32_t)r[k], o * lanestep);
      if (o < extent && coord >= o) r[k] += u;
    }
  }
}

template <int WP>
struct DecShared {
  int32_t info[WP * 64];
  int32_t end[WP * 4];
  uint4 xch[WP * XCH];  // one block per wave: y/z running sums
};

// wave-level ordering of LDS accesses among the lanes of one wave
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// inclusive running sum of v along x inside brick rows of rowq lanes (one
// block per wave): DPP row shifts when rows tile the 16-lane DPP rows,
// the full wave for 1-d blocks, lane shuffles otherwise
__device__ __forceinline__ uint32_t row_scan64(uint32_t v, int xq, int rowq) {
  if (rowq == 64) return seg_scan_add<64>(v);
  if (rowq <= 16 && (16 % rowq) == 0) {
    // every lane computes the shifted value (pinned there); the select follows
    if (rowq > 1) { const uint32_t t = pin(row_shr<1>(v)); v += xq >= 1 ? t : 0u; }
    if (rowq > 2) { const uint32_t t = pin(row_shr<2>(v)); v += xq >= 2 ? t : 0u; }
    if (rowq > 4) { const uint32_t t = pin(row_shr<4>(v)); v += xq >= 4 ? t : 0u; }
    if (rowq > 8) { const uint32_t t = pin(row_shr<8>(v)); v += xq >= 8 ? t : 0u; }
    return v;
  }
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t u = (uint32_t)__shfl_up((int)v, (unsigned)o, 64);
    if (o < rowq && xq >= o) v += u;
  }
  return v;
}

// undo one x difference: running sums along x inside the brick row
__device__ __forceinline__ void undo_x64(uint32_t r[4], int xq, int rowq) {
  r[1] += r[0];
  r[2] += r[1];
  r[3] += r[2];
  const uint32_t inc = row_scan64(r[3], xq, rowq);
  const uint32_t ex = inc - r[3];
#pragma unroll
  for (int k = 0; k < 4; k++) r[k] += ex;
}

// undo one difference along an axis whose neighbour is `step` lanes back
// (coordinate coord < extent): log-step running sums through the wave's
// LDS exchange (entry XCH - 1 is zero)
__device__ __forceinline__ void undo_axis64(uint32_t r[4], int coord, int extent, int step, uint4* xch) {
  const int lane = lane_id();
  for (int o = 1; o < extent; o <<= 1) {
    xch[lane] = make_uint4(r[0], r[1], r[2], r[3]);
    wave_sync();
    const uint4 q = xch[coord >= o ? lane - o * step : XCH - 1];
    wave_sync();
    r[0] += q.x;
    r[1] += q.y;
    r[2] += q.z;
    r[3] += q.w;
  }
}

// One block per wave (blocks of up to 256 samples in 64 groups): the header,
// stream id and code are wave-uniform, the JEE token parse works on 64-bit
// nibble masks, the exponents come from two DPP scans (a running sum of the
// differences and a running max that carries the last absolute exponent),
// and only the inverse differences of the block's own stream run.  Checks
// are those of the general tile below.
template <typename T, int NDIM, int WP, bool DOT>
__device__ __forceinline__ void decode_tile64(const DecArgs& A, const int64_t tile, DecShared<WP>& sm,
                                              uint32_t* lds, const T* __restrict__ w, double* dot) {
  constexpr int H = Traits<T>::H;
  constexpr int W = Traits<T>::W;
  constexpr int MAXEPS = W == 32 ? 31 : W;
  const Geo& g = A.g;
  const int wave = threadIdx.x >> 6;
  const int lane = lane_id();
  const int gi = lane;

  if (tile == 0 && threadIdx.x < 16) {
    const uint32_t* h = reinterpret_cast<const uint32_t*>(A.in);
    if (h[threadIdx.x] != A.hdr[threadIdx.x]) atomicOr(A.status, ST_CORRUPT);
  }
  const int64_t j = tile * WP + wave;  // wave-uniform
  if (j >= g.nblocks) return;
  const LaneMap<64> L = lane_map<64>(g);
  const bool act = gi < g.G;
  const int mode = __builtin_amdgcn_readfirstlane(g.mode);  // wave-uniform
  const bool variable = mode != M_RATE;
  bool bad = false;

  // ---- block offset and length (wave-uniform)
  uint64_t off;
  int len;
  bool ubad = false;
  if (variable) {
    const int64_t jb = (j >> 6) << 6;
    uint32_t l = (jb + gi < j) ? (uint32_t)A.lens[jb + gi] : 0u;
    const uint32_t acc = (uint32_t)__builtin_amdgcn_readlane((int)seg_scan_add<64>(l), 63);
    const uint64_t sb = A.sbo[j >> 6];
    // a superblock offset past the payload is corrupt (checked before the
    // addition, which could otherwise wrap)
    ubad = sb > A.payload_words;
    off = ubad ? A.payload_words : sb + (uint64_t)acc;
    len = A.lens[j];
  } else {
    off = (uint64_t)j * (uint64_t)g.budget;
    len = g.budget;
  }
  if (ubad || len < 1 || (variable && len > g.maxw) || off > A.payload_words ||
      (uint64_t)len > A.payload_words - off) {
    ubad = true;
    len = 0;
  }

  // ---- stage the block words in LDS (two zero words after them)
  const int stride = g.ldsw;
  uint32_t* buf = lds + wave * stride;
  const int lim = len + 2 < stride ? len + 2 : stride;
  for (int q = gi; q < lim; q += 64) buf[q] = q < len ? A.words[off + q] : 0u;
  // words past the LDS buffer (fixed rate with a budget above any encoding)
  // can only be padding
  for (int q = stride + gi; q < len; q += 64)
    if (A.words[off + q]) bad = true;
  sm.info[wave * 64 + gi] = 0;
  wave_sync();

  // ---- block header (wave-uniform)
  const uint32_t w0 = (uint32_t)__builtin_amdgcn_readfirstlane((int)buf[0]);
  const uint32_t w1 = (uint32_t)__builtin_amdgcn_readfirstlane((int)buf[1]);
  const int st = (int)(w0 & 7u);
  const int e0 = (int)((w0 >> 3) & 31u);
  int c;
  uint32_t rsv;
  if constexpr (H == 32) {
    c = ((int32_t)(w0 << 14)) >> 22;
    rsv = w0 >> 18;
  } else {
    c = (int32_t)(int16_t)(uint16_t)((w0 >> 8) & 0xFFFFu);
    rsv = (w0 >> 24) | (w1 & 0xFFFFu);
  }
  const bool verb = st == 7;
  ubad |= rsv != 0u;
  ubad |= !((g.mask >> st) & 1u);
  ubad |= mode == M_LOSSLESS ? (c != 0) : (c < g.cmin || c > g.cmax);
  ubad |= 32 * len < H;
  if (verb) ubad |= e0 != 0 || 32 * len < H + g.B * W;
  else ubad |= e0 > MAXEPS;

  int pw = 0, pay0 = H;
  if (!verb) {
    // ---- JEE token parse: nibbles gi and 64 + gi of the token section
    auto nib_at = [&](int n) -> int {
      const int bit = H + 4 * n;
      const int q = bit >> 5;
      return q < stride ? (int)((buf[q] >> (bit & 31)) & 15u) : 0;
    };
    const int nb0 = nib_at(gi), nb1 = nib_at(64 + gi);
    const uint64_t vt = __ballot(act);
    const uint64_t E0 = __ballot(nb0 >= 14) & vt, E1 = __ballot(nb1 >= 14) & vt;
    uint64_t llo, lhi;
    low_half_mask(E0, E1, llo, lhi);
    const uint64_t S0 = vt & ~llo, S1 = vt & ~lhi;   // token starts (where inside the section)
    const uint64_t P0 = __ballot(nb0 <= 8) & S0, P1 = __ballot(nb1 <= 8) & S1;  // pairs
    // groups covered by the tokens before this one: pairs cover two
    const int cov0 = below_in_seg<64>(P0, 0) + below_in_seg<64>(S0, 0);
    const int cov1 = __popcll(P0) + __popcll(S0) + below_in_seg<64>(P1, 0) + below_in_seg<64>(S1, 0);
    // the nibble after each one (DPP lane shifts; lane 63 takes nibble 64)
    const int nb1_0 = __builtin_amdgcn_readlane(nb1, 0);
    const int sh0 = (int)pin(shl1((uint32_t)nb0));
    const int nxt0 = gi < 63 ? sh0 : nb1_0;
    const int nxt1 = (int)pin(shl1((uint32_t)nb1));
    int32_t* info = sm.info + wave * 64;
    const int G = g.G;
    int tend = -1;  // nibbles of the token section (this lane's view)
    auto place = [&](bool s, int v, int cov, int nxt, int n) {
      const int g0 = 1 + cov;
      if (!s || g0 > G - 1) return;
      if (v <= 8) {
        if (g0 + 1 > G - 1) { bad = true; return; }
        info[g0] = (1 << 8) | ((v / 3 - 1) & 0xFF);
        info[g0 + 1] = (1 << 8) | ((v % 3 - 1) & 0xFF);
        if (g0 + 1 == G - 1) tend = n + 1;
      } else if (v <= 13) {
        info[g0] = (1 << 8) | ((v - 11) & 0xFF);
        if (g0 == G - 1) tend = n + 1;
      } else {
        if (n + 1 >= 128) { bad = true; return; }
        info[g0] = (2 << 8) | (16 * (v - 14) + nxt);
        if (g0 == G - 1) tend = n + 2;
      }
    };
    place(__builtin_amdgcn_inverse_ballot_w64(S0), nb0, cov0, nxt0, gi);
    place(__builtin_amdgcn_inverse_ballot_w64(S1), nb1, cov1, nxt1, 64 + gi);
    if (gi == 0) info[0] = (2 << 8) | e0;
    wave_sync();

    // ---- exponents: running sum of the differences, and the last absolute
    // exponent (minus the running sum there) carried by a running max of
    // keys (position << 9 | value + 256); lanes without a group are absolute 0
    const int32_t iv = act ? info[gi] : (2 << 8);
    const int kind = iv >> 8;
    if (act && kind == 0) bad = true;  // a group no token covers
    const int32_t dl = kind == 1 ? (int32_t)(int8_t)(iv & 0xFF) : 0;
    const int32_t sum = (int32_t)seg_scan_add<64>((uint32_t)dl);
    const uint32_t key = kind == 2 ? ((uint32_t)gi << 9) | (uint32_t)((iv & 0xFF) - sum + 256) : 0u;
    const uint32_t mk = seg_scan_max<64>(key);
    int eps = (int)(mk & 511u) - 256 + sum;
    if (act && (eps < 0 || eps > MAXEPS)) bad = true;
    if (!act) eps = 0;
    pw = (W == 32 && eps == 31) ? 32 : eps;
    // the token section ends after the token that covers group G - 1
    const int te = __builtin_amdgcn_readfirstlane(
        (int)seg_last<64>(seg_scan_max<64>((uint32_t)(tend + 1)), 0)) - 1;
    if (te < 0) ubad = true;
    pay0 = H + 4 * (te < 0 ? 0 : te);
  }
  const uint32_t incl = seg_scan_add<64>((uint32_t)(4 * pw));
  const int pex = (int)incl - 4 * pw;
  const int total = verb ? (H + g.B * W) : pay0 + __builtin_amdgcn_readlane((int)incl, 63);
  if (total > 32 * len) ubad = true;

  // ---- extract values: p-bit fields at o, o + p, ... (funnel shifts of word pairs)
  uint32_t r[4];
  {
    const int width = verb ? W : pw;
    const int o = verb ? H + 4 * gi * W : pay0 + pex;
#pragma unroll
    for (int k = 0; k < 4; k++) {
      const int bit = o + k * width;
      int q = bit >> 5;
      q = q < 0 ? 0 : (q > stride - 2 ? stride - 2 : q);
      const uint32_t lo = buf[q], hi = buf[q + 1];
      const uint32_t raw = (uint32_t)((((uint64_t)hi << 32) | lo) >> (bit & 31));
      r[k] = width >= 32 ? raw : (uint32_t)__builtin_amdgcn_sbfe((int)raw, 0, width);
    }
  }
  // padding after the last used bit must be zero
  if (total <= 32 * len) {
    const int wfirst = (total + 31) >> 5;
    const int wlast = len < stride ? len : stride;
    for (int q = wfirst + gi; q < wlast; q += 64)
      if (buf[q]) bad = true;
    if (gi == 0 && (total & 31) && (buf[total >> 5] >> (total & 31))) bad = true;
  }

  // ---- undo the derivative stream (running sums, mod 2^W); st is wave-uniform
  if (NDIM == 1 && st == 3) unfilter(r, gi, g.fk, g.fneg, 4 * g.G);
  if (st == 1 || st == 2 || st == 5 || st == 6) undo_x64(r, L.xq, g.rowq);
  if (st == 2) undo_x64(r, L.xq, g.rowq);
  uint4* xch = sm.xch + wave * XCH;
  if (NDIM >= 2 && (st == 3 || st == 5 || st == 6 || st == 4)) {
    if (lane == 0) xch[XCH - 1] = make_uint4(0u, 0u, 0u, 0u);
    if (st != 4) undo_axis64(r, L.y, g.b[1], g.rowq, xch);
    if (NDIM == 3 && (st == 4 || st == 6)) undo_axis64(r, L.z, g.b[0], g.plane, xch);
  }

  if ((__ballot(bad) || ubad) && lane == 0) atomicOr(A.status, ST_CORRUPT);

  // ---- dequantize and store
  int64_t base;
  uint32_t doff;
  const bool aligned = (((uintptr_t)A.y) & (4 * sizeof(T) - 1)) == 0;
  const bool dense = aligned && dense_block<NDIM, 64>(g, L, j, base, doff);
  int nvalid = 4;
  int64_t idx = 0;
  if (!dense) {
    if (act) idx = group_index<NDIM, 64>(g, L, j, nvalid);
    else nvalid = 0;
  } else {
    idx = base + doff;
  }
  T out[4];
  const double R = inv_mantissa(c);
  const int e = -(c >> 4);
#pragma unroll
  for (int k = 0; k < 4; k++) {
    const int32_t av = wrapw<W>(r[k]);
    if (mode == M_LOSSLESS) out[k] = (T)av;
    else out[k] = to_out<T>(dequant_rk(av, R, e));
  }
  if constexpr (DOT) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < 4; k++)
      if (k < nvalid) s += (double)out[k] * (double)w[idx + k];
    *dot += s;
  } else {
    if (dense) store4_full<T>((T*)A.y + idx, out);
    else if (act) store4<T>((T*)A.y, idx, nvalid, out);
  }
}

// One tile (WP waves x 64/LPB blocks) of one stream.  DOT: instead of storing
// the decoded samples, add their products with w (same layout) into *dot
// (this lane's binary64 partial) -- decode-on-read for a consumer.
template <typename T, int LPB, int NDIM, int WP, bool DOT = false>
__device__ __forceinline__ void decode_tile(const DecArgs& A, const int64_t tile, DecShared<WP>& sm,
                                            uint32_t* lds, const T* __restrict__ w = nullptr,
                                            double* dot = nullptr) {
  if constexpr (LPB == 64) {
    decode_tile64<T, NDIM, WP, DOT>(A, tile, sm, lds, w, dot);
    return;
  }
  constexpr int BPW = 64 / LPB;
  constexpr int H = Traits<T>::H;
  constexpr int W = Traits<T>::W;
  constexpr int MAXEPS = W == 32 ? 31 : W;
  const Geo& g = A.g;
  int32_t* s_info = sm.info;
  int32_t* s_end = sm.end;

  const int wave = threadIdx.x >> 6;
  const int lane = lane_id();
  const LaneMap<LPB> L = lane_map<LPB>(g);
  const int seg = L.seg, gi = L.gi;
  const int64_t j = (tile * WP + wave) * BPW + seg;
  const bool blk_ok = j < g.nblocks;
  const bool act = blk_ok && gi < g.G;
  const bool variable = g.mode != M_RATE;
  bool bad = false;

  if (tile == 0 && threadIdx.x < 16) {
    const uint32_t* h = reinterpret_cast<const uint32_t*>(A.in);
    if (h[threadIdx.x] != A.hdr[threadIdx.x]) atomicOr(A.status, ST_CORRUPT);
  }

  // ---- block offset and length
  uint64_t off = 0;
  int len = 0;
  if (variable) {
    int64_t jb = (j >> 6) << 6;
    int acc = 0;
    if (blk_ok)
      for (int64_t r = jb + gi; r < j; r += LPB) acc += A.lens[r];
    acc = seg_sum<LPB>(acc);
    if (blk_ok) {
      const uint64_t sb = A.sbo[j >> 6];
      // a superblock offset past the payload is corrupt (checked before the
      // addition, which could otherwise wrap)
      if (sb > A.payload_words) bad = true;
      off = sb > A.payload_words ? A.payload_words : sb + (uint64_t)acc;
      len = A.lens[j];
    }
  } else if (blk_ok) {
    off = (uint64_t)j * (uint64_t)g.budget;
    len = g.budget;
  }
  if (blk_ok && (bad || len < 1 || (variable && len > g.maxw) || off > A.payload_words ||
                 (uint64_t)len > A.payload_words - off)) {
    bad = true;
    len = 0;
  }

  // ---- stage block words in LDS
  const int stride = g.ldsw;
  uint32_t* buf = lds + (wave * BPW + seg) * stride;
  for (int w = gi; w < stride; w += LPB) buf[w] = w < len ? A.words[off + w] : 0u;
  // words past the LDS buffer (fixed rate with a budget above any encoding)
  // can only be padding
  for (int w = stride + gi; w < len; w += LPB)
    if (A.words[off + w]) bad = true;
  s_info[wave * 64 + seg * LPB + gi] = 0;
  if (gi == 0) s_end[wave * BPW + seg] = -1;
  __syncthreads();

  // ---- block header
  const uint32_t w0 = buf[0], w1 = buf[1];
  const int st = (int)(w0 & 7u);
  const int e0 = (int)((w0 >> 3) & 31u);
  int c;
  uint32_t rsv;
  if constexpr (H == 32) {
    c = ((int32_t)(w0 << 14)) >> 22;
    rsv = w0 >> 18;
  } else {
    c = (int32_t)(int16_t)(uint16_t)((w0 >> 8) & 0xFFFFu);
    rsv = (w0 >> 24) | (w1 & 0xFFFFu);
  }
  const bool verb = st == 7;
  if (blk_ok) {
    bad |= rsv != 0u;
    bad |= !((g.mask >> st) & 1u);
    bad |= g.mode == M_LOSSLESS ? (c != 0) : (c < g.cmin || c > g.cmax);
    bad |= 32 * len < H;
    if (verb) bad |= e0 != 0 || 32 * len < H + g.B * W;
    else bad |= e0 > MAXEPS;
  }

  // ---- JEE token parse (nibbles gi and LPB + gi of the token section)
  auto nib_at = [&](int n) -> int {
    int bit = H + 4 * n;
    int w = bit >> 5;
    if (w >= stride) return 0;
    return (int)((buf[w] >> (bit & 31)) & 15u);
  };
  const bool tk = act && !verb;
  const int nb0 = nib_at(gi), nb1 = nib_at(LPB + gi);
  const uint64_t E0 = __ballot(tk && nb0 >= 14), E1 = __ballot(tk && nb1 >= 14);
  uint64_t slo, shi;
  if constexpr (LPB == 64) {
    slo = E0;
    shi = E1;
  } else {
    const uint64_t msk = (1ull << LPB) - 1ull;
    slo = ((E0 >> (LPB * seg)) & msk) | (((E1 >> (LPB * seg)) & msk) << LPB);
    shi = 0;
  }
  uint64_t llo, lhi;
  low_half_mask(slo, shi, llo, lhi);
  bool low0, low1;
  if constexpr (LPB == 64) {
    low0 = (llo >> gi) & 1;
    low1 = (lhi >> gi) & 1;
  } else {
    low0 = (llo >> gi) & 1;
    low1 = (llo >> (LPB + gi)) & 1;
  }
  const bool s0 = tk && !low0, s1 = tk && !low1;
  const uint64_t P0 = __ballot(s0 && nb0 <= 8), Q0 = __ballot(s0 && nb0 >= 9);
  const uint64_t P1 = __ballot(s1 && nb1 <= 8), Q1 = __ballot(s1 && nb1 >= 9);
  const uint64_t sbm = seg_bits<LPB>(seg);
  const int cov0 = 2 * below_in_seg<LPB>(P0, seg) + below_in_seg<LPB>(Q0, seg);
  const int cov1 = 2 * (__popcll(P0 & sbm) + below_in_seg<LPB>(P1, seg)) +
                   (__popcll(Q0 & sbm) + below_in_seg<LPB>(Q1, seg));
  // low nibble following each position
  const int nxt0_a = dn<LPB>(nb0, 1), nxt0_b = seg_shfl<LPB>(nb1, 0);
  const int nxt0 = gi < LPB - 1 ? nxt0_a : nxt0_b;
  const int nxt1 = dn<LPB>(nb1, 1);
  int32_t* info = s_info + wave * 64 + seg * LPB;
  const int G = g.G;
  bool tbad = false;
  auto place = [&](bool s, int v, int cov, int nxt, int n) {
    if (!s) return;
    int g0 = 1 + cov;
    if (g0 > G - 1) return;
    int end;
    if (v <= 8) {
      if (g0 + 1 > G - 1) { tbad = true; return; }
      info[g0] = (1 << 8) | ((v / 3 - 1) & 0xFF);
      info[g0 + 1] = (1 << 8) | ((v % 3 - 1) & 0xFF);
      end = n + 1;
      if (g0 + 1 == G - 1) s_end[wave * BPW + seg] = end;
    } else if (v <= 13) {
      info[g0] = (1 << 8) | ((v - 11) & 0xFF);
      end = n + 1;
      if (g0 == G - 1) s_end[wave * BPW + seg] = end;
    } else {
      if (n + 1 >= 2 * LPB) { tbad = true; return; }
      info[g0] = (2 << 8) | (16 * (v - 14) + nxt);
      end = n + 2;
      if (g0 == G - 1) s_end[wave * BPW + seg] = end;
    }
  };
  place(s0, nb0, cov0, nxt0, gi);
  place(s1, nb1, cov1, (gi < LPB - 1) ? nxt1 : 0, LPB + gi);
  if (act && gi == 0) info[0] = (2 << 8) | e0;
  bad |= tbad;
  __syncthreads();

  // ---- exponents: segmented scan (absolute tokens reset the running sum)
  int32_t iv = act ? info[gi] : (2 << 8);
  const int kind = iv >> 8;
  if (act && !verb && kind == 0) bad = true;
  int32_t f = kind == 2 ? 1 : 0;
  int32_t x = kind == 2 ? (iv & 0xFF) : (int32_t)(int8_t)(iv & 0xFF);
#pragma unroll
  for (int o = 1; o < LPB; o <<= 1) {
    int32_t fo = up<LPB>(f, o), xo = up<LPB>(x, o);
    if (gi >= o && !f) {
      x += xo;
      f = fo;
    }
  }
  int eps = x;
  if (tk && (eps < 0 || eps > MAXEPS)) bad = true;
  if (!tk) eps = 0;
  const int pw = (W == 32 && eps == 31) ? 32 : eps;
  const int tend = s_end[wave * BPW + seg];
  if (blk_ok && !verb && tend < 0) bad = true;
  const int pay0 = H + 4 * (tend < 0 ? 0 : tend);
  const int pex = seg_excl_scan<LPB>(4 * pw, gi);
  const int total = verb ? (H + g.B * W) : (pay0 + seg_sum<LPB>(4 * pw));
  if (blk_ok && total > 32 * len) bad = true;

  // ---- extract values
  uint32_t r[4];
#pragma unroll
  for (int k = 0; k < 4; k++) {
    int width = verb ? W : pw;
    int bit = verb ? H + (4 * gi + k) * W : pay0 + pex + k * pw;
    int w = bit >> 5;
    w = w < 0 ? 0 : (w > stride - 2 ? stride - 2 : w);
    uint64_t both = ((uint64_t)buf[w + 1] << 32) | buf[w];
    uint32_t raw = (uint32_t)(both >> (bit & 31));
    r[k] = width == 0 ? 0u : (width >= 32 ? raw : (uint32_t)(((int32_t)(raw << (32 - width))) >> (32 - width)));
  }
  // padding after the last used bit must be zero
  if (blk_ok && total <= 32 * len) {
    int wfirst = (total + 31) >> 5;
    int wlast = len < stride ? len : stride;
    for (int w = wfirst + gi; w < wlast; w += LPB)
      if (buf[w]) bad = true;
    if (gi == 0 && (total & 31) && (buf[total >> 5] >> (total & 31))) bad = true;
  }

  // ---- undo the derivative stream (running sums, mod 2^W)
  {
    uint32_t u[4] = {r[0], r[1], r[2], r[3]};
    if constexpr (NDIM == 1) {
      if (g.fk) {  // the filter stream (every lane takes part; segments with st 3 keep it)
        unfilter(u, gi, g.fk, g.fneg, 4 * g.G);
#pragma unroll
        for (int k = 0; k < 4; k++) r[k] = st == 3 ? u[k] : r[k];
#pragma unroll
        for (int k = 0; k < 4; k++) u[k] = r[k];
      }
    }
    const bool dx1 = st == 1 || st == 2 || st == 5 || st == 6;
    sum_x<LPB>(u, L.xq, g.rowq);
#pragma unroll
    for (int k = 0; k < 4; k++) r[k] = dx1 ? u[k] : r[k];
#pragma unroll
    for (int k = 0; k < 4; k++) u[k] = r[k];
    sum_x<LPB>(u, L.xq, g.rowq);
#pragma unroll
    for (int k = 0; k < 4; k++) r[k] = st == 2 ? u[k] : r[k];
    if constexpr (NDIM >= 2) {
#pragma unroll
      for (int k = 0; k < 4; k++) u[k] = r[k];
      sum_axis<LPB>(u, L.y, g.b[1], g.rowq);
      const bool dy = st == 3 || st == 5 || st == 6;
#pragma unroll
      for (int k = 0; k < 4; k++) r[k] = dy ? u[k] : r[k];
    }
    if constexpr (NDIM == 3) {
#pragma unroll
      for (int k = 0; k < 4; k++) u[k] = r[k];
      sum_axis<LPB>(u, L.z, g.b[0], g.plane);
      const bool dz = st == 4 || st == 6;
#pragma unroll
      for (int k = 0; k < 4; k++) r[k] = dz ? u[k] : r[k];
    }
  }

  if (__ballot(bad) && lane == 0) atomicOr(A.status, ST_CORRUPT);

  // ---- dequantize and store
  if (act) {
    int nvalid = 0;
    int64_t idx = group_index<NDIM, LPB>(g, L, j, nvalid);
    T out[4];
    const double R = inv_mantissa(c);
    const int e = -(c >> 4);
#pragma unroll
    for (int k = 0; k < 4; k++) {
      int32_t av = wrapw<W>(r[k]);
      if (g.mode == M_LOSSLESS) out[k] = (T)av;
      else out[k] = to_out<T>(dequant_rk(av, R, e));
    }
    if constexpr (DOT) {
      double sum = 0.0;
#pragma unroll
      for (int k = 0; k < 4; k++)
        if (k < nvalid) sum += (double)out[k] * (double)w[idx + k];
      *dot += sum;
    } else {
      store4<T>((T*)A.y, idx, nvalid, out);
    }
  }
}

}  // namespace apax
