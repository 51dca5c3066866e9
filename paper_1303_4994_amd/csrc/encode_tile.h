// encode_tile.h -- one tile of the APAX encoder (Sec. 6), shared by the
// single-array kernel and the persistent batch kernel.
//
// Per block: coalesced loads of its groups, block max -> code bracket, gain
// choice (lossless: 0; fixed quality: clamp(c*); fixed rate: cap-and-descend
// search), every candidate stream costed in registers, the cheapest emitted
// into a zeroed LDS buffer with ds_or (header | JEE tokens | BFPE payload),
// then copied out with coalesced word stores.  Fixed rate places block j at
// j * budget words.  Variable-size modes take runs of RUN consecutive tiles
// per work-queue ticket: every tile of the run is analysed and assembled in
// LDS and publishes its word count first, then the run's first tile finds
// its offset with a single-pass decoupled look-back (64 predecessors per
// probe) and the others follow by addition, then all are stored.  Publishing
// every count before any wait keeps the runs of different workgroups
// independent, and one ticket per run cuts the atomics on the shared ticket.
#pragma once
#include "block.h"
#include "kernels.h"

namespace apax {

__device__ __forceinline__ void or_bits(uint32_t* buf, int bitpos, uint32_t val, int len) {
  if (len <= 0) return;
  int w = bitpos >> 5, sh = bitpos & 31;
  uint32_t lo = val << sh;
  if (lo) atomicOr(&buf[w], lo);
  if (sh && sh + len > 32) {
    uint32_t hi = val >> (32 - sh);
    if (hi) atomicOr(&buf[w + 1], hi);
  }
}

// OR the bits of val into the buffer from bit position bitpos on (the two
// words it may touch; zero bits leave a word unchanged)
__device__ __forceinline__ void or_word2(uint32_t* buf, int bitpos, uint32_t val) {
  const uint64_t r = (uint64_t)val << (bitpos & 31);
  uint32_t* q = buf + (bitpos >> 5);
  atomicOr(q, (uint32_t)r);
  atomicOr(q + 1, (uint32_t)(r >> 32));
}

__device__ __forceinline__ uint32_t low_bits(int32_t v, int n) {
  return n >= 32 ? (uint32_t)v : ((uint32_t)v & ((1u << n) - 1u));
}

__device__ __forceinline__ uint64_t wave_sum64(uint64_t v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += (uint64_t)__shfl_xor((unsigned long long)v, o, 64);
  return v;
}

// Decoupled look-back over per-tile word counts, run by one full wave.  Each
// tile publishes its aggregate (flag A), then the wave reads the states of
// the 64 nearest unconsumed predecessors in one round trip: aggregates are
// summed up to and including the nearest inclusive prefix (flag P); a
// predecessor that has not published yet is waited for.  The value travels
// in the same 64-bit word as its flag, so relaxed device-scope atomics
// suffice (no cache invalidation per probe).  Tiles are started in
// increasing order, so every tile waited on is already running; the wait is
// still bounded in time and reports ST_INTERNAL if the bound is ever hit.
// Returns the exclusive prefix (words before this tile).
constexpr uint64_t LB_FLAG_A = 1ull << 62, LB_FLAG_P = 2ull << 62, LB_VAL = LB_FLAG_A - 1;

// publish a tile's own word count (tile 0: its inclusive prefix)
__device__ __forceinline__ void lb_publish(uint64_t* ts, int64_t tile, uint64_t agg) {
  __hip_atomic_store(&ts[tile], (tile == 0 ? LB_FLAG_P : LB_FLAG_A) | agg, __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void lb_prefix(uint64_t* ts, int64_t tile, uint64_t incl) {
  __hip_atomic_store(&ts[tile], LB_FLAG_P | incl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t lookback(uint64_t* ts, int64_t tile, uint32_t* status) {
  const uint64_t FLAG_P = LB_FLAG_P, VAL = LB_VAL;
  const int lane = lane_id();
  if (tile == 0) return 0;
  uint64_t base = 0;
  int64_t end = tile - 1;
  const uint64_t t0 = wall_clock64();
  for (;;) {
    const int64_t idx = end - lane;
    const uint64_t s = idx >= 0 ? __hip_atomic_load(&ts[idx], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                                : FLAG_P;
    const uint32_t flag = (uint32_t)(s >> 62);
    const uint64_t mz = __ballot(flag == 0), mp = __ballot(flag == 2);
    const int fz = mz ? __builtin_ctzll(mz) : 64;
    const int fp = mp ? __builtin_ctzll(mp) : 64;
    const int take = fp < fz ? fp + 1 : fz;  // lanes [0, take) are consumed
    base += wave_sum64(lane < take ? (s & VAL) : 0);
    if (fp < fz) break;
    end -= take;
    if (take == 0) {
      if (wall_clock64() - t0 > 400000000ull) {  // 4 s of the 100 MHz clock
        if (lane == 0) atomicOr(status, ST_INTERNAL);
        break;
      }
      __builtin_amdgcn_s_sleep(1);
    }
  }
  return base;
}

template <int WP>
struct EncShared {
  int64_t tile;
  uint64_t agg[RUN];          // words of each tile of the run
  uint32_t item[RUN];         // batch: item of each tile of the run
  uint32_t nw[RUN][WP * 4];   // words of each block
  uint64_t off[RUN][WP * 4];  // word offset of each block
  uint4 xch[WP * XCH];
};

__device__ __forceinline__ bool profiled_point(const EncArgs& A, const Geo& g, int32_t& code,
                                               uint32_t& mask) {
  return operating_point(A.sel, A.status, g.cmin, g.cmax, g.code, g.mask, code, mask);
}

// Analysis of one block (the wave segment's): samples, bracket, operating
// point c, quantized samples a, chosen stream st and its size best (bits);
// fixed rate: after the cap-and-descend search (c final, a at c).
template <typename T, int LPB, int NDIM>
__device__ __forceinline__ void analyze_block(const EncArgs& A, Blk<T, LPB, NDIM>& b, int mode, int code0,
                                              uint32_t emask, int& c, int& st, int32_t& best, int32_t a[4]) {
  using B_ = Blk<T, LPB, NDIM>;
  const Geo& g = A.g;
  {
    T xv4[4];
    b.fetch((const T*)A.x, g, xv4);
    if (mode == M_LOSSLESS) b.template take<false>(g, xv4);  // code 0: no bracket
    else b.take(g, xv4);
  }
  if (__ballot(b.act && b.nonfinite) && lane_id() == 0) atomicOr(A.status, ST_NONFINITE);
  c = 0;
  if (mode != M_LOSSLESS) c = clampc(code0, b.cf, b.cc);
  b.quantize(c, mode == M_LOSSLESS, a);
  if (A.lag) {  // lagged choice (lossless): the previous block's best stream,
                // or verbatim where that would code the block above verbatim size
    Costs C;
    b.costs(g, emask, a, C);
    st = b.j == 0 ? 0 : (b.blk_ok ? A.lag[b.j - 1] : 0);
    if constexpr (LPB == 64) st = __builtin_amdgcn_readfirstlane(st);
    best = B_::size_sel(C, st);
    if (best > C.sz[7]) {
      st = 7;
      best = C.sz[7];
    }
  } else {
    st = b.best_stream(g, emask, a, best);
  }
  if constexpr (LPB == 64) {
    st = __builtin_amdgcn_readfirstlane(st);
    best = __builtin_amdgcn_readfirstlane(best);
  }
  if (mode == M_RATE) {
    const bool need = b.act && best > 32 * g.budget;
    if (__ballot(need)) {
      // some block of this wave does not fit at its start code: search (the
      // stream stays the one chosen at the start code), then quantize at the
      // final code
      c = b.rate_search(g, emask, c, st, need);
      if constexpr (LPB == 64) c = __builtin_amdgcn_readfirstlane(c);
      b.quantize(c, false, a);
    }
  }
}

// One block's encoding at code c with stream st, assembled in the segment's
// LDS buffer `buf` (its nw words zeroed first): header | JEE tokens | BFPE
// payload (verbatim: the W-bit samples).  Every lane of the wave takes part.
template <typename T, int LPB, int NDIM>
__device__ __forceinline__ void emit_block(const Geo& g, const Blk<T, LPB, NDIM>& b, int c, int st, uint32_t emask,
                                           const int32_t a[4], uint32_t* buf, int nw) {
  constexpr int H = Traits<T>::H;
  constexpr int W = Traits<T>::W;
  using B_ = Blk<T, LPB, NDIM>;
  // the chosen stream's values, exponent and payload width
  const bool verb = st == 7;  // LPB = 64: wave-uniform
  int32_t vv[4] = {0, 0, 0, 0};
  int e = 0, p = 0;
  if constexpr (LPB == 64) {  // one block per wave: form the chosen stream alone
    if (!verb) {
      b.stream_one(g, st, a, vv);
      b.eps_of(vv, e, p);
    }
  } else {  // every lane takes part: the streams move values across lanes
    int32_t v[7][4];
    b.streams(g, a, v, emask | 1u);
    B_::select_stream(st, v, vv);
    b.eps_of(vv, e, p);
    if (verb) { e = 0; p = 0; }
  }
  // zero the words the block will hold (this wave's own buffer: LDS
  // accesses of one wave complete in order)
  const int seg = b.L.seg, gi = b.L.gi;
  const int stride = g.ldsw;
  const int nz = nw < stride ? nw : stride;
  for (int w = 4 * gi; w < nz; w += 4 * LPB) *reinterpret_cast<uint4*>(buf + w) = make_uint4(0, 0, 0, 0);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

  // JEE tokens of the chosen stream.  Exponent differences: the
  // predecessor's exponent arrives negated through a DPP add (lane 0 of a
  // segment gets a value it never uses).
  const int d = (int)((uint32_t)e + shr1(0u - (uint32_t)e));
  uint64_t vp;
  if constexpr (LPB == 64) vp = verb ? 0ull : b.vpos;
  else vp = __ballot(b.act && gi >= 1 && !verb);
  const uint64_t m1 = __ballot((uint32_t)(d + 1) <= 2u) & vp;
  const uint64_t m2 = __ballot((uint32_t)(d + 2) <= 4u) & vp;
  const uint64_t Tm = jee_token_starts(m1);
  const uint64_t starts = Tm | (~m1 & vp);
  const uint64_t ab = ~m2 & vp;
  const uint64_t pairs = Tm & (m1 >> 1);  // a pair token: its second difference is small too
  const int dnext = (int)pin(shl1((uint32_t)d));
  const int ntot = seg_popc<LPB>(starts, seg) + seg_popc<LPB>(ab, seg);
  const int pay0 = H + 4 * ntot;
  const int pex = (int)seg_scan_add<LPB>((uint32_t)(4 * p)) - 4 * p;
  if (__builtin_amdgcn_inverse_ballot_w64(starts)) {
    const int nib_off = below_in_seg<LPB>(starts, seg) + below_in_seg<LPB>(ab, seg);
    const bool pr = __builtin_amdgcn_inverse_ballot_w64(pairs), isab = __builtin_amdgcn_inverse_ballot_w64(ab);
    const uint32_t tabs = (uint32_t)(14 + (e >> 4)) | ((uint32_t)(e & 15) << 4);
    const uint32_t tok = pr ? (uint32_t)(3 * d + dnext + 4) : (isab ? tabs : (uint32_t)(11 + d));
    or_word2(buf, H + 4 * nib_off, tok);
  }
  if (!verb) {
    // the 4 fields of the group, p bits each, from bit pay0 + pex on; lanes
    // with p = 0 (and lanes without a group) OR zeros
    const uint32_t msk = (uint32_t)(1ull << p) - 1u;
    const int o = pay0 + pex;
#pragma unroll
    for (int k = 0; k < 4; k++) or_word2(buf, o + k * p, (uint32_t)vv[k] & msk);
  } else if (b.act) {
#pragma unroll
    for (int k = 0; k < 4; k++) or_bits(buf, H + (4 * gi + k) * W, low_bits(a[k], W), W);
  }
  if (b.act && gi == 0) {
    uint32_t cm = H == 32 ? 0x3FFu : 0xFFFFu;
    uint32_t hdr = (uint32_t)st | ((uint32_t)e << 3) | (((uint32_t)c & cm) << 8);
    or_bits(buf, 0, hdr, 32);
  }
}

// Phase 1 for one tile (WP waves x 64/LPB blocks) of one array: analyse
// every block, assemble it in LDS region r of the run (block slots of
// `slot` >= g.ldsw words, the same for every tile of a run), record the
// block word counts and publish the tile's count (variable-size modes).
template <typename T, int LPB, int NDIM, int WP>
__device__ __forceinline__ void encode_analyze(const EncArgs& A, const int64_t tile, const int r,
                                               const int slot, EncShared<WP>& sm, uint32_t* lds) {
  constexpr int BPW = 64 / LPB;
  using B_ = Blk<T, LPB, NDIM>;
  const Geo& g = A.g;
  // wave-uniform by construction (batches read their arguments from memory,
  // where the compiler cannot see that)
  const int mode = __builtin_amdgcn_readfirstlane(g.mode);
  uint32_t* s_nw = sm.nw[r];
  const int wave = threadIdx.x >> 6;
  const bool variable = mode != M_RATE;
  int32_t code0;  // operating point, read before the block so the loads overlap
  uint32_t mask0;
  profiled_point(A, g, code0, mask0);
  B_ b;
  const int lane = lane_id();
  b.init(g, (tile * WP + wave) * BPW + lane / LPB, NDIM >= 2 ? sm.xch + wave * XCH : nullptr);
  const uint32_t emask = mode == M_RATE ? (mask0 & 0x7Fu) : mask0;
  int c, st;
  int32_t best, a[4];
  analyze_block<T, LPB, NDIM>(A, b, mode, code0, emask, c, st, best, a);
  const int nw = !b.blk_ok ? 0 : (mode == M_RATE ? g.budget : ((best + 31) >> 5));
  const int seg = b.L.seg, gi = b.L.gi;
  uint32_t* buf = lds + ((r * WP + wave) * BPW + seg) * slot;
  emit_block<T, LPB, NDIM>(g, b, c, st, emask, a, buf, nw);
  if (gi == 0) s_nw[wave * BPW + seg] = (uint32_t)nw;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t agg = 0;
    for (int i = 0; i < WP * BPW; i++) agg += s_nw[i];
    sm.agg[r] = agg;
    if (variable) lb_publish(A.tile_state, tile, agg);
  }
}

// The stream header (lanes 0-15 of the calling wave, one word each, read
// from `hsrc`: the argument block in memory, so no scalar registers are held
// for it across the kernel) and the index padding; in variable-size modes
// words 14-15 (the payload size) and the byte count are written by whoever
// knows the total.
__device__ __forceinline__ void write_stream_header(const EncArgs& A, const uint32_t* hsrc, bool variable) {
  const Geo& g = A.g;
  const int lane = lane_id();
  if (lane >= 16) return;
  uint32_t* h = reinterpret_cast<uint32_t*>(A.out_base);
  uint32_t w = hsrc[lane];
  if (A.sel && (lane == 2 || lane == 3)) {  // operating point adopted on the device
    int32_t code0;
    uint32_t mask0;
    const bool ok = profiled_point(A, g, code0, mask0);
    if (!ok && lane == 2) atomicOr(A.status, ST_NOPROFILE);
    w = lane == 2 ? ((w & ~0xFF00u) | ((mask0 & 0xFFu) << 8)) : (uint32_t)code0;
  }
  if (lane < 14 || !variable) h[lane] = w;
  if (lane == 0) {
    for (uint64_t i = A.zpad[0]; i < A.zpad[1]; i++) A.out_base[i] = 0;
    for (uint64_t i = A.zpad[2]; i < A.zpad[3]; i++) A.out_base[i] = 0;
    if (!variable) *A.d_nbytes = A.area + 4 * (uint64_t)g.budget * (uint64_t)g.nblocks;
  }
}

// Phase 2 for one tile, run by wave 0 in run order: the tile's offset (`base`
// in: offset of the previous tile of the run when `chain`, else unknown),
// the stream header and length fields it owns, the block offsets.
template <int WP, int BPW, int MODE = -1>  // MODE: M_RATE when known fixed rate, else runtime
__device__ __forceinline__ void encode_place(const EncArgs& A, const uint32_t* hsrc, const int64_t tile,
                                             const int r, EncShared<WP>& sm, bool chain, uint64_t& base) {
  const Geo& g = A.g;
  const int lane = lane_id();
  const bool variable = MODE == M_RATE ? false : g.mode != M_RATE;
  const uint64_t agg = sm.agg[r];
  if (variable) {
    if (!chain) base = lookback(A.tile_state, tile, A.status);
    if (tile > 0 && lane == 0) lb_prefix(A.tile_state, tile, base + agg);
    if (tile == A.ntiles - 1 && lane == 0) {
      const uint64_t total = base + agg;
      *reinterpret_cast<uint64_t*>(A.out_base + 56) = total;
      *A.d_nbytes = A.area + 4 * total;
    }
  } else {
    base = (uint64_t)tile * (WP * BPW) * (uint64_t)g.budget;
  }
  if (tile == 0) write_stream_header(A, hsrc, variable);
  if (lane == 0) {
    uint64_t acc = base;
    for (int i = 0; i < WP * BPW; i++) {
      sm.off[r][i] = acc;
      acc += sm.nw[r][i];
    }
  }
}

// Phase 3 for one tile: coalesced word stores of its LDS blocks and, in
// variable-size modes, their length and superblock-offset fields.
template <int LPB, int WP>
__device__ __forceinline__ void encode_store(const EncArgs& A, const int64_t tile, const int r,
                                             const int slot, EncShared<WP>& sm, const uint32_t* lds) {
  constexpr int BPW = 64 / LPB;
  const Geo& g = A.g;
  const int wave = threadIdx.x >> 6;
  const int lane = lane_id();
  const int seg = lane / LPB, gi = lane % LPB;
  const int64_t j = (tile * WP + wave) * BPW + seg;
  if (j >= g.nblocks) return;
  const int stride = g.ldsw;
  const uint32_t* buf = lds + ((r * WP + wave) * BPW + seg) * slot;
  const int nw = (int)sm.nw[r][wave * BPW + seg];
  const uint64_t off = sm.off[r][wave * BPW + seg];
  uint32_t* dst = A.out_words + off;
  for (int w = gi; w < nw; w += LPB) dst[w] = w < stride ? buf[w] : 0u;
  if (g.mode != M_RATE && gi == 0) {
    A.lens[j] = (uint16_t)nw;
    if ((j & 63) == 0) A.sbo[j >> 6] = off;
  }
}

// A whole run of tiles [t0, t0 + n) of one array (n <= RUN; fixed rate: 1).
template <typename T, int LPB, int NDIM, int WP>
__device__ __forceinline__ void encode_run(const EncArgs& A, const uint32_t* hsrc, const int64_t t0,
                                           const int n, EncShared<WP>& sm, uint32_t* lds) {
  constexpr int BPW = 64 / LPB;
#pragma unroll 1
  for (int r = 0; r < n; r++) encode_analyze<T, LPB, NDIM, WP>(A, t0 + r, r, A.g.ldsw, sm, lds);
  if ((threadIdx.x >> 6) == 0) {
    uint64_t base = 0;
#pragma unroll 1
    for (int r = 0; r < n; r++) {
      if (r > 0) base += sm.agg[r - 1];
      encode_place<WP, BPW>(A, hsrc, t0 + r, r, sm, r > 0, base);
    }
  }
  __syncthreads();
#pragma unroll 1
  for (int r = 0; r < n; r++) encode_store<LPB, WP>(A, t0 + r, r, A.g.ldsw, sm, lds);
}

}  // namespace apax
