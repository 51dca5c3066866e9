// profile.hip -- profiler kernels (Sec. 4) for gfx950.
//
// Every pass visits blocks with the encoder's own per-block machinery
// (bracket, quantizer, stream sizes, fixed-rate search), so the profiler sees
// exactly what the encoder will produce.  Persistent workgroups loop over
// tiles; each lane accumulates its statistics in binary64 (the terms scaled
// by a power of two chosen from max|x|, which is exact).  Lanes reduce once
// per workgroup (wave butterflies, then LDS) into a partial record; a
// one-workgroup kernel then
// reduces the records in a fixed order, so results are deterministic, and
// runs the next control step of the profile.  No global atomics in the
// passes.  grid.y indexes the gain codes evaluated in one launch.
#include "block.h"
#include "totals.h"
#include "kernels.h"
#include "encode_tile.h"

namespace apax {

__device__ void ctl_step(const CtlArgs& C);

// The profiler state is staged in LDS for the reduce kernels, so the
// one-thread control step runs on LDS instead of dependent global loads; a
// second copy keeps the state as read.
__device__ __forceinline__ void st_copy(PState* dst, PState* was, const PState* src) {
  constexpr int NW = (int)(sizeof(PState) / 4);
  const uint32_t* s = (const uint32_t*)src;
  uint32_t* d = (uint32_t*)dst;
  uint32_t* w = (uint32_t*)was;
  for (int i = threadIdx.x; i < NW; i += blockDim.x) {
    const uint32_t v = s[i];
    d[i] = v;
    w[i] = v;
  }
}

// The words of the state this kernel changed, back from LDS.  Reduce
// kernels of passes on two streams (the curve beside the metrics and
// centred passes) run at the same time and change different fields, so
// neither writes back a field it did not change; nor are the status and
// ticket words written, which other kernels change atomically.
__device__ __forceinline__ void st_copy_back(PState* dst, const PState* now, const PState* was) {
  constexpr int NW = (int)(sizeof(PState) / 4);
  constexpr int W0 = (int)(offsetof(PState, maxbits) / 4);
  static_assert(offsetof(PState, status) == 0 && offsetof(PState, ticket) == 4 && W0 == 2,
                "status and ticket lead the state");
  const uint32_t* n = (const uint32_t*)now;
  const uint32_t* w = (const uint32_t*)was;
  uint32_t* d = (uint32_t*)dst;
  for (int i = W0 + threadIdx.x; i < NW; i += blockDim.x)
    if (n[i] != w[i]) d[i] = n[i];
}


// ---------------------------------------------------------------- max |x|
// Streaming pass: max |x| as magnitude bit patterns (monotone in value) and
// the non-finite flag, 16-byte loads; one partial per workgroup, reduced by
// the last workgroup, which then brackets the codes (control step C_INIT).
struct PMaxPart {
  uint64_t key;
  uint32_t nf, pad;
};

template <typename T>
__device__ __forceinline__ void pmax_take(T v, uint64_t& key, uint32_t& nf) {
  uint64_t k;
  if constexpr (Traits<T>::isint) {
    const int64_t iv = (int64_t)v;
    k = __builtin_bit_cast(uint64_t, (double)(iv < 0 ? -iv : iv));
  } else if constexpr (sizeof(T) == 4) {
    const uint32_t m = __builtin_bit_cast(uint32_t, v) & 0x7FFFFFFFu;
    const uint32_t bad = m >= 0x7F800000u;
    nf |= bad;
    k = bad ? 0 : __builtin_bit_cast(uint64_t, (double)__builtin_bit_cast(float, m));
  } else {
    const uint64_t m = __builtin_bit_cast(uint64_t, v) & 0x7FFFFFFFFFFFFFFFull;
    const uint32_t bad = m >= 0x7FF0000000000000ull;
    nf |= bad;
    k = bad ? 0 : m;
  }
  key = k > key ? k : key;
}

template <typename T>
__global__ __launch_bounds__(256) void k_pmax(const T* __restrict__ x, uint64_t n, PMaxPart* parts) {
  constexpr int PER = 16 / sizeof(T);
  constexpr int U = 4;  // independent 16-byte loads in flight per thread
  __shared__ uint64_t s_key[4];
  __shared__ uint32_t s_nf[4];
  const uint64_t nvec = (((uintptr_t)x) & 15) == 0 ? n / PER : 0;
  uint64_t key = 0;
  uint32_t nf = 0;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  typedef unsigned int v4u __attribute__((ext_vector_type(4)));
  const v4u* xv = reinterpret_cast<const v4u*>(x);
  uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (; i + (U - 1) * stride < nvec; i += U * stride) {
    v4u u[U];
#pragma unroll
    for (int r = 0; r < U; r++) u[r] = __builtin_nontemporal_load(xv + i + r * stride);
#pragma unroll
    for (int r = 0; r < U; r++) {
      T v[PER];
      __builtin_memcpy(v, &u[r], 16);
#pragma unroll
      for (int k = 0; k < PER; k++) pmax_take<T>(v[k], key, nf);
    }
  }
  for (; i < nvec; i += stride) {
    v4u u = xv[i];
    T v[PER];
    __builtin_memcpy(v, &u, 16);
#pragma unroll
    for (int k = 0; k < PER; k++) pmax_take<T>(v[k], key, nf);
  }
  for (uint64_t t = nvec * PER + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += stride)
    pmax_take<T>(x[t], key, nf);
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint64_t t = (uint64_t)__shfl_xor((unsigned long long)key, o, 64);
    key = t > key ? t : key;
  }
  const int wave = threadIdx.x >> 6;
  const bool wnf = __ballot(nf != 0) != 0;
  if (lane_id() == 0) {
    s_key[wave] = key;
    s_nf[wave] = wnf;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t k = s_key[0];
    uint32_t f = s_nf[0];
    for (int w = 1; w < 4; w++) {
      k = s_key[w] > k ? s_key[w] : k;
      f |= s_nf[w];
    }
    parts[blockIdx.x].key = k;
    parts[blockIdx.x].nf = f;
  }
}

// One workgroup: max over the partials of the max pass, then C_INIT.
__global__ __launch_bounds__(256) void k_pmax_reduce(const PMaxPart* parts, int nparts, CtlArgs C) {
  __shared__ uint64_t s_key[4];
  __shared__ uint32_t s_nf[4];
  __shared__ PState s_st, s_was;
  uint64_t k = 0;
  uint32_t f = 0;
  // the first record of every thread is loaded before the state is copied
  // into LDS, so the two loads are in flight together
  const int w0 = threadIdx.x;
  const uint64_t k0 = w0 < nparts ? parts[w0].key : 0;
  const uint32_t f0 = w0 < nparts ? parts[w0].nf : 0;
  st_copy(&s_st, &s_was, C.st);
  k = k0;
  f = f0;
  for (int w = w0 + blockDim.x; w < nparts; w += blockDim.x) {
    const uint64_t kw = parts[w].key;
    k = kw > k ? kw : k;
    f |= parts[w].nf;
  }
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    uint64_t t = (uint64_t)__shfl_xor((unsigned long long)k, o, 64);
    k = t > k ? t : k;
  }
  const bool anyf = __ballot(f != 0) != 0;
  const int wave = threadIdx.x >> 6;
  if (lane_id() == 0) {
    s_key[wave] = k;
    s_nf[wave] = anyf;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    bool nfa = anyf;
    for (int w = 1; w < 4; w++) {
      k = s_key[w] > k ? s_key[w] : k;
      nfa |= s_nf[w] != 0;
    }
    s_st.maxbits[0] = k;
    if (nfa) {
      s_st.status |= ST_NONFINITE;
      atomicOr(&C.st->status, ST_NONFINITE);
    }
    CtlArgs D = C;
    D.st = &s_st;
    ctl_step(D);
  }
  __syncthreads();
  st_copy_back(C.st, &s_st, &s_was);
}

// ---------------------------------------------------------------- block passes
// Fixed-order reduction of the partial records of one pass (one workgroup,
// 256 threads): each code's records are split over Lc lanes, lane k taking
// records k, k + Lc, ... in order (U records loaded together), then a
// butterfly inside the wave and an ordered merge of the waves.  OPK / HIST
// name the pass, so only its fields are loaded.  The first batch is loaded
// before the profiler state is copied into LDS (S, and S0 as read), so both
// are in flight together; the results are written into S.
template <int OPK, bool HIST>
__device__ void reduce_recs(const ProfArgs& A, PState* S, PState* S0) {
  constexpr int I0 = OPK == P_STATS ? 0 : (OPK == P_CURVE ? S_XX : (OPK == P_CENTER ? S_CXX : NSUM));
  constexpr int I1 = (OPK == P_STATS || OPK == P_CURVE) ? S_CXX : NSUM;
  constexpr int NS = I1 - I0;  // sums of the pass
  constexpr int NSA = NS > 0 ? NS : 1;
  constexpr bool WORDS = OPK == P_STATS || OPK == P_CURVE || HIST;
  constexpr bool DMAX = OPK == P_STATS;
  constexpr bool FITS = OPK == P_FITS;
  constexpr int U = OPK == P_CURVE ? 16 : 8;
  __shared__ double s_ff[4][NSA];
  __shared__ uint64_t s_c64[4][2];
  __shared__ uint32_t s_c32[4][9];
  const int mc = A.maxcodes;  // <= MAXCODES, so every code gets Lc >= 8 lanes
  const int64_t nwg = A.nwg;
  const PParts P = pparts(A.parts, (int64_t)mc * nwg);
  int Lc = 256;
  while (Lc > 1 && Lc * mc > 256) Lc >>= 1;
  const int ci = (int)threadIdx.x / Lc;
  const int k = (int)threadIdx.x % Lc;
  const bool in_code = ci < mc;
  const int64_t r0 = (int64_t)(in_code ? ci : 0) * nwg;
  double acc[NSA];
#pragma unroll
  for (int i = 0; i < NSA; i++) acc[i] = 0.0;
  uint64_t w = 0, dm = 0;
  uint32_t fit = 0, h[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  auto batch = [&](const int64_t q0, const bool copy_state) {
    double v[NSA][U];
    uint64_t wv[U], dv[U];
    uint32_t fv[U], hv[8][U];
#pragma unroll
    for (int u = 0; u < U; u++) {
      const int64_t q = q0 + (int64_t)u * Lc;
      const bool in = in_code && q < nwg;
#pragma unroll
      for (int i = 0; i < NS; i++) v[i][u] = in ? P.s[(int64_t)(I0 + i) * P.R + r0 + q] : 0.0;
      if (WORDS) wv[u] = in ? P.words[r0 + q] : 0;
      if (DMAX) dv[u] = in ? P.dmax[r0 + q] : 0;
      if (FITS) fv[u] = in ? P.nfit[r0 + q] : 0;
      if (HIST) {
#pragma unroll
        for (int t = 0; t < 8; t++) hv[t][u] = in ? P.hist[(int64_t)t * P.R + r0 + q] : 0;
      }
    }
    if (copy_state) st_copy(S, S0, A.st);
#pragma unroll
    for (int u = 0; u < U; u++) {
#pragma unroll
      for (int i = 0; i < NS; i++) acc[i] += v[i][u];
      if (WORDS) w += wv[u];
      if (DMAX) dm = dv[u] > dm ? dv[u] : dm;
      if (FITS) fit += fv[u];
      if (HIST) {
#pragma unroll
        for (int t = 0; t < 8; t++) h[t] += hv[t][u];
      }
    }
  };
  batch(k, true);
  for (int64_t q0 = k + (int64_t)U * Lc; q0 < nwg; q0 += (int64_t)U * Lc) batch(q0, false);
  __syncthreads();  // the state copy is complete
  const int nset = A.final_code ? 1 : S->ncodes;
  const int ncodes = nset < mc ? nset : mc;

  // butterfly inside the code's lanes of one wave
  const int Lw = Lc < 64 ? Lc : 64;
  for (int o = 1; o < Lw; o <<= 1) {
#pragma unroll
    for (int i = 0; i < NS; i++) acc[i] += __shfl_xor(acc[i], o, 64);
    if (WORDS) w += (uint64_t)__shfl_xor((unsigned long long)w, o, 64);
    if (DMAX) {
      const uint64_t d2 = (uint64_t)__shfl_xor((unsigned long long)dm, o, 64);
      dm = d2 > dm ? d2 : dm;
    }
    if (FITS) fit += __shfl_xor(fit, o, 64);
    if (HIST) {
#pragma unroll
      for (int t = 0; t < 8; t++) h[t] += __shfl_xor(h[t], o, 64);
    }
  }
  // codes spanning several waves (Lc > 64): merge the waves in order
  if (Lc > 64) {
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
      for (int i = 0; i < NS; i++) s_ff[wave][i] = acc[i];
      s_c64[wave][0] = w;
      s_c64[wave][1] = dm;
      s_c32[wave][0] = fit;
#pragma unroll
      for (int t = 0; t < 8; t++) s_c32[wave][1 + t] = h[t];
    }
    __syncthreads();
    if (k == 0) {
      const int wb = (int)threadIdx.x >> 6, nw = Lc / 64;
      for (int j = 1; j < nw; j++) {
#pragma unroll
        for (int i = 0; i < NS; i++) acc[i] += s_ff[wb + j][i];
        w += s_c64[wb + j][0];
        dm = s_c64[wb + j][1] > dm ? s_c64[wb + j][1] : dm;
        fit += s_c32[wb + j][0];
#pragma unroll
        for (int t = 0; t < 8; t++) h[t] += s_c32[wb + j][1 + t];
      }
    }
  }
  if (ci < ncodes && k == 0) {
#pragma unroll
    for (int i = 0; i < NS; i++) S->sums[ci][I0 + i] = acc[i];
    if (FITS) S->fits[ci] = fit;
    if (HIST && ci == 0) {
      for (int t = 0; t < 8; t++) S->hist[t] = h[t];
      S->sub_samples = w;
    }
    if (OPK == P_STATS || OPK == P_CURVE) S->words[ci] = w;
    if (DMAX) S->maxbits[1] = dm;
  }
}

// OPK: the pass (P_FITS, P_STATS, P_CENTER, P_CURVE).  The statistics passes
// over 1-4 byte samples are held to five waves per SIMD (a few spilled
// values cost less than the latency the fifth wave hides).
template <typename T, int LPB, int NDIM, int OPK>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(OPK == P_CURVE && sizeof(T) <= 4 ? 6 : ((OPK == P_STATS || OPK == P_MENC) && sizeof(T) <= 4 ? 5 : 1)))) void k_profile(ProfArgs A) {
  constexpr int OP = (OPK == P_CURVE || OPK == P_MENC) ? P_STATS : OPK;
  // P_MENC: the fixed-rate metrics pass also writes each block's encoded
  // words (its code and stream are the encoder's), assembled in the
  // dynamic LDS, one ldsw-word buffer per block of the tile
  constexpr bool MENC = OPK == P_MENC;
  extern __shared__ __align__(16) uint32_t enc_lds[];
  A.curve = OPK == P_CURVE;
  if (OPK == P_CURVE) A.rule = R_QUALITY;  // curve codes are fixed per block
  constexpr int BPW = 64 / LPB;
  using B_ = Blk<T, LPB, NDIM>;
  const Geo& g = A.g;
  PState* st = A.st;
  constexpr int NL = S_CXX;  // accumulator slots; the centred pass uses slots S_XX..S_DD
  __shared__ double s_red[WPG][NL];
  __shared__ uint64_t s_w[WPG], s_dm[WPG];
  __shared__ uint32_t s_fit[WPG], s_hist[WPG][8];
  __shared__ uint4 s_xch[NDIM >= 2 ? WPG * XCH : 1];

  // (workgroup of the code, code): blockIdx, or with the XCD map, id =
  // ((q * maxcodes + code) * 8 + x) for workgroup 8 q + x of the code --
  // consecutive ids go to consecutive XCDs, so every id of workgroup 8 q + x
  // lands on XCD x, and the codes' workgroups over the same tiles run there
  // close together
  int64_t wgx;
  int ci;
  if (A.xcd_map) {
    const uint32_t id = blockIdx.x, k = id >> 3;
    ci = (int)(k % (uint32_t)A.maxcodes);
    wgx = (int64_t)(k / (uint32_t)A.maxcodes) * 8 + (id & 7u);
  } else {
    wgx = blockIdx.x;
    ci = blockIdx.y;
  }
  const int nset = A.final_code ? 1 : st->ncodes;
  const int ncodes = nset < A.maxcodes ? nset : A.maxcodes;
  if (ci >= ncodes) return;  // uniform per workgroup
  if (OP == P_CENTER && st->centred) return;  // the metrics pass's moments gave the centred sums
  const int wave = threadIdx.x >> 6;
  const int lane = lane_id();
  const int code = A.final_code ? st->code : st->codes[ci];
  const int escale = st->escale;
  uint32_t mask;
  if (A.mask_sel == 0) mask = st->mask_probe;
  else if (A.mask_sel == 1) mask = st->mask_out | 0x81u;
  else mask = A.rule == R_RATE ? ((st->mask_out & 0x7Fu) | 1u) : (st->mask_out | 0x81u);
  const double s1 = ldexp(1.0, -escale);
  const double s2 = ldexp(1.0, -2 * escale);
  const double mx = st->mean[0], my = st->mean[1], md = st->mean[2];
  // active accumulator slots of this pass
  constexpr int L0 = OP == P_STATS ? (OPK == P_CURVE ? S_XX : 0) : S_XX;
  constexpr int L1 = OP == P_STATS ? NL : (OP == P_CENTER ? S_DS : 0);
  constexpr int NA = L1 > L0 ? L1 - L0 : 1;
  // each lane sums its groups' binary64 terms over up to 64 tiles, then
  // adds the partial (scaled by a power of two) to the accumulators that
  // every further reduction level uses; those are only touched by these
  // adds, so they live in LDS (one slot per thread)
  __shared__ double s_acc[NA][WPG * 64];
#pragma unroll
  for (int i = 0; i < NA; i++) s_acc[i][threadIdx.x] = 0.0;
  double lacc[NL];
#pragma unroll
  for (int i = 0; i < NL; i++) lacc[i] = 0.0;
  int lcount = 0;
  auto flush = [&]() {
#pragma unroll
    for (int i = L0; i < L1; i++) {
      s_acc[i - L0][threadIdx.x] += lacc[i] * (i < S_XX ? s1 : s2);
    }
#pragma unroll
    for (int i = 0; i < NL; i++) lacc[i] = 0.0;
    lcount = 0;
  };
  double dmax = 0.0;
  uint32_t nfit = 0;
  uint32_t hcnt[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // wave-uniform
  unsigned long long wsum = 0;

  // block of this lane in tile t (past the end: an empty block)
  auto block_of = [&](int64_t t) -> int64_t {
    const int64_t jj = (t * WPG + wave) * BPW + lane / LPB;
    return jj < A.nbe ? jj * A.jstride : g.nblocks;
  };
  uint4* xw = NDIM >= 2 ? s_xch + wave * XCH : nullptr;
  // the samples of the next tile are fetched while the current one is
  // evaluated (a tile past the end fetches nothing)
  B_ nb;
  T nv[4];
  nb.init(g, block_of(wgx), xw);
  nb.fetch((const T*)A.x, g, nv);
  for (int64_t tile = wgx; tile < A.ntiles; tile += A.nwg) {
    B_ b = nb;
    T cv[4];
#pragma unroll
    for (int k = 0; k < 4; k++) cv[k] = nv[k];
    if (tile + A.nwg < A.ntiles) {
      nb.init(g, block_of(tile + A.nwg), xw);
      nb.fetch((const T*)A.x, g, nv);
    }
    if (OP == P_CENTER && A.rule != R_QUALITY) b.template take<false>(g, cv);
    else b.take(g, cv);
    int32_t a[4];
    int32_t best;
    if (OP == P_FITS) {
      // argmin over the mask at the clamped code: fit test + stream histogram
      int c = A.rule == R_LOSSLESS ? 0 : clampc(code, b.cf, b.cc);
      b.quantize(c, A.rule == R_LOSSLESS, a);
      if (!A.hist) {  // bisection probe: the fit test alone
        if (b.fits(g, mask, a, 32 * g.budget) && b.blk_ok && b.L.gi == 0) nfit++;
        continue;
      }
      int s_ = b.best_stream(g, mask, a, best);
      if (b.blk_ok && b.L.gi == 0 && best <= 32 * g.budget) nfit++;
      if (A.hist) {
        if (b.act) wsum += (unsigned long long)b.nvalid;  // samples of the subsample
        const bool lead = b.blk_ok && b.L.gi == 0;
#pragma unroll
        for (int t = 0; t < 8; t++) hcnt[t] += (uint32_t)__popcll(__ballot(lead && s_ == t));
      }
      continue;
    }
    // P_STATS / P_CENTER: operating point of the block, decoded values
    int c = 0;
    int s_enc = 0;        // P_MENC: the block's stream
    bool have_a = false;  // a[] already holds the block quantized at c
    if (A.rule == R_QUALITY) {
      c = clampc(code, b.cf, b.cc);
    } else if (A.rule == R_RATE) {
      if (OP == P_CENTER) {
        c = b.blk_ok ? A.cj[b.j] : 0;
      } else {
        c = clampc(code, b.cf, b.cc);
        const uint32_t m7 = mask & 0x7Fu;
        b.quantize(c, false, a);
        int s_ = b.best_stream(g, m7, a, best);
        bool need = b.act && best > 32 * g.budget;
        if (__ballot(need)) c = b.rate_search(g, g.mask, c, s_, need);
        else have_a = true;
        if (A.store_cj && b.blk_ok && b.L.gi == 0) {
          A.cj[b.j] = c;
          if (A.bst) A.bst[b.j] = (uint8_t)s_;  // the encoder's choice at this block
        }
        s_enc = s_;
      }
    }
    if (!have_a) b.quantize(c, A.rule == R_LOSSLESS, a);
    if constexpr (MENC) {
      // the block's budget words at code c with stream s_enc (the encoder's
      // mask is the metrics pass's: stream-histogram mask, verbatim allowed)
      const int nwb = b.blk_ok ? g.budget : 0;
      uint32_t* buf = enc_lds + (wave * BPW + b.L.seg) * g.ldsw;
      emit_block<T, LPB, NDIM>(g, b, c, s_enc, mask & 0x7Fu, a, buf, nwb);
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
      __builtin_amdgcn_wave_barrier();
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
      uint32_t* dst = A.enc_words + (uint64_t)(b.blk_ok ? b.j : 0) * (uint64_t)g.budget;
      for (int w = b.L.gi; w < nwb; w += LPB) dst[w] = w < g.ldsw ? buf[w] : 0u;
    }
    if (OP == P_STATS) {
      int nw;
      if (A.rule != R_RATE) {
        const int s_ = b.best_stream(g, mask, a, best);
        nw = (best + 31) >> 5;
        if (A.bst && b.blk_ok && b.L.gi == 0) {  // the encoder's size pass, done here
          A.bst[b.j] = (uint8_t)s_;
          A.lens[b.j] = (uint16_t)nw;
          atomicAdd(&A.ssum[b.j >> 6], (uint32_t)nw);
        }
      } else {
        nw = g.budget;
      }
      if (b.blk_ok && b.L.gi == 0) wsum += (unsigned long long)nw;
    }
    // the group's terms are summed first (4 terms), then added to the
    // lane's partial
    double t[NL];
#pragma unroll
    for (int i = 0; i < NL; i++) t[i] = 0.0;
    const double Rq = inv_mantissa(c);
    const int eq = -(c >> 4);
    // a sample past the edge (or of a lane without a group) is 0 and
    // decodes to 0, so its terms of the plain sums are +0 and change nothing:
    // the statistics passes add them unconditionally
#pragma unroll
    for (int k = 0; k < 4; k++) {
      if (OP != P_STATS && !(b.act && b.valid(k))) continue;
      double x = b.xv(k);
      double y;
      if (A.rule == R_LOSSLESS) y = (double)a[k];
      else y = (double)to_out<T>(dequant_rk(a[k], Rq, eq));
      double d = x - y;
      if (OP == P_STATS) {
        if (!A.curve) {
          t[S_X] += x;
          t[S_Y] += y;
          t[S_D] += d;
          double ad = __builtin_fabs(d);
          dmax = ad > dmax ? ad : dmax;
        }
        // products fused into the adds (one rounding instead of two: the
        // sums stay within the 1e-9 the statistics promise, at fewer
        // instructions)
        t[S_XX] = __builtin_fma(x, x, t[S_XX]);
        t[S_YY] = __builtin_fma(y, y, t[S_YY]);
        t[S_DD] = __builtin_fma(d, d, t[S_DD]);
        t[S_DS] = __builtin_fma(d, x + y, t[S_DS]);
      } else {
        double ex = x - mx, ey = y - my, ed = d - md;
        t[S_XX] = __builtin_fma(ex, ex, t[S_XX]);  // slots of the centred sums S_CXX, S_CYY, S_CDD
        t[S_YY] = __builtin_fma(ey, ey, t[S_YY]);
        t[S_DD] = __builtin_fma(ed, ed, t[S_DD]);
      }
    }
#pragma unroll
    for (int i = 0; i < NL; i++) lacc[i] += t[i];
    if (++lcount == 64) flush();
  }
  flush();

  // ---- workgroup partial record
  if constexpr (L1 > L0) {
    double part[L1 - L0];
#pragma unroll
    for (int i = 0; i < L1 - L0; i++) part[i] = s_acc[i][threadIdx.x];
    const double tot = wave_totals<L1 - L0>(part, lane);
    const int idx = wave_totals_index<L1 - L0>(lane);
    if (lane < 8 && idx < L1 - L0) {
      s_red[wave][L0 + idx] = tot;
    }
  }
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    double tt = __shfl_xor(dmax, o, 64);
    dmax = tt > dmax ? tt : dmax;
    wsum += __shfl_xor(wsum, o, 64);
    nfit += __shfl_xor(nfit, o, 64);
  }
  if (lane == 0) {
    s_w[wave] = wsum;
    s_dm[wave] = __builtin_bit_cast(uint64_t, dmax);
    s_fit[wave] = nfit;
#pragma unroll
    for (int t = 0; t < 8; t++) s_hist[wave][t] = hcnt[t];
  }
  __syncthreads();
  const PParts P = pparts(A.parts, (int64_t)A.maxcodes * A.nwg);
  const int64_t r = (int64_t)ci * A.nwg + wgx;
  if (threadIdx.x < NL) {
    const int i = threadIdx.x;
    if (i >= L0 && i < L1) {
      double tt = s_red[0][i];
      for (int w = 1; w < WPG; w++) tt += s_red[w][i];
      const int si = OP == P_CENTER ? i - S_XX + S_CXX : i;  // sum index of the slot
      P.s[(int64_t)si * P.R + r] = tt;
    }
  } else if (threadIdx.x == 64) {
    uint64_t ww = 0, dm = 0;
    uint32_t nf = 0;
    for (int w = 0; w < WPG; w++) {
      ww += s_w[w];
      dm = s_dm[w] > dm ? s_dm[w] : dm;
      nf += s_fit[w];
    }
    P.words[r] = ww;
    P.dmax[r] = dm;
    P.nfit[r] = nf;
  } else if (threadIdx.x >= 128 && threadIdx.x < 136) {
    const int t = threadIdx.x - 128;
    uint32_t h = 0;
    for (int w = 0; w < WPG; w++) h += s_hist[w][t];
    P.hist[(int64_t)t * P.R + r] = h;
  }
}

// the probe records (fit counts only) of up to MAXCODES codes x 2048
// workgroups fit the partial region sized for 2048 + 2 MAXCODES full records
static_assert((int64_t)MAXCODES * 2048 * 4 <= (2048 + 2 * (int64_t)MAXCODES) * PPART_BYTES, "probe records");

// Bisection probes of a fixed-rate profile (the fit test alone) with every
// code of the launch tested on a tile that is loaded and bracketed once:
// each persistent workgroup takes tiles wgx, wgx + nwg, ... and, per tile,
// quantizes and tests its blocks at each code in turn; the fits of code ci
// go to record ci * nwg + wgx, the layout of the one-code-per-workgroup
// passes, so the same reduce kernel follows.
template <typename T, int LPB, int NDIM>
__global__ __launch_bounds__(256) void k_probe_all(ProfArgs A) {
  constexpr int BPW = 64 / LPB;
  using B_ = Blk<T, LPB, NDIM>;
  const Geo& g = A.g;
  const PState* st = A.st;
  __shared__ uint4 s_xch[NDIM >= 2 ? WPG * XCH : 1];
  __shared__ uint32_t s_fit[WPG][MAXCODES];
  __shared__ int32_t s_code[MAXCODES];
  const int wave = threadIdx.x >> 6;
  const int lane = lane_id();
  const int nset = st->ncodes;
  const int ncodes = nset < A.maxcodes ? nset : A.maxcodes;
  if (threadIdx.x < MAXCODES) s_code[threadIdx.x] = st->codes[threadIdx.x];
  if (lane < MAXCODES) s_fit[wave][lane] = 0;
  __syncthreads();
  const uint32_t mask = st->mask_probe;
  const int64_t wgx = blockIdx.x;
  auto block_of = [&](int64_t t) -> int64_t {
    const int64_t jj = (t * WPG + wave) * BPW + lane / LPB;
    return jj < A.nbe ? jj * A.jstride : g.nblocks;
  };
  uint4* xw = NDIM >= 2 ? s_xch + wave * XCH : nullptr;
  B_ nb;
  T nv[4];
  nb.init(g, block_of(wgx), xw);
  nb.fetch((const T*)A.x, g, nv);
  for (int64_t tile = wgx; tile < A.ntiles; tile += A.nwg) {
    B_ b = nb;
    T cv[4];
#pragma unroll
    for (int k = 0; k < 4; k++) cv[k] = nv[k];
    if (tile + A.nwg < A.ntiles) {
      nb.init(g, block_of(tile + A.nwg), xw);
      nb.fetch((const T*)A.x, g, nv);
    }
    b.take(g, cv);
    const bool lead = b.blk_ok && b.L.gi == 0;
#pragma unroll 1
    for (int ci = 0; ci < ncodes; ci++) {
      const int c = clampc(s_code[ci], b.cf, b.cc);
      int32_t a[4];
      b.quantize(c, false, a);
      const bool f = b.fits(g, mask, a, 32 * g.budget);
      const uint32_t n = (uint32_t)__popcll(__ballot(f && lead));
      if (lane == 0) s_fit[wave][ci] += n;
    }
  }
  __syncthreads();
  const PParts P = pparts(A.parts, (int64_t)A.maxcodes * A.nwg);
  if (threadIdx.x < ncodes) {
    const int ci = threadIdx.x;
    uint32_t n = 0;
    for (int w = 0; w < WPG; w++) n += s_fit[w][ci];
    P.nfit[(int64_t)ci * A.nwg + wgx] = n;
  }
}

// One workgroup: fixed-order reduction of the records of the preceding
// pass, then its control step.
template <int OPK, bool HIST>
__global__ __launch_bounds__(256) void k_reduce(ProfArgs A) {
  if (OPK == P_CENTER && A.st->centred) return;  // no centred pass ran
  __shared__ PState s_st, s_was;
  reduce_recs<OPK, HIST>(A, &s_st, &s_was);
  __syncthreads();
  if (threadIdx.x == 0 && A.C.step != C_NONE) {
    CtlArgs C = A.C;
    C.st = &s_st;
    ctl_step(C);
  }
  __syncthreads();
  st_copy_back(A.st, &s_st, &s_was);
}

// ---------------------------------------------------------------- control
__device__ int ctl_largest(double M, double lim, int cmin, int cmax) {
  if (M * gain_of(cmax) <= lim) return cmax;
  int lo = cmin, hi = cmax;
  while (hi - lo > 1) {
    int mid = lo + ((hi - lo) >> 1);
    if (M * gain_of(mid) <= lim) lo = mid;
    else hi = mid;
  }
  return lo;
}

// pre-order nodes of the bisection decision tree of the next `depth` steps
// (a node, then its left and right subtrees), depth <= D; unrolled at
// compile time, so no stack array (a dynamically indexed local array becomes
// compare-and-select chains on the one thread that runs this)
template <int D>
__device__ __forceinline__ void ctl_tree_rec(int l, int h, int d, int32_t* out, int& n) {
  if (d == 0 || h - l <= 1 || n >= MAXCODES) return;
  const int mid = l + ((h - l) >> 1);
  out[n++] = mid;
  if constexpr (D > 1) {
    ctl_tree_rec<D - 1>(l, mid, d - 1, out, n);
    ctl_tree_rec<D - 1>(mid, h, d - 1, out, n);
  }
}

constexpr int CTL_MAX_DEPTH = 4;  // 15 nodes + the cap fit MAXCODES
__device__ int ctl_tree(int lo, int hi, int depth, int32_t* out, int n) {
  ctl_tree_rec<CTL_MAX_DEPTH>(lo, hi, depth < CTL_MAX_DEPTH ? depth : CTL_MAX_DEPTH, out, n);
  return n;
}

__device__ void r_from(const double* S, double& r) {
  double sxx = S[S_XX], syy = S[S_YY], sdd = S[S_DD], sds = S[S_DS];
  if (sxx == 0.0 && syy == 0.0) { r = 1.0; return; }
  if (sxx == 0.0 || syy == 0.0) { r = 0.0; return; }
  double nx = sqrt(sxx), ny = sqrt(syy);
  double dn = sds / (nx + ny);
  r = 1.0 - (sdd - dn * dn) / (2.0 * nx * ny);
}

constexpr double CENTRED_K = 1000.0;

__device__ void ctl_zero(PState* st) {
  for (int i = 0; i < MAXCODES; i++) { st->fits[i] = 0; st->words[i] = 0; }
}

__device__ void ctl_step(const CtlArgs& C) {
  PState* st = C.st;
  const bool fr = C.mode == M_RATE;
  switch (C.step) {
    case C_INIT: {
      double M = __builtin_bit_cast(double, st->maxbits[0]);
      int CF = ctl_largest(M, 0.5, C.cmin, C.cmax);
      int CC = C.isint ? 0 : ctl_largest(M, 2147483647.0, C.cmin, C.cmax);
      int ex = 0;
      if (M > 0) frexp(M, &ex);
      st->cf = CF; st->cc = CC; st->escale = ex;
      st->need = (uint32_t)((9 * C.nsub + 9) / 10);
      st->mask_probe = fr ? (C.mask_user & 0x7Fu) : C.mask_user;
      st->flags = 0; st->n_probes = 0;
      ctl_zero(st);
      if (C.mode == M_LOSSLESS || (st->status & ST_NONFINITE) || CF >= CC) {
        st->code = C.mode == M_LOSSLESS ? 0 : CC;
        st->done = 1; st->ncodes = 0;
      } else {
        st->lo = CF; st->hi = CC; st->first = 1; st->done = 0;
        st->probe[0] = CC;
        int n = ctl_tree(CF, CC, C.depth, st->probe, 1);
        for (int i = 0; i < n; i++) st->codes[i] = st->probe[i];
        st->ncodes = n;
      }
      break;
    }
    case C_DECIDE: {
      if (st->done || st->ncodes == 0) { st->ncodes = 0; break; }
      const int n = st->ncodes;
      // the predicate and the tie flag of every probed code, as bit masks
      uint32_t pred = 0, near = 0;
      for (int i = 0; i < n; i++) {
        if (fr) {
          pred |= (st->fits[i] >= st->need ? 1u : 0u) << i;
        } else {
          double r;
          r_from(st->sums[i], r);
          pred |= (r >= C.target ? 1u : 0u) << i;
          near |= (fabs(r - C.target) < 1e-11 ? 1u : 0u) << i;
        }
      }
      int k = 0;
      if (st->first) {
        st->first = 0;
        st->n_probes++;
        if (near & 1u) st->flags |= 1;
        if (fr ? (pred & 1u) : !(pred & 1u)) {  // all fit at the cap / target unreachable
          st->code = st->cc; st->done = 1; st->ncodes = 0;
          break;
        }
        k = 1;
      }
      int lo = st->lo, hi = st->hi;
      while (hi - lo > 1) {
        int mid = lo + ((hi - lo) >> 1);
        while (k < n && st->probe[k] != mid) k++;
        if (k >= n) break;
        st->n_probes++;
        if ((near >> k) & 1u) st->flags |= 1;
        const bool pk = (pred >> k) & 1u;
        if (fr) { if (pk) lo = mid; else hi = mid; }
        else { if (pk) hi = mid; else lo = mid; }
      }
      st->lo = lo; st->hi = hi;
      ctl_zero(st);
      if (hi - lo <= 1) {
        st->code = fr ? lo : hi; st->done = 1; st->ncodes = 0;
      } else {
        int m = ctl_tree(lo, hi, C.depth, st->probe, 0);
        for (int i = 0; i < m; i++) st->codes[i] = st->probe[i];
        st->ncodes = m;
      }
      break;
    }
    case C_MASK: {  // histogram launch comes next: probe the chosen code
      st->codes[0] = st->code; st->ncodes = 1;
      for (int t = 0; t < 8; t++) st->hist[t] = 0;
      ctl_zero(st);
      break;
    }
    case C_CURVE: {  // after the histogram: stream mask, then the curve codes
      uint64_t thresh = (C.nsub + 99) / 100;
      if (thresh < 1) thresh = 1;
      uint32_t mask = 0x81u;
      for (int t = 0; t < 8; t++)
        if (st->hist[t] >= thresh) mask |= 1u << t;
      st->mask_out = mask & (C.mask_user | 0x81u);
      // the operating point an encode of this workspace may adopt on the device
      st->sel[0] = st->code;
      st->sel[1] = (int32_t)(fr ? ((st->mask_out & 0x7Fu) | 1u) : (st->mask_out | 0x81u));
      for (int t = 0; t < NCURVE; t++) {
        int ct = st->code + 4 * (t - NCURVE / 2);
        ct = ct < C.cmin ? C.cmin : (ct > C.cmax ? C.cmax : ct);
        st->codes[t] = ct;
        st->curve_codes[t] = ct;
      }
      st->ncodes = NCURVE;
      // the metrics pass (at st->code alone) comes next, then the centred
      // and curve passes; codes[] keeps the curve codes until then
      st->maxbits[1] = 0;
      ctl_zero(st);
      break;
    }
    case C_KEEP_CURVE: {  // after the curve pass: keep its sums
      for (int t = 0; t < NCURVE; t++) {
        st->curve_sums[t][0] = st->sums[t][S_XX];
        st->curve_sums[t][1] = st->sums[t][S_YY];
        st->curve_sums[t][2] = st->sums[t][S_DD];
        st->curve_sums[t][3] = st->sums[t][S_DS];
        st->curve_words[t] = st->words[t];
      }
      break;
    }
    case C_MEANS: {  // after the metrics pass: keep it, means for the centred pass
      for (int i = 0; i < NSUM; i++) st->msums[i] = st->sums[0][i];
      st->mwords = st->words[0];
      double n = (double)(C.nsamples ? C.nsamples : 1);
      st->mean[0] = ldexp(st->sums[0][S_X], st->escale) / n;
      st->mean[1] = ldexp(st->sums[0][S_Y], st->escale) / n;
      st->mean[2] = ldexp(st->sums[0][S_D], st->escale) / n;
      // The centred sums S2 - S^2 / n from the raw moments, where that is
      // well conditioned: mean^2 <= CENTRED_K var for x, y and d (or every
      // term zero).  The binary64 sums carry relative errors below ~4e-14 (of
      // S2, and of sum |x| for S), so the variance's relative error stays
      // below 4e-14 (1 + 3 CENTRED_K) ~ 1.2e-10; otherwise the centred pass
      // sums (x - mean)^2 itself.
      auto direct = [&](int is, int iq, int ic) -> bool {
        const double S = st->sums[0][is], Q = st->sums[0][iq];
        const double m2n = S * (S / n);
        const double c = Q - m2n;
        if (Q == 0.0) { st->sums[0][ic] = 0.0; return true; }
        if (c > 0.0 && m2n <= CENTRED_K * c) { st->sums[0][ic] = c; return true; }
        return false;
      };
      const bool dx = direct(S_X, S_XX, S_CXX), dy = direct(S_Y, S_YY, S_CYY), dd = direct(S_D, S_DD, S_CDD);
      st->centred = dx && dy && dd ? 1 : 0;
      break;
    }
  }
}

__global__ void k_ctl(CtlArgs C) {
  if (threadIdx.x == 0 && blockIdx.x == 0) ctl_step(C);
}

int64_t prof_tiles(const Geo& g, int64_t nbe) {
  int lpb = g.G <= 16 ? 16 : (g.G <= 32 ? 32 : 64);
  int64_t per = (int64_t)WPG * (64 / lpb);
  return (nbe + per - 1) / per;
}

// persistent workgroups per code: about 2048 in flight over all codes
int64_t prof_wgs(int64_t ntiles, int ncodes) {
  int64_t w = (2048 + ncodes - 1) / ncodes;
  return ntiles < w ? ntiles : w;
}

// Workgroups of `kernel` (256 threads) the whole chip holds at once, at most
// 2048: the persistent passes launch about this many, so every SIMD runs the
// same number of waves from start to end.
template <void (*KERNEL)(ProfArgs)>
static int64_t resident_wgs() {
  // (queried once per kernel, on the device current at the first launch)
  static const int64_t r = [] {
    int n = 0, dev = 0, cus = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, (const void*)KERNEL, WPG * 64, 0) != hipSuccess || n < 1)
      n = 8;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
      cus = 256;
    const int64_t t = (int64_t)n * cus;
    return t < 2048 ? t : (int64_t)2048;
  }();
  return r;
}

// Persistent workgroups of a one-wave-per-block pass: a one-code pass runs
// the resident count (every SIMD keeps the same number of waves to the end);
// several codes share about 2048 workgroups (measured faster than the
// resident count for the curve), in whole groups of 8 per code mapped onto
// the XCDs; the fixed-rate probes test every code in each workgroup.
static void plan_wgs(ProfArgs& A, int64_t resident) {
  A.xcd_map = 0;
  if (A.maxcodes > 1) resident = 2048;
  if (A.probe_all) {
    A.nwg = A.ntiles < resident ? A.ntiles : resident;
    return;
  }
  int64_t per = resident / A.maxcodes;
  if (per < 1) per = 1;
  A.nwg = A.ntiles < per ? A.ntiles : per;
  if (A.maxcodes > 1 && A.nwg >= 8) {
    A.nwg = A.nwg / 8 * 8;
    A.xcd_map = 1;
  }
}

template <typename T, int LPB, int NDIM>
static hipError_t launch_t(ProfArgs& A, hipStream_t s) {
  if (A.op == P_FITS && A.probe_all) plan_wgs(A, resident_wgs<k_probe_all<T, LPB, NDIM>>());
  else if (A.op == P_FITS) plan_wgs(A, resident_wgs<k_profile<T, LPB, NDIM, P_FITS>>());
  else if (A.op == P_STATS && A.curve) plan_wgs(A, resident_wgs<k_profile<T, LPB, NDIM, P_CURVE>>());
  else if (A.op == P_STATS && A.enc_words) plan_wgs(A, resident_wgs<k_profile<T, LPB, NDIM, P_MENC>>());
  else if (A.op == P_STATS) plan_wgs(A, resident_wgs<k_profile<T, LPB, NDIM, P_STATS>>());
  else plan_wgs(A, resident_wgs<k_profile<T, LPB, NDIM, P_CENTER>>());
  const dim3 grid = A.xcd_map ? dim3((unsigned)(A.nwg * A.maxcodes), 1) : dim3((unsigned)A.nwg, A.maxcodes);
  const dim3 block(WPG * 64);
  if (A.op == P_FITS && A.probe_all) {
    hipLaunchKernelGGL((k_probe_all<T, LPB, NDIM>), dim3((unsigned)A.nwg), block, 0, s, A);
    return hipGetLastError();
  }
  if (A.op == P_FITS) hipLaunchKernelGGL((k_profile<T, LPB, NDIM, P_FITS>), grid, block, 0, s, A);
  else if (A.op == P_STATS && A.curve) hipLaunchKernelGGL((k_profile<T, LPB, NDIM, P_CURVE>), grid, block, 0, s, A);
  else if (A.op == P_STATS && A.enc_words)
    hipLaunchKernelGGL((k_profile<T, LPB, NDIM, P_MENC>), grid, block, (size_t)WPG * (64 / LPB) * A.g.ldsw * 4, s, A);
  else if (A.op == P_STATS) hipLaunchKernelGGL((k_profile<T, LPB, NDIM, P_STATS>), grid, block, 0, s, A);
  else hipLaunchKernelGGL((k_profile<T, LPB, NDIM, P_CENTER>), grid, block, 0, s, A);
  return hipGetLastError();
}

template <typename T, int NDIM>
static hipError_t launch_lpb(ProfArgs& A, hipStream_t s) {
  if (A.g.G <= 16) return launch_t<T, 16, NDIM>(A, s);
  if (A.g.G <= 32) return launch_t<T, 32, NDIM>(A, s);
  return launch_t<T, 64, NDIM>(A, s);
}

template <typename T>
static hipError_t launch_nd(ProfArgs& A, int ndim, hipStream_t s) {
  if (ndim == 1) return launch_lpb<T, 1>(A, s);
  if (ndim == 2) return launch_lpb<T, 2>(A, s);
  return launch_lpb<T, 3>(A, s);
}

hipError_t launch_profile(int dtype, int ndim, ProfArgs& A, hipStream_t s, hipEvent_t* ev, hipStream_t rs,
                          hipEvent_t fork) {
  // blocks of more than 64 groups, or groups of 8: one workgroup per block
  const bool wide = A.g.G > 64 || A.g.gq == 2;
  A.ntiles = wide ? A.nbe : prof_tiles(A.g, A.nbe);
  // (the one-wave-per-block passes size their grid at launch: plan_wgs)
  A.nwg = prof_wgs(A.ntiles, A.maxcodes);
  A.xcd_map = 0;
  // fixed-rate bisection probes: every code of the launch tested on each
  // tile, loaded and bracketed once
  A.probe_all = !wide && A.op == P_FITS && !A.hist && !A.final_code && A.rule == R_RATE && A.maxcodes > 1;
  if (A.ntiles == 0) return hipSuccess;
  hipError_t e;
  if (ev && (e = hipEventRecord(ev[0], s)) != hipSuccess) return e;
  if (wide) e = launch_wide_profile(dtype, ndim, A, s);
  else switch (dtype) {
    case DT_I8: e = launch_nd<int8_t>(A, ndim, s); break;
    case DT_I16: e = launch_nd<int16_t>(A, ndim, s); break;
    case DT_I32: e = launch_nd<int32_t>(A, ndim, s); break;
    case DT_F32: e = launch_nd<float>(A, ndim, s); break;
    default: e = launch_nd<double>(A, ndim, s); break;
  }
  if (e != hipSuccess) return e;
  if (ev && (e = hipEventRecord(ev[1], s)) != hipSuccess) return e;
  // the reduce on another stream, forked once the pass is done
  if (rs) {
    if ((e = hipEventRecord(fork, s)) != hipSuccess || (e = hipStreamWaitEvent(rs, fork, 0)) != hipSuccess) return e;
    s = rs;
  }
  if (A.op == P_FITS && A.hist) hipLaunchKernelGGL((k_reduce<P_FITS, true>), dim3(1), dim3(256), 0, s, A);
  else if (A.op == P_FITS) hipLaunchKernelGGL((k_reduce<P_FITS, false>), dim3(1), dim3(256), 0, s, A);
  else if (A.op == P_STATS && A.curve) hipLaunchKernelGGL((k_reduce<P_CURVE, false>), dim3(1), dim3(256), 0, s, A);
  else if (A.op == P_STATS) hipLaunchKernelGGL((k_reduce<P_STATS, false>), dim3(1), dim3(256), 0, s, A);
  else hipLaunchKernelGGL((k_reduce<P_CENTER, false>), dim3(1), dim3(256), 0, s, A);
  return hipGetLastError();
}

hipError_t launch_pmax(int dtype, const void* x, uint64_t n, void* parts, const CtlArgs& C,
                       hipStream_t s, hipEvent_t* ev) {
  if (n == 0) return hipSuccess;
  const unsigned grid = PMAX_WGS;
  PMaxPart* P = reinterpret_cast<PMaxPart*>(parts);
  if (ev && hipEventRecord(ev[0], s) != hipSuccess) return hipErrorUnknown;
  switch (dtype) {
    case DT_I8: hipLaunchKernelGGL(k_pmax<int8_t>, dim3(grid), dim3(256), 0, s, (const int8_t*)x, n, P); break;
    case DT_I16: hipLaunchKernelGGL(k_pmax<int16_t>, dim3(grid), dim3(256), 0, s, (const int16_t*)x, n, P); break;
    case DT_I32: hipLaunchKernelGGL(k_pmax<int32_t>, dim3(grid), dim3(256), 0, s, (const int32_t*)x, n, P); break;
    case DT_F32: hipLaunchKernelGGL(k_pmax<float>, dim3(grid), dim3(256), 0, s, (const float*)x, n, P); break;
    default: hipLaunchKernelGGL(k_pmax<double>, dim3(grid), dim3(256), 0, s, (const double*)x, n, P); break;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (ev && (e = hipEventRecord(ev[1], s)) != hipSuccess) return e;
  hipLaunchKernelGGL(k_pmax_reduce, dim3(1), dim3(256), 0, s, (const PMaxPart*)P, (int)grid, C);
  return hipGetLastError();
}

hipError_t launch_ctl(const CtlArgs& C, hipStream_t s) {
  hipLaunchKernelGGL(k_ctl, dim3(1), dim3(64), 0, s, C);
  return hipGetLastError();
}

}  // namespace apax
