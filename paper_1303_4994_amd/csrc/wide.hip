// wide.hip -- encode and decode kernels for blocks of more than 256 samples
// (G > 64 groups, up to the 16384 samples Sec. 6 allows): one workgroup per
// block, the block staged in LDS (wide.h).
#include "decode_tile.h"
#include "encode_tile.h"
#include "wide.h"

namespace apax {

enum { WK_RATE = 0, WK_SIZE = 1, WK_EMIT = 2, WK_CHOICE = 3, WK_TABLE = 4 };

template <typename T, int NDIM>
struct WEnc {
  static constexpr int W = Traits<T>::W;
  static constexpr int H = Traits<T>::H;
  static constexpr bool ISINT = Traits<T>::isint;
  static constexpr uint32_t NDMASK = NDIM == 1 ? 0x0Fu : (NDIM == 2 ? 0x2Fu : 0x7Fu);  // 1-d: 3 = filter
  using S = typename std::conditional<ISINT, int32_t, double>::type;

  const Geo* g;
  WGeo wg;
  int64_t j;
  int tid;
  S xs[WIDE_GPT][4];  // samples of groups tid + m * nt (0 past the edge)
  int cf, cc;
  bool nonfinite;
  uint32_t* qa;   // LDS: quantized block, then the block's encoding
  uint8_t* eps;   // LDS: exponent rows, stream s at eps + s * G (row 7: the chosen stream)
  WideShared* sh;
  int qc;         // code of the block in qa (qa empty: a value no code takes)
  int32_t bits[7];

  __device__ __forceinline__ void init(const Geo& g_, int64_t j_, uint32_t* lds, WideShared& sh_) {
    g = &g_;
    j = j_;
    wg.init(g_, j_);
    tid = threadIdx.x;
    qa = lds;
    eps = reinterpret_cast<uint8_t*>(lds + wide_qw(g_));
    sh = &sh_;
    qc = 0x7FFFFFFF;
    cf = cc = 0;
    nonfinite = false;
  }

  // samples of the thread's groups; BRACKET: the block's code bracket too
  template <bool BRACKET>
  __device__ __forceinline__ void load(const T* __restrict__ x) {
    uint64_t key = 0;
#pragma unroll
    for (int m = 0; m < WIDE_GPT; m++) {
      const int gi = tid + m * wg.nt;
      T v[4] = {(T)0, (T)0, (T)0, (T)0};
      if (gi < g->G) {
        int z, y, xq;
        wg.coords(*g, gi, z, y, xq);
        int64_t idx;
        const int nv = wg.nvalid(*g, z, y, xq, idx);
        load4<T>(x, idx, nv, v);
      }
#pragma unroll
      for (int k = 0; k < 4; k++) {
        xs[m][k] = (S)v[k];
        if constexpr (ISINT) {
          const int32_t s = (int32_t)v[k];
          key = max(key, (uint64_t)(s < 0 ? 0u - (uint32_t)s : (uint32_t)s));
        } else if constexpr (sizeof(T) == 4) {
          key = max(key, (uint64_t)(__builtin_bit_cast(uint32_t, (float)v[k]) & 0x7FFFFFFFu));
        } else {
          key = max(key, __builtin_bit_cast(uint64_t, (double)v[k]) & 0x7FFFFFFFFFFFFFFFull);
        }
      }
    }
    if constexpr (!BRACKET) return;
    if (tid == 0) sh->key = 0;
    __syncthreads();
    if (key) atomicMax((unsigned long long*)&sh->key, (unsigned long long)key);
    __syncthreads();
    key = sh->key;
    uint64_t m;
    int e;
    if constexpr (ISINT) {
      bracket_me<false>(key, 0, g->cmin, g->cmax, true, cf, cc);
    } else if constexpr (sizeof(T) == 4) {
      nonfinite = key >= 0x7F800000u;
      const uint32_t E = (uint32_t)key >> 23;
      m = (uint64_t)(((uint32_t)key & 0x7FFFFFu) | (E ? 0x800000u : 0u));
      e = E ? (int)E - 150 : -149;
      bracket_me<false>(m, e, g->cmin, g->cmax, false, cf, cc);
    } else {
      const uint32_t hi = (uint32_t)(key >> 32);
      nonfinite = hi >= 0x7FF00000u;
      const uint32_t E = hi >> 20;
      m = (key & 0xFFFFFFFFFFFFFull) | (E ? (1ull << 52) : 0ull);
      e = E ? (int)E - 1075 : -1074;
      bracket_me<true>(m, e, g->cmin, g->cmax, false, cf, cc);
    }
  }

  // the block quantized at code c into qa (lossless integers: the samples)
  __device__ __forceinline__ void quantize(int c, bool lossless) {
    if (c == qc) return;
    const double gv = gain_of(c);
#pragma unroll
    for (int m = 0; m < WIDE_GPT; m++) {
      const int gi = tid + m * wg.nt;
      if (gi >= g->G) break;
      int32_t a[4];
#pragma unroll
      for (int k = 0; k < 4; k++) {
        if constexpr (ISINT) a[k] = lossless ? xs[m][k] : quant((double)xs[m][k], gv);
        else a[k] = quant(xs[m][k], gv);
      }
      *reinterpret_cast<uint4*>(qa + 4 * gi) = make_uint4((uint32_t)a[0], (uint32_t)a[1], (uint32_t)a[2], (uint32_t)a[3]);
    }
    __syncthreads();
    qc = c;
  }

  // the filter stream x[n] - s x[n-k] of group gi of a 1-d block (Sec. 5 / Sec. 6)
  __device__ __forceinline__ void group_filter(int gi, const uint32_t P[6], uint32_t u[4]) const {
#pragma unroll
    for (int m = 0; m < 4; m++) {
      const int p = 4 * gi + m;
      const uint32_t prev = p >= g->fk ? qa[p - g->fk] : 0u;
      u[m] = g->fneg ? P[m + 2] + prev : P[m + 2] - prev;
    }
  }

  // values of stream st (0..6) for group gi: wrapped to W bits, 0 past the edge
  __device__ __forceinline__ void group_stream(int st, int gi, int32_t v[4]) const {
    int z, y, xq;
    wg.coords(*g, gi, z, y, xq);
    int64_t idx;
    const int nv = wg.nvalid(*g, z, y, xq, idx);
    uint32_t P[6], Y[6], Z[6], ZY[6];
    wide_row6(qa, *g, z, y, xq, P);
    const uint32_t bit = 1u << st;
    if (bit & 0x68u) wide_row6(qa, *g, z, y - 1, xq, Y);
    if (bit & 0x50u) wide_row6(qa, *g, z - 1, y, xq, Z);
    if (bit & 0x40u) wide_row6(qa, *g, z - 1, y - 1, xq, ZY);
    uint32_t u[4];
    if (NDIM == 1 && st == 3) group_filter(gi, P, u);
    else wide_stream(st, P, Y, Z, ZY, u);
#pragma unroll
    for (int k = 0; k < 4; k++) v[k] = k < nv ? wrapw<W>(u[k]) : 0;
  }

  // bits of every stream in `need` (a subset of 0x7F) at the quantized block;
  // returns their sum (with one stream: its bits).  Exponent positions of
  // g->gq groups of 4 (groups of 4 or 8 samples, Sec. 6); each thread takes
  // CP consecutive positions.
  __device__ __forceinline__ int32_t cost(uint32_t need) {
    need &= NDMASK;
    const int G = g->G, gq = g->gq, NP = G / gq;
    const int CP = (NP + wg.nt - 1) / wg.nt, pp0 = tid * CP;
    int32_t pay[7] = {0, 0, 0, 0, 0, 0, 0};
    for (int q = 0; q < CP; q++) {
      const int pos = pp0 + q;
      if (pos >= NP) break;
      int em[7] = {0, 0, 0, 0, 0, 0, 0}, pm[7] = {0, 0, 0, 0, 0, 0, 0};
      for (int r = 0; r < gq; r++) {
        const int gi = pos * gq + r;
        int z, y, xq;
        wg.coords(*g, gi, z, y, xq);
        int64_t idx;
        const int nv = wg.nvalid(*g, z, y, xq, idx);
        uint32_t P[6], Y[6] = {0, 0, 0, 0, 0, 0}, Z[6] = {0, 0, 0, 0, 0, 0}, ZY[6] = {0, 0, 0, 0, 0, 0};
        wide_row6(qa, *g, z, y, xq, P);
        if (need & 0x68u) wide_row6(qa, *g, z, y - 1, xq, Y);
        if (need & 0x50u) wide_row6(qa, *g, z - 1, y, xq, Z);
        if (need & 0x40u) wide_row6(qa, *g, z - 1, y - 1, xq, ZY);
#pragma unroll
        for (int st = 0; st < 7; st++) {
          if (!((need >> st) & 1u)) continue;
          uint32_t u[4];
          if (NDIM == 1 && st == 3) group_filter(gi, P, u);
          else wide_stream(st, P, Y, Z, ZY, u);
          int32_t v[4];
#pragma unroll
          for (int k = 0; k < 4; k++) v[k] = k < nv ? wrapw<W>(u[k]) : 0;
          int e, pw;
          group_eps<W>(v, e, pw);
          em[st] = max(em[st], e);
          pm[st] = max(pm[st], pw);
        }
      }
#pragma unroll
      for (int st = 0; st < 7; st++) {
        if (!((need >> st) & 1u)) continue;
        eps[st * G + pos] = (uint8_t)em[st];
        pay[st] += 4 * gq * pm[st];
      }
    }
    wg_sum<7>(pay, *sh);  // its barriers also publish the exponent rows
    int32_t last[7];
#pragma unroll
    for (int st = 0; st < 7; st++) last[st] = ((need >> st) & 1u) ? wide_last_big(eps + st * G, NP, pp0, CP) : -1;
    wg_excl_max<7>(last, *sh);
    int32_t nib[7];
#pragma unroll
    for (int st = 0; st < 7; st++)
      nib[st] = ((need >> st) & 1u) ? wide_jee_count(eps + st * G, NP, pp0, CP, last[st]) : 0;
    wg_sum<7>(nib, *sh);
    int32_t sum = 0;
#pragma unroll
    for (int st = 0; st < 7; st++) {
      bits[st] = ((need >> st) & 1u) ? H + 4 * nib[st] + pay[st] : 0x7FFFFFFF;
      sum += ((need >> st) & 1u) ? bits[st] : 0;
    }
    return sum;
  }

  __device__ __forceinline__ int32_t verbatim_bits() const { return H + g->B * W; }

  // cheapest stream of `mask` at the quantized block (ties: the lowest id)
  __device__ __forceinline__ int choose(uint32_t mask, int32_t& best) {
    cost(mask & 0x7Fu);
    best = 0x7FFFFFFF;
    int st = 0;
#pragma unroll
    for (int s = 0; s < 8; s++) {
      if (!((mask >> s) & 1u)) continue;
      const int32_t b = s == 7 ? verbatim_bits() : bits[s];
      if (b < best) {
        best = b;
        st = s;
      }
    }
    return st;
  }

  __device__ __forceinline__ int32_t cost_one(int st) {
    if (st == 7) return verbatim_bits();
    return cost(1u << st);
  }

  // fixed rate, from the block's start code c (quantized, stream st chosen
  // there, size best): step down an octave at a time until the block fits the
  // budget (c_floor always fits), then bisect between the last fitting and the
  // last failing code
  __device__ __forceinline__ int rate_search(int c, int st, int32_t best) {
    const int32_t budget = 32 * g->budget;
    if (best <= budget) return c;
    int hi = c;
    for (;;) {
      c = c - 16 < cf ? cf : c - 16;
      quantize(c, false);
      if (cost_one(st) <= budget) break;
      hi = c;
    }
    int lo = c;
    while (hi - lo > 1) {
      const int mid = lo + ((hi - lo) >> 1);
      quantize(mid, false);
      if (cost_one(st) <= budget) lo = mid;
      else hi = mid;
    }
    return lo;
  }

  // the block's encoding at code c (quantized in qa) with stream st, nw words
  // stored at dst (words past the LDS buffer are zero padding).  The thread
  // takes CP consecutive exponent positions, i.e. their gq * CP groups of 4.
  __device__ __forceinline__ void emit(int c, int st, int nw, uint32_t* __restrict__ dst) {
    const int G = g->G, gq = g->gq, NP = G / gq;
    const int CP = (NP + wg.nt - 1) / wg.nt, pp0 = tid * CP, q0 = pp0 * gq, nq = CP * gq;
    const bool verb = st == 7;
    uint8_t* e7 = eps + 7 * G;
    uint32_t vv[WIDE_GPT][4];
    int32_t pwq[WIDE_GPT];  // payload width of each group's position
    int32_t pay = 0;
#pragma unroll
    for (int lq = 0; lq < WIDE_GPT; lq++) {
      const int gi = q0 + lq;
      pwq[lq] = 0;
#pragma unroll
      for (int k = 0; k < 4; k++) vv[lq][k] = 0u;
      if (lq >= nq || gi >= G) continue;
      if (verb) {
        const uint4 a = *reinterpret_cast<const uint4*>(qa + 4 * gi);
        vv[lq][0] = a.x; vv[lq][1] = a.y; vv[lq][2] = a.z; vv[lq][3] = a.w;
      } else {
        int32_t v[4];
        group_stream(st, gi, v);
        int e, pw;
        group_eps<W>(v, e, pw);
        pwq[lq] = (e << 8) | pw;  // combined per position below
#pragma unroll
        for (int k = 0; k < 4; k++) vv[lq][k] = (uint32_t)v[k];
      }
    }
    if (!verb) {  // exponent and width of each position: the widest of its groups
#pragma unroll
      for (int lq = 0; lq < WIDE_GPT; lq++) {
        // gq = 2: groups lq & ~1 and lq | 1 share a position (the even one
        // already holds the pair's maximum when the odd one comes)
        const int a = lq & ~1, b = (lq | 1) < WIDE_GPT ? (lq | 1) : lq;
        const int m = gq == 1 ? pwq[lq] : max(pwq[a], pwq[b]);
        const bool head = gq == 1 || (lq & 1) == 0;
        const int pos = pp0 + (gq == 1 ? lq : (lq >> 1));
        if (head && lq < nq && pos < NP) {
          e7[pos] = (uint8_t)(m >> 8);
          pay += 4 * gq * (m & 0xFF);
        }
        pwq[lq] = m;
      }
    }
    int32_t s1[1] = {pay}, t1[1];
    wg_excl_sum<1>(s1, t1, *sh);  // its barriers publish row 7 and end the reads of qa
    int32_t payoff = s1[0];
    int32_t last[1] = {verb ? -1 : wide_last_big(e7, NP, pp0, CP)};
    wg_excl_max<1>(last, *sh);
    int32_t n1[1] = {verb ? 0 : wide_jee_count(e7, NP, pp0, CP, last[0])}, ntot[1];
    wg_excl_sum<1>(n1, ntot, *sh);
    const int e0 = verb ? 0 : (int)e7[0];
    uint32_t* buf = qa;
    const int nz = nw < g->ldsw ? nw : g->ldsw;
    for (int w = tid; w < nz; w += wg.nt) buf[w] = 0u;
    __syncthreads();
    if (!verb) {
      // JEE tokens of the thread's positions
      int lst = last[0], noff = n1[0];
      for (int q = 0; q < CP; q++) {
        const int i = pp0 + q;
        if (i >= NP) break;
        if (i == 0) {
          lst = 0;
          continue;
        }
        const int d = (int)e7[i] - (int)e7[i - 1];
        const int ad = d < 0 ? -d : d;
        if (ad <= 1) {
          if ((i - lst) & 1) {
            const int d2 = i + 1 < NP ? (int)e7[i + 1] - (int)e7[i] : 9;
            const bool pair = d2 >= -1 && d2 <= 1;
            const uint32_t tok = pair ? (uint32_t)(3 * (d + 1) + (d2 + 1)) : (uint32_t)(11 + d);
            or_word2(buf, H + 4 * noff, tok);
            noff += 1;
          }
        } else {
          lst = i;
          const int ei = e7[i];
          if (ad == 2) {
            or_word2(buf, H + 4 * noff, (uint32_t)(11 + d));
            noff += 1;
          } else {
            or_word2(buf, H + 4 * noff, (uint32_t)(14 + (ei >> 4)) | ((uint32_t)(ei & 15) << 4));
            noff += 2;
          }
        }
      }
      // BFPE payload: 4 gq fields of pw bits per position, its groups in order
      int o = H + 4 * ntot[0] + payoff;
#pragma unroll
      for (int lq = 0; lq < WIDE_GPT; lq++) {
        if (lq >= nq || q0 + lq >= G) break;
        const int pw = pwq[lq] & 0xFF;
        if (pw) {
          const uint32_t msk = (uint32_t)((1ull << pw) - 1u);
#pragma unroll
          for (int k = 0; k < 4; k++) or_word2(buf, o + k * pw, vv[lq][k] & msk);
        }
        o += 4 * pw;
      }
    } else {
#pragma unroll
      for (int lq = 0; lq < WIDE_GPT; lq++) {
        const int gi = q0 + lq;
        if (lq >= nq || gi >= G) break;
#pragma unroll
        for (int k = 0; k < 4; k++) or_word2(buf, H + (4 * gi + k) * W, low_bits((int32_t)vv[lq][k], W));
      }
    }
    if (tid == 0) {
      const uint32_t cm = H == 32 ? 0x3FFu : 0xFFFFu;
      or_bits(buf, 0, (uint32_t)st | ((uint32_t)e0 << 3) | (((uint32_t)c & cm) << 8), 32);
    }
    __syncthreads();
    for (int w = tid; w < nw; w += wg.nt) dst[w] = w < g->ldsw ? buf[w] : 0u;
    qc = 0x7FFFFFFF;
  }
};

// One block per workgroup.  KIND: WK_RATE fixed rate (search and store at
// j * budget), WK_SIZE variable-size first pass (length, chosen stream,
// superblock sums), WK_EMIT second pass (store at the block's offset),
// WK_CHOICE the lagged choice's first pass (each block's own best stream into
// aux, int32 per block), WK_TABLE the adaptive rate's transition map of the
// block (aux: 64 bytes per block).
template <typename T, int NDIM, int KIND>
__global__ __launch_bounds__(WIDE_MAXT) void k_wide_enc(EncArgs A, void* aux) {
  extern __shared__ __align__(16) uint32_t lds[];
  __shared__ WideShared sh;
  const uint32_t* hsrc =
      (const uint32_t*)((const uint8_t*)__builtin_amdgcn_kernarg_segment_ptr() + offsetof(EncArgs, hdr));
  const Geo& g = A.g;
  const int64_t j = blockIdx.x;
  const int mode = g.mode;
  int32_t code0;
  uint32_t mask0;
  profiled_point(A, g, code0, mask0);
  if (A.bcode) code0 = A.bcode[j];  // adaptive rate: the block's own requested code
  if ((KIND == WK_RATE || KIND == WK_EMIT) && j == 0 && threadIdx.x < 64)
    write_stream_header(A, hsrc, KIND == WK_EMIT);
  WEnc<T, NDIM> b;
  b.init(g, j, lds, sh);
  if (mode == M_LOSSLESS) b.template load<false>((const T*)A.x);
  else b.template load<true>((const T*)A.x);
  if (b.nonfinite && threadIdx.x == 0) atomicOr(A.status, ST_NONFINITE);
  const int c0 = mode == M_LOSSLESS ? 0 : clampc(code0, b.cf, b.cc);
  b.quantize(c0, mode == M_LOSSLESS);
  if constexpr (KIND == WK_CHOICE) {
    int32_t best;
    const int st = b.choose(g.mask, best);
    if (threadIdx.x == 0) static_cast<int32_t*>(aux)[j] = st;
  } else if constexpr (KIND == WK_TABLE) {
    uint8_t* row = static_cast<uint8_t*>(aux) + 64 * j;
    int cprev = 0x7FFFFFFF, nprev = 0;
    for (int w = 0; w < 64; w++) {
      if (w >= g.awd) {
        if (threadIdx.x == 0) row[w] = (uint8_t)w;
        continue;
      }
      const int c = clampc(g.alo + w, b.cf, b.cc);
      if (c != cprev) {
        b.quantize(c, false);
        int32_t best;
        b.choose(g.mask, best);
        nprev = (best + 31) >> 5;
        cprev = c;
      }
      if (threadIdx.x == 0) row[w] = adapt_next(w, nprev, g.target, g.awd);
    }
  } else if constexpr (KIND == WK_RATE) {
    const uint32_t emask = mask0 & 0x7Fu;
    int32_t best;
    const int st = b.choose(emask, best);
    const int c = b.rate_search(c0, st, best);
    b.quantize(c, false);
    b.emit(c, st, g.budget, A.out_words + (uint64_t)j * (uint64_t)g.budget);
  } else if constexpr (KIND == WK_SIZE) {
    int32_t best;
    int st;
    if (A.lag) {  // lossless, lagged: the previous block's choice, verbatim if that is larger
      st = j == 0 ? 0 : A.lag[j - 1];
      best = b.cost_one(st);
      if (best > b.verbatim_bits()) {
        st = 7;
        best = b.verbatim_bits();
      }
    } else {
      st = b.choose(mask0, best);
    }
    if (threadIdx.x == 0) {
      const uint32_t nw = (uint32_t)((best + 31) >> 5);
      A.lens[j] = (uint16_t)nw;
      A.bst[j] = (uint8_t)st;
      atomicAdd(&A.ssum[j >> 6], nw);
    }
  } else {  // WK_EMIT
    const int st = A.bst[j];
    const int nw = A.lens[j];
    int32_t l[1] = {0};
    const int64_t jb = (j >> 6) << 6;
    if (threadIdx.x < 64 && jb + (int64_t)threadIdx.x < j) l[0] = A.lens[jb + threadIdx.x];
    wg_sum<1>(l, sh);
    const uint64_t off = A.sbo[j >> 6] + (uint64_t)l[0];
    b.emit(c0, st, nw, A.out_words + off);
  }
}

// ---- decoder: one block per workgroup
template <typename T, int NDIM, bool DOT>
__global__ __launch_bounds__(WIDE_MAXT) void k_wide_dec(DecArgs A, const T* __restrict__ w, double* partial) {
  constexpr int H = Traits<T>::H;
  constexpr int W = Traits<T>::W;
  constexpr int MAXEPS = W == 32 ? 31 : W;
  extern __shared__ __align__(16) uint32_t lds[];
  __shared__ WideShared sh;
  __shared__ double s_dot[WIDE_MAXT / 64];
  const Geo& g = A.g;
  const int64_t j = blockIdx.x;
  const int tid = threadIdx.x;
  WGeo wg;
  wg.init(g, j);
  const int nt = wg.nt, G = g.G, C = wg.C, p0 = tid * C;
  // exponent positions (groups of 4 or 8 samples: gq groups of 4 each); the
  // thread takes CP consecutive positions, i.e. groups q0 .. q0 + nq - 1
  const int gq = g.gq, NP = G / gq, CP = (NP + nt - 1) / nt, pp0 = tid * CP, q0 = pp0 * gq, nq = CP * gq;
  const int mode = g.mode;
  const bool variable = mode != M_RATE;
  uint32_t* buf = lds;
  const int stride = g.ldsw;
  int32_t* info = reinterpret_cast<int32_t*>(lds + wide_qw(g) + 2 * G);
  bool bad = false;

  if (j == 0 && tid < 16) {
    const uint32_t* h = reinterpret_cast<const uint32_t*>(A.in);
    if (h[tid] != A.hdr[tid]) atomicOr(A.status, ST_CORRUPT);
  }

  // ---- block offset and length (workgroup-uniform)
  uint64_t off;
  int len;
  bool ubad = false;
  if (variable) {
    int32_t l[1] = {0};
    const int64_t jb = (j >> 6) << 6;
    if (tid < 64 && jb + tid < j) l[0] = A.lens[jb + tid];
    wg_sum<1>(l, sh);
    const uint64_t sb = A.sbo[j >> 6];
    ubad = sb > A.payload_words;  // checked before the addition, which could wrap
    off = ubad ? A.payload_words : sb + (uint64_t)(uint32_t)l[0];
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
  // ---- stage the words (two zero words after them); words past the LDS
  // buffer (a fixed-rate budget above any encoding) can only be padding
  {
    const int lim = len + 2 < stride ? len + 2 : stride;
    for (int q = tid; q < lim; q += nt) buf[q] = q < len ? A.words[off + q] : 0u;
    for (int q = stride + tid; q < len; q += nt)
      if (A.words[off + q]) bad = true;
  }
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
  ubad |= rsv != 0u;
  ubad |= !((g.mask >> st) & 1u);
  ubad |= mode == M_LOSSLESS ? (c != 0) : (c < g.cmin || c > g.cmax);
  ubad |= 32 * len < H;
  if (verb) ubad |= e0 != 0 || 32 * len < H + g.B * W;
  else ubad |= e0 > MAXEPS;

  // ---- JEE tokens: starts, positions, token area length
  int tend = 0;
  if (!verb && !ubad) {
    const int K = 2 * (NP - 1);                 // nibbles the tokens can take at most
    const int avail = (32 * len - H) / 4;      // nibbles before the block's end
    const int Kw = K < avail ? K : avail;
    const int NC = (K + nt - 1) / nt;          // nibbles per thread
    const int k0 = tid * NC;
    auto nib = [&](int k) -> int { const int b = H + 4 * k; return (int)((buf[b >> 5] >> (b & 31)) & 15u); };
    // per-position token data: (1 << 16) | difference (16 bits) or (2 << 16) | absolute exponent
    auto rel = [](int d) -> int32_t { return (1 << 16) | (int32_t)(uint16_t)(int16_t)d; };
    // last non-escape nibble before each nibble
    int32_t lne[1] = {-1};
    for (int q = 0; q < NC; q++) {
      const int k = k0 + q;
      if (k >= Kw) break;
      if (nib(k) < 14) lne[0] = k;
    }
    wg_excl_max<1>(lne, sh);
    // positions covered by the thread's tokens
    int32_t np[1] = {0};
    {
      int last = lne[0];
      for (int q = 0; q < NC; q++) {
        const int k = k0 + q;
        if (k >= Kw) break;
        const int t = nib(k);
        if (((k - last - 1) & 1) == 0) np[0] += t <= 8 ? 2 : 1;
        if (t < 14) last = k;
      }
    }
    int32_t ptot[1];
    wg_excl_sum<1>(np, ptot, sh);
    if (tid == 0) sh.tend = -1;
    __syncthreads();
    {
      int last = lne[0];
      int pos = 1 + np[0];
      for (int q = 0; q < NC; q++) {
        const int k = k0 + q;
        if (k >= Kw || pos > NP - 1) break;
        const int t = nib(k);
        const bool start = ((k - last - 1) & 1) == 0;
        if (t < 14) last = k;
        if (!start) continue;
        int cover = 1, nn = 1;
        if (t <= 8) {
          cover = 2;
          if (pos + 1 > NP - 1) bad = true;
          info[pos] = rel(t / 3 - 1);
          if (pos + 1 <= NP - 1) info[pos + 1] = rel(t % 3 - 1);
        } else if (t <= 13) {
          info[pos] = rel(t - 11);
        } else {
          nn = 2;
          if (k + 1 >= avail) {
            bad = true;
          } else {
            info[pos] = (2 << 16) | ((t - 14) * 16 + nib(k + 1));
          }
        }
        if (pos + cover > NP - 1 && pos <= NP - 1) sh.tend = k + nn;  // the token that covers the last position
        pos += cover;
      }
    }
    __syncthreads();
    tend = sh.tend;
    if (tend < 0) ubad = true;  // the tokens end before the last position
  }

  // ---- exponents: running sums of the differences, restarted by absolute tokens
  int32_t pwv[WIDE_GPT];
#pragma unroll
  for (int q = 0; q < WIDE_GPT; q++) pwv[q] = 0;
  if (!verb && !ubad) {
    int32_t rs[1] = {0};
    for (int q = 0; q < CP; q++) {
      const int i = pp0 + q;
      if (i >= NP || i == 0) continue;
      const int32_t v = info[i];
      if ((v >> 16) == 1) rs[0] += (int16_t)(v & 0xFFFF);
    }
    int32_t rtot[1];
    wg_excl_sum<1>(rs, rtot, sh);
    // key of the last absolute exponent: (position << 16) | (value - running sum + 32768)
    int32_t key[1] = {-1};
    {
      int32_t s = rs[0];
      for (int q = 0; q < CP; q++) {
        const int i = pp0 + q;
        if (i >= NP) break;
        if (i == 0) {
          key[0] = e0 + 32768;
          continue;
        }
        const int32_t v = info[i];
        if ((v >> 16) == 2) key[0] = (i << 16) | ((v & 0xFFFF) - s + 32768);
        else s += (int16_t)(v & 0xFFFF);
      }
    }
    wg_excl_max<1>(key, sh);
    int32_t s = rs[0], kk = key[0];
#pragma unroll
    for (int q = 0; q < WIDE_GPT; q++) {
      const int i = pp0 + q;
      if (q >= CP || i >= NP) break;
      int eps;
      if (i == 0) {
        eps = e0;
        kk = e0 + 32768;
      } else {
        const int32_t v = info[i];
        if ((v >> 16) == 2) {
          kk = (i << 16) | ((v & 0xFFFF) - s + 32768);
        } else {
          s += (int16_t)(v & 0xFFFF);
        }
        eps = (kk & 0xFFFF) - 32768 + s;
      }
      if (eps < 0 || eps > MAXEPS) bad = true;
      const int e = eps < 0 ? 0 : (eps > MAXEPS ? MAXEPS : eps);
      pwv[q] = (W == 32 && e == 31) ? 32 : e;
    }
  }
  // ---- payload offsets and extraction (4 gq fields of a position's width)
  int32_t po[1] = {0};
#pragma unroll
  for (int q = 0; q < WIDE_GPT; q++) po[0] += 4 * gq * pwv[q];
  int32_t ptot[1];
  wg_excl_sum<1>(po, ptot, sh);
  const int pay0 = H + 4 * tend;
  const int total = verb ? (H + g.B * W) : (pay0 + ptot[0]);
  ubad |= total > 32 * len;
  uint32_t r[WIDE_GPT][4];
  {
    int o = pay0 + po[0];
#pragma unroll
    for (int lq = 0; lq < WIDE_GPT; lq++) {
      const int gi = q0 + lq;
      int pq = 0;  // width of the group's position
#pragma unroll
      for (int q = 0; q < WIDE_GPT; q++) pq = q == lq / gq ? pwv[q] : pq;
#pragma unroll
      for (int k = 0; k < 4; k++) {
        const int width = verb ? W : pq;
        const int bit = verb ? H + (4 * gi + k) * W : o + k * pq;
        int wd = bit >> 5;
        wd = wd < 0 ? 0 : (wd > stride - 2 ? stride - 2 : wd);
        const uint64_t both = ((uint64_t)buf[wd + 1] << 32) | buf[wd];
        const uint32_t raw = (uint32_t)(both >> (bit & 31));
        r[lq][k] = (ubad || lq >= nq || gi >= G || width == 0)
                       ? 0u
                       : (width >= 32 ? raw : (uint32_t)(((int32_t)(raw << (32 - width))) >> (32 - width)));
      }
      o += 4 * pq;
    }
  }
  // padding after the last used bit must be zero
  if (!ubad) {
    const int wfirst = (total + 31) >> 5;
    const int wlast = len < stride ? len : stride;
    for (int wd = wfirst + tid; wd < wlast; wd += nt)
      if (buf[wd]) bad = true;
    if (tid == 0 && (total & 31) && (buf[total >> 5] >> (total & 31))) bad = true;
  }
  __syncthreads();  // the words are read: the buffer takes the values
  uint32_t* v = lds;
#pragma unroll
  for (int lq = 0; lq < WIDE_GPT; lq++) {
    const int gi = q0 + lq;
    if (lq < nq && gi < G)
      *reinterpret_cast<uint4*>(v + 4 * gi) = make_uint4(r[lq][0], r[lq][1], r[lq][2], r[lq][3]);
  }
  __syncthreads();

  // ---- undo the stream: running sums along x, y, z (log-step, mod 2^32)
  auto run_sum = [&](int axis) {
    const int L = g.b[axis];
    const int sstride = axis == 2 ? 1 : (axis == 1 ? g.b[2] : g.b[2] * g.b[1]);
    for (int s = 1; s < L; s <<= 1) {
      uint32_t nv[WIDE_GPT][4];
#pragma unroll
      for (int q = 0; q < WIDE_GPT; q++) {
        const int gi = p0 + q;
        if (q >= C || gi >= G) continue;
        int z, y, xq;
        wg.coords(g, gi, z, y, xq);
#pragma unroll
        for (int k = 0; k < 4; k++) {
          const int p = 4 * gi + k;
          const int coord = axis == 2 ? 4 * xq + k : (axis == 1 ? y : z);
          nv[q][k] = v[p] + (coord >= s ? v[p - s * sstride] : 0u);
        }
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < WIDE_GPT; q++) {
        const int gi = p0 + q;
        if (q >= C || gi >= G) continue;
        *reinterpret_cast<uint4*>(v + 4 * gi) = make_uint4(nv[q][0], nv[q][1], nv[q][2], nv[q][3]);
      }
      __syncthreads();
    }
  };
  // the filter stream's inverse a[p] = v[p] + s a[p - k]: log-step sums over
  // multiples of k (the first step carries the sign)
  auto run_filter = [&]() {
    bool first = true;
    for (int D = g.fk; D < g.B; D <<= 1) {
      uint32_t nv[WIDE_GPT][4];
#pragma unroll
      for (int q = 0; q < WIDE_GPT; q++) {
        const int gi = p0 + q;
        if (q >= C || gi >= G) continue;
#pragma unroll
        for (int k = 0; k < 4; k++) {
          const int p = 4 * gi + k;
          const uint32_t prev = p >= D ? v[p - D] : 0u;
          nv[q][k] = (first && g.fneg) ? v[p] - prev : v[p] + prev;
        }
      }
      __syncthreads();
#pragma unroll
      for (int q = 0; q < WIDE_GPT; q++) {
        const int gi = p0 + q;
        if (q >= C || gi >= G) continue;
        *reinterpret_cast<uint4*>(v + 4 * gi) = make_uint4(nv[q][0], nv[q][1], nv[q][2], nv[q][3]);
      }
      __syncthreads();
      first = false;
    }
  };
  if (!ubad) {
    if (NDIM == 1 && st == 3) run_filter();
    if (st == 1 || st == 2 || st == 5 || st == 6) run_sum(2);
    if (st == 2) run_sum(2);
    if (NDIM >= 2 && (st == 3 || st == 5 || st == 6)) run_sum(1);
    if (NDIM == 3 && (st == 4 || st == 6)) run_sum(0);
  }
  if (__syncthreads_or(bad || ubad) && tid == 0) atomicOr(A.status, ST_CORRUPT);

  // ---- dequantize and store
  double dot = 0.0;
  const double R = inv_mantissa(c);
  const int ek = -(c >> 4);
#pragma unroll
  for (int q = 0; q < WIDE_GPT; q++) {
    const int gi = p0 + q;
    if (q >= C || gi >= G) continue;
    int z, y, xq;
    wg.coords(g, gi, z, y, xq);
    int64_t idx;
    const int nv = wg.nvalid(g, z, y, xq, idx);
    const uint4 u = *reinterpret_cast<const uint4*>(v + 4 * gi);
    const uint32_t uu[4] = {u.x, u.y, u.z, u.w};
    T out[4];
#pragma unroll
    for (int k = 0; k < 4; k++) {
      const int32_t av = wrapw<W>(uu[k]);
      if (mode == M_LOSSLESS) out[k] = (T)av;
      else out[k] = to_out<T>(dequant_rk(av, R, ek));
    }
    if constexpr (DOT) {
      for (int k = 0; k < 4; k++)
        if (k < nv) dot += (double)out[k] * (double)w[idx + k];
    } else {
      store4<T>((T*)A.y, idx, nv, out);
    }
  }
  if constexpr (DOT) {
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) dot += __shfl_down(dot, o, 64);
    if ((tid & 63) == 0) s_dot[tid >> 6] = dot;
    __syncthreads();
    if (tid == 0) {
      double t = s_dot[0];
      for (int i = 1; i < wg_nwaves(); i++) t += s_dot[i];
      partial[j] = t;
    }
  }
}

// ------------------------------------------------------------ launchers
template <typename K>
static hipError_t wide_lds_attr(K kernel, size_t lds) {
  if (lds <= 65536) return hipSuccess;
  return hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

template <typename T, int NDIM, int KIND>
static hipError_t wide_enc_t(const EncArgs& A, void* best, hipStream_t s) {
  const size_t lds = wide_lds_bytes(A.g);
  hipError_t e = wide_lds_attr(k_wide_enc<T, NDIM, KIND>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_wide_enc<T, NDIM, KIND>), dim3((unsigned)A.g.nblocks), dim3(wide_threads(A.g.G)), lds, s,
                     A, best);
  return hipGetLastError();
}

template <typename T, int NDIM>
static hipError_t wide_encode_nd(const EncArgs& A, hipStream_t s) {
  if (A.g.mode == M_RATE) return wide_enc_t<T, NDIM, WK_RATE>(A, nullptr, s);
  const int64_t nsuper = (A.g.nblocks + 63) / 64;
  launch_encode_reset(A.ssum, nsuper, s);
  hipError_t e = wide_enc_t<T, NDIM, WK_SIZE>(A, nullptr, s);
  if (e != hipSuccess) return e;
  launch_encode_scan(A, nsuper, s);
  return wide_enc_t<T, NDIM, WK_EMIT>(A, nullptr, s);
}

template <typename T>
static hipError_t wide_encode_t(const EncArgs& A, int ndim, hipStream_t s) {
  if (ndim == 1) return wide_encode_nd<T, 1>(A, s);
  if (ndim == 2) return wide_encode_nd<T, 2>(A, s);
  return wide_encode_nd<T, 3>(A, s);
}

hipError_t launch_wide_encode(int dtype, int ndim, EncArgs& A, hipStream_t s) {
  A.ntiles = A.g.nblocks;
  if (A.g.nblocks == 0) return hipSuccess;
  switch (dtype) {
    case DT_I8: return wide_encode_t<int8_t>(A, ndim, s);
    case DT_I16: return wide_encode_t<int16_t>(A, ndim, s);
    case DT_I32: return wide_encode_t<int32_t>(A, ndim, s);
    case DT_F32: return wide_encode_t<float>(A, ndim, s);
    default: return wide_encode_t<double>(A, ndim, s);
  }
}

template <typename T>
static hipError_t wide_choice_t(const EncArgs& A, int ndim, int32_t* best, hipStream_t s) {
  if (ndim == 1) return wide_enc_t<T, 1, WK_CHOICE>(A, best, s);
  if (ndim == 2) return wide_enc_t<T, 2, WK_CHOICE>(A, best, s);
  return wide_enc_t<T, 3, WK_CHOICE>(A, best, s);
}

template <typename T>
static hipError_t wide_table_t(const EncArgs& A, int ndim, uint8_t* tab, hipStream_t s) {
  if (ndim == 1) return wide_enc_t<T, 1, WK_TABLE>(A, tab, s);
  if (ndim == 2) return wide_enc_t<T, 2, WK_TABLE>(A, tab, s);
  return wide_enc_t<T, 3, WK_TABLE>(A, tab, s);
}

hipError_t launch_wide_table(int dtype, int ndim, const EncArgs& A, uint8_t* tab, hipStream_t s) {
  if (A.g.nblocks == 0) return hipSuccess;
  switch (dtype) {
    case DT_I8: return wide_table_t<int8_t>(A, ndim, tab, s);
    case DT_I16: return wide_table_t<int16_t>(A, ndim, tab, s);
    case DT_I32: return wide_table_t<int32_t>(A, ndim, tab, s);
    case DT_F32: return wide_table_t<float>(A, ndim, tab, s);
    default: return wide_table_t<double>(A, ndim, tab, s);
  }
}

hipError_t launch_wide_choice(int dtype, int ndim, const EncArgs& A, int32_t* best, hipStream_t s) {
  if (A.g.nblocks == 0) return hipSuccess;
  switch (dtype) {  // lossless: integer dtypes only
    case DT_I8: return wide_choice_t<int8_t>(A, ndim, best, s);
    case DT_I16: return wide_choice_t<int16_t>(A, ndim, best, s);
    default: return wide_choice_t<int32_t>(A, ndim, best, s);
  }
}

template <typename T, int NDIM, bool DOT>
static hipError_t wide_dec_t(const DecArgs& A, const void* w, double* partial, hipStream_t s) {
  const size_t lds = wide_lds_bytes(A.g);
  hipError_t e = wide_lds_attr(k_wide_dec<T, NDIM, DOT>, lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_wide_dec<T, NDIM, DOT>), dim3((unsigned)A.g.nblocks), dim3(wide_threads(A.g.G)), lds, s,
                     A, (const T*)w, partial);
  return hipGetLastError();
}

template <typename T, bool DOT>
static hipError_t wide_decode_t(const DecArgs& A, int ndim, const void* w, double* partial, hipStream_t s) {
  if (ndim == 1) return wide_dec_t<T, 1, DOT>(A, w, partial, s);
  if (ndim == 2) return wide_dec_t<T, 2, DOT>(A, w, partial, s);
  return wide_dec_t<T, 3, DOT>(A, w, partial, s);
}

template <bool DOT>
static hipError_t wide_decode_dt(int dtype, int ndim, const DecArgs& A, const void* w, double* partial,
                                 hipStream_t s) {
  switch (dtype) {
    case DT_I8: return wide_decode_t<int8_t, DOT>(A, ndim, w, partial, s);
    case DT_I16: return wide_decode_t<int16_t, DOT>(A, ndim, w, partial, s);
    case DT_I32: return wide_decode_t<int32_t, DOT>(A, ndim, w, partial, s);
    case DT_F32: return wide_decode_t<float, DOT>(A, ndim, w, partial, s);
    default: return wide_decode_t<double, DOT>(A, ndim, w, partial, s);
  }
}

hipError_t launch_wide_decode(int dtype, int ndim, DecArgs& A, hipStream_t s) {
  A.ntiles = A.g.nblocks;
  if (A.g.nblocks == 0) return hipSuccess;
  return wide_decode_dt<false>(dtype, ndim, A, nullptr, nullptr, s);
}

hipError_t launch_wide_decode_dot(int dtype, int ndim, DecArgs& A, const void* w, double* partial, double* out,
                                  hipStream_t s) {
  A.ntiles = A.g.nblocks;
  if (A.g.nblocks == 0) return hipSuccess;
  hipError_t e = wide_decode_dt<true>(dtype, ndim, A, w, partial, s);
  if (e != hipSuccess) return e;
  launch_dot_reduce(partial, A.g.nblocks, out, s);
  return hipGetLastError();
}

}  // namespace apax
