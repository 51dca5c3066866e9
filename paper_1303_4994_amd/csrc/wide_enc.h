// wide_enc.h -- the encoder's analysis of one block of more than 256 samples
// (or of groups of 8) by one workgroup, the block staged in LDS: bracket,
// quantizer, candidate streams, BFPE exponents, JEE token counts, stream
// choice, fixed-rate search and emission.  Used by the encode kernels and by
// the profiler's passes over such blocks.
#pragma once
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

}  // namespace apax
