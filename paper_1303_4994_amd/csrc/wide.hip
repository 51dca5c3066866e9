// wide.hip -- encode and decode kernels for blocks of more than 256 samples
// (G > 64 groups, up to the 16384 samples Sec. 6 allows): one workgroup per
// block, the block staged in LDS (wide.h).
#include "decode_tile.h"
#include "wide_enc.h"

namespace apax {

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
