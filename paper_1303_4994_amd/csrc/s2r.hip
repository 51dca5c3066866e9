// s2r.hip -- the 2-sigma signal-to-residual margin (Sec. 4, Window 4): the
// nearest-rank 4.5th percentile of the per-sample ratio |x| / |x - y| over
// the whole array, y the decoded array at the profile's operating point.
//
// Exact selection without sorting: the ratio's binary64 bit pattern is a
// monotone 64-bit key (non-negative; d = 0 gives the key of +inf).  Five
// passes select its digits from the top (13, 13, 13, 13, 12 bits); each pass
// recomputes the keys from x (quantize at the block's code, dequantize),
// histograms the next digit of the keys that match the digits chosen so far
// (per-workgroup LDS histogram, then one global add per non-empty bin), and a
// one-workgroup control kernel picks the bin holding the wanted rank.  The
// third pass also keeps the keys that match its 26-bit prefix (few, as a
// rule): when they all fit, the last two passes select from them alone.
#include "block.h"
#include "kernels.h"
#include "wide_enc.h"

namespace apax {

constexpr int S2R_BINS = 8192;
__host__ __device__ constexpr int s2r_width(int level) { return level < 4 ? 13 : 12; }
__host__ __device__ constexpr int s2r_shift(int level) { return level < 4 ? 51 - 13 * level : 0; }

// The digit selection of one pass, shared by the one-wave and the
// one-workgroup-per-block kernels.
struct S2RPass {
  int level, shift, width, code;
  uint64_t prefix;
  __device__ __forceinline__ void init(const PState* st) {
    level = st->s2r_level;
    prefix = st->s2r_prefix;
    shift = s2r_shift(level);
    width = s2r_width(level);
    code = st->code;
  }
};

// Passes after the one that kept its matching keys, when they all fit: the
// digits of the kept keys alone.  Returns false when the pass has to read the
// array instead.  Every thread of the workgroup takes the same path.
__device__ __forceinline__ bool s2r_from_kept(const S2RArgs& A, const S2RPass& P, uint32_t* s_hist) {
  if (P.level < 3) return false;
  const uint64_t nc = *A.ncand;
  if (nc > A.cand_cap) return false;
  // workgroups past the last one return before any barrier
  if ((uint64_t)blockIdx.x * blockDim.x >= nc) return true;
  __syncthreads();
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nc; i += stride) {
    const uint64_t key = A.cand[i];
    if ((key >> (P.shift + P.width)) == P.prefix)
      atomicAdd(&s_hist[(uint32_t)(key >> P.shift) & ((1u << P.width) - 1u)], 1u);
  }
  __syncthreads();
  for (int i = threadIdx.x; i < S2R_BINS; i += blockDim.x)
    if (s_hist[i]) atomicAdd(&A.hist[i], s_hist[i]);
  return true;
}

// One sample (x, its decoded value y; `valid` false: no sample): its key,
// the LDS histogram add of its digit if it matches, and at level 2 the kept
// key (one counter add per wave: every lane of the wave calls this together).
__device__ __forceinline__ void s2r_take(const S2RArgs& A, const S2RPass& P, uint32_t* s_hist, bool valid,
                                         double x, double y) {
  bool match = false;
  uint32_t digit = 0;
  uint64_t key = 0;
  if (valid) {
    const double d = x - y;
    key = d == 0.0 ? 0x7FF0000000000000ull : __builtin_bit_cast(uint64_t, __builtin_fabs(x) / __builtin_fabs(d));
    match = P.level == 0 || (key >> (P.shift + P.width)) == P.prefix;
    digit = (uint32_t)(key >> P.shift) & ((1u << P.width) - 1u);
  }
  if (P.level == 2) {  // keep the matching keys
    const uint64_t bal = __ballot(match);
    if (bal) {
      const int lane = lane_id();
      const int lead = __builtin_ctzll(bal);
      unsigned long long base = 0;
      if (lane == lead) base = atomicAdd((unsigned long long*)A.ncand, (unsigned long long)__popcll(bal));
      base = __shfl(base, lead, 64);
      const uint64_t idx = base + (uint64_t)__popcll(bal & ((1ull << lane) - 1ull));
      if (match && idx < A.cand_cap) A.cand[idx] = key;
    }
  }
  // one LDS add per matching lane: the digits of neighbouring ratios differ
  // (the residual is noise-like), so grouping lanes by digit costs more
  // rounds than the adds it saves
  if (match) atomicAdd(&s_hist[digit], 1u);
}

template <typename T, int LPB, int NDIM>
__global__ __launch_bounds__(256) void k_s2r(S2RArgs A) {
  constexpr int BPW = 64 / LPB;
  using B_ = Blk<T, LPB, NDIM>;
  const Geo& g = A.g;
  __shared__ uint32_t s_hist[S2R_BINS];
  for (int i = threadIdx.x; i < S2R_BINS; i += blockDim.x) s_hist[i] = 0;
  S2RPass P;
  P.init(A.st);
  if (s2r_from_kept(A, P, s_hist)) return;
  __syncthreads();
  const int wave = threadIdx.x >> 6;
  const int lane = lane_id();
  for (int64_t tile = blockIdx.x; tile < A.ntiles; tile += gridDim.x) {
    const int64_t jj = (tile * WPG + wave) * BPW + lane / LPB;
    B_ b;
    b.init(g, jj < g.nblocks ? jj : g.nblocks, nullptr);
    b.load((const T*)A.x, g);
    int c = 0;
    if (A.rule == R_QUALITY) c = clampc(P.code, b.cf, b.cc);
    else if (A.rule == R_RATE) c = b.blk_ok ? A.cj[b.j] : 0;
    int32_t a[4];
    b.quantize(c, A.rule == R_LOSSLESS, a);
    const double Rq = inv_mantissa(c);
    const int eq = -(c >> 4);
#pragma unroll
    for (int k = 0; k < 4; k++) {
      const bool valid = b.act && b.valid(k);
      const double x = valid ? b.xv(k) : 0.0;
      const double y = A.rule == R_LOSSLESS ? (double)a[k] : (double)to_out<T>(dequant_rk(a[k], Rq, eq));
      s2r_take(A, P, s_hist, valid, x, y);
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < S2R_BINS; i += blockDim.x)
    if (s_hist[i]) atomicAdd(&A.hist[i], s_hist[i]);
}

// Blocks of more than 64 groups, or groups of 8: one workgroup per block
// (the encoder's wide-block bracket and quantizer), blocks blockIdx.x,
// blockIdx.x + gridDim.x, ...
template <typename T, int NDIM>
__global__ __launch_bounds__(WIDE_MAXT) void k_ws2r(S2RArgs A) {
  extern __shared__ __align__(16) uint32_t lds[];
  __shared__ WideShared sh;
  __shared__ uint32_t s_hist[S2R_BINS];
  const Geo& g = A.g;
  for (int i = threadIdx.x; i < S2R_BINS; i += blockDim.x) s_hist[i] = 0;
  S2RPass P;
  P.init(A.st);
  if (s2r_from_kept(A, P, s_hist)) return;
  __syncthreads();
  WEnc<T, NDIM> b;
  for (int64_t j = blockIdx.x; j < g.nblocks; j += gridDim.x) {
    b.init(g, j, lds, sh);
    if (A.rule == R_QUALITY) b.template load<true>((const T*)A.x);
    else b.template load<false>((const T*)A.x);
    int c = 0;
    if (A.rule == R_QUALITY) c = clampc(P.code, b.cf, b.cc);
    else if (A.rule == R_RATE) c = A.cj[j];
    b.quantize(c, A.rule == R_LOSSLESS);
    const double Rq = inv_mantissa(c);
    const int eq = -(c >> 4);
#pragma unroll
    for (int m = 0; m < WIDE_GPT; m++) {
      const int gi = threadIdx.x + m * b.wg.nt;
      int nv = 0;
      uint4 q4 = make_uint4(0u, 0u, 0u, 0u);
      if (gi < g.G) {
        int z, y_, xq;
        b.wg.coords(g, gi, z, y_, xq);
        int64_t idx;
        nv = b.wg.nvalid(g, z, y_, xq, idx);
        q4 = *reinterpret_cast<const uint4*>(b.qa + 4 * gi);
      }
      const int32_t qv[4] = {(int32_t)q4.x, (int32_t)q4.y, (int32_t)q4.z, (int32_t)q4.w};
#pragma unroll
      for (int k = 0; k < 4; k++) {
        const bool valid = k < nv;
        const double x = valid ? (double)b.xs[m][k] : 0.0;
        const double y = A.rule == R_LOSSLESS ? (double)qv[k] : (double)to_out<T>(dequant_rk(qv[k], Rq, eq));
        s2r_take(A, P, s_hist, valid, x, y);
      }
    }
  }
  __syncthreads();
  for (int i = threadIdx.x; i < S2R_BINS; i += blockDim.x)
    if (s_hist[i]) atomicAdd(&A.hist[i], s_hist[i]);
}

// One workgroup: the bin of this level's digit that holds the wanted rank;
// appends it to the prefix, keeps the rank within the bin, clears the bins.
__global__ __launch_bounds__(256) void k_s2r_ctl(PState* st, uint32_t* hist) {
  constexpr int PER = S2R_BINS / 256;
  __shared__ uint64_t s_sum[256];
  __shared__ int s_bin;
  __shared__ uint64_t s_before;
  const int t = threadIdx.x;
  uint64_t sum = 0;
  for (int i = 0; i < PER; i++) sum += hist[t * PER + i];
  s_sum[t] = sum;
  if (t == 0) s_bin = -1;
  __syncthreads();
  if (t == 0) {
    const uint64_t rank = st->s2r_rank;  // 1-based, >= 1
    uint64_t cum = 0;
    int th = 0;
    while (th < 256 && cum + s_sum[th] < rank) cum += s_sum[th++];
    if (th < 256) {
      int b = th * PER;
      while (cum + hist[b] < rank) cum += hist[b++];
      s_bin = b;
      s_before = cum;
    }
  }
  __syncthreads();
  if (t == 0) {
    const int level = st->s2r_level;
    if (s_bin < 0) {
      st->status |= ST_INTERNAL;  // fewer keys than the rank: cannot happen
    } else {
      st->s2r_prefix = (st->s2r_prefix << s2r_width(level)) | (uint64_t)s_bin;
      st->s2r_rank -= s_before;
    }
    st->s2r_level = level + 1;
  }
  for (int i = 0; i < PER; i++) hist[t * PER + i] = 0;
}

__global__ void k_s2r_init(PState* st, uint32_t* hist, uint64_t* ncand, uint64_t rank) {
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    st->s2r_level = 0;
    st->s2r_prefix = 0;
    st->s2r_rank = rank;
    *ncand = 0;
  }
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < S2R_BINS; i += gridDim.x * blockDim.x) hist[i] = 0;
}

template <typename T, int LPB, int NDIM>
static hipError_t launch_t(const S2RArgs& A, hipStream_t s) {
  hipLaunchKernelGGL((k_s2r<T, LPB, NDIM>), dim3((unsigned)A.nwg), dim3(WPG * 64), 0, s, A);
  return hipGetLastError();
}

template <typename T, int NDIM>
static hipError_t launch_wide_t(const S2RArgs& A, hipStream_t s) {
  const size_t lds = wide_lds_bytes(A.g);
  if (lds > 65536) {
    const hipError_t e = hipFuncSetAttribute((const void*)k_ws2r<T, NDIM>,
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL((k_ws2r<T, NDIM>), dim3((unsigned)A.nwg), dim3(wide_threads(A.g.G)), lds, s, A);
  return hipGetLastError();
}

template <typename T, int NDIM>
static hipError_t launch_lpb(const S2RArgs& A, hipStream_t s) {
  if (A.g.G > 64 || A.g.gq == 2) return launch_wide_t<T, NDIM>(A, s);
  if (A.g.G <= 16) return launch_t<T, 16, NDIM>(A, s);
  if (A.g.G <= 32) return launch_t<T, 32, NDIM>(A, s);
  return launch_t<T, 64, NDIM>(A, s);
}

template <typename T>
static hipError_t launch_nd(const S2RArgs& A, int ndim, hipStream_t s) {
  if (ndim == 1) return launch_lpb<T, 1>(A, s);
  if (ndim == 2) return launch_lpb<T, 2>(A, s);
  return launch_lpb<T, 3>(A, s);
}

hipError_t launch_s2r(int dtype, int ndim, S2RArgs& A, uint64_t rank, hipStream_t s) {
  const int lpb = A.g.G <= 16 ? 16 : (A.g.G <= 32 ? 32 : 64);
  const int64_t per = A.g.G > 64 || A.g.gq == 2 ? 1 : (int64_t)WPG * (64 / lpb);  // blocks per tile
  A.ntiles = (A.g.nblocks + per - 1) / per;
  A.nwg = A.ntiles < 2048 ? A.ntiles : 2048;
  hipLaunchKernelGGL(k_s2r_init, dim3(8), dim3(256), 0, s, A.st, A.hist, A.ncand, rank);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess || A.ntiles == 0) return e;
  for (int level = 0; level < 5; level++) {
    switch (dtype) {
      case DT_I8: e = launch_nd<int8_t>(A, ndim, s); break;
      case DT_I16: e = launch_nd<int16_t>(A, ndim, s); break;
      case DT_I32: e = launch_nd<int32_t>(A, ndim, s); break;
      case DT_F32: e = launch_nd<float>(A, ndim, s); break;
      default: e = launch_nd<double>(A, ndim, s); break;
    }
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_s2r_ctl, dim3(1), dim3(256), 0, s, A.st, A.hist);
    if ((e = hipGetLastError()) != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace apax
