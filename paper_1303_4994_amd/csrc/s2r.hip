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

namespace apax {

constexpr int S2R_BINS = 8192;
__host__ __device__ constexpr int s2r_width(int level) { return level < 4 ? 13 : 12; }
__host__ __device__ constexpr int s2r_shift(int level) { return level < 4 ? 51 - 13 * level : 0; }

template <typename T, int LPB, int NDIM>
__global__ __launch_bounds__(256) void k_s2r(S2RArgs A) {
  constexpr int BPW = 64 / LPB;
  using B_ = Blk<T, LPB, NDIM>;
  const Geo& g = A.g;
  __shared__ uint32_t s_hist[S2R_BINS];
  for (int i = threadIdx.x; i < S2R_BINS; i += blockDim.x) s_hist[i] = 0;
  const PState* st = A.st;
  const int level = st->s2r_level;
  const uint64_t prefix = st->s2r_prefix;
  const int shift = s2r_shift(level), width = s2r_width(level);
  const int code = st->code;
  if (level >= 3) {
    const uint64_t nc = *A.ncand;
    if (nc <= A.cand_cap) {
      // the kept keys hold every key the remaining digits can match;
      // workgroups past the last one return before any barrier
      if ((uint64_t)blockIdx.x * blockDim.x >= nc) return;
      __syncthreads();
      const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
      for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nc; i += stride) {
        const uint64_t key = A.cand[i];
        if ((key >> (shift + width)) == prefix) atomicAdd(&s_hist[(uint32_t)(key >> shift) & ((1u << width) - 1u)], 1u);
      }
      __syncthreads();
      for (int i = threadIdx.x; i < S2R_BINS; i += blockDim.x)
        if (s_hist[i]) atomicAdd(&A.hist[i], s_hist[i]);
      return;
    }
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6;
  const int lane = lane_id();
  for (int64_t tile = blockIdx.x; tile < A.ntiles; tile += gridDim.x) {
    const int64_t jj = (tile * WPG + wave) * BPW + lane / LPB;
    B_ b;
    b.init(g, jj < g.nblocks ? jj : g.nblocks, nullptr);
    b.load((const T*)A.x, g);
    int c = 0;
    if (A.rule == R_QUALITY) c = clampc(code, b.cf, b.cc);
    else if (A.rule == R_RATE) c = b.blk_ok ? A.cj[b.j] : 0;
    int32_t a[4];
    b.quantize(c, A.rule == R_LOSSLESS, a);
    const double Rq = inv_mantissa(c);
    const int eq = -(c >> 4);
#pragma unroll
    for (int k = 0; k < 4; k++) {
      bool match = false;
      uint32_t digit = 0;
      uint64_t key = 0;
      if (b.act && b.valid(k)) {
        const double x = b.xv(k);
        const double y = A.rule == R_LOSSLESS ? (double)a[k] : (double)to_out<T>(dequant_rk(a[k], Rq, eq));
        const double d = x - y;
        key = d == 0.0 ? 0x7FF0000000000000ull
                       : __builtin_bit_cast(uint64_t, __builtin_fabs(x) / __builtin_fabs(d));
        match = level == 0 || (key >> (shift + width)) == prefix;
        digit = (uint32_t)(key >> shift) & ((1u << width) - 1u);
      }
      if (level == 2) {  // keep the matching keys: one counter add per wave
        const uint64_t bal = __ballot(match);
        if (bal) {
          const int lead = __builtin_ctzll(bal);
          unsigned long long base = 0;
          if (lane == lead) base = atomicAdd((unsigned long long*)A.ncand, (unsigned long long)__popcll(bal));
          base = __shfl(base, lead, 64);
          const uint64_t idx = base + (uint64_t)__popcll(bal & ((1ull << lane) - 1ull));
          if (match && idx < A.cand_cap) A.cand[idx] = key;
        }
      }
      // one LDS add per matching lane: the digits of neighbouring ratios
      // differ (the residual is noise-like), so grouping lanes by digit
      // costs more rounds than the adds it saves
      if (match) atomicAdd(&s_hist[digit], 1u);
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
static hipError_t launch_lpb(const S2RArgs& A, hipStream_t s) {
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
  const int64_t per = (int64_t)WPG * (64 / lpb);
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
