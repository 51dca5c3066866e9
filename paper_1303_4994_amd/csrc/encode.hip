// encode.hip -- single-array APAX encoder kernel for gfx950: fixed rate, one
// workgroup per tile; variable-size modes, one workgroup per run of RUN tiles
// taken from an atomic ticket, so runs start in order (the look-back in
// encode_tile.h relies on it).
#include "encode_tile.h"

namespace apax {

__global__ void k_encode_reset(uint32_t* ticket, uint32_t* status_unused, uint64_t* tile_state,
                               int64_t ntiles) {
  int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) *ticket = 0;
  for (; i < ntiles; i += (int64_t)gridDim.x * blockDim.x) tile_state[i] = 0;
  (void)status_unused;
}

// VAR: variable-size modes (runs of RUN tiles from the ticket, look-back);
// else fixed rate (one tile per workgroup, offsets known up front).
template <typename T, int LPB, int NDIM, int WP, bool VAR>
__global__ __launch_bounds__(WP * 64) void k_encode(EncArgs A) {
  constexpr int BPW = 64 / LPB;
  // the header words as the argument block holds them in memory
  const uint32_t* hsrc =
      (const uint32_t*)((const uint8_t*)__builtin_amdgcn_kernarg_segment_ptr() + offsetof(EncArgs, hdr));
  extern __shared__ __align__(16) uint32_t lds[];
  __shared__ EncShared<WP> sm;
  if constexpr (VAR) {
    if (threadIdx.x == 0) sm.tile = (int64_t)atomicAdd(A.ticket, (uint32_t)RUN);
    __syncthreads();
    const int64_t t0 = sm.tile;
    const int64_t left = A.ntiles - t0;
    encode_run<T, LPB, NDIM, WP>(A, hsrc, t0, left < RUN ? (int)left : RUN, sm, lds);
  } else {
    const int64_t t = blockIdx.x;
    encode_analyze<T, LPB, NDIM, WP>(A, t, 0, A.g.ldsw, sm, lds);
    if ((threadIdx.x >> 6) == 0) {
      uint64_t base = 0;
      encode_place<WP, BPW, M_RATE>(A, hsrc, t, 0, sm, false, base);
    }
    __syncthreads();
    encode_store<LPB, WP>(A, t, 0, A.g.ldsw, sm, lds);
  }
}

// Lagged choice, first pass: every block's own best stream (lossless).
template <typename T, int LPB, int NDIM>
__global__ __launch_bounds__(WPG * 64) void k_stream_choice(EncArgs A, int32_t* best_st) {
  constexpr int BPW = 64 / LPB;
  using B_ = Blk<T, LPB, NDIM>;
  __shared__ uint4 s_xch[NDIM >= 2 ? WPG * XCH : 1];
  const Geo& g = A.g;
  const int wave = threadIdx.x >> 6;
  const int lane = lane_id();
  B_ b;
  b.init(g, ((int64_t)blockIdx.x * WPG + wave) * BPW + lane / LPB, NDIM >= 2 ? s_xch + wave * XCH : nullptr);
  b.template load<false>((const T*)A.x, g);
  int32_t a[4];
  Costs C;
  int32_t best;
  b.quantize(0, true, a);
  b.costs(g, g.mask, a, C);
  const int st = B_::argmin(C, g.mask, best);
  if (b.blk_ok && b.L.gi == 0) best_st[b.j] = st;
}

template <typename T, int LPB, int NDIM>
static hipError_t launch_choice_t(const EncArgs& A, int32_t* best, hipStream_t s) {
  hipLaunchKernelGGL((k_stream_choice<T, LPB, NDIM>), dim3((unsigned)encode_tiles(A.g)), dim3(WPG * 64), 0, s,
                     A, best);
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_choice_nd(const EncArgs& A, int ndim, int32_t* best, hipStream_t s) {
  const int G = A.g.G;
#define APAX_CHOICE_LPB(ND)                                            \
  if (G <= 16) return launch_choice_t<T, 16, ND>(A, best, s);         \
  if (G <= 32) return launch_choice_t<T, 32, ND>(A, best, s);         \
  return launch_choice_t<T, 64, ND>(A, best, s);
  if (ndim == 1) { APAX_CHOICE_LPB(1) }
  if (ndim == 2) { APAX_CHOICE_LPB(2) }
  APAX_CHOICE_LPB(3)
#undef APAX_CHOICE_LPB
}

hipError_t launch_stream_choice(int dtype, int ndim, const EncArgs& A, int32_t* best, hipStream_t s) {
  switch (dtype) {  // lossless: integer dtypes only
    case DT_I8: return launch_choice_nd<int8_t>(A, ndim, best, s);
    case DT_I16: return launch_choice_nd<int16_t>(A, ndim, best, s);
    default: return launch_choice_nd<int32_t>(A, ndim, best, s);
  }
}

// ------------------------------------------------------------ launcher
template <typename T, int LPB, int NDIM>
static hipError_t launch_t(const EncArgs& A, hipStream_t s) {
  constexpr int BPW = 64 / LPB;
  const bool variable = A.g.mode != M_RATE;
  const int run = variable ? RUN : 1;
  size_t lds = (size_t)run * WPG * BPW * A.g.ldsw * 4;
  const int64_t grid = (A.ntiles + run - 1) / run;
  if (variable)
    hipLaunchKernelGGL((k_encode<T, LPB, NDIM, WPG, true>), dim3((unsigned)grid), dim3(WPG * 64), lds, s, A);
  else
    hipLaunchKernelGGL((k_encode<T, LPB, NDIM, WPG, false>), dim3((unsigned)grid), dim3(WPG * 64), lds, s, A);
  return hipGetLastError();
}

template <typename T, int NDIM>
static hipError_t launch_lpb(const EncArgs& A, hipStream_t s) {
  if (A.g.G <= 16) return launch_t<T, 16, NDIM>(A, s);
  if (A.g.G <= 32) return launch_t<T, 32, NDIM>(A, s);
  return launch_t<T, 64, NDIM>(A, s);
}

template <typename T>
static hipError_t launch_nd(const EncArgs& A, int ndim, hipStream_t s) {
  if (ndim == 1) return launch_lpb<T, 1>(A, s);
  if (ndim == 2) return launch_lpb<T, 2>(A, s);
  return launch_lpb<T, 3>(A, s);
}

int lpb_of(const Geo& g) { return g.G <= 16 ? 16 : (g.G <= 32 ? 32 : 64); }


int64_t encode_tiles_wp(const Geo& g, int wp) {
  int64_t per = (int64_t)wp * (64 / lpb_of(g));
  return (g.nblocks + per - 1) / per;
}

int64_t encode_tiles(const Geo& g) { return encode_tiles_wp(g, WPG); }

hipError_t launch_encode(int dtype, int ndim, EncArgs& A, hipStream_t s) {
  A.ntiles = encode_tiles(A.g);
  if (A.ntiles == 0) return hipSuccess;
  if (A.g.mode != M_RATE) {
    int64_t nb = (A.ntiles + 255) / 256;
    unsigned grid = (unsigned)(nb > 1024 ? 1024 : (nb < 1 ? 1 : nb));
    hipLaunchKernelGGL(k_encode_reset, dim3(grid), dim3(256), 0, s, A.ticket, A.status,
                       A.tile_state, A.ntiles);
  }
  switch (dtype) {
    case DT_I8: return launch_nd<int8_t>(A, ndim, s);
    case DT_I16: return launch_nd<int16_t>(A, ndim, s);
    case DT_I32: return launch_nd<int32_t>(A, ndim, s);
    case DT_F32: return launch_nd<float>(A, ndim, s);
    default: return launch_nd<double>(A, ndim, s);
  }
}

}  // namespace apax
