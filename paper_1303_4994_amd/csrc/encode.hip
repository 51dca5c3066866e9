// encode.hip -- single-array APAX encoder kernel for gfx950: fixed rate, one
// workgroup per tile; variable-size modes, one workgroup per run of RUN tiles
// taken from an atomic ticket, so runs start in order (the look-back in
// encode_tile.h relies on it).
#include "encode_tile.h"

namespace apax {

// adaptive rate: the block's own requested code (wave-uniform with one block
// per wave)
template <int LPB>
__device__ __forceinline__ void block_code(const EncArgs& A, bool ok, int64_t j, int32_t& code0) {
  code0 = ok ? A.bcode[j] : 0;
  if constexpr (LPB == 64) code0 = __builtin_amdgcn_readfirstlane(code0);
}

// zero the superblock word counts of a variable-size encode
__global__ void k_encode_reset(uint32_t* ssum, int64_t nsuper) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nsuper; i += (int64_t)gridDim.x * blockDim.x)
    ssum[i] = 0;
}

// Variable-size modes, first pass (one tile per workgroup): each block's
// analysis -- operating point, quantization, every allowed stream costed --
// gives its chosen stream and word count; the counts go to the stream's
// block-length index and are summed per superblock of 64 blocks.
template <typename T, int LPB, int NDIM, int WP>
__global__ __launch_bounds__(WP * 64) void k_encode_size(EncArgs A) {
  constexpr int BPW = 64 / LPB;
  using B_ = Blk<T, LPB, NDIM>;
  __shared__ uint4 s_xch[NDIM >= 2 ? WP * XCH : 1];
  const Geo& g = A.g;
  const int mode = __builtin_amdgcn_readfirstlane(g.mode);
  int32_t code0;
  uint32_t mask0;
  profiled_point(A, g, code0, mask0);
  const int wave = threadIdx.x >> 6;
  B_ b;
  b.init(g, ((int64_t)blockIdx.x * WP + wave) * BPW + lane_id() / LPB,
         NDIM >= 2 ? s_xch + wave * XCH : nullptr);
  if (A.bcode) block_code<LPB>(A, b.blk_ok, b.j, code0);
  int c, st;
  int32_t best, a[4];
  analyze_block<T, LPB, NDIM>(A, b, mode, code0, mask0, c, st, best, a);
  uint32_t nw = 0;
  if (b.blk_ok && b.L.gi == 0) {
    nw = (uint32_t)((best + 31) >> 5);
    A.lens[b.j] = (uint16_t)nw;
    A.bst[b.j] = (uint8_t)st;
  }
  // the workgroup's blocks are consecutive and inside one superblock (64 is
  // a multiple of WPG * BPW): one add per workgroup, not one per block (the
  // adds of a superblock's blocks to one word serialize at the memory side)
  static_assert(64 % (WP * BPW) == 0, "a workgroup's blocks lie in one superblock");
  __shared__ uint32_t s_nw[WP];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) nw += __shfl_xor(nw, o, 64);
  if (lane_id() == 0) s_nw[wave] = nw;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
#pragma unroll
    for (int w = 0; w < WP; w++) t += s_nw[w];
    const int64_t j0 = (int64_t)blockIdx.x * WP * BPW;
    if (t) atomicAdd(&A.ssum[j0 >> 6], t);
  }
}

// Variable-size modes: superblock word offsets (exclusive running sum of the
// superblock counts, one workgroup, fixed order), the payload size in the
// stream header and the stream's byte count.
__global__ __launch_bounds__(1024) void k_encode_scan(EncArgs A, int64_t nsuper) {
  __shared__ uint64_t s_part[1024];
  const int t = threadIdx.x;
  const int64_t per = (nsuper + 1023) / 1024;
  const int64_t lo = t * per, hi = lo + per < nsuper ? lo + per : nsuper;
  uint64_t sum = 0;
  for (int64_t i = lo; i < hi; i++) sum += A.ssum[i];
  s_part[t] = sum;
  __syncthreads();
  for (int o = 1; o < 1024; o <<= 1) {
    const uint64_t v = t >= o ? s_part[t - o] : 0;
    __syncthreads();
    s_part[t] += v;
    __syncthreads();
  }
  uint64_t acc = s_part[t] - sum;
  for (int64_t i = lo; i < hi; i++) {
    A.sbo[i] = acc;
    acc += A.ssum[i];
  }
  if (t == 1023) {
    const uint64_t total = s_part[1023];
    *reinterpret_cast<uint64_t*>(A.out_base + 56) = total;
    *A.d_nbytes = A.area + 4 * total;
  }
}

// Variable-size modes, second pass (one tile per workgroup): each block is
// quantized again at its operating point, its chosen stream (first pass)
// assembled in LDS and stored at its offset: the superblock's offset plus the
// lengths of the blocks before it in the superblock.  Tile 0 writes the
// stream header.
template <typename T, int LPB, int NDIM>
__global__ __launch_bounds__(WPG * 64) void k_encode_emit(EncArgs A) {
  constexpr int BPW = 64 / LPB;
  using B_ = Blk<T, LPB, NDIM>;
  const uint32_t* hsrc =
      (const uint32_t*)((const uint8_t*)__builtin_amdgcn_kernarg_segment_ptr() + offsetof(EncArgs, hdr));
  extern __shared__ __align__(16) uint32_t lds[];
  __shared__ uint4 s_xch[NDIM >= 2 ? WPG * XCH : 1];
  const Geo& g = A.g;
  const int mode = __builtin_amdgcn_readfirstlane(g.mode);
  int32_t code0;
  uint32_t mask0;
  profiled_point(A, g, code0, mask0);
  const int wave = threadIdx.x >> 6;
  const int lane = lane_id();
  if (blockIdx.x == 0 && wave == 0) write_stream_header(A, hsrc, true);
  B_ b;
  b.init(g, ((int64_t)blockIdx.x * WPG + wave) * BPW + lane / LPB, NDIM >= 2 ? s_xch + wave * XCH : nullptr);
  if (A.bcode) block_code<LPB>(A, b.blk_ok, b.j, code0);
  {
    T xv4[4];
    b.fetch((const T*)A.x, g, xv4);
    if (mode == M_LOSSLESS) b.template take<false>(g, xv4);
    else b.take(g, xv4);
  }
  const int c = mode == M_LOSSLESS ? 0 : clampc(code0, b.cf, b.cc);
  int32_t a[4];
  b.quantize(c, mode == M_LOSSLESS, a);
  const int seg = b.L.seg, gi = b.L.gi;
  const int64_t j = b.j;
  int st = b.blk_ok ? (int)A.bst[j] : 0;
  int nw = b.blk_ok ? (int)A.lens[j] : 0;
  // offset: superblock offset + lengths of the blocks before j in its superblock
  const int64_t jb = (j >> 6) << 6;
  uint32_t acc = 0;
  if (b.blk_ok)
    for (int64_t r = jb + gi; r < j; r += LPB) acc += A.lens[r];
  acc = (uint32_t)seg_sum<LPB>((int32_t)acc);
  uint64_t off = b.blk_ok ? A.sbo[j >> 6] + (uint64_t)acc : 0;
  if constexpr (LPB == 64) {
    st = __builtin_amdgcn_readfirstlane(st);
    nw = __builtin_amdgcn_readfirstlane(nw);
  }
  uint32_t* buf = lds + (wave * BPW + seg) * g.ldsw;
  emit_block<T, LPB, NDIM>(g, b, c, st, mask0, a, buf, nw);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  uint32_t* dst = A.out_words + off;
  const int stride = g.ldsw;
  for (int w = gi; w < nw; w += LPB) dst[w] = w < stride ? buf[w] : 0u;
}

// The stream header of a fixed-rate encode whose blocks the profile's
// metrics pass writes (one wave; the operating point from the profile).
__global__ __launch_bounds__(64) void k_encode_header(EncArgs A) {
  const uint32_t* hsrc =
      (const uint32_t*)((const uint8_t*)__builtin_amdgcn_kernarg_segment_ptr() + offsetof(EncArgs, hdr));
  write_stream_header(A, hsrc, false);
}

hipError_t launch_encode_header(const EncArgs& A, hipStream_t s) {
  hipLaunchKernelGGL(k_encode_header, dim3(1), dim3(64), 0, s, A);
  return hipGetLastError();
}

// Fixed rate: one workgroup per tile, block j at j * budget words.  (VAR is
// kept for the template's shape; variable-size single arrays use the size /
// scan / emit kernels below.)
template <typename T, int LPB, int NDIM, int WP, bool VAR>
__global__ __launch_bounds__(WP * 64) void k_encode(EncArgs A) {
  constexpr int BPW = 64 / LPB;
  // the header words as the argument block holds them in memory
  const uint32_t* hsrc =
      (const uint32_t*)((const uint8_t*)__builtin_amdgcn_kernarg_segment_ptr() + offsetof(EncArgs, hdr));
  extern __shared__ __align__(16) uint32_t lds[];
  __shared__ EncShared<WP> sm;
  static_assert(!VAR, "variable-size single arrays use k_encode_size / k_encode_scan / k_encode_emit");
  {
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
  int32_t best;
  b.quantize(0, true, a);
  const int st = b.best_stream(g, g.mask, a, best);
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
void launch_encode_reset(uint32_t* ssum, int64_t nsuper, hipStream_t s) {
  const int64_t nb = (nsuper + 255) / 256;
  hipLaunchKernelGGL(k_encode_reset, dim3((unsigned)(nb > 1024 ? 1024 : (nb < 1 ? 1 : nb))), dim3(256), 0, s,
                     ssum, nsuper);
}

void launch_encode_scan(const EncArgs& A, int64_t nsuper, hipStream_t s) {
  hipLaunchKernelGGL(k_encode_scan, dim3(1), dim3(1024), 0, s, A, nsuper);
}

template <typename T, int LPB, int NDIM>
static hipError_t launch_t(const EncArgs& A, hipStream_t s) {
  constexpr int BPW = 64 / LPB;
  const size_t lds = (size_t)WPG * BPW * A.g.ldsw * 4;
  const unsigned grid = (unsigned)A.ntiles;
  if (A.g.mode == M_RATE) {
    hipLaunchKernelGGL((k_encode<T, LPB, NDIM, WPG, false>), dim3(grid), dim3(WPG * 64), lds, s, A);
    return hipGetLastError();
  }
  const int64_t nsuper = (A.g.nblocks + 63) / 64;
  launch_encode_reset(A.ssum, nsuper, s);
  // first pass: 1-d blocks (few registers) with up to 16 waves per
  // workgroup, so each superblock word takes at most 4 adds; 2-/3-d blocks
  // keep 4 waves, as 16-wave workgroups would not fill a SIMD's wave slots at
  // their register counts
  constexpr int SWP = NDIM == 1 ? (64 / BPW > 16 ? 16 : 64 / BPW) : WPG;
  const unsigned sgrid = (unsigned)((A.g.nblocks + SWP * BPW - 1) / (SWP * BPW));
  hipLaunchKernelGGL((k_encode_size<T, LPB, NDIM, SWP>), dim3(sgrid), dim3(SWP * 64), 0, s, A);
  launch_encode_scan(A, nsuper, s);
  hipLaunchKernelGGL((k_encode_emit<T, LPB, NDIM>), dim3(grid), dim3(WPG * 64), lds, s, A);
  return hipGetLastError();
}

template <typename T, int LPB, int NDIM>
static hipError_t launch_profiled_t(const EncArgs& A, const int32_t* cj, hipStream_t s) {
  (void)cj;
  constexpr int BPW = 64 / LPB;
  const size_t lds = (size_t)WPG * BPW * A.g.ldsw * 4;
  const unsigned grid = (unsigned)A.ntiles;
  // (fixed rate: the metrics pass writes the blocks, launch_encode_header the header)
  if (A.g.mode == M_RATE) return hipErrorInvalidValue;
  launch_encode_scan(A, (A.g.nblocks + 63) / 64, s);
  hipLaunchKernelGGL((k_encode_emit<T, LPB, NDIM>), dim3(grid), dim3(WPG * 64), lds, s, A);
  return hipGetLastError();
}

template <typename T>
static hipError_t launch_profiled_nd(const EncArgs& A, int ndim, const int32_t* cj, hipStream_t s) {
  const int G = A.g.G;
#define APAX_PROF_LPB(ND)                                      \
  if (G <= 16) return launch_profiled_t<T, 16, ND>(A, cj, s);  \
  if (G <= 32) return launch_profiled_t<T, 32, ND>(A, cj, s);  \
  return launch_profiled_t<T, 64, ND>(A, cj, s);
  if (ndim == 1) { APAX_PROF_LPB(1) }
  if (ndim == 2) { APAX_PROF_LPB(2) }
  APAX_PROF_LPB(3)
#undef APAX_PROF_LPB
}

hipError_t launch_encode_profiled(int dtype, int ndim, EncArgs& A, const int32_t* cj, hipStream_t s) {
  A.ntiles = encode_tiles(A.g);
  if (A.ntiles == 0) return hipSuccess;
  switch (dtype) {
    case DT_I8: return launch_profiled_nd<int8_t>(A, ndim, cj, s);
    case DT_I16: return launch_profiled_nd<int16_t>(A, ndim, cj, s);
    case DT_I32: return launch_profiled_nd<int32_t>(A, ndim, cj, s);
    case DT_F32: return launch_profiled_nd<float>(A, ndim, cj, s);
    default: return launch_profiled_nd<double>(A, ndim, cj, s);
  }
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
  if (g.G > 64) return g.nblocks;  // blocks above 256 samples: one workgroup each
  int64_t per = (int64_t)wp * (64 / lpb_of(g));
  return (g.nblocks + per - 1) / per;
}

int64_t encode_tiles(const Geo& g) { return encode_tiles_wp(g, WPG); }

hipError_t launch_encode(int dtype, int ndim, EncArgs& A, hipStream_t s) {
  A.ntiles = encode_tiles(A.g);
  if (A.ntiles == 0) return hipSuccess;
  switch (dtype) {
    case DT_I8: return launch_nd<int8_t>(A, ndim, s);
    case DT_I16: return launch_nd<int16_t>(A, ndim, s);
    case DT_I32: return launch_nd<int32_t>(A, ndim, s);
    case DT_F32: return launch_nd<float>(A, ndim, s);
    default: return launch_nd<double>(A, ndim, s);
  }
}

}  // namespace apax
