// wide.h -- blocks of more than 256 samples (Sec. 6 allows 64 to 16384): one
// workgroup per block.
//
// The block is too large for one wave's registers, so it is staged in LDS:
// each thread loads up to four groups (coalesced, group gi = tid + m * nt) and
// keeps their samples in registers for every quantization of the block; the
// quantized block goes to LDS, where the candidate streams read their x, y
// and z predecessors directly.  Streams are costed with one thread per run of
// C consecutive groups: the group exponents of every candidate stream go to
// LDS, JEE token counts follow from one exclusive max-scan per stream (the
// last position whose exponent difference is not small: the pair tokens of a
// run of small differences start at odd distances from it), and block sizes
// from workgroup sums.  Emission assembles header | tokens | payload in the
// same LDS words the quantized block used, with ds_or, and copies them out.
// The decoder stages the block's words in LDS, finds token starts with the
// same max-scan over nibbles (an escape nibble 14/15 at an even distance
// after the last non-escape nibble starts a token), places tokens by a scan of
// the positions they cover, rebuilds the exponents with a segmented scan,
// extracts the payload, and undoes the stream with log-step running sums
// along each brick axis in LDS.
#pragma once
#include <type_traits>

#include "block.h"
#include "kernels.h"

namespace apax {

constexpr int WIDE_MAXT = 1024;  // threads of one block's workgroup at most
constexpr int WIDE_GPT = 4;      // groups per thread at most (G <= 4096)

// threads of the workgroup that handles a block of G groups
__host__ __device__ inline int wide_threads(int G) {
  const int t = (G + 63) / 64 * 64;
  return t > WIDE_MAXT ? WIDE_MAXT : t;
}
// LDS words of the block buffer: the quantized block, then the block's
// encoding (at most g.ldsw words), or the decoder's staged words, then values
__host__ __device__ inline int wide_qw(const Geo& g) {
  const int q = g.B > g.ldsw ? g.B : g.ldsw;
  return (q + 3) / 4 * 4;
}
// dynamic LDS bytes of the wide kernels: block buffer, eight exponent rows of
// G bytes, G words of per-position token data
__host__ __device__ inline size_t wide_lds_bytes(const Geo& g) {
  return 4 * ((size_t)wide_qw(g) + 2 * (size_t)g.G + (size_t)g.G);
}

struct WideShared {
  int32_t red[16][8];  // per-wave partials of the workgroup scans (up to 8 values)
  uint64_t key;        // block max magnitude key
  int32_t pay[8];      // payload bits per stream
  int32_t nib[8];      // JEE nibbles per stream
  int32_t tend;        // decoder: nibbles of the token area (-1: not found)
  int32_t acc;         // decoder: words of the blocks before this one in its superblock
};

// ---- workgroup collectives (every thread calls them; they end with a
// barrier, so WideShared::red can be reused at once)
__device__ __forceinline__ int wg_nwaves() { return (blockDim.x + 63) >> 6; }

// sums of N values over the workgroup
template <int N>
__device__ __forceinline__ void wg_sum(int32_t v[N], WideShared& sh) {
  const int lane = lane_id(), wave = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < N; i++) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v[i] += __shfl_xor(v[i], o, 64);
  }
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < N; i++) sh.red[wave][i] = v[i];
  }
  __syncthreads();
  const int nw = wg_nwaves();
#pragma unroll
  for (int i = 0; i < N; i++) {
    int32_t t = 0;
    for (int w = 0; w < nw; w++) t += sh.red[w][i];
    v[i] = t;
  }
  __syncthreads();
}

// exclusive prefix sums (thread order) of N values; total[i] = the sum
template <int N>
__device__ __forceinline__ void wg_excl_sum(int32_t v[N], int32_t total[N], WideShared& sh) {
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  int32_t inc[N];
#pragma unroll
  for (int i = 0; i < N; i++) {
    inc[i] = v[i];
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int32_t u = __shfl_up(inc[i], (unsigned)o, 64);
      if (lane >= o) inc[i] += u;
    }
  }
  if (lane == 63) {
#pragma unroll
    for (int i = 0; i < N; i++) sh.red[wave][i] = inc[i];
  }
  __syncthreads();
  const int nw = wg_nwaves();
#pragma unroll
  for (int i = 0; i < N; i++) {
    int32_t before = 0, t = 0;
    for (int w = 0; w < nw; w++) {
      const int32_t r = sh.red[w][i];
      before += w < wave ? r : 0;
      t += r;
    }
    v[i] = before + inc[i] - v[i];
    total[i] = t;
  }
  __syncthreads();
}

// exclusive prefix maxima (thread order) of N values >= -1 (-1 before the first)
template <int N>
__device__ __forceinline__ void wg_excl_max(int32_t v[N], WideShared& sh) {
  const int lane = lane_id(), wave = threadIdx.x >> 6;
  int32_t inc[N];
#pragma unroll
  for (int i = 0; i < N; i++) {
    inc[i] = v[i];
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const int32_t u = __shfl_up(inc[i], (unsigned)o, 64);
      if (lane >= o) inc[i] = max(inc[i], u);
    }
  }
  if (lane == 63) {
#pragma unroll
    for (int i = 0; i < N; i++) sh.red[wave][i] = inc[i];
  }
  __syncthreads();
#pragma unroll
  for (int i = 0; i < N; i++) {
    int32_t before = -1;
    for (int w = 0; w < wave; w++) before = max(before, sh.red[w][i]);
    int32_t ex = __shfl_up(inc[i], 1u, 64);
    if (lane == 0) ex = -1;
    v[i] = max(before, ex);
  }
  __syncthreads();
}

// ---- geometry of one block held by a workgroup
struct WGeo {
  int64_t bz, by, bx;  // brick coordinates of the block
  int nt, C;           // threads, consecutive groups per thread

  __device__ __forceinline__ void init(const Geo& g, int64_t j) {
    const uint32_t jj = (uint32_t)j;  // j < 2^31
    const uint32_t t = fdiv(jj, g.nbx_m, g.nbx_s);
    bx = jj - t * (uint32_t)g.nbx;
    const uint32_t z = fdiv(t, g.nby_m, g.nby_s);
    by = t - z * (uint32_t)g.nby;
    bz = z;
    nt = blockDim.x;
    C = (g.G + nt - 1) / nt;
  }
  // brick coordinates of group gi: z, y (rows), xq (group along the row)
  __device__ __forceinline__ void coords(const Geo& g, int gi, int& z, int& y, int& xq) const {
    z = (int)fdiv((uint32_t)gi, g.plane_m, g.plane_s);
    const int r = gi - z * g.plane;
    y = (int)fdiv((uint32_t)r, g.rowq_m, g.rowq_s);
    xq = r - y * g.rowq;
  }
  // valid samples (0..4) of the group at brick coordinates (z, y, xq) and the
  // array index of its sample 0
  __device__ __forceinline__ int nvalid(const Geo& g, int z, int y, int xq, int64_t& idx) const {
    const int64_t X = bx * g.b[2] + 4 * xq, Y = by * g.b[1] + y, Z = bz * g.b[0] + z;
    idx = 0;
    if (X >= g.n[2] || Y >= g.n[1] || Z >= g.n[0]) return 0;
    idx = (Z * g.n[1] + Y) * g.n[2] + X;
    const int64_t rem = g.n[2] - X;
    return rem >= 4 ? 4 : (int)rem;
  }
};

// quantized samples x-2 .. x+3 of brick row (z, y) around group xq (zero for
// rows and samples before the brick)
__device__ __forceinline__ void wide_row6(const uint32_t* qa, const Geo& g, int z, int y, int xq, uint32_t r[6]) {
  if (z < 0 || y < 0) {
#pragma unroll
    for (int k = 0; k < 6; k++) r[k] = 0u;
    return;
  }
  const int base = (z * g.b[1] + y) * g.b[2] + 4 * xq;
  const uint4 c = *reinterpret_cast<const uint4*>(qa + base);
  const uint2 p = xq > 0 ? *reinterpret_cast<const uint2*>(qa + base - 2) : make_uint2(0u, 0u);
  r[0] = p.x; r[1] = p.y; r[2] = c.x; r[3] = c.y; r[4] = c.z; r[5] = c.w;
}

// stream st (0..6) of one group from its rows: P the group's own, Y the row
// before in y, Z the row before in z, ZY both; mod 2^32 (the caller wraps)
__device__ __forceinline__ void wide_stream(int st, const uint32_t P[6], const uint32_t Y[6], const uint32_t Z[6],
                                            const uint32_t ZY[6], uint32_t v[4]) {
#pragma unroll
  for (int k = 0; k < 4; k++) {
    const int i = k + 2;
    uint32_t r;
    switch (st) {
      case 0: r = P[i]; break;
      case 1: r = P[i] - P[i - 1]; break;
      case 2: r = P[i] - 2u * P[i - 1] + P[i - 2]; break;
      case 3: r = P[i] - Y[i]; break;
      case 4: r = P[i] - Z[i]; break;
      case 5: r = (P[i] - Y[i]) - (P[i - 1] - Y[i - 1]); break;
      default: {
        const uint32_t t0 = (P[i] - Z[i]) - (Y[i] - ZY[i]);
        const uint32_t t1 = (P[i - 1] - Z[i - 1]) - (Y[i - 1] - ZY[i - 1]);
        r = t0 - t1;
      }
    }
    v[k] = r;
  }
}

// JEE nibbles of the exponent row e[0..G) for this thread's positions
// [p0, p0 + C): returns the count; `last` in: the last position before p0
// whose difference is not small (position 0 counts as such)
__device__ __forceinline__ int wide_jee_count(const uint8_t* e, int G, int p0, int C, int last) {
  int nib = 0;
  for (int q = 0; q < C; q++) {
    const int i = p0 + q;
    if (i >= G) break;
    if (i == 0) {
      last = 0;
      continue;
    }
    const int d = (int)e[i] - (int)e[i - 1];
    const int ad = d < 0 ? -d : d;
    if (ad <= 1) {
      nib += (i - last) & 1;
    } else {
      last = i;
      nib += ad == 2 ? 1 : 2;
    }
  }
  return nib;
}

// the last position in [p0, p0 + C) whose exponent difference is not small
// (position 0 included), or -1
__device__ __forceinline__ int wide_last_big(const uint8_t* e, int G, int p0, int C) {
  int last = -1;
  for (int q = 0; q < C; q++) {
    const int i = p0 + q;
    if (i >= G) break;
    if (i == 0) {
      last = 0;
      continue;
    }
    const int d = (int)e[i] - (int)e[i - 1];
    if (d < -1 || d > 1) last = i;
  }
  return last;
}

}  // namespace apax
