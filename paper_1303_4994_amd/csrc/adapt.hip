// adapt.hip -- the sequential adaptive loop (Sec. 6: the attenuator's gain
// follows a feedback loop towards the desired packet size) as a parallel scan.
//
// The controller's state between blocks is a requested code in a window of
// at most 64 codes; block j maps state w to w + sign(T - n_j(w)), clamped to
// the window, where n_j(w) is the block's size in words at code
// clamp(lo + w, c_floor_j, c_cap_j).  Every block's map is a 64-entry table,
// computed independently for all blocks (one evaluation per code).  Maps
// compose associatively, so the states of all blocks follow from a scan:
// groups of 256 maps are composed into one map per group (64 lanes, one per
// state, walk the group's maps in LDS), level by level until one group
// remains; then, top-down, one lane per group walks its 256 maps from the
// group's entry state and writes the entry state of every item.  The bottom
// level's entry states are the blocks' requested codes; the encode then
// codes each block at its own code (variable-size size / scan / emit).
#include "kernels.h"
#include "block.h"

namespace apax {

// Transition table of every block (one wave segment per block): entry w of
// block j at tab[64 j + w]; entries past the window width map to themselves.
template <typename T, int LPB, int NDIM>
__global__ __launch_bounds__(WPG * 64) void k_adapt_table(EncArgs A, uint8_t* __restrict__ tab) {
  constexpr int BPW = 64 / LPB;
  using B_ = Blk<T, LPB, NDIM>;
  __shared__ uint4 s_xch[NDIM >= 2 ? WPG * XCH : 1];
  const Geo& g = A.g;
  const int wave = threadIdx.x >> 6;
  B_ b;
  b.init(g, ((int64_t)blockIdx.x * WPG + wave) * BPW + lane_id() / LPB, NDIM >= 2 ? s_xch + wave * XCH : nullptr);
  b.load((const T*)A.x, g);
  if (__ballot(b.act && b.nonfinite) && lane_id() == 0) atomicOr(A.status, ST_NONFINITE);
  const int wd = g.awd, Tw = g.target;
  int cprev = 0x7FFFFFFF, nprev = 0;
  uint8_t* row = tab + 64 * b.j;
  const bool lead = b.blk_ok && b.L.gi == 0;
  for (int w = 0; w < 64; w++) {
    if (w >= wd) {  // uniform
      if (lead) row[w] = (uint8_t)w;
      continue;
    }
    const int c = clampc(g.alo + w, b.cf, b.cc);
    if (__ballot(b.act && c != cprev)) {  // some block of the wave needs a new evaluation
      int32_t a[4];
      int32_t best;
      b.quantize(c, false, a);
      b.best_stream(g, g.mask, a, best);
      nprev = (best + 31) >> 5;
      cprev = c;
    }
    if (lead) row[w] = adapt_next(w, nprev, Tw, wd);
  }
}

// Groups of 256 consecutive maps of `in` (m maps) composed into one map each.
__global__ __launch_bounds__(256) void k_adapt_compose(const uint8_t* __restrict__ in, int64_t m,
                                                       uint8_t* __restrict__ out) {
  __shared__ uint4 s[256 * 4];
  const int64_t base = (int64_t)blockIdx.x * 256;
  const int cnt = m - base < 256 ? (int)(m - base) : 256;
  const uint4* src = reinterpret_cast<const uint4*>(in + 64 * base);
  for (int i = threadIdx.x; i < cnt * 4; i += 256) s[i] = src[i];
  __syncthreads();
  if (threadIdx.x < 64) {
    const uint8_t* t = reinterpret_cast<const uint8_t*>(s);
    int st = threadIdx.x;
    for (int k = 0; k < cnt; k++) st = t[64 * k + st];
    out[64 * blockIdx.x + threadIdx.x] = (uint8_t)st;
  }
}

// One lane per group of 256 maps: from the group's entry state (entry_in, or
// w0 for the single top group) the state before each item, into entry_out
// (levels above the blocks) or as a requested code into bcode (blocks).
__global__ __launch_bounds__(64) void k_adapt_walk(const uint8_t* __restrict__ tab, int64_t m,
                                                   const uint8_t* __restrict__ entry_in, int w0,
                                                   uint8_t* __restrict__ entry_out, int32_t* __restrict__ bcode,
                                                   int alo) {
  __shared__ uint4 s[256 * 4];
  const int64_t base = (int64_t)blockIdx.x * 256;
  const int cnt = m - base < 256 ? (int)(m - base) : 256;
  const uint4* src = reinterpret_cast<const uint4*>(tab + 64 * base);
  for (int i = threadIdx.x; i < cnt * 4; i += 64) s[i] = src[i];
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint8_t* t = reinterpret_cast<const uint8_t*>(s);
    int st = entry_in ? entry_in[blockIdx.x] : w0;
    for (int k = 0; k < cnt; k++) {
      if (entry_out) entry_out[base + k] = (uint8_t)st;
      if (bcode) bcode[base + k] = alo + st;
      st = t[64 * k + st];
    }
  }
}

template <typename T, int LPB, int NDIM>
static hipError_t table_t(const EncArgs& A, uint8_t* tab, hipStream_t s) {
  hipLaunchKernelGGL((k_adapt_table<T, LPB, NDIM>), dim3((unsigned)encode_tiles(A.g)), dim3(WPG * 64), 0, s, A,
                     tab);
  return hipGetLastError();
}

template <typename T>
static hipError_t table_nd(const EncArgs& A, int ndim, uint8_t* tab, hipStream_t s) {
  const int G = A.g.G;
#define APAX_ADAPT_LPB(ND)                                \
  if (G <= 16) return table_t<T, 16, ND>(A, tab, s);     \
  if (G <= 32) return table_t<T, 32, ND>(A, tab, s);     \
  return table_t<T, 64, ND>(A, tab, s);
  if (ndim == 1) { APAX_ADAPT_LPB(1) }
  if (ndim == 2) { APAX_ADAPT_LPB(2) }
  APAX_ADAPT_LPB(3)
#undef APAX_ADAPT_LPB
}

// Map levels of n blocks: m[0] = n, m[l + 1] = ceil(m[l] / 256), composed at
// least once and until one map remains; returns the number of levels above
// the blocks (L, with m[L] = 1).
int adapt_levels(int64_t n, int64_t m[16]) {
  int L = 0;
  m[0] = n;
  do {
    m[L + 1] = (m[L] + 255) / 256;
    L++;
  } while (m[L] > 1 && L < 15);
  return L;
}

uint64_t adapt_bytes(int64_t n) {
  int64_t m[16];
  const int L = adapt_levels(n, m);
  uint64_t b = 0;
  for (int l = 0; l <= L; l++) b += ((uint64_t)64 * m[l] + 255) / 256 * 256;  // maps
  for (int l = 1; l <= L; l++) b += ((uint64_t)m[l] + 255) / 256 * 256;       // entry states
  return b;
}

hipError_t launch_adapt(int dtype, int ndim, const EncArgs& A, void* region, int32_t* bcode, hipStream_t s) {
  const Geo& g = A.g;
  if (g.nblocks == 0) return hipSuccess;
  int64_t m[16];
  const int L = adapt_levels(g.nblocks, m);
  uint8_t* tabs[16];
  uint8_t* ents[16];
  uint8_t* p = (uint8_t*)region;
  for (int l = 0; l <= L; l++) {
    tabs[l] = p;
    p += ((uint64_t)64 * m[l] + 255) / 256 * 256;
  }
  ents[0] = nullptr;
  for (int l = 1; l <= L; l++) {
    ents[l] = p;
    p += ((uint64_t)m[l] + 255) / 256 * 256;
  }
  hipError_t e;
  if (g.G > 64 || g.gq == 2) e = launch_wide_table(dtype, ndim, A, tabs[0], s);
  else {
    switch (dtype) {
      case DT_I8: e = table_nd<int8_t>(A, ndim, tabs[0], s); break;
      case DT_I16: e = table_nd<int16_t>(A, ndim, tabs[0], s); break;
      case DT_I32: e = table_nd<int32_t>(A, ndim, tabs[0], s); break;
      case DT_F32: e = table_nd<float>(A, ndim, tabs[0], s); break;
      default: e = table_nd<double>(A, ndim, tabs[0], s); break;
    }
  }
  if (e != hipSuccess) return e;
  for (int l = 0; l < L; l++)
    hipLaunchKernelGGL(k_adapt_compose, dim3((unsigned)m[l + 1]), dim3(256), 0, s, (const uint8_t*)tabs[l], m[l],
                       tabs[l + 1]);
  const int w0 = g.code - g.alo;
  for (int l = L - 1; l >= 0; l--) {
    const uint8_t* ein = l == L - 1 ? nullptr : ents[l + 1];
    hipLaunchKernelGGL(k_adapt_walk, dim3((unsigned)m[l + 1]), dim3(64), 0, s, (const uint8_t*)tabs[l], m[l], ein,
                       w0, l > 0 ? ents[l] : nullptr, l == 0 ? bcode : nullptr, g.alo);
  }
  return hipGetLastError();
}

}  // namespace apax
