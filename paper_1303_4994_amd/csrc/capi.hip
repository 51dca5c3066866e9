// capi.hip -- host side of libapax: parameter validation, stream container
// layout, workspace layout, kernel launches and the profiler's control loop.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <chrono>
#include <deque>
#include <mutex>
#include <vector>

#include "apax.h"
#include "kernels.h"
#include "monitor.h"
#include "spectra.h"
#include "wide.h"

using namespace apax;

namespace {

constexpr uint32_t MAGIC = 0x58415041u;  // "APAX"
constexpr uint32_t ND_ALLOWED[4] = {0u, 0x87u, 0xAFu, 0xFFu};

struct HG {
  Geo g;
  int dtype, mode, ndim, esz, W, H;
  bool isint;
  bool lagged;  // APAX_FLAG_LAGGED
  uint64_t nsamples;
};

int floordiv16(int c) { return c >> 4; }

double host_gain(int c) { return ldexp((double)(16 + (c & 15)), floordiv16(c) - 4); }

// Largest code in [cmin, cmax] with fl64(M * g(c)) <= lim (monotone in c).
int host_largest(double M, double lim, int cmin, int cmax) {
  if (M * host_gain(cmax) <= lim) return cmax;
  int lo = cmin, hi = cmax;
  while (hi - lo > 1) {
    int mid = lo + ((hi - lo) >> 1);
    if (M * host_gain(mid) <= lim) lo = mid;
    else hi = mid;
  }
  return lo;
}

// Multiplier and shift for n / d with n < 2^31, 1 <= d < 2^31:
// m = ceil(2^(31+l) / d), l = ceil(log2 d); then n / d = (n * m) >> (31 + l).
void magic(int64_t d, uint32_t& m, int32_t& sh) {
  int l = 0;
  while ((1ll << l) < d) l++;
  const unsigned __int128 num = (unsigned __int128)1 << (31 + l);
  m = (uint32_t)((num + (unsigned __int128)(d - 1)) / (unsigned __int128)d);
  sh = 31 + l;
}

// Validation of apax_params (the rules of include/apax.h).  forced_budget >= 0
// takes the fixed-rate budget from a stream header instead of the rate.
// the budget field of a stream header as setup()'s forced budget: fixed rate
// (words per block) and adaptive rate (target words per block) only
int header_budget(uint32_t mode, int budget) {
  return (mode == APAX_FIXED_RATE || mode == APAX_ADAPTIVE_RATE) ? budget : -1;
}

int setup(const apax_params* p, HG& h, int forced_budget = -1) {
  memset(&h, 0, sizeof(h));
  if (!p || p->size != sizeof(apax_params)) return APAX_E_INVALID;
  if (p->dtype < APAX_I8 || p->dtype > APAX_F64) return APAX_E_INVALID;
  if (p->ndim < 1 || p->ndim > 3) return APAX_E_INVALID;
  if (p->mode > APAX_ADAPTIVE_RATE) return APAX_E_INVALID;
  if (p->flags & ~(APAX_FLAG_LAGGED | APAX_FILTER(31, 1) | APAX_FLAG_GROUP8)) return APAX_E_INVALID;
  if ((p->flags & APAX_FLAG_LAGGED) && p->mode != APAX_LOSSLESS) return APAX_E_INVALID;
  // filter stream: 1-d only, stride 1..16, a sign only with a stride
  const int fk = (int)((p->flags >> 8) & 0x1Fu), fneg = (p->flags & APAX_FILTER_NEG) ? 1 : 0;
  if (fk > 16 || (fneg && !fk) || (fk && p->ndim != 1)) return APAX_E_INVALID;
  h.lagged = (p->flags & APAX_FLAG_LAGGED) != 0;
  static const int ESZ[6] = {0, 1, 2, 4, 4, 8};
  static const int WQ[6] = {0, 8, 16, 32, 32, 32};
  h.dtype = (int)p->dtype;
  h.mode = (int)p->mode;
  h.ndim = (int)p->ndim;
  h.esz = ESZ[h.dtype];
  h.W = WQ[h.dtype];
  h.isint = h.dtype <= APAX_I32;
  h.H = h.isint ? 32 : 48;
  if (h.mode == APAX_LOSSLESS && !h.isint) return APAX_E_UNSUPPORTED;
  int64_t n[3] = {1, 1, 1}, b[3] = {1, 1, 1};
  int off = 3 - h.ndim;
  int64_t B = 1;
  for (int i = 0; i < h.ndim; i++) {
    if (p->brick[i] < 1 || p->brick[i] > 16384) return APAX_E_INVALID;
    if (p->dims[i] > (1ull << 40)) return APAX_E_INVALID;
    n[off + i] = (int64_t)p->dims[i];
    b[off + i] = p->brick[i];
    B *= p->brick[i];
  }
  if (B < 64 || B > 16384 || B % 4 != 0 || b[2] % 4 != 0) return APAX_E_INVALID;
  Geo& g = h.g;
  // groups of 8 samples per exponent: B and the brick rows multiples of 8
  g.gq = (p->flags & APAX_FLAG_GROUP8) ? 2 : 1;
  if (g.gq == 2 && (B % 8 != 0 || b[2] % 8 != 0)) return APAX_E_INVALID;
  for (int i = 0; i < 3; i++) { g.n[i] = n[i]; g.b[i] = (int32_t)b[i]; }
  g.B = (int32_t)B;
  g.G = (int32_t)(B / 4);
  g.rowq = g.b[2] / 4;
  g.plane = g.b[1] * g.rowq;
  // block counts and sample counts must not wrap: the kernels index blocks
  // with 31 bits and samples with 64-bit offsets in bytes
  int64_t nb[3];
  g.nblocks = 1;
  int64_t ns = 1;
  for (int i = 0; i < 3; i++) {
    nb[i] = (n[i] + b[i] - 1) / b[i];
    if (__builtin_mul_overflow(g.nblocks, nb[i], &g.nblocks)) return APAX_E_UNSUPPORTED;
    if (__builtin_mul_overflow(ns, n[i], &ns)) return APAX_E_UNSUPPORTED;
  }
  int64_t nbytes_in;
  if (__builtin_mul_overflow(ns, (int64_t)h.esz, &nbytes_in) || nbytes_in > ((int64_t)1 << 56))
    return APAX_E_UNSUPPORTED;
  g.nbx = nb[2] ? nb[2] : 1;
  g.nby = nb[1] ? nb[1] : 1;
  if (g.nblocks > (int64_t)0x7FFFFFFF) return APAX_E_UNSUPPORTED;
  h.nsamples = (uint64_t)ns;
  uint32_t allowed = ND_ALLOWED[h.ndim] | (fk ? 0x08u : 0u);
  g.fk = fk;
  g.fneg = fneg;
  uint32_t m = p->stream_mask ? p->stream_mask : allowed;
  if (m & ~allowed) return APAX_E_INVALID;
  m = h.mode == APAX_FIXED_RATE ? ((m | 1u) & 0x7Fu) : (m | 0x81u);
  g.mask = m;
  g.mode = h.mode;
  g.cmin = h.isint ? -512 : -17120;
  g.cmax = h.isint ? 0 : 16383;
  g.code = 0;
  if (h.mode != APAX_LOSSLESS) {
    if (p->code < g.cmin || p->code > g.cmax) return APAX_E_INVALID;
    g.code = p->code;
  }
  g.maxw = (h.H + g.B * h.W + 31) / 32;
  g.ldsw = ((h.H + 8 * (g.G - 1) + g.B * h.W + 31) / 32 + 2 + 3) / 4 * 4;
  g.budget = 0;
  if (h.mode == APAX_FIXED_RATE) {
    double words;
    if (forced_budget >= 0) {
      words = forced_budget;
    } else {
      if (!(p->rate > 0.0) || !isfinite(p->rate)) return APAX_E_INVALID;
      words = floor((double)g.B * 8.0 * h.esz / (p->rate * 32.0));
    }
    int min_words = (h.H + 4 * (g.G / g.gq / 2) + 31) / 32;
    if (words < min_words || words > 65535.0) return APAX_E_INVALID;
    g.budget = (int32_t)words;
  }
  if (h.mode == APAX_FIXED_QUALITY && forced_budget < 0) {
    if (!(p->target_corr > 0.0 && p->target_corr <= 1.0)) return APAX_E_INVALID;
  }
  g.target = g.alo = g.awd = 0;
  if (h.mode == APAX_ADAPTIVE_RATE) {
    // target words per block (from the rate as in fixed rate) and the
    // controller's window of requested codes around the start code
    double words;
    if (forced_budget >= 0) {
      words = forced_budget;
    } else {
      if (!(p->rate > 0.0) || !isfinite(p->rate)) return APAX_E_INVALID;
      words = floor((double)g.B * 8.0 * h.esz / (p->rate * 32.0));
    }
    if (words < 1.0 || words > 65535.0) return APAX_E_INVALID;
    g.target = (int32_t)words;
    g.alo = std::max(g.cmin, g.code - APAX_ADAPT_HALF);
    g.awd = std::min(g.cmax, g.code + APAX_ADAPT_HALF - 1) - g.alo + 1;
  }
  g.sz = (int64_t)g.b[0] * g.n[1] * g.n[2];
  g.sy = (int64_t)g.b[1] * g.n[2];
  g.fbx = (int32_t)(g.n[2] / g.b[2]);
  g.fby = (int32_t)(g.n[1] / g.b[1]);
  g.fbz = (int32_t)(g.n[0] / g.b[0]);
  {
    const int64_t span = ((int64_t)(g.b[0] - 1) * g.n[1] + (g.b[1] - 1)) * g.n[2] + g.b[2];
    g.dense_ok = span < ((int64_t)1 << 31) && (h.ndim == 1 || g.n[2] % 4 == 0);
  }
  magic(g.nbx, g.nbx_m, g.nbx_s);
  magic(g.nby, g.nby_m, g.nby_s);
  magic(g.rowq, g.rowq_m, g.rowq_s);
  magic(g.plane, g.plane_m, g.plane_s);
  return APAX_OK;
}

uint64_t lens_bytes(const HG& h) { return ((uint64_t)h.g.nblocks * 2 + 7) / 8 * 8; }
uint64_t sbo_count(const HG& h) { return ((uint64_t)h.g.nblocks + 63) / 64; }

uint64_t area_offset(const HG& h) {
  if (h.mode == APAX_FIXED_RATE) return 64;
  uint64_t o = 64 + lens_bytes(h) + 8 * sbo_count(h);
  return (o + 15) / 16 * 16;
}

uint64_t bound_of(const HG& h) {
  uint64_t per = h.g.budget ? (uint64_t)h.g.budget : (uint64_t)h.g.maxw;
  return area_offset(h) + 4 * per * (uint64_t)h.g.nblocks;
}

void make_header(const apax_params* p, const HG& h, uint32_t hdr[16]) {
  uint8_t b[64];
  memset(b, 0, sizeof(b));
  auto put16 = [&](int o, uint16_t v) { memcpy(b + o, &v, 2); };
  auto put32 = [&](int o, uint32_t v) { memcpy(b + o, &v, 4); };
  auto put64 = [&](int o, uint64_t v) { memcpy(b + o, &v, 8); };
  put32(0, MAGIC);
  put16(4, 1);
  b[6] = (uint8_t)h.dtype;
  b[7] = (uint8_t)h.mode;
  b[8] = (uint8_t)(h.ndim | (h.g.gq == 2 ? 0x10 : 0));  // bit 4: groups of 8
  b[9] = (uint8_t)h.g.mask;
  put16(10, (uint16_t)(h.mode == APAX_ADAPTIVE_RATE ? h.g.target : h.g.budget));
  put32(12, (uint32_t)h.g.code);
  for (int i = 0; i < 3; i++) put64(16 + 8 * i, i < h.ndim ? p->dims[i] : 0);
  for (int i = 0; i < 3; i++) put16(40 + 2 * i, (uint16_t)(i < h.ndim ? p->brick[i] : 0));
  b[46] = (uint8_t)h.g.fk;  // filter stream: stride and sign (0 0: none)
  b[47] = (uint8_t)h.g.fneg;
  put64(48, (uint64_t)h.g.nblocks);
  put64(56, h.mode == APAX_FIXED_RATE ? (uint64_t)h.g.budget * (uint64_t)h.g.nblocks : 0);
  memcpy(hdr, b, 64);
}

// ---- workspace layout: [PState][tile states][per-block codes][partials]
uint64_t al256(uint64_t b) { return (b + 255) / 256 * 256; }
uint64_t tiles_enc(const HG& h) { return (uint64_t)encode_tiles(h.g); }

// partial records of one profile launch: at most about 2048 workgroups over
// all codes (prof_wgs), or the max pass's PMAX_WGS
uint64_t partial_bytes(const HG& h) {
  uint64_t recs = 2048 + 2 * (uint64_t)MAXCODES;
  // also: one binary64 partial per tile of a decode-on-read consumer
  return std::max<uint64_t>(std::max<uint64_t>(recs * PPART_BYTES, (uint64_t)PMAX_WGS * 16),
                            8 * (uint64_t)encode_tiles(h.g));
}

// [PState][chosen stream per block][words per superblock][int32 per block][partials]
uint64_t ws_bst_off(const HG& h) { (void)h; return al256(sizeof(PState)); }
uint64_t ws_ssum_off(const HG& h) { return ws_bst_off(h) + al256((uint64_t)h.g.nblocks); }
uint64_t ws_cj_off(const HG& h) { return ws_ssum_off(h) + al256(4 * (((uint64_t)h.g.nblocks + 63) / 64)); }
uint64_t ws_part_off(const HG& h) { return ws_cj_off(h) + al256(4 * (uint64_t)h.g.nblocks); }
// adaptive rate: the controller's maps and states after the per-block codes
uint64_t adapt_need(const HG& h) { return h.mode == APAX_ADAPTIVE_RATE ? adapt_bytes(h.g.nblocks) : 0; }
// two partial-record regions: a profile with a side stream runs its curve
// pass beside the metrics pass, each with its own records
uint64_t ws_need(const HG& h) { return ws_part_off(h) + std::max(2 * al256(partial_bytes(h)), adapt_need(h)); }

void* partials_ptr(void* ws, const HG& h) { return (uint8_t*)ws + ws_part_off(h); }
void* partials2_ptr(void* ws, const HG& h) { return (uint8_t*)partials_ptr(ws, h) + al256(partial_bytes(h)); }
int32_t* cj_ptr(void* ws, const HG& h) { return (int32_t*)((uint8_t*)ws + ws_cj_off(h)); }

int hip_err(hipError_t e) { return e == hipSuccess ? APAX_OK : APAX_E_HIP; }

__global__ void k_clear(uint32_t* p, int nwords) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nwords) p[i] = 0u;
}

void clear_words(uint32_t* p, int nwords, hipStream_t s) {
  if (nwords > 0) hipLaunchKernelGGL(k_clear, dim3((unsigned)((nwords + 255) / 256)), dim3(256), 0, s, p, nwords);
}

__global__ void k_copy_word(uint32_t* dst, const uint32_t* src) {
  if (threadIdx.x == 0) *dst = *src;
}

// OR the per-item status words of a batch into the workspace status word
__global__ void k_fold_status(const uint32_t* item_status, uint32_t n, uint32_t* status) {
  uint32_t acc = 0;
  for (uint32_t i = threadIdx.x; i < n; i += blockDim.x) acc |= item_status[i];
  if (acc) atomicOr(status, acc);
}

// the operating point of one workspace's profile, into another workspace
__global__ void k_adopt_point(const PState* from, PState* to) {
  if (threadIdx.x < 2) to->sel[threadIdx.x] = from->sel[threadIdx.x];
}

__global__ void k_header_only(HdrArgs A) {
  if (threadIdx.x == 0) {
    uint32_t h[16];
    for (int i = 0; i < 16; i++) h[i] = A.hdr[i];
    if (A.sel) {
      int32_t code;
      uint32_t mask;
      if (!operating_point(A.sel, A.status, A.cmin, A.cmax, A.ucode, A.umask, code, mask))
        atomicOr(A.status, ST_NOPROFILE);
      h[2] = (h[2] & ~0xFF00u) | ((mask & 0xFFu) << 8);
      h[3] = (uint32_t)code;
    }
    for (int i = 0; i < 16; i++) A.out[i] = h[i];
    *A.d_nbytes = A.nbytes;
  }
}

// r from the four sums, cancellation-free form of the printed formula (Sec. 4)
void r_of(double sxx, double syy, double sdd, double sds, double& r, double& omr) {
  if (sxx == 0.0 && syy == 0.0) { r = 1.0; omr = 0.0; return; }
  if (sxx == 0.0 || syy == 0.0) { r = 0.0; omr = 1.0; return; }
  double nx = sqrt(sxx), ny = sqrt(syy);
  double dn = sds / (nx + ny);
  omr = (sdd - dn * dn) / (2.0 * nx * ny);
  r = 1.0 - omr;
}

// ---- batch plans
struct BatchClass {
  int lpb, ndim;
  std::vector<uint32_t> items;  // indices into the plan's items
  int64_t total_tiles = 0;
  int maxldsw = 0;
  uint64_t items_off = 0, starts_off = 0, tstate_off = 0, ticket_off = 0;
  int grid = 0;
};

}  // namespace

struct apax_batch {
  int op = 0;
  apax_tune tune{};
  std::vector<apax_batch_item> items;
  std::vector<HG> geo;
  std::vector<BatchClass> classes;
  // items the shared launch does not take (blocks of more than 64 groups,
  // groups of 8, the lagged choice, adaptive rate): single-array calls in
  // the same run, each with its own workspace region and copy of the header
  std::vector<uint32_t> solo;
  std::vector<uint64_t> solo_off;
  std::vector<std::array<uint8_t, 64>> solo_hdr;
  uint64_t ws_bytes = 0;
  uint64_t istat_off = 0;       // per-item status words in the workspace
  void* d_ws = nullptr;
  std::vector<uint8_t> tables;  // host image of [descriptors | starts] of every class
  void* pinned = nullptr;       // pinned staging copy of `tables` (async upload)
  hipEvent_t upload_done = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

// ======================================================================== C ABI

extern "C" {

const char* apax_strerror(int code) {
  switch (code) {
    case APAX_OK: return "ok";
    case APAX_E_INVALID: return "invalid parameters";
    case APAX_E_UNSUPPORTED: return "unsupported parameters";
    case APAX_E_CAPACITY: return "buffer too small";
    case APAX_E_CORRUPT: return "corrupt stream";
    case APAX_E_NONFINITE: return "non-finite input";
    case APAX_E_HIP: return "HIP runtime error";
    case APAX_E_INTERNAL: return "device safety limit";
    default: return "unknown error";
  }
}

int apax_encode_bound(const apax_params* p, uint64_t* bytes) {
  if (!p || !bytes) return APAX_E_INVALID;
  apax_params q = *p;
  if (q.code == APAX_CODE_PROFILED) q.code = 0;  // the bound does not depend on the code
  HG h;
  int e = setup(&q, h);
  if (e) return e;
  *bytes = bound_of(h);
  return APAX_OK;
}

int apax_workspace_size(const apax_params* p, uint64_t* bytes) {
  apax_params q = *p;
  q.code = 0;
  HG h;
  int e = setup(&q, h);
  if (e) return e;
  *bytes = ws_need(h);
  return APAX_OK;
}

int apax_stream_info(const void* h_hdr, uint64_t n, apax_params* out) {
  if (!h_hdr || n < 64 || !out) return APAX_E_CORRUPT;
  const uint8_t* b = (const uint8_t*)h_hdr;
  uint32_t magic;
  uint16_t ver, budget, rsv, brick[3];
  int32_t code;
  uint64_t dims[3], nblocks;
  memcpy(&magic, b, 4);
  memcpy(&ver, b + 4, 2);
  memcpy(&budget, b + 10, 2);
  memcpy(&code, b + 12, 4);
  memcpy(dims, b + 16, 24);
  memcpy(brick, b + 40, 6);
  memcpy(&rsv, b + 46, 2);  // filter stream: stride, sign
  memcpy(&nblocks, b + 48, 8);
  if (magic != MAGIC || ver != 1) return APAX_E_CORRUPT;
  const uint32_t hk = b[46], hn = b[47];
  if (hk > 16 || hn > 1 || (hn && !hk)) return APAX_E_CORRUPT;
  apax_params p;
  memset(&p, 0, sizeof(p));
  p.size = sizeof(p);
  p.dtype = b[6];
  p.mode = b[7];
  p.ndim = b[8] & 0x0Fu;
  if (b[8] & 0xE0u) return APAX_E_CORRUPT;
  p.stream_mask = b[9];
  p.code = code;
  p.flags = (hk ? APAX_FILTER(hk, hn) : 0u) | ((b[8] & 0x10u) ? APAX_FLAG_GROUP8 : 0u);
  if (p.ndim < 1 || p.ndim > 3) return APAX_E_CORRUPT;
  for (int i = 0; i < 3; i++) {
    if (i < (int)p.ndim) { p.dims[i] = dims[i]; p.brick[i] = brick[i]; }
    else if (dims[i] || brick[i]) return APAX_E_CORRUPT;
  }
  p.target_corr = 0.5;
  if (p.mode == APAX_FIXED_RATE || p.mode == APAX_ADAPTIVE_RATE) {
    if (budget == 0) return APAX_E_CORRUPT;
  } else if (budget != 0) {
    return APAX_E_CORRUPT;
  }
  HG h;
  if (setup(&p, h, header_budget(p.mode, budget)) != APAX_OK) return APAX_E_CORRUPT;
  if (h.g.mask != p.stream_mask || (uint64_t)h.g.nblocks != nblocks) return APAX_E_CORRUPT;
  if (p.mode == APAX_FIXED_RATE || p.mode == APAX_ADAPTIVE_RATE) {
    uint32_t B = 1;
    for (int i = 0; i < (int)p.ndim; i++) B *= p.brick[i];
    p.rate = (double)B * 8.0 * h.esz / (32.0 * (double)budget);
  }
  *out = p;
  return APAX_OK;
}

int apax_stream_size(const void* h_hdr, uint64_t n, uint64_t* nbytes) {
  if (!nbytes) return APAX_E_INVALID;
  apax_params p;
  const int e = apax_stream_info(h_hdr, n, &p);
  if (e) return e;
  HG h;
  if (setup(&p, h, header_budget(p.mode, ((const uint16_t*)h_hdr)[5])) != APAX_OK)
    return APAX_E_CORRUPT;
  uint64_t words;
  memcpy(&words, (const uint8_t*)h_hdr + 56, 8);
  const uint64_t per = h.g.budget ? (uint64_t)h.g.budget : (uint64_t)h.g.maxw;
  if (words > per * (uint64_t)h.g.nblocks) return APAX_E_CORRUPT;
  if (h.mode == APAX_FIXED_RATE && words != per * (uint64_t)h.g.nblocks) return APAX_E_CORRUPT;
  *nbytes = area_offset(h) + 4 * words;
  return APAX_OK;
}

int apax_status_clear(void* d_ws, hipStream_t stream) {
  if (!d_ws) return APAX_E_INVALID;
  hipLaunchKernelGGL(k_clear, dim3(1), dim3(64), 0, stream, (uint32_t*)d_ws, 1);
  return hip_err(hipGetLastError());
}

int apax_status(const void* d_ws, hipStream_t stream) {
  if (!d_ws) return APAX_E_INVALID;
  uint32_t st = 0;
  if (hipStreamSynchronize(stream) != hipSuccess) return APAX_E_HIP;
  if (hipMemcpy(&st, d_ws, 4, hipMemcpyDeviceToHost) != hipSuccess) return APAX_E_HIP;
  if (st & ST_NONFINITE) return APAX_E_NONFINITE;
  if (st & ST_CORRUPT) return APAX_E_CORRUPT;
  if (st & ST_INTERNAL) return APAX_E_INTERNAL;
  if (st & ST_NOPROFILE) return APAX_E_INVALID;
  return APAX_OK;
}

}  // extern "C"

namespace {

// Workspace bytes an encode itself uses: the state block (status word), one
// chosen stream per block and one word count per superblock of 64 blocks
// (variable-size modes) and, for the lagged choice, one best stream per block.
uint64_t enc_need(const HG& h) {
  if (h.mode == APAX_ADAPTIVE_RATE) return ws_part_off(h) + adapt_need(h);
  return ws_cj_off(h) + (h.lagged ? al256(4 * (uint64_t)h.g.nblocks) : 0);
}

// Blocks above 256 samples run one workgroup per block with the block staged
// in LDS; the current device must give a workgroup that much.
// extra: static LDS of the kernel beyond WideShared (the profile passes' wave partials)
bool wide_fits(const Geo& g, size_t extra = 256) {
  static int cache[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return false;
  int v = dev >= 0 && dev < 64 ? cache[dev] : 0;
  if (v == 0) {
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) return false;
    if (dev >= 0 && dev < 64) cache[dev] = v;
  }
  return wide_lds_bytes(g) + sizeof(WideShared) + extra <= (size_t)v;
}

// The encoder's kernel arguments for array d_x, stream d_stream, workspace d_ws.
void enc_args(const void* d_x, const apax_params* p, const HG& h, bool profiled, void* d_stream,
              uint64_t* d_nbytes, void* d_ws, EncArgs& A) {
  memset(&A, 0, sizeof(A));
  A.g = h.g;
  A.x = d_x;
  A.out_base = (uint8_t*)d_stream;
  A.area = area_offset(h);
  A.out_words = (uint32_t*)((uint8_t*)d_stream + A.area);
  A.lens = (uint16_t*)((uint8_t*)d_stream + 64);
  A.sbo = (uint64_t*)((uint8_t*)d_stream + 64 + lens_bytes(h));
  A.d_nbytes = d_nbytes;
  A.status = &((PState*)d_ws)->status;
  A.ticket = &((PState*)d_ws)->ticket;
  A.bst = (uint8_t*)d_ws + ws_bst_off(h);
  A.ssum = (uint32_t*)((uint8_t*)d_ws + ws_ssum_off(h));
  make_header(p, h, A.hdr);
  if (h.mode != APAX_FIXED_RATE) {
    A.zpad[0] = (uint64_t)(64 + 2 * (uint64_t)h.g.nblocks);
    A.zpad[1] = (uint64_t)(64 + lens_bytes(h));
    A.zpad[2] = (uint64_t)(64 + lens_bytes(h) + 8 * sbo_count(h));
    A.zpad[3] = A.area;
  }
  if (profiled) A.sel = ((PState*)d_ws)->sel;
}

// apax_encode's work once the parameters are set up and the buffers checked:
// d_ws holds at least enc_need(h) bytes.
int encode_enqueue(const void* d_x, const apax_params* p, const HG& h, bool profiled, void* d_stream,
                   uint64_t* d_nbytes, void* d_ws, hipStream_t stream) {
  int e;
  EncArgs A;
  enc_args(d_x, p, h, profiled, d_stream, d_nbytes, d_ws, A);
  const bool wide = h.g.G > 64 || h.g.gq == 2;
  if (wide && h.g.nblocks && !wide_fits(h.g)) return APAX_E_UNSUPPORTED;
  if (h.lagged && h.g.nblocks) {
    int32_t* best = cj_ptr(d_ws, h);  // each block's own best stream
    if ((e = hip_err(wide ? launch_wide_choice(h.dtype, h.ndim, A, best, stream)
                          : launch_stream_choice(h.dtype, h.ndim, A, best, stream))))
      return e;
    A.lag = best;
  }
  if (h.mode == APAX_ADAPTIVE_RATE && h.g.nblocks) {
    // the loop's requested code of every block, then the encode at those codes
    int32_t* bcode = cj_ptr(d_ws, h);
    if ((e = hip_err(launch_adapt(h.dtype, h.ndim, A, (uint8_t*)d_ws + ws_part_off(h), bcode, stream)))) return e;
    A.bcode = bcode;
  }
  if (h.g.nblocks == 0) {
    HdrArgs Hd;
    memset(&Hd, 0, sizeof(Hd));
    Hd.out = (uint32_t*)d_stream;
    Hd.d_nbytes = d_nbytes;
    Hd.nbytes = A.area;
    memcpy(Hd.hdr, A.hdr, 64);
    Hd.sel = A.sel;
    Hd.status = A.status;
    Hd.cmin = h.g.cmin;
    Hd.cmax = h.g.cmax;
    Hd.ucode = h.g.code;
    Hd.umask = h.g.mask;
    hipLaunchKernelGGL(k_header_only, dim3(1), dim3(64), 0, stream, Hd);
    return hip_err(hipGetLastError());
  }
  return hip_err(wide ? launch_wide_encode(h.dtype, h.ndim, A, stream) : launch_encode(h.dtype, h.ndim, A, stream));
}

// ---- scratch of the allocation-free encode: one copy per GPU, held until
// the process ends.  Host code never passes `scratch` itself to a kernel
// (on the host it names a stand-in, not device memory); it passes the
// device address hipGetSymbolAddress returns for the current device.
constexpr uint64_t NOALLOC_BYTES = APAX_NOALLOC_SCRATCH_BYTES;
__device__ __align__(256) uint8_t scratch[NOALLOC_BYTES];

constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// device address of the current device's scratch (looked up once per device)
int scratch_of_current_device(void** out) {
  int dev = -1;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= NOALLOC_MAX_DEVICES) return APAX_E_HIP;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return APAX_E_HIP;
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return APAX_OK;
}

// the encode's device status word as an APAX code, into the caller's word
__global__ void k_status_code(const uint32_t* status, int32_t* out) {
  if (threadIdx.x == 0) {
    const uint32_t st = *status;
    *out = (st & ST_NONFINITE) ? APAX_E_NONFINITE : ((st & ST_INTERNAL) ? APAX_E_INTERNAL : APAX_OK);
  }
}

}  // namespace

extern "C" {

int apax_encode(const void* d_x, const apax_params* p, void* d_stream, uint64_t cap,
                uint64_t* d_nbytes, void* d_ws, uint64_t ws_bytes, hipStream_t stream) {
  HG h;
  const bool profiled = p && p->code == APAX_CODE_PROFILED;
  int e;
  if (profiled && p->mode == APAX_ADAPTIVE_RATE) return APAX_E_UNSUPPORTED;  // needs its start code
  if (profiled) {
    apax_params q = *p;
    q.code = 0;  // placeholder; the kernels read the profiled code on the device
    e = setup(&q, h);
  } else {
    e = setup(p, h);
  }
  if (e) return e;
  if (!d_stream || !d_nbytes || !d_ws || (!d_x && h.nsamples)) return APAX_E_INVALID;
  if (((uintptr_t)d_stream & 15) || ((uintptr_t)d_ws & 15)) return APAX_E_INVALID;
  if (cap < bound_of(h)) return APAX_E_CAPACITY;
  if (ws_bytes < ws_need(h)) return APAX_E_CAPACITY;
  return encode_enqueue(d_x, p, h, profiled, d_stream, d_nbytes, d_ws, stream);
}

int apax_encode_noalloc(const void* d_x, const apax_params* p, void* d_stream, uint64_t cap,
                        uint64_t* d_nbytes, int32_t* d_status, hipStream_t stream) {
  if (p && p->code == APAX_CODE_PROFILED) return APAX_E_INVALID;  // no profile writes the scratch
  HG h;
  int e = setup(p, h);
  if (e) return e;
  if (!d_stream || !d_nbytes || (!d_x && h.nsamples)) return APAX_E_INVALID;
  if ((uintptr_t)d_stream & 15) return APAX_E_INVALID;
  if (cap < bound_of(h)) return APAX_E_CAPACITY;
  if (enc_need(h) > NOALLOC_BYTES) return APAX_E_CAPACITY;  // larger than the library's scratch
  void* ws = nullptr;
  if ((e = scratch_of_current_device(&ws))) return e;
  // the status word starts at zero (a fill kernel: no memset node if captured);
  // the superblock counts are reset by the encode's own first kernel
  clear_words((uint32_t*)ws, 1, stream);
  if ((e = hip_err(hipGetLastError()))) return e;
  if ((e = encode_enqueue(d_x, p, h, false, d_stream, d_nbytes, ws, stream))) return e;
  if (d_status) {
    hipLaunchKernelGGL(k_status_code, dim3(1), dim3(64), 0, stream, (const uint32_t*)ws, d_status);
    return hip_err(hipGetLastError());
  }
  return APAX_OK;
}

// Header checks and kernel arguments of a decode (no output pointer yet).
static int decode_setup(const void* h_hdr, const void* d_stream, uint64_t nbytes, void* d_ws, uint64_t ws_bytes,
                        HG& h, DecArgs& A) {
  apax_params p;
  int e = apax_stream_info(h_hdr, 64, &p);
  if (e) return e;
  uint16_t budget;
  memcpy(&budget, (const uint8_t*)h_hdr + 10, 2);
  e = setup(&p, h, header_budget(p.mode, budget));
  if (e) return e == APAX_E_UNSUPPORTED ? e : APAX_E_CORRUPT;
  if (!d_stream || !d_ws) return APAX_E_INVALID;
  if (((uintptr_t)d_stream & 15) || ((uintptr_t)d_ws & 15)) return APAX_E_INVALID;
  if (ws_bytes < ws_need(h)) return APAX_E_CAPACITY;
  uint64_t pw;
  memcpy(&pw, (const uint8_t*)h_hdr + 56, 8);
  uint64_t area = area_offset(h);
  if (h.mode == APAX_FIXED_RATE && pw != (uint64_t)h.g.budget * (uint64_t)h.g.nblocks) return APAX_E_CORRUPT;
  if (nbytes < area || (nbytes - area) / 4 < pw) return APAX_E_CORRUPT;
  memset(&A, 0, sizeof(A));
  A.g = h.g;
  A.in = (const uint8_t*)d_stream;
  A.words = (const uint32_t*)((const uint8_t*)d_stream + area);
  A.lens = (const uint16_t*)((const uint8_t*)d_stream + 64);
  A.sbo = (const uint64_t*)((const uint8_t*)d_stream + 64 + lens_bytes(h));
  A.status = &((PState*)d_ws)->status;
  A.payload_words = pw;
  memcpy(A.hdr, h_hdr, 64);
  return APAX_OK;
}

int apax_decode(const void* h_hdr, const void* d_stream, uint64_t nbytes, void* d_y, uint64_t cap,
                void* d_ws, uint64_t ws_bytes, hipStream_t stream) {
  HG h;
  DecArgs A;
  int e = decode_setup(h_hdr, d_stream, nbytes, d_ws, ws_bytes, h, A);
  if (e) return e;
  if (!d_y && h.nsamples) return APAX_E_INVALID;
  if (cap < h.nsamples * (uint64_t)h.esz) return APAX_E_CAPACITY;
  A.y = d_y;
  if (h.g.G > 64 || h.g.gq == 2) {
    if (h.g.nblocks && !wide_fits(h.g)) return APAX_E_UNSUPPORTED;
    return hip_err(launch_wide_decode(h.dtype, h.ndim, A, stream));
  }
  return hip_err(launch_decode(h.dtype, h.ndim, A, stream));
}

int apax_decode_dot(const void* h_hdr, const void* d_stream, uint64_t nbytes, const void* d_w, double* d_out,
                    void* d_ws, uint64_t ws_bytes, hipStream_t stream) {
  HG h;
  DecArgs A;
  int e = decode_setup(h_hdr, d_stream, nbytes, d_ws, ws_bytes, h, A);
  if (e) return e;
  if (!d_out || (!d_w && h.nsamples)) return APAX_E_INVALID;
  if (h.g.nblocks == 0) {
    hipLaunchKernelGGL(k_clear, dim3(1), dim3(64), 0, stream, (uint32_t*)d_out, 2);
    return hip_err(hipGetLastError());
  }
  if (h.g.G > 64 || h.g.gq == 2) {
    if (!wide_fits(h.g)) return APAX_E_UNSUPPORTED;
    return hip_err(launch_wide_decode_dot(h.dtype, h.ndim, A, d_w, (double*)partials_ptr(d_ws, h), d_out, stream));
  }
  return hip_err(launch_decode_dot(h.dtype, h.ndim, A, d_w, (double*)partials_ptr(d_ws, h), d_out, stream));
}

int apax_dot(const void* d_x, const void* d_w, uint32_t dtype, uint64_t n, double* d_out, void* d_ws,
             uint64_t ws_bytes, hipStream_t stream) {
  if (dtype < APAX_I8 || dtype > APAX_F64 || !d_out || !d_ws || (n && (!d_x || !d_w))) return APAX_E_INVALID;
  if (ws_bytes < APAX_DOT_WGS * 8) return APAX_E_CAPACITY;
  if (n == 0) {
    hipLaunchKernelGGL(k_clear, dim3(1), dim3(64), 0, stream, (uint32_t*)d_out, 2);
    return hip_err(hipGetLastError());
  }
  return hip_err(launch_dot_plain((int)dtype, d_x, d_w, (int64_t)n, (double*)d_ws, APAX_DOT_WGS, d_out, stream));
}

// Subsample of the profiler's statistics passes: every 16th block once the
// array has 1024 blocks, else every block.
static int64_t sub_count(const Geo& g, int64_t* stride = nullptr) {
  const int64_t sub_stride = g.nblocks >= 1024 ? 16 : 1;
  if (stride) *stride = sub_stride;
  return (g.nblocks + sub_stride - 1) / sub_stride;
}

static int profile_setup(const void* d_x, const apax_params* p, const void* d_ws, uint64_t ws_bytes, HG& h) {
  if (!p) return APAX_E_INVALID;
  apax_params q = *p;
  q.code = 0;
  int e = setup(&q, h);
  if (e) return e;
  // blocks of more than 64 groups (or groups of 8) take one workgroup each,
  // staged in LDS beside the wave partials of the pass
  if ((h.g.G > 64 || h.g.gq == 2) && h.g.nblocks && !wide_fits(h.g, 2048)) return APAX_E_UNSUPPORTED;
  if (h.mode == APAX_ADAPTIVE_RATE) return APAX_E_UNSUPPORTED;  // the loop sets its own codes
  if (!d_ws || (!d_x && h.nsamples)) return APAX_E_INVALID;
  if ((uintptr_t)d_ws & 15) return APAX_E_INVALID;
  if (ws_bytes < ws_need(h)) return APAX_E_CAPACITY;
  return APAX_OK;
}

// The whole profile as one asynchronous launch sequence on `stream`; its
// result stays in the workspace's PState.
// ev (optional): 2 * APAX_NPASS events, a pair around the kernel of each
// pass that runs (bit of *ran set)
// enc (optional): an encode of the same array at the profiled operating
// point, enqueued right after the metrics pass from that pass's per-block
// results (the encoder's own per-block search and stream choice, run there);
// `encoded` is recorded once it is complete, before the centred and curve
// passes.  side (optional, with the event `forked`): the curve pass runs on
// `side` from the end of the histogram pass on (beside the metrics pass),
// and the centred pass there once the metrics pass is done (beside the
// encode on `stream`).
static int profile_enqueue(const void* d_x, const apax_params* p, const HG& h, void* d_ws, hipStream_t stream,
                           hipEvent_t* ev = nullptr, uint32_t* ran = nullptr,
                           hipEvent_t point_ready = nullptr, EncArgs* enc = nullptr,
                           hipEvent_t encoded = nullptr, hipStream_t side = nullptr,
                           hipEvent_t forked = nullptr) {
  int e;
  hipStream_t ps = stream;  // the stream of the passes still to come
  if (ran) *ran = 0;
  auto pair = [&](int pass) -> hipEvent_t* {
    if (!ev) return nullptr;
    *ran |= 1u << pass;
    return ev + 2 * pass;
  };
  const Geo& g = h.g;
  PState* st = (PState*)d_ws;
  int64_t sub_stride;
  const int64_t sub_n = sub_count(g, &sub_stride);
  const int rule = h.mode == APAX_LOSSLESS ? R_LOSSLESS : (h.mode == APAX_FIXED_RATE ? R_RATE : R_QUALITY);
  const bool fr = h.mode == APAX_FIXED_RATE;
  const uint64_t in_bytes = h.nsamples * (uint64_t)h.esz;
  // bisection batches: each probe launch evaluates the decision tree of the
  // next `depth` steps; fixed quality re-reads the whole array per code, so
  // it evaluates one code per launch once the array outgrows the last-level cache
  const int depth = fr ? 3 : (in_bytes <= (96ull << 20) ? 3 : 1);
  // c_cap - c_floor <= 512 (the gain grid spans 2^32 in 512 codes), so the
  // bisection takes at most 9 steps after the first probe at c_cap
  const int nbatch = (9 + depth - 1) / depth;
  const int tree_n = (1 << depth) - 1 + 1;

  CtlArgs C;
  memset(&C, 0, sizeof(C));
  C.st = st;
  C.mode = h.mode;
  C.isint = h.isint;
  C.depth = depth;
  C.cmin = g.cmin;
  C.cmax = g.cmax;
  C.mask_user = g.mask;
  C.nsub = (uint64_t)sub_n;
  C.nsamples = h.nsamples;
  C.target = p->target_corr;
  auto ctl = [&](int step) { C.step = step; return hip_err(launch_ctl(C, ps)); };
  // one pass over blocks; its last workgroup reduces and runs control step `next`
  auto run = [&](int op, int rl, int mask_sel, bool sub, int maxcodes, int next, int flags, int pass) -> int {
    ProfArgs A;
    memset(&A, 0, sizeof(A));
    A.x = d_x;
    A.st = st;
    A.g = g;
    A.op = op;
    A.rule = rl;
    A.mask_sel = mask_sel;
    A.jstride = sub ? sub_stride : 1;
    A.nbe = sub ? sub_n : g.nblocks;
    A.maxcodes = maxcodes;
    A.parts = (flags & 32) ? partials2_ptr(d_ws, h) : partials_ptr(d_ws, h);
    A.cj = cj_ptr(d_ws, h);
    A.hist = (flags & 1) != 0;
    A.final_code = (flags & 2) != 0;
    A.curve = (flags & 4) != 0;
    A.store_cj = (flags & 8) != 0;
    if ((flags & 16) && enc) {
      A.bst = enc->bst;
      A.lens = enc->lens;
      A.ssum = enc->ssum;
      if (fr) {  // fixed rate: the pass writes the blocks too (no stream choice to hand over)
        A.enc_words = enc->out_words;
        A.bst = nullptr;
      }
    }
    A.C = C;
    A.C.step = next;
    // F_SPLIT: the reduce on `side`, forked after the pass kernel
    return hip_err(launch_profile(h.dtype, h.ndim, A, ps, pair(pass), (flags & 64) ? side : nullptr, forked));
  };
  // F_PARTS2: the second partial-record region (a pass beside another)
  enum { F_HIST = 1, F_FINAL = 2, F_CURVE = 4, F_STORE = 8, F_ENC = 16, F_PARTS2 = 32, F_SPLIT = 64 };

  // whole profile, asynchronously: clear, max |x| (-> bracket), bisection
  // batches, histogram at the chosen code (-> mask, curve codes), curve
  // (-> metrics set-up), metrics (-> means), centred metrics; one read-back
  hipLaunchKernelGGL(k_clear, dim3((unsigned)((sizeof(PState) / 4 + 255) / 256)), dim3(256), 0,
                     stream, (uint32_t*)st, (int)(sizeof(PState) / 4));
  if ((e = hip_err(hipGetLastError()))) return e;
  if (g.nblocks) {
    C.step = C_INIT;
    if ((e = hip_err(launch_pmax(h.dtype, d_x, h.nsamples, partials_ptr(d_ws, h), C, stream,
                                 pair(APAX_PASS_MAX)))))
      return e;
    for (int b = 0; b < nbatch && (fr || h.mode == APAX_FIXED_QUALITY); b++) {
      if (fr) e = run(P_FITS, R_RATE, 0, true, tree_n, C_DECIDE, 0, APAX_PASS_PROBE0 + b);
      else e = run(P_STATS, R_QUALITY, 0, false, tree_n, C_DECIDE, 0, APAX_PASS_PROBE0 + b);
      if (e) return e;
    }
    if ((e = run(P_FITS, rule, 0, true, 1, C_CURVE, F_HIST | F_FINAL, APAX_PASS_HIST))) return e;
    if (point_ready && hipEventRecord(point_ready, stream) != hipSuccess) return APAX_E_HIP;
    // side stream: `side` forks here and runs the curve (its codes are set)
    // beside the metrics pass, with its own partial records; the two
    // passes' reduce kernels change different fields of the state and write
    // back only those
    auto fork = [&]() -> int {
      if (hipEventRecord(forked, stream) != hipSuccess || hipStreamWaitEvent(side, forked, 0) != hipSuccess)
        return APAX_E_HIP;
      return APAX_OK;
    };
    if (side) {
      if ((e = fork())) return e;
      ps = side;
      if ((e = run(P_STATS, R_QUALITY, 1, true, NCURVE, C_KEEP_CURVE, F_CURVE | F_PARTS2, APAX_PASS_CURVE)))
        return e;
      ps = stream;
    }
    // metrics at the operating point (fixed rate: each block's code kept
    // for the centred pass), then the encode that may follow it (it reads
    // the per-block codes and streams the pass stored and the operating point
    // the histogram's control step set, nothing of the metrics' reduce), the
    // centred sums and, without a side stream, the curve.  With a side
    // stream and an encode, `side` forks once the metrics pass kernel is
    // done and runs its reduce (means) and the centred pass beside the
    // encode; that reduce writes back only the state words it changed, none
    // of which the encode reads
    if (enc && !fr) launch_encode_reset(enc->ssum, (g.nblocks + 63) / 64, stream);
    // fixed rate: the stream header now (the operating point is set), the
    // blocks from the metrics pass itself
    if (enc && fr && (e = hip_err(launch_encode_header(*enc, stream)))) return e;
    const int split = side && enc ? F_SPLIT : 0;
    if ((e = run(P_STATS, rule, 2, false, 1, C_MEANS, F_FINAL | F_STORE | F_ENC | split, APAX_PASS_METRICS)))
      return e;
    if (side) {
      if (!split && (e = fork())) return e;
      ps = side;
    }
    if (enc) {
      if (!fr && (e = hip_err(launch_encode_profiled(h.dtype, h.ndim, *enc, cj_ptr(d_ws, h), stream)))) return e;
      if (encoded && hipEventRecord(encoded, stream) != hipSuccess) return APAX_E_HIP;
    }
    if ((e = run(P_CENTER, rule, 2, false, 1, C_NONE, F_FINAL, APAX_PASS_CENTRED))) return e;
    if (!side && (e = run(P_STATS, R_QUALITY, 1, true, NCURVE, C_KEEP_CURVE, F_CURVE, APAX_PASS_CURVE))) return e;
  } else {
    if ((e = ctl(C_INIT))) return e;
    if ((e = ctl(C_MASK))) return e;
    if ((e = ctl(C_CURVE))) return e;
    if (point_ready && hipEventRecord(point_ready, stream) != hipSuccess) return APAX_E_HIP;
  }
  return APAX_OK;
}

// Result record of a finished profile from the host copy of its PState.
static int profile_finish(const HG& h, const PState& hs, apax_profile_result* out) {
  memset(out, 0, sizeof(*out));
  out->size = sizeof(*out);
  const Geo& g = h.g;
  const bool fr = h.mode == APAX_FIXED_RATE;
  out->n_sub = (uint32_t)sub_count(g);
  if (hs.status & ST_NONFINITE) return APAX_E_NONFINITE;
  if (hs.status & ST_INTERNAL) return APAX_E_INTERNAL;

  out->c_floor = hs.cf;
  out->c_cap = hs.cc;
  out->code = hs.code;
  out->flags = (uint32_t)hs.flags;
  out->n_probes = (uint32_t)hs.n_probes;
  out->stream_mask = hs.mask_out;
  const int es = hs.escale;
  auto unscale = [&](double v, int i) { return ldexp(v, i >= S_XX ? 2 * es : es); };
  const double in_bits = (double)hs.sub_samples * 8.0 * h.esz;  // counted by the histogram pass
  for (int t = 0; t < APAX_NCURVE; t++) {
    out->curve[t].code = hs.curve_codes[t];
    double r = 1.0, omr = 0.0, ob = 0.0;
    if (g.nblocks) {
      r_of(hs.curve_sums[t][0], hs.curve_sums[t][1], hs.curve_sums[t][2], hs.curve_sums[t][3], r, omr);
      ob = 32.0 * (double)hs.curve_words[t];
    }
    out->curve[t].ratio = ob > 0 ? in_bits / ob : 0.0;
    out->curve[t].r = r;
  }
  apax_metrics& m = out->m;
  m.n = h.nsamples;
  if (g.nblocks) {
    m.sum_x = unscale(hs.msums[S_X], S_X);
    m.sum_y = unscale(hs.msums[S_Y], S_Y);
    m.sum_d = unscale(hs.msums[S_D], S_D);
    m.sxx = unscale(hs.msums[S_XX], S_XX);
    m.syy = unscale(hs.msums[S_YY], S_YY);
    m.sdd = unscale(hs.msums[S_DD], S_DD);
    m.sds = unscale(hs.msums[S_DS], S_DS);
    memcpy(&m.max_abs_d, &hs.maxbits[1], 8);
  }
  r_of(m.sxx, m.syy, m.sdd, m.sds, m.r, m.one_minus_r);
  if (m.sdd == 0.0) { m.snr_db = INFINITY; m.rms_pct = 0.0; m.rms_db = -INFINITY; }
  else if (m.sxx == 0.0) { m.snr_db = -INFINITY; m.rms_pct = INFINITY; m.rms_db = INFINITY; }
  else {
    m.snr_db = 10.0 * log10(m.sxx / m.sdd);
    m.rms_pct = 100.0 * sqrt(m.sdd / m.sxx);
    m.rms_db = -m.snr_db;
  }
  double nn = (double)(m.n ? m.n : 1);
  m.mean_x = m.sum_x / nn;
  m.mean_y = m.sum_y / nn;
  m.mean_d = m.sum_d / nn;
  m.enc_bytes = area_offset(h) + 4 * (fr ? (uint64_t)g.budget * (uint64_t)g.nblocks : hs.mwords);
  m.ratio = m.enc_bytes ? (double)(h.nsamples * (uint64_t)h.esz) / (double)m.enc_bytes : 0.0;
  if (g.nblocks) {
    m.std_x = sqrt(unscale(hs.sums[0][S_CXX], S_CXX) / nn);
    m.std_y = sqrt(unscale(hs.sums[0][S_CYY], S_CYY) / nn);
    m.std_d = sqrt(unscale(hs.sums[0][S_CDD], S_CDD) / nn);
  }
  return APAX_OK;
}

int apax_profile(const void* d_x, const apax_params* p, apax_profile_result* out, void* d_ws,
                 uint64_t ws_bytes, hipStream_t stream) {
  if (!out) return APAX_E_INVALID;
  HG h;
  int e = profile_setup(d_x, p, d_ws, ws_bytes, h);
  if (e) return e;
  if ((e = profile_enqueue(d_x, p, h, d_ws, stream))) return e;
  return apax_profile_read(p, out, d_ws, stream);
}

// A profile (and, with enc, the encode at its point) with HIP events around
// each pass kernel; synchronous.
static int profile_timed(const void* d_x, const apax_params* p, const HG& h, void* d_ws, hipStream_t stream,
                         EncArgs* enc, apax_profile_result* out, float* pass_ms) {
  int e = 0;
  hipEvent_t ev[2 * APAX_NPASS];
  int made = 0;
  for (; made < 2 * APAX_NPASS; made++)
    if (hipEventCreate(&ev[made]) != hipSuccess) break;
  uint32_t ran = 0;
  if (made < 2 * APAX_NPASS) e = APAX_E_HIP;
  if (!e) e = profile_enqueue(d_x, p, h, d_ws, stream, ev, &ran, nullptr, enc);
  if (!e) e = apax_profile_read(p, out, d_ws, stream);  // waits for the stream
  for (int i = 0; i < APAX_NPASS; i++) {
    pass_ms[i] = -1.0f;
    if (!e && ((ran >> i) & 1) && hipEventElapsedTime(&pass_ms[i], ev[2 * i], ev[2 * i + 1]) != hipSuccess)
      e = APAX_E_HIP;
  }
  for (int i = 0; i < made; i++) (void)hipEventDestroy(ev[i]);
  return e;
}

int apax_profile_timed(const void* d_x, const apax_params* p, apax_profile_result* out,
                       float* pass_ms, void* d_ws, uint64_t ws_bytes, hipStream_t stream) {
  if (!out || !pass_ms) return APAX_E_INVALID;
  HG h;
  int e = profile_setup(d_x, p, d_ws, ws_bytes, h);
  if (e) return e;
  return profile_timed(d_x, p, h, d_ws, stream, nullptr, out, pass_ms);
}

int apax_profile_encode_timed(const void* d_x, const apax_params* p, apax_profile_result* out, float* pass_ms,
                              void* d_ws, uint64_t ws_bytes, void* d_stream, uint64_t cap, uint64_t* d_nbytes,
                              hipStream_t stream) {
  if (!out || !pass_ms) return APAX_E_INVALID;
  HG h;
  int e = profile_setup(d_x, p, d_ws, ws_bytes, h);
  if (e) return e;
  if (!d_stream || !d_nbytes || ((uintptr_t)d_stream & 15)) return APAX_E_INVALID;
  if (cap < bound_of(h)) return APAX_E_CAPACITY;
  if (h.lagged || h.g.nblocks == 0 || h.g.G > 64 || h.g.gq == 2) return APAX_E_UNSUPPORTED;
  apax_params q = *p;
  q.code = 0;
  EncArgs A;
  enc_args(d_x, &q, h, true, d_stream, d_nbytes, d_ws, A);
  return profile_timed(d_x, p, h, d_ws, stream, &A, out, pass_ms);
}

int apax_s2r_margin(const void* d_x, const apax_params* p, double* h_ratio, double* h_db, void* d_ws,
                    uint64_t ws_bytes, hipStream_t stream) {
  if (!h_ratio || !h_db) return APAX_E_INVALID;
  HG h;
  int e = profile_setup(d_x, p, d_ws, ws_bytes, h);
  if (e) return e;
  // one workgroup per block: the block in LDS beside the digit histogram
  if ((h.g.G > 64 || h.g.gq == 2) && h.g.nblocks && !wide_fits(h.g, S2R_HIST_BYTES + 256))
    return APAX_E_UNSUPPORTED;
  *h_ratio = NAN;
  *h_db = NAN;
  if (h.nsamples == 0) return APAX_OK;
  S2RArgs A;
  memset(&A, 0, sizeof(A));
  A.x = d_x;
  A.st = (PState*)d_ws;
  A.cj = cj_ptr(d_ws, h);
  // the profile's partial records are spent: 8192 bins, the kept-key count,
  // then as many kept keys as the rest of the region holds
  uint8_t* part = (uint8_t*)partials_ptr(d_ws, h);
  A.hist = (uint32_t*)part;
  A.ncand = (uint64_t*)(part + S2R_HIST_BYTES);
  A.cand = (uint64_t*)(part + S2R_HIST_BYTES + 256);
  const uint64_t region = partial_bytes(h);
  A.cand_cap = region > S2R_HIST_BYTES + 256 ? (region - S2R_HIST_BYTES - 256) / 8 : 0;
  A.rule = h.mode == APAX_LOSSLESS ? R_LOSSLESS : (h.mode == APAX_FIXED_RATE ? R_RATE : R_QUALITY);
  A.g = h.g;
  const uint64_t rank = (45 * h.nsamples + 999) / 1000;  // ceil(0.045 n), n >= 1
  if ((e = hip_err(launch_s2r(h.dtype, h.ndim, A, rank, stream)))) return e;
  PState hs;
  if (hipMemcpyAsync(&hs, d_ws, sizeof(PState), hipMemcpyDeviceToHost, stream) != hipSuccess) return APAX_E_HIP;
  if (hipStreamSynchronize(stream) != hipSuccess) return APAX_E_HIP;
  if (hs.status & ST_NONFINITE) return APAX_E_NONFINITE;
  if (hs.status & ST_INTERNAL) return APAX_E_INTERNAL;
  double r;
  memcpy(&r, &hs.s2r_prefix, 8);
  *h_ratio = r;
  *h_db = r == 0.0 ? -INFINITY : (isinf(r) ? INFINITY : 20.0 * log10(r));
  return APAX_OK;
}

// Spectral workspace: window and twiddle table, PSD partials and sums, then
// the monitor's autocorrelation partials, sums and end samples.
static constexpr uint64_t SPEC_TABLE = 8 * 1024 + 16 * 1024;
static constexpr uint64_t SPEC_PSD_OUT = SPEC_TABLE + (uint64_t)PSD_MAX_WGS * 3 * 512 * 8;
static constexpr uint64_t SPEC_ACF = SPEC_PSD_OUT + 3 * 512 * 8;
static constexpr uint64_t SPEC_ACF_OUT = SPEC_ACF + (uint64_t)ACF_MAX_WGS * (ACF_LAGS + 1) * 8;
static constexpr uint64_t SPEC_ENDS = SPEC_ACF_OUT + 256;
static constexpr uint64_t SPEC_BYTES = SPEC_ENDS + 256;

uint64_t apax_spectral_workspace_bytes(void) { return SPEC_BYTES; }

// The Hann window and the twiddles, written into d_ws on the stream.
static int spectral_tables(uint8_t* w, hipStream_t stream) {
  return hip_err(launch_psd_tables((double*)w, stream));
}

int apax_spectral_metrics(const void* d_x, const void* d_y, uint32_t dtype, uint64_t n, apax_spectral* out,
                          void* d_ws, uint64_t ws_bytes, hipStream_t stream) {
  if (!out || dtype < APAX_I8 || dtype > APAX_F64) return APAX_E_INVALID;
  memset(out, 0, sizeof(*out));
  const double nan = NAN;
  double* fields[10] = {&out->peak_x, &out->floor_x, &out->peak_y, &out->floor_y, &out->peak_d,
                        &out->floor_d, &out->resid_mean, &out->dr, &out->srr, &out->fft_s2r_margin};
  for (double* f : fields) *f = nan;
  if (n < 1024) return APAX_OK;
  if (!d_x || !d_y || !d_ws) return APAX_E_INVALID;
  if (((uintptr_t)d_ws & 15) || ws_bytes < apax_spectral_workspace_bytes()) return APAX_E_CAPACITY;
  const uint64_t K = 1 + (n - 1024) / 512;
  uint8_t* w = (uint8_t*)d_ws;
  int e = spectral_tables(w, stream);
  if (e) return e;
  PsdArgs A;
  A.x = d_x;
  A.y = d_y;
  A.window = (const double*)w;
  A.twiddle = w + 8 * 1024;
  A.partial = (double*)(w + SPEC_TABLE);
  A.out = (double*)(w + SPEC_PSD_OUT);
  A.segments = (int64_t)K;
  A.nsig = 3;
  A.pad = 0;
  e = hip_err(launch_psd((int)dtype, A, stream));
  if (e) return e;
  double P[3 * 512];
  if (hipMemcpyAsync(P, A.out, sizeof(P), hipMemcpyDeviceToHost, stream) != hipSuccess) return APAX_E_HIP;
  if (hipStreamSynchronize(stream) != hipSuccess) return APAX_E_HIP;
  auto db = [](double v) { return v > 0.0 ? 10.0 * log10(v) : -INFINITY; };
  double peak[3], floor_[3], mean_d = 0.0;
  for (int s = 0; s < 3; s++) {
    double v[512];
    for (int f = 0; f < 512; f++) v[f] = P[s * 512 + f] / (double)K;
    double mx = v[0];
    for (int f = 1; f < 512; f++) mx = v[f] > mx ? v[f] : mx;
    if (s == 2) {
      double sum = 0.0;
      for (int f = 0; f < 512; f++) sum += v[f];
      mean_d = sum / 512.0;
    }
    std::nth_element(v, v + 255, v + 512);  // nearest-rank median: the 256th smallest
    peak[s] = db(mx);
    floor_[s] = db(v[255]);
  }
  out->segments = K;
  out->peak_x = peak[0];
  out->floor_x = floor_[0];
  out->peak_y = peak[1];
  out->floor_y = floor_[1];
  out->peak_d = peak[2];
  out->floor_d = floor_[2];
  out->resid_mean = db(mean_d);
  out->dr = out->peak_x - out->floor_x;
  out->srr = out->peak_x - out->resid_mean;
  out->fft_s2r_margin = out->floor_x - out->resid_mean;
  return APAX_OK;
}

// Sec. 6 signal monitor.  The lag sums and the spectrum run on the device;
// the host assembles the scalars from the 512 bins, the 17 sums and the 32
// end samples.
int apax_signal_monitor(const void* d_x, uint32_t dtype, uint64_t n, apax_monitor* out, void* d_ws,
                        uint64_t ws_bytes, hipStream_t stream) {
  if (!out || dtype < APAX_I8 || dtype > APAX_F64) return APAX_E_INVALID;
  memset(out, 0, sizeof(*out));
  out->center_freq = out->peak_db = out->floor_db = out->snr_db = out->gain_db = NAN;
  if (n == 0) return APAX_OK;
  if (!d_x || !d_ws) return APAX_E_INVALID;
  if (((uintptr_t)d_ws & 15) || ws_bytes < SPEC_BYTES) return APAX_E_CAPACITY;
  uint8_t* w = (uint8_t*)d_ws;
  AcfArgs C;
  C.x = d_x;
  C.n = (int64_t)n;
  C.partial = (double*)(w + SPEC_ACF);
  C.out = (double*)(w + SPEC_ACF_OUT);
  C.ends = (double*)(w + SPEC_ENDS);
  int e = hip_err(launch_acf((int)dtype, C, stream));
  if (e) return e;
  double R[ACF_LAGS + 1], ends[2 * ACF_LAGS];
  if (hipMemcpyAsync(R, C.out, sizeof(R), hipMemcpyDeviceToHost, stream) != hipSuccess) return APAX_E_HIP;
  if (hipMemcpyAsync(ends, C.ends, sizeof(ends), hipMemcpyDeviceToHost, stream) != hipSuccess) return APAX_E_HIP;
  uint64_t K = 0;
  double P[512];
  if (n >= 1024) {
    K = 1 + (n - 1024) / 512;
    e = spectral_tables(w, stream);
    if (e) return e;
    PsdArgs A;
    A.x = d_x;
    A.y = d_x;
    A.window = (const double*)w;
    A.twiddle = w + 8 * 1024;
    A.partial = (double*)(w + SPEC_TABLE);
    A.out = (double*)(w + SPEC_PSD_OUT);
    A.segments = (int64_t)K;
    A.nsig = 1;
    A.pad = 0;
    e = hip_err(launch_psd((int)dtype, A, stream));
    if (e) return e;
    if (hipMemcpyAsync(P, A.out, sizeof(P), hipMemcpyDeviceToHost, stream) != hipSuccess) return APAX_E_HIP;
  }
  if (hipStreamSynchronize(stream) != hipSuccess) return APAX_E_HIP;
  // acf[k] = (R[k] / (n - k)) / (R[0] / n) for the lags the array has
  if (R[0] > 0.0)
    for (uint64_t k = 0; k <= ACF_LAGS && k < n; k++) out->acf[k] = (R[k] / (double)(n - k)) / (R[0] / (double)n);
  if (n < 1024) return APAX_OK;
  auto db = [](double v) { return v > 0.0 ? 10.0 * log10(v) : -INFINITY; };
  double v[512], sum = 0.0;
  int b = 1;
  for (int f = 0; f < 512; f++) {
    v[f] = P[f] / (double)K;
    if (v[f] > v[b - 1]) b = f + 1;  // the first largest bin
    sum += v[f];
  }
  const double peak = v[b - 1];
  std::nth_element(v, v + 255, v + 512);  // nearest-rank median: the 256th smallest
  out->segments = K;
  out->peak_bin = b;
  out->center_freq = b / 1024.0;
  out->peak_db = db(peak);
  out->floor_db = db(v[255]);
  out->snr_db = db(sum / 512.0) - out->floor_db;
  // the lag whose phase at bin b lies nearest a multiple of half a turn
  int k = 1, dist = 1024;
  for (int j = 1; j <= ACF_LAGS; j++) {
    const int r = (b * j) & 511, d = r < 512 - r ? r : 512 - r;
    if (d < dist) dist = d, k = j;
  }
  const int m = (b * k) & 1023;
  const int sg = (m <= 256 || m >= 768) ? 1 : -1;
  out->stride = k;
  out->sign = sg;
  // energy in: sum_{i >= k} x_i^2 = R0 - head; energy out: the filtered
  // samples' squares summed directly on the device
  double head = 0.0;
  for (int j = 0; j < k; j++) head += ends[j] * ends[j];
  const double e_in = R[0] - head;
  double* d_eout = C.out + (ACF_LAGS + 1);
  e = hip_err(launch_resid((int)dtype, d_x, (int64_t)n, k, sg, C.partial, d_eout, stream));
  if (e) return e;
  double e_out = 0.0;
  if (hipMemcpyAsync(&e_out, d_eout, sizeof(double), hipMemcpyDeviceToHost, stream) != hipSuccess) return APAX_E_HIP;
  if (hipStreamSynchronize(stream) != hipSuccess) return APAX_E_HIP;
  out->gain_db = db(e_in) - db(e_out);
  return APAX_OK;
}

int apax_profile_async(const void* d_x, const apax_params* p, void* d_ws, uint64_t ws_bytes,
                       hipStream_t stream) {
  HG h;
  int e = profile_setup(d_x, p, d_ws, ws_bytes, h);
  if (e) return e;
  return profile_enqueue(d_x, p, h, d_ws, stream);
}

int apax_profile_async_point(const void* d_x, const apax_params* p, void* d_ws, uint64_t ws_bytes,
                             hipStream_t stream, hipEvent_t point_ready) {
  if (!point_ready) return APAX_E_INVALID;
  HG h;
  int e = profile_setup(d_x, p, d_ws, ws_bytes, h);
  if (e) return e;
  return profile_enqueue(d_x, p, h, d_ws, stream, nullptr, nullptr, point_ready);
}

int apax_profile_encode_async(const void* d_x, const apax_params* p, void* d_ws, uint64_t ws_bytes,
                              void* d_stream, uint64_t cap, uint64_t* d_nbytes, hipStream_t stream,
                              hipEvent_t encoded, hipStream_t side, hipEvent_t forked) {
  HG h;
  int e = profile_setup(d_x, p, d_ws, ws_bytes, h);
  if (e) return e;
  if (!d_stream || !d_nbytes || ((uintptr_t)d_stream & 15)) return APAX_E_INVALID;
  if (side && (!forked || side == stream)) return APAX_E_INVALID;
  if (cap < bound_of(h)) return APAX_E_CAPACITY;
  apax_params q = *p;
  q.code = 0;  // the header's code and mask are the profile's, written on the device
  if (h.lagged || h.g.nblocks == 0 || h.g.G > 64 || h.g.gq == 2) {
    // the lagged choice codes block j with block j-1's stream, which the
    // metrics pass does not record, and the one-workgroup-per-block passes
    // record no per-block choices: the profile, then the plain encode
    if ((e = profile_enqueue(d_x, p, h, d_ws, stream))) return e;
    if ((e = encode_enqueue(d_x, &q, h, true, d_stream, d_nbytes, d_ws, stream))) return e;
    if (encoded && hipEventRecord(encoded, stream) != hipSuccess) return APAX_E_HIP;
    return APAX_OK;
  }
  EncArgs A;
  enc_args(d_x, &q, h, true, d_stream, d_nbytes, d_ws, A);
  return profile_enqueue(d_x, p, h, d_ws, stream, nullptr, nullptr, nullptr, &A, encoded, side, forked);
}

int apax_adopt_point(const void* d_ws_from, void* d_ws_to, hipStream_t stream) {
  if (!d_ws_from || !d_ws_to) return APAX_E_INVALID;
  hipLaunchKernelGGL(k_adopt_point, dim3(1), dim3(64), 0, stream, (const PState*)d_ws_from, (PState*)d_ws_to);
  return hip_err(hipGetLastError());
}

int apax_profile_read(const apax_params* p, apax_profile_result* out, const void* d_ws,
                        hipStream_t stream) {
  if (!p || !out || !d_ws) return APAX_E_INVALID;
  apax_params q = *p;
  q.code = 0;
  HG h;
  int e = setup(&q, h);
  if (e) return e;
  PState hs;
  if (hipMemcpyAsync(&hs, d_ws, sizeof(PState), hipMemcpyDeviceToHost, stream) != hipSuccess) return APAX_E_HIP;
  if (hipStreamSynchronize(stream) != hipSuccess) return APAX_E_HIP;
  return profile_finish(h, hs, out);
}

static int batch_error(int e, uint32_t i) { (void)i; return e; }

int apax_batch_create(int op, const apax_batch_item* h_items, uint32_t n, const apax_tune* tune,
                      apax_batch** out, uint64_t* ws_bytes) {
  if (!out || !ws_bytes || (n && !h_items) || (op != APAX_OP_ENCODE && op != APAX_OP_DECODE))
    return APAX_E_INVALID;
  *out = nullptr;
  apax_tune t = tune ? *tune : apax_tune{};
  if (t.waves_per_wg == 0) t.waves_per_wg = 4;
  if (t.wgs_per_cu == 0) t.wgs_per_cu = 8;
  if (t.tiles_per_ticket == 0) t.tiles_per_ticket = RUN;
  if ((t.waves_per_wg != 2 && t.waves_per_wg != 4 && t.waves_per_wg != 8) || t.wgs_per_cu > 64 ||
      t.tiles_per_ticket > 64)
    return APAX_E_INVALID;
  apax_batch* b = new apax_batch();
  b->op = op;
  b->tune = t;
  b->items.assign(h_items, h_items + n);
  b->geo.resize(n);
  for (uint32_t i = 0; i < n; i++) {
    const apax_batch_item& it = h_items[i];
    HG& h = b->geo[i];
    int e;
    if (op == APAX_OP_ENCODE) {
      if ((e = setup(&it.p, h))) { delete b; return batch_error(e, i); }
      if (!it.d_out || !it.d_nbytes || (!it.d_in && h.nsamples) || ((uintptr_t)it.d_out & 15)) {
        delete b;
        return batch_error(APAX_E_INVALID, i);
      }
      if (it.cap < bound_of(h)) { delete b; return batch_error(APAX_E_CAPACITY, i); }
      if (h.lagged || h.mode == APAX_ADAPTIVE_RATE || h.g.G > 64 || h.g.gq == 2) {
        if ((h.g.G > 64 || h.g.gq == 2) && h.g.nblocks && !wide_fits(h.g)) {
          delete b;
          return batch_error(APAX_E_UNSUPPORTED, i);
        }
        b->solo.push_back(i);
        b->solo_hdr.push_back({});
        continue;
      }
    } else {
      apax_params q;
      if (!it.h_hdr || (e = apax_stream_info(it.h_hdr, 64, &q))) { delete b; return batch_error(APAX_E_CORRUPT, i); }
      uint16_t budget;
      memcpy(&budget, (const uint8_t*)it.h_hdr + 10, 2);
      if ((e = setup(&q, h, header_budget(q.mode, budget)))) { delete b; return batch_error(e, i); }
      uint64_t pw;
      memcpy(&pw, (const uint8_t*)it.h_hdr + 56, 8);
      uint64_t area = area_offset(h);
      if (!it.d_in || ((uintptr_t)it.d_in & 15) || (!it.d_out && h.nsamples)) { delete b; return batch_error(APAX_E_INVALID, i); }
      if (it.in_bytes < area || (it.in_bytes - area) / 4 < pw) { delete b; return batch_error(APAX_E_CORRUPT, i); }
      if (h.mode == APAX_FIXED_RATE && pw != (uint64_t)h.g.budget * (uint64_t)h.g.nblocks) { delete b; return batch_error(APAX_E_CORRUPT, i); }
      if (it.cap < h.nsamples * (uint64_t)h.esz) { delete b; return batch_error(APAX_E_CAPACITY, i); }
      if (h.mode == APAX_ADAPTIVE_RATE || h.g.G > 64 || h.g.gq == 2) {
        if ((h.g.G > 64 || h.g.gq == 2) && h.g.nblocks && !wide_fits(h.g)) {
          delete b;
          return batch_error(APAX_E_UNSUPPORTED, i);
        }
        b->solo.push_back(i);
        b->solo_hdr.emplace_back();
        memcpy(b->solo_hdr.back().data(), it.h_hdr, 64);
        continue;
      }
    }
    int lpb = lpb_of(h.g);
    BatchClass* c = nullptr;
    for (auto& k : b->classes)
      if (k.lpb == lpb && k.ndim == h.ndim) c = &k;
    if (!c) {
      b->classes.push_back(BatchClass{});
      c = &b->classes.back();
      c->lpb = lpb;
      c->ndim = h.ndim;
    }
    c->items.push_back(i);
    c->total_tiles += std::max<int64_t>(1, encode_tiles_wp(h.g, (int)t.waves_per_wg));
    c->maxldsw = std::max(c->maxldsw, h.g.ldsw);
  }
  int dev = 0, ncu = 256;
  if (hipGetDevice(&dev) == hipSuccess)
    hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  const size_t desc = op == APAX_OP_ENCODE ? sizeof(BatchEnc) : sizeof(BatchDec);
  uint64_t off = al256(sizeof(PState));
  uint64_t tab = 0;
  for (auto& c : b->classes) {
    c.items_off = tab;
    tab += al256(desc * c.items.size());
    c.starts_off = tab;
    tab += al256(8 * c.items.size());
  }
  b->tables.assign(tab, 0);
  uint64_t tables_off = off;
  off += tab;
  b->istat_off = off;
  off += al256(4 * (uint64_t)std::max<uint32_t>(n, 1));
  for (uint32_t i : b->solo) {
    b->solo_off.push_back(off);
    off += al256(ws_need(b->geo[i]));
  }
  for (auto& c : b->classes) {
    c.ticket_off = off;
    off += 256;
    c.tstate_off = off;
    off += al256(8 * (uint64_t)c.total_tiles);
    int64_t g = (int64_t)ncu * t.wgs_per_cu;
    c.grid = (int)std::min<int64_t>(std::max<int64_t>(1, c.total_tiles), g);
    c.items_off += tables_off;
    c.starts_off += tables_off;
  }
  b->ws_bytes = off;
  *ws_bytes = off;
  *out = b;
  return APAX_OK;
}

}  // extern "C"

namespace {

// Fill the plan's descriptor tables for workspace d_ws, copy them from the
// pinned buffer `staging` (>= tables bytes; the caller keeps it untouched
// until the copy has run) and clear the status words.
int batch_upload_from(apax_batch* b, void* d_ws, uint64_t ws_bytes, hipStream_t stream, void* staging) {
  if (!b || !d_ws || ((uintptr_t)d_ws & 255)) return APAX_E_INVALID;
  if (ws_bytes < b->ws_bytes) return APAX_E_CAPACITY;
  b->d_ws = d_ws;
  uint8_t* ws = (uint8_t*)d_ws;
  const uint64_t tables_off = al256(sizeof(PState));
  const int wp = (int)b->tune.waves_per_wg;
  for (auto& c : b->classes) {
    int64_t start = 0;
    for (size_t k = 0; k < c.items.size(); k++) {
      const uint32_t i = c.items[k];
      const apax_batch_item& it = b->items[i];
      const HG& h = b->geo[i];
      int64_t nt = std::max<int64_t>(1, encode_tiles_wp(h.g, wp));
      uint8_t* dst = b->tables.data() + (c.items_off - tables_off) + k * (b->op == APAX_OP_ENCODE ? sizeof(BatchEnc) : sizeof(BatchDec));
      if (b->op == APAX_OP_ENCODE) {
        BatchEnc E;
        memset(&E, 0, sizeof(E));
        E.dtype = h.dtype;
        E.ndim = h.ndim;
        E.tile_start = start;
        EncArgs& A = E.a;
        A.g = h.g;
        A.x = it.d_in;
        A.out_base = (uint8_t*)it.d_out;
        A.area = area_offset(h);
        A.out_words = (uint32_t*)((uint8_t*)it.d_out + A.area);
        A.lens = (uint16_t*)((uint8_t*)it.d_out + 64);
        A.sbo = (uint64_t*)((uint8_t*)it.d_out + 64 + lens_bytes(h));
        A.d_nbytes = it.d_nbytes;
        A.status = (uint32_t*)(ws + b->istat_off) + i;
        A.ticket = nullptr;
        A.tile_state = (uint64_t*)(ws + c.tstate_off) + start;
        A.ntiles = nt;
        make_header(&it.p, h, A.hdr);
        if (h.mode != APAX_FIXED_RATE) {
          A.zpad[0] = 64 + 2 * (uint64_t)h.g.nblocks;
          A.zpad[1] = 64 + lens_bytes(h);
          A.zpad[2] = 64 + lens_bytes(h) + 8 * sbo_count(h);
          A.zpad[3] = A.area;
        }
        memcpy(dst, &E, sizeof(E));
      } else {
        BatchDec D;
        memset(&D, 0, sizeof(D));
        D.dtype = h.dtype;
        D.ndim = h.ndim;
        D.tile_start = start;
        DecArgs& A = D.a;
        A.g = h.g;
        uint64_t area = area_offset(h);
        A.in = (const uint8_t*)it.d_in;
        A.words = (const uint32_t*)((const uint8_t*)it.d_in + area);
        A.lens = (const uint16_t*)((const uint8_t*)it.d_in + 64);
        A.sbo = (const uint64_t*)((const uint8_t*)it.d_in + 64 + lens_bytes(h));
        A.y = it.d_out;
        A.status = (uint32_t*)(ws + b->istat_off) + i;
        memcpy(&A.payload_words, (const uint8_t*)it.h_hdr + 56, 8);
        A.ntiles = nt;
        memcpy(A.hdr, it.h_hdr, 64);
        memcpy(dst, &D, sizeof(D));
      }
      memcpy(b->tables.data() + (c.starts_off - tables_off) + 8 * k, &start, 8);
      start += nt;
    }
  }
  if (!b->tables.empty()) {
    memcpy(staging, b->tables.data(), b->tables.size());
    if (hipMemcpyAsync(ws + tables_off, staging, b->tables.size(), hipMemcpyHostToDevice, stream) != hipSuccess)
      return APAX_E_HIP;
  }
  clear_words((uint32_t*)d_ws, 1, stream);
  clear_words((uint32_t*)(ws + b->istat_off), (int)b->items.size(), stream);
  for (uint64_t o : b->solo_off) clear_words((uint32_t*)(ws + o), 1, stream);
  return hip_err(hipGetLastError());
}

}  // namespace

extern "C" {

int apax_batch_upload(apax_batch* b, void* d_ws, uint64_t ws_bytes, hipStream_t stream) {
  if (!b || !d_ws || ((uintptr_t)d_ws & 255)) return APAX_E_INVALID;
  if (ws_bytes < b->ws_bytes) return APAX_E_CAPACITY;
  if (!b->tables.empty()) {
    // stage in pinned memory owned by the plan, so the copy can stay
    // asynchronous (the plan outlives it)
    if (!b->pinned && hipHostMalloc(&b->pinned, b->tables.size(), hipHostMallocDefault) != hipSuccess) {
      b->pinned = nullptr;
      return APAX_E_HIP;
    }
    if (!b->upload_done && hipEventCreateWithFlags(&b->upload_done, hipEventDisableTiming) != hipSuccess) {
      b->upload_done = nullptr;
      return APAX_E_HIP;
    }
    if (hipEventSynchronize(b->upload_done) != hipSuccess) return APAX_E_HIP;  // staging reused
  }
  int e = batch_upload_from(b, d_ws, ws_bytes, stream, b->pinned);
  if (e) return e;
  if (b->upload_done && hipEventRecord(b->upload_done, stream) != hipSuccess) return APAX_E_HIP;
  return APAX_OK;
}

int apax_batch_run(apax_batch* b, hipStream_t stream) {
  if (!b || !b->d_ws) return APAX_E_INVALID;
  uint8_t* ws = (uint8_t*)b->d_ws;
  const int wp = (int)b->tune.waves_per_wg;
  for (auto& c : b->classes) {
    BatchArgs B;
    memset(&B, 0, sizeof(B));
    B.items = ws + c.items_off;
    B.starts = (const int64_t*)(ws + c.starts_off);
    B.ticket = (uint32_t*)(ws + c.ticket_off);
    B.tile_state = (uint64_t*)(ws + c.tstate_off);
    B.total_tiles = c.total_tiles;
    B.n = (uint32_t)c.items.size();
    B.tiles_per_ticket = b->tune.tiles_per_ticket;
    B.ldsw = c.maxldsw;
    int e = hip_err(launch_batch_reset(B.ticket, B.tile_state, b->op == APAX_OP_ENCODE ? c.total_tiles : 0, stream));
    if (e) return e;
    const int run = b->op == APAX_OP_ENCODE ? RUN : 1;  // encode keeps a run of tiles in LDS
    size_t lds = (size_t)run * wp * (64 / c.lpb) * (size_t)c.maxldsw * 4;
    if (b->op == APAX_OP_ENCODE) e = hip_err(launch_encode_batch(c.lpb, c.ndim, wp, B, c.grid, lds, stream));
    else e = hip_err(launch_decode_batch(c.lpb, c.ndim, wp, B, c.grid, lds, stream));
    if (e) return e;
  }
  for (size_t k = 0; k < b->solo.size(); k++) {
    const uint32_t i = b->solo[k];
    const apax_batch_item& it = b->items[i];
    const HG& h = b->geo[i];
    uint8_t* sws = ws + b->solo_off[k];
    const uint64_t swb = ws_need(h);
    int e;
    if (b->op == APAX_OP_ENCODE) {
      e = encode_enqueue(it.d_in, &it.p, h, false, it.d_out, it.d_nbytes, sws, stream);
    } else {
      HG hd;
      DecArgs A;
      e = decode_setup(b->solo_hdr[k].data(), it.d_in, it.in_bytes, sws, swb, hd, A);
      if (!e) {
        A.y = it.d_out;
        e = hip_err(hd.g.G > 64 || hd.g.gq == 2 ? launch_wide_decode(hd.dtype, hd.ndim, A, stream)
                                                 : launch_decode(hd.dtype, hd.ndim, A, stream));
      }
    }
    if (e) return e;
    hipLaunchKernelGGL(k_copy_word, dim3(1), dim3(64), 0, stream, (uint32_t*)(ws + b->istat_off) + i,
                       (const uint32_t*)sws);
    if ((e = hip_err(hipGetLastError()))) return e;
  }
  if (!b->items.empty()) {
    hipLaunchKernelGGL(k_fold_status, dim3(1), dim3(256), 0, stream, (const uint32_t*)(ws + b->istat_off),
                       (uint32_t)b->items.size(), &((PState*)ws)->status);
    return hip_err(hipGetLastError());
  }
  return APAX_OK;
}

int apax_batch_capture(apax_batch* b) {
  if (!b || !b->d_ws) return APAX_E_INVALID;
  if (b->exec) { hipGraphExecDestroy(b->exec); b->exec = nullptr; }
  if (b->graph) { hipGraphDestroy(b->graph); b->graph = nullptr; }
  hipStream_t cs;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) != hipSuccess) return APAX_E_HIP;
  int e = APAX_OK;
  if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) != hipSuccess) e = APAX_E_HIP;
  if (!e) {
    int e2 = apax_batch_run(b, cs);
    if (hipStreamEndCapture(cs, &b->graph) != hipSuccess) e2 = APAX_E_HIP;
    e = e2;
  }
  if (!e && hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0) != hipSuccess) e = APAX_E_HIP;
  hipStreamDestroy(cs);
  return e;
}

int apax_batch_launch(apax_batch* b, hipStream_t stream) {
  if (!b) return APAX_E_INVALID;
  if (!b->exec) return apax_batch_run(b, stream);
  return hipGraphLaunch(b->exec, stream) == hipSuccess ? APAX_OK : APAX_E_HIP;
}

void apax_batch_destroy(apax_batch* b) {
  if (!b) return;
  if (b->exec) hipGraphExecDestroy(b->exec);
  if (b->graph) hipGraphDestroy(b->graph);
  if (b->upload_done) {
    hipEventSynchronize(b->upload_done);  // an upload may still read the staging buffer
    hipEventDestroy(b->upload_done);
  }
  if (b->pinned) hipHostFree(b->pinned);
  delete b;
}

// ---------------------------------------------------------------- serving
// Continuous batching: submitted requests wait in a FIFO; poll() retires the
// groups whose completion event has fired, then admits FIFO-head requests
// onto every free slot while their footprint fits the budget, and launches
// each admitted group as one persistent batch on the slot's stream.  Slots
// run concurrently, so a group admitted while others run overlaps them.

}  // extern "C"

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct SrvReq {
  uint64_t id = 0;
  apax_request r{};
  hipEvent_t ready = nullptr;  // recorded on the submitter's stream (APAX_REQ_AFTER)
  uint8_t hdr[64];
  uint64_t footprint = 0;
  double t_submit = 0.0;
  bool alone = false;  // runs as a single call whatever its size (no shared launch takes it)
};

struct SrvSlot {
  hipStream_t stream = nullptr;
  hipEvent_t done = nullptr;
  void* ws[2] = {nullptr, nullptr};     // resident codec state: encode, decode
  uint8_t* staging = nullptr;           // pinned: descriptor tables, then item status
  uint32_t* h_status[2] = {nullptr, nullptr};  // pinned copies of per-item status
  apax_batch* plan[2] = {nullptr, nullptr};
  std::vector<SrvReq> reqs;
  std::vector<uint32_t> which[2];       // request index in reqs for each plan item
  std::vector<uint32_t> solo;           // requests run as single calls (request index)
  uint32_t* d_solo = nullptr;           // their status words (device), then
  uint32_t* h_solo = nullptr;           // pinned copies
  bool busy = false;
};

// Requests of at least this many payload bytes run as single apax_encode /
// apax_decode calls on the slot's stream (the single-array kernels are faster
// than the batch kernels on large arrays); smaller ones share batch launches.
constexpr uint64_t SOLO_BYTES = 16ull << 20;

uint64_t req_footprint(const apax_request& q, const HG& h) {
  const uint64_t in = q.op == APAX_OP_ENCODE ? h.nsamples * (uint64_t)h.esz : q.item.in_bytes;
  return in + q.item.cap;
}

}  // namespace

struct apax_server {
  int dev = 0;
  uint64_t budget = 0, used = 0, ws_bytes = 0, staging_bytes = 0;
  uint32_t max_group = 0;
  apax_tune tune{};
  uint64_t next_id = 1;
  std::deque<SrvReq> queue;
  std::vector<SrvSlot> slots;
  std::deque<apax_completion> ready;
  std::vector<hipEvent_t> events;  // free submit events (APAX_REQ_AFTER)
  uint64_t groups = 0;
};

namespace {

void server_free(apax_server* s) {
  for (auto& sl : s->slots) {
    if (sl.stream) hipStreamSynchronize(sl.stream);
    if (sl.d_solo) hipFree(sl.d_solo);
    for (int k = 0; k < 2; k++) {
      if (sl.plan[k]) apax_batch_destroy(sl.plan[k]);
      if (sl.ws[k]) hipFree(sl.ws[k]);
    }
    if (sl.staging) hipHostFree(sl.staging);
    if (sl.done) hipEventDestroy(sl.done);
    if (sl.stream) hipStreamDestroy(sl.stream);
  }
  for (auto& q : s->queue)
    if (q.ready) hipEventDestroy(q.ready);
  for (hipEvent_t ev : s->events) hipEventDestroy(ev);
  delete s;
}

// launch one admitted group on a free slot
// workspace bytes of a single call for request q (0 if it cannot be found)
uint64_t solo_ws(const SrvReq& q) {
  apax_params p = q.r.item.p;
  if (q.r.op == APAX_OP_DECODE && apax_stream_info(q.hdr, 64, &p) != APAX_OK) return 0;
  uint64_t need = 0;
  return apax_workspace_size(&p, &need) == APAX_OK ? need : 0;
}

int server_launch(apax_server* s, SrvSlot& sl) {
  // the group starts after every submitter's stream point it was ordered after
  for (const SrvReq& q : sl.reqs)
    if (q.ready && hipStreamWaitEvent(sl.stream, q.ready, 0) != hipSuccess) return APAX_E_HIP;
  std::vector<apax_batch_item> items[2];
  for (int k = 0; k < 2; k++) sl.which[k].clear();
  sl.solo.clear();
  for (uint32_t i = 0; i < sl.reqs.size(); i++) {
    const SrvReq& q = sl.reqs[i];
    const int k = q.r.op == APAX_OP_ENCODE ? 0 : 1;
    const uint64_t w = q.alone || q.footprint - q.r.item.cap >= SOLO_BYTES ? solo_ws(q) : 0;
    if (w && w <= s->ws_bytes) {
      sl.solo.push_back(i);
      continue;
    }
    items[k].push_back(q.r.item);
    if (k == 1) items[k].back().h_hdr = q.hdr;
    sl.which[k].push_back(i);
  }
  uint64_t soff = 0;
  // large requests: single calls, each status word kept on the device, then
  // one copy of them all
  if (!sl.solo.empty()) {
    for (uint32_t n = 0; n < sl.solo.size(); n++) {
      const SrvReq& q = sl.reqs[sl.solo[n]];
      const apax_batch_item& it = q.r.item;
      const int k = q.r.op == APAX_OP_ENCODE ? 0 : 1;
      int e = apax_status_clear(sl.ws[k], sl.stream);
      if (!e)
        e = k == 0 ? apax_encode(it.d_in, &it.p, it.d_out, it.cap, it.d_nbytes, sl.ws[k], s->ws_bytes, sl.stream)
                   : apax_decode(q.hdr, it.d_in, it.in_bytes, it.d_out, it.cap, sl.ws[k], s->ws_bytes, sl.stream);
      if (e) return e;
      hipLaunchKernelGGL(k_copy_word, dim3(1), dim3(64), 0, sl.stream, sl.d_solo + n,
                         (const uint32_t*)sl.ws[k]);
      if (hipGetLastError() != hipSuccess) return APAX_E_HIP;
    }
    const uint64_t nst = 4 * sl.solo.size();
    sl.h_solo = (uint32_t*)(sl.staging + soff);
    soff += (nst + 255) / 256 * 256;
    if (hipMemcpyAsync(sl.h_solo, sl.d_solo, nst, hipMemcpyDeviceToHost, sl.stream) != hipSuccess)
      return APAX_E_HIP;
  }
  for (int k = 0; k < 2; k++) {
    if (items[k].empty()) continue;
    uint64_t wsb = 0;
    int e = apax_batch_create(k == 0 ? APAX_OP_ENCODE : APAX_OP_DECODE, items[k].data(),
                              (uint32_t)items[k].size(), &s->tune, &sl.plan[k], &wsb);
    if (e) return e;
    if (wsb > s->ws_bytes || soff + sl.plan[k]->tables.size() > s->staging_bytes) return APAX_E_CAPACITY;
    e = batch_upload_from(sl.plan[k], sl.ws[k], s->ws_bytes, sl.stream, sl.staging + soff);
    soff += (sl.plan[k]->tables.size() + 255) / 256 * 256;
    if (e) return e;
    if ((e = apax_batch_run(sl.plan[k], sl.stream))) return e;
    const uint64_t nst = 4 * items[k].size();
    if (soff + nst > s->staging_bytes) return APAX_E_CAPACITY;
    sl.h_status[k] = (uint32_t*)(sl.staging + soff);
    soff += (nst + 255) / 256 * 256;
    if (hipMemcpyAsync(sl.h_status[k], (uint8_t*)sl.ws[k] + sl.plan[k]->istat_off, nst,
                       hipMemcpyDeviceToHost, sl.stream) != hipSuccess)
      return APAX_E_HIP;
  }
  if (hipEventRecord(sl.done, sl.stream) != hipSuccess) return APAX_E_HIP;
  sl.busy = true;
  s->groups++;
  return APAX_OK;
}

int status_code(uint32_t bits) {
  if (bits & ST_NONFINITE) return APAX_E_NONFINITE;
  if (bits & ST_CORRUPT) return APAX_E_CORRUPT;
  if (bits & ST_INTERNAL) return APAX_E_INTERNAL;
  if (bits & ST_NOPROFILE) return APAX_E_INVALID;
  return APAX_OK;
}

}  // namespace

extern "C" {

int apax_server_create(uint64_t budget_bytes, uint32_t n_slots, uint32_t max_group, uint64_t ws_bytes,
                       const apax_tune* tune, apax_server** out) {
  if (!out || n_slots == 0 || n_slots > 16 || max_group == 0 || max_group > 65536 || ws_bytes < 4096)
    return APAX_E_INVALID;
  *out = nullptr;
  apax_server* s = new apax_server();
  ws_bytes = (ws_bytes + 255) / 256 * 256;
  // workspace and staging are reserved for the server's lifetime and count
  // against the budget
  const uint64_t reserved = (uint64_t)n_slots * 2 * ws_bytes;
  if (budget_bytes <= reserved) { delete s; return APAX_E_CAPACITY; }
  s->budget = budget_bytes - reserved;
  s->ws_bytes = ws_bytes;
  s->max_group = max_group;
  if (tune) s->tune = *tune;
  // descriptor tables (<= 1 KiB per item) + three status arrays + alignment
  s->staging_bytes = (uint64_t)max_group * (sizeof(BatchEnc) > sizeof(BatchDec) ? sizeof(BatchEnc) : sizeof(BatchDec))
                     + (uint64_t)max_group * 16 + 16 * 4096;
  if (hipGetDevice(&s->dev) != hipSuccess) { delete s; return APAX_E_HIP; }
  s->slots.resize(n_slots);
  for (auto& sl : s->slots) {
    bool ok = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) == hipSuccess &&
              hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) == hipSuccess &&
              hipMalloc(&sl.ws[0], ws_bytes) == hipSuccess && hipMalloc(&sl.ws[1], ws_bytes) == hipSuccess &&
              hipMalloc((void**)&sl.d_solo, 4 * (uint64_t)max_group) == hipSuccess &&
              hipHostMalloc((void**)&sl.staging, s->staging_bytes, hipHostMallocDefault) == hipSuccess;
    if (!ok) { server_free(s); return APAX_E_HIP; }
  }
  *out = s;
  return APAX_OK;
}

int apax_server_submit(apax_server* s, const apax_request* q, uint64_t* id) {
  if (!s || !q || !id || (q->op != APAX_OP_ENCODE && q->op != APAX_OP_DECODE)) return APAX_E_INVALID;
  if (q->flags & ~APAX_REQ_AFTER) return APAX_E_INVALID;
  SrvReq r;
  r.r = *q;
  HG h;
  int e;
  if (q->op == APAX_OP_ENCODE) {
    if ((e = setup(&q->item.p, h))) return e;
    if (q->item.cap < bound_of(h)) return APAX_E_CAPACITY;
    r.alone = h.lagged || h.g.G > 64 || h.g.gq == 2 || h.mode == APAX_ADAPTIVE_RATE;
    memset(r.hdr, 0, 64);
  } else {
    apax_params p;
    if (!q->item.h_hdr || apax_stream_info(q->item.h_hdr, 64, &p)) return APAX_E_CORRUPT;
    uint16_t budget;
    memcpy(&budget, (const uint8_t*)q->item.h_hdr + 10, 2);
    if ((e = setup(&p, h, header_budget(p.mode, budget)))) return e;
    r.alone = h.g.G > 64 || h.g.gq == 2 || h.mode == APAX_ADAPTIVE_RATE;
    memcpy(r.hdr, q->item.h_hdr, 64);
    r.r.item.h_hdr = nullptr;
  }
  // requests no shared launch takes run alone in the slot's codec workspace
  if (r.alone) {
    if ((h.g.G > 64 || h.g.gq == 2) && h.g.nblocks && !wide_fits(h.g)) return APAX_E_UNSUPPORTED;
    if (ws_need(h) > s->ws_bytes) return APAX_E_CAPACITY;
  }
  r.footprint = req_footprint(*q, h);
  if (r.footprint > s->budget) return APAX_E_CAPACITY;
  if (q->flags & APAX_REQ_AFTER) {
    if (s->events.empty()) {
      hipEvent_t ev;
      if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) return APAX_E_HIP;
      s->events.push_back(ev);
    }
    r.ready = s->events.back();
    if (hipEventRecord(r.ready, q->after) != hipSuccess) return APAX_E_HIP;
    s->events.pop_back();
  }
  r.id = s->next_id++;
  r.t_submit = now_s();
  *id = r.id;
  s->queue.push_back(r);
  return APAX_OK;
}

int apax_server_poll(apax_server* s, apax_completion* done, uint32_t max_done, uint32_t* n_done) {
  if (!s || !n_done || (max_done && !done)) return APAX_E_INVALID;
  *n_done = 0;
  int dev0 = -1;
  hipGetDevice(&dev0);
  if (dev0 != s->dev) hipSetDevice(s->dev);
  int err = APAX_OK;
  // retire finished groups
  for (uint32_t k = 0; k < s->slots.size(); k++) {
    SrvSlot& sl = s->slots[k];
    if (!sl.busy) continue;
    hipError_t q = hipEventQuery(sl.done);
    if (q == hipErrorNotReady) continue;
    if (q != hipSuccess) { err = APAX_E_HIP; break; }
    const double t = now_s();
    for (uint32_t n = 0; n < sl.solo.size(); n++) {
      const SrvReq& r = sl.reqs[sl.solo[n]];
      s->ready.push_back(apax_completion{r.id, r.r.tag, status_code(sl.h_solo[n]), k, t - r.t_submit});
      s->used -= r.footprint;
    }
    sl.solo.clear();
    for (int p = 0; p < 2; p++) {
      for (uint32_t i = 0; i < sl.which[p].size(); i++) {
        const SrvReq& r = sl.reqs[sl.which[p][i]];
        apax_completion c;
        c.id = r.id;
        c.tag = r.r.tag;
        c.status = status_code(sl.h_status[p][i]);
        c.slot = k;
        c.latency_s = t - r.t_submit;
        s->ready.push_back(c);
        s->used -= r.footprint;
      }
      if (sl.plan[p]) { apax_batch_destroy(sl.plan[p]); sl.plan[p] = nullptr; }
      sl.which[p].clear();
    }
    for (auto& r : sl.reqs)
      if (r.ready) s->events.push_back(r.ready);
    sl.reqs.clear();
    sl.busy = false;
  }
  // admit FIFO-head requests onto free slots
  for (auto& sl : s->slots) {
    if (err || s->queue.empty()) break;
    if (sl.busy) continue;
    while (!s->queue.empty() && sl.reqs.size() < s->max_group &&
           s->used + s->queue.front().footprint <= s->budget) {
      s->used += s->queue.front().footprint;
      sl.reqs.push_back(s->queue.front());
      s->queue.pop_front();
    }
    if (sl.reqs.empty()) break;  // the head waits for memory
    int e = server_launch(s, sl);
    if (e) {
      // the group could not be launched: complete its requests with the error
      hipStreamSynchronize(sl.stream);
      for (auto& r : sl.reqs) {
        s->ready.push_back(apax_completion{r.id, r.r.tag, e, 0, now_s() - r.t_submit});
        s->used -= r.footprint;
      }
      for (int p = 0; p < 2; p++)
        if (sl.plan[p]) { apax_batch_destroy(sl.plan[p]); sl.plan[p] = nullptr; }
      for (auto& r : sl.reqs)
        if (r.ready) s->events.push_back(r.ready);
      sl.reqs.clear();
      sl.busy = false;
    }
  }
  while (*n_done < max_done && !s->ready.empty()) {
    done[(*n_done)++] = s->ready.front();
    s->ready.pop_front();
  }
  if (dev0 >= 0 && dev0 != s->dev) hipSetDevice(dev0);
  return err;
}

int apax_server_stats(const apax_server* s, uint64_t* queued, uint64_t* in_flight_bytes, uint64_t* groups) {
  if (!s) return APAX_E_INVALID;
  if (queued) *queued = s->queue.size();
  if (in_flight_bytes) *in_flight_bytes = s->used;
  if (groups) *groups = s->groups;
  return APAX_OK;
}

void apax_server_destroy(apax_server* s) {
  if (s) server_free(s);
}

}  // extern "C"
