// profile.hip -- profiler kernels (Sec. 4) for gfx950.
//
// Every pass visits blocks with the encoder's own per-block machinery
// (bracket, quantizer, stream sizes, fixed-rate search), so the profiler sees
// exactly what the encoder will produce.  Persistent workgroups loop over
// tiles; each lane accumulates its statistics in FP32 float-float pairs
// (TwoSum, Knuth; renormalised with Fast2Sum), every binary64 term split
// exactly into hi + lo first and scaled by a power of two chosen from max|x|
// so FP32 never overflows.  Lanes reduce once per workgroup (wave
// butterflies, then LDS), workgroups in a fixed-order final pass, so results
// are deterministic.  grid.y indexes the gain codes evaluated in one launch.
#include "block.h"
#include "kernels.h"

namespace apax {

struct FF {
  float hi, lo;
};

__device__ __forceinline__ FF fast2sum(float a, float b) {
  float s = a + b;
  float e = b - (s - a);
  return {s, e};
}

__device__ __forceinline__ FF ff_add(FF a, FF b) {
  float s = a.hi + b.hi;
  float bb = s - a.hi;
  float e = (a.hi - (s - bb)) + (b.hi - bb);
  e += a.lo + b.lo;
  return fast2sum(s, e);
}

__device__ __forceinline__ FF ff_of(double t) {
  float hi = (float)t;
  float lo = (float)(t - (double)hi);
  return {hi, lo};
}

__device__ __forceinline__ FF ff_shfl_xor(FF a, int o) {
  return {__shfl_xor(a.hi, o, 64), __shfl_xor(a.lo, o, 64)};
}

template <typename T, int LPB, int NDIM>
__global__ __launch_bounds__(256) void k_profile(ProfArgs A) {
  constexpr int BPW = 64 / LPB;
  using B_ = Blk<T, LPB, NDIM>;
  const Geo& g = A.g;
  __shared__ float s_red[WPG][NSUM][2];
  __shared__ uint4 s_xch[NDIM >= 2 ? WPG * 64 : 1];

  const int wave = threadIdx.x >> 6;
  const int lane = lane_id();
  const int ci = blockIdx.y;
  int code = 0;
#pragma unroll
  for (int t = 0; t < MAXCODES; t++) code |= (int)pick(ci == t, (uint32_t)A.codes[t]);
  const double s1 = ldexp(1.0, -A.escale);
  const double s2 = ldexp(1.0, -2 * A.escale);
  FF acc[NSUM];
#pragma unroll
  for (int i = 0; i < NSUM; i++) acc[i] = {0.f, 0.f};
  double dmax = 0.0, xmax = 0.0;
  uint32_t nfit = 0;
  unsigned long long wsum = 0;
  bool nonfinite = false;

  for (int64_t tile = blockIdx.x; tile < A.ntiles; tile += A.nwg) {
    const int64_t jj = (tile * WPG + wave) * BPW + lane / LPB;
    B_ b;
    b.init(g, jj < A.nbe ? jj * A.jstride : g.nblocks, NDIM >= 2 ? s_xch + wave * 64 : nullptr);
    b.load((const T*)A.x, g);
    nonfinite |= b.act && b.nonfinite;
    if (A.op == P_MAX) {
      xmax = b.act && b.M > xmax ? b.M : xmax;
      continue;
    }
    int32_t a[4], v[7][4];
    int eps[7], pw[7];
    Costs C;
    int32_t best;
    if (A.op == P_FITS) {
      // argmin over the mask at the clamped code: fit test + stream histogram
      int c = A.rule == R_LOSSLESS ? 0 : clampc(code, b.cf, b.cc);
      b.quantize(c, A.rule == R_LOSSLESS, a);
      b.sizes(g, A.mask, a, v, eps, pw, C);
      int st = B_::argmin(C, A.mask, best);
      if (b.blk_ok && b.L.gi == 0) {
        if (best <= 32 * g.budget) nfit++;
        if (ci == A.hist_code) atomicAdd(&A.hist[st], 1u);
      }
      continue;
    }
    // P_STATS / P_CENTER: operating point of the block, decoded values
    int c = 0;
    if (A.rule == R_QUALITY) {
      c = clampc(code, b.cf, b.cc);
    } else if (A.rule == R_RATE) {
      if (A.op == P_CENTER) {
        c = b.blk_ok ? A.cj[b.j] : 0;
      } else {
        c = clampc(code, b.cf, b.cc);
        const uint32_t m7 = A.mask & 0x7Fu;
        b.quantize(c, false, a);
        b.sizes(g, m7, a, v, eps, pw, C);
        int st = B_::argmin(C, m7, best);
        bool need = b.act && best > 32 * g.budget;
        if (__ballot(need)) c = b.rate_search(g, c, st, need);
        if (A.store_cj && b.blk_ok && b.L.gi == 0) A.cj[b.j] = c;
      }
    }
    b.quantize(c, A.rule == R_LOSSLESS, a);
    if (A.op == P_STATS) {
      int nw;
      if (A.rule != R_RATE) {
        b.sizes(g, A.mask, a, v, eps, pw, C);
        B_::argmin(C, A.mask, best);
        nw = (best + 31) >> 5;
      } else {
        nw = g.budget;
      }
      if (b.blk_ok && b.L.gi == 0) wsum += (unsigned long long)nw;
    }
#pragma unroll
    for (int k = 0; k < 4; k++) {
      if (!(b.act && b.valid(k))) continue;
      double x = b.xd[k];
      double y;
      if (A.rule == R_LOSSLESS) y = (double)a[k];
      else y = (double)to_out<T>(dequant(a[k], c));
      double d = x - y;
      if (A.op == P_STATS) {
        acc[S_X] = ff_add(acc[S_X], ff_of(x * s1));
        acc[S_Y] = ff_add(acc[S_Y], ff_of(y * s1));
        acc[S_D] = ff_add(acc[S_D], ff_of(d * s1));
        acc[S_XX] = ff_add(acc[S_XX], ff_of((x * x) * s2));
        acc[S_YY] = ff_add(acc[S_YY], ff_of((y * y) * s2));
        acc[S_DD] = ff_add(acc[S_DD], ff_of((d * d) * s2));
        acc[S_DS] = ff_add(acc[S_DS], ff_of((d * (x + y)) * s2));
        double ad = __builtin_fabs(d);
        dmax = ad > dmax ? ad : dmax;
      } else {
        double ex = x - A.mean_x, ey = y - A.mean_y, ed = d - A.mean_d;
        acc[S_CXX] = ff_add(acc[S_CXX], ff_of((ex * ex) * s2));
        acc[S_CYY] = ff_add(acc[S_CYY], ff_of((ey * ey) * s2));
        acc[S_CDD] = ff_add(acc[S_CDD], ff_of((ed * ed) * s2));
      }
    }
  }

  if (__ballot(nonfinite) && lane == 0) atomicOr(A.status, ST_NONFINITE);
  if (A.op == P_MAX) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      double t = __shfl_xor(xmax, o, 64);
      xmax = t > xmax ? t : xmax;
    }
    if (lane == 0) atomicMax(&A.maxbits[0], (unsigned long long)__builtin_bit_cast(uint64_t, xmax));
    return;
  }
  if (A.op == P_FITS) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) nfit += __shfl_xor(nfit, o, 64);
    if (lane == 0 && nfit) atomicAdd(&A.fits[ci], nfit);
    return;
  }
  // wave reduction of the sums this op produced
  const int i0 = A.op == P_STATS ? 0 : S_CXX;
  const int i1 = A.op == P_STATS ? S_CXX : NSUM;
#pragma unroll
  for (int i = 0; i < NSUM; i++) {
    if (i < i0 || i >= i1) continue;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) acc[i] = ff_add(acc[i], ff_shfl_xor(acc[i], o));
  }
  if (A.op == P_STATS) {
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      double t = __shfl_xor(dmax, o, 64);
      dmax = t > dmax ? t : dmax;
      wsum += __shfl_xor(wsum, o, 64);
    }
    if (lane == 0) {
      atomicMax(&A.maxbits[1], (unsigned long long)__builtin_bit_cast(uint64_t, dmax));
      if (wsum) atomicAdd(&A.words[ci], wsum);
    }
  }
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < NSUM; i++) {
      s_red[wave][i][0] = acc[i].hi;
      s_red[wave][i][1] = acc[i].lo;
    }
  }
  __syncthreads();
  if (threadIdx.x < NSUM) {
    int i = threadIdx.x;
    FF t = {s_red[0][i][0], s_red[0][i][1]};
    for (int w = 1; w < WPG; w++) t = ff_add(t, FF{s_red[w][i][0], s_red[w][i][1]});
    float* p = A.partials + (((int64_t)ci * A.nwg + blockIdx.x) * NSUM + i) * 2;
    p[0] = t.hi;
    p[1] = t.lo;
  }
}

// Fixed-order reduction of the per-workgroup partials of every code.
__global__ __launch_bounds__(256) void k_finalize(const float* partials, int64_t nwg,
                                                  double* out) {
  __shared__ float s[256][2];
  const int ci = blockIdx.x / NSUM, i = blockIdx.x % NSUM;
  FF acc = {0.f, 0.f};
  for (int64_t t = threadIdx.x; t < nwg; t += 256) {
    const float* p = partials + ((ci * nwg + t) * NSUM + i) * 2;
    acc = ff_add(acc, FF{p[0], p[1]});
  }
  s[threadIdx.x][0] = acc.hi;
  s[threadIdx.x][1] = acc.lo;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      FF a = {s[threadIdx.x][0], s[threadIdx.x][1]};
      FF b = {s[threadIdx.x + w][0], s[threadIdx.x + w][1]};
      FF r = ff_add(a, b);
      s[threadIdx.x][0] = r.hi;
      s[threadIdx.x][1] = r.lo;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[ci * NSUM + i] = (double)s[0][0] + (double)s[0][1];
}

int64_t prof_tiles(const Geo& g, int64_t nbe) {
  int lpb = g.G <= 16 ? 16 : (g.G <= 32 ? 32 : 64);
  int64_t per = (int64_t)WPG * (64 / lpb);
  return (nbe + per - 1) / per;
}

// persistent workgroups per code: enough to fill 256 CUs several times over
int64_t prof_wgs(int64_t ntiles) { return ntiles < 2048 ? ntiles : 2048; }

template <typename T, int LPB, int NDIM>
static hipError_t launch_t(const ProfArgs& A, hipStream_t s) {
  hipLaunchKernelGGL((k_profile<T, LPB, NDIM>), dim3((unsigned)A.nwg, A.ncodes), dim3(WPG * 64),
                     0, s, A);
  return hipGetLastError();
}

template <typename T, int NDIM>
static hipError_t launch_lpb(const ProfArgs& A, hipStream_t s) {
  if (A.g.G <= 16) return launch_t<T, 16, NDIM>(A, s);
  if (A.g.G <= 32) return launch_t<T, 32, NDIM>(A, s);
  return launch_t<T, 64, NDIM>(A, s);
}

template <typename T>
static hipError_t launch_nd(const ProfArgs& A, int ndim, hipStream_t s) {
  if (ndim == 1) return launch_lpb<T, 1>(A, s);
  if (ndim == 2) return launch_lpb<T, 2>(A, s);
  return launch_lpb<T, 3>(A, s);
}

hipError_t launch_profile(int dtype, int ndim, ProfArgs& A, hipStream_t s) {
  A.ntiles = prof_tiles(A.g, A.nbe);
  A.nwg = prof_wgs(A.ntiles);
  if (A.ntiles == 0) return hipSuccess;
  switch (dtype) {
    case DT_I8: return launch_nd<int8_t>(A, ndim, s);
    case DT_I16: return launch_nd<int16_t>(A, ndim, s);
    case DT_I32: return launch_nd<int32_t>(A, ndim, s);
    case DT_F32: return launch_nd<float>(A, ndim, s);
    default: return launch_nd<double>(A, ndim, s);
  }
}

hipError_t launch_finalize(const float* partials, int64_t nwg, int ncodes, double* out,
                           hipStream_t s) {
  if (nwg == 0) return hipSuccess;
  hipLaunchKernelGGL(k_finalize, dim3((unsigned)(ncodes * NSUM)), dim3(256), 0, s, partials,
                     nwg, out);
  return hipGetLastError();
}

}  // namespace apax
