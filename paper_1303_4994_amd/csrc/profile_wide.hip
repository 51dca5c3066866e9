// profile_wide.hip -- the profiler's passes (Sec. 4) over blocks of more than
// 256 samples, or of groups of 8 samples per exponent (Sec. 6): one workgroup
// per block at a time, with the encoder's own wide-block analysis (bracket,
// quantizer, stream sizes, stream choice, fixed-rate search; wide_enc.h), so
// the profiler sees exactly what the encoder produces.  Each workgroup visits
// blocks blockIdx.x, blockIdx.x + nwg, ... of the pass (grid.y: the codes
// evaluated in one launch) and writes the same per-(code, workgroup) partial
// record as the one-wave passes; the same one-workgroup kernel reduces the
// records in a fixed order and runs the next control step.
#include "totals.h"
#include "kernels.h"
#include "wide_enc.h"

namespace apax {

template <typename T, int NDIM, int OPK>
__global__ __launch_bounds__(WIDE_MAXT) void k_wprofile(ProfArgs A) {
  extern __shared__ __align__(16) uint32_t lds[];
  __shared__ WideShared sh;
  constexpr int OP = OPK == P_CURVE ? P_STATS : OPK;
  constexpr int NL = S_CXX;  // accumulator slots; the centred pass uses slots S_XX..S_DD
  constexpr int MAXW = WIDE_MAXT / 64;
  __shared__ double s_red[MAXW][NL];
  __shared__ uint64_t s_dm[MAXW];
  A.curve = OPK == P_CURVE;
  if (OPK == P_CURVE) A.rule = R_QUALITY;  // curve codes are fixed per block
  const Geo& g = A.g;
  const PState* st = A.st;
  const int ci = blockIdx.y;
  const int nset = A.final_code ? 1 : st->ncodes;
  const int ncodes = nset < (int)gridDim.y ? nset : (int)gridDim.y;
  if (ci >= ncodes) return;  // uniform per workgroup
  if (OP == P_CENTER && st->centred) return;  // the metrics pass's moments gave the centred sums
  const int tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
  const int code = A.final_code ? st->code : st->codes[ci];
  const int escale = st->escale;
  uint32_t mask;
  if (A.mask_sel == 0) mask = st->mask_probe;
  else if (A.mask_sel == 1) mask = st->mask_out | 0x81u;
  else mask = A.rule == R_RATE ? ((st->mask_out & 0x7Fu) | 1u) : (st->mask_out | 0x81u);
  const double s1 = ldexp(1.0, -escale);
  const double s2 = ldexp(1.0, -2 * escale);
  const double mx = st->mean[0], my = st->mean[1], md = st->mean[2];
  constexpr int L0 = OP == P_STATS ? (OPK == P_CURVE ? S_XX : 0) : S_XX;
  constexpr int L1 = OP == P_STATS ? NL : (OP == P_CENTER ? S_DS : 0);
  constexpr int NA = L1 > L0 ? L1 - L0 : 1;
  const bool lossless = A.rule == R_LOSSLESS;
  // the centred pass of a fixed-rate profile takes each block's code from
  // the metrics pass, so it needs no bracket (nor does a lossless pass)
  const bool bracket = !(lossless || (OP == P_CENTER && A.rule == R_RATE));

  // each thread sums its groups' binary64 terms over up to 64 blocks, then
  // adds the partial (scaled by a power of two) to its accumulators
  double acc[NA];
#pragma unroll
  for (int i = 0; i < NA; i++) acc[i] = 0.0;
  double lacc[NL];
#pragma unroll
  for (int i = 0; i < NL; i++) lacc[i] = 0.0;
  int lcount = 0;
  auto flush = [&]() {
#pragma unroll
    for (int i = L0; i < L1; i++) acc[i - L0] += lacc[i] * (i < S_XX ? s1 : s2);
#pragma unroll
    for (int i = 0; i < NL; i++) lacc[i] = 0.0;
    lcount = 0;
  };
  double dmax = 0.0;
  // per-block counts, kept by thread 0
  uint32_t nfit = 0;
  uint32_t hcnt[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  unsigned long long wsum = 0;

  WEnc<T, NDIM> b;
  for (int64_t jj = blockIdx.x; jj < A.nbe; jj += A.nwg) {
    const int64_t j = jj * A.jstride;
    b.init(g, j, lds, sh);
    if (bracket) b.template load<true>((const T*)A.x);
    else b.template load<false>((const T*)A.x);
    int32_t best;
    if (OP == P_FITS) {
      // argmin over the mask at the clamped code: fit test + stream histogram
      const int c = lossless ? 0 : clampc(code, b.cf, b.cc);
      b.quantize(c, lossless);
      const int s_ = b.choose(mask, best);
      if (tid == 0) {
        if (best <= 32 * g.budget) nfit++;
        if (A.hist) {
          hcnt[s_]++;
          int64_t nv = 1;  // samples of the block inside the array
#pragma unroll
          for (int d = 0; d < 3; d++) {
            const int64_t bc = d == 0 ? b.wg.bz : (d == 1 ? b.wg.by : b.wg.bx);
            const int64_t rem = g.n[d] - bc * g.b[d];
            nv *= rem < g.b[d] ? rem : g.b[d];
          }
          wsum += (unsigned long long)nv;
        }
      }
      continue;
    }
    // P_STATS / P_CENTER: operating point of the block, decoded values
    int c = 0;
    if (A.rule == R_QUALITY) {
      c = clampc(code, b.cf, b.cc);
    } else if (A.rule == R_RATE) {
      if (OP == P_CENTER) {
        c = A.cj[j];
      } else {
        c = clampc(code, b.cf, b.cc);
        b.quantize(c, false);
        const int s_ = b.choose(mask & 0x7Fu, best);
        c = b.rate_search(c, s_, best);
        if (A.store_cj && tid == 0) A.cj[j] = c;
      }
    }
    b.quantize(c, lossless);
    if (OP == P_STATS) {
      int nw;
      if (A.rule != R_RATE) {
        b.choose(mask, best);
        nw = (best + 31) >> 5;
      } else {
        nw = g.budget;
      }
      if (tid == 0) wsum += (unsigned long long)nw;
    }
    // the thread's groups: binary64 terms into the accumulators
    double* t = lacc;
    const double Rq = inv_mantissa(c);
    const int eq = -(c >> 4);
#pragma unroll
    for (int m = 0; m < WIDE_GPT; m++) {
      const int gi = tid + m * b.wg.nt;
      if (gi >= g.G) break;
      int z, y_, xq;
      b.wg.coords(g, gi, z, y_, xq);
      int64_t idx;
      const int nv = b.wg.nvalid(g, z, y_, xq, idx);
      const uint4 q4 = *reinterpret_cast<const uint4*>(b.qa + 4 * gi);
      const int32_t qv[4] = {(int32_t)q4.x, (int32_t)q4.y, (int32_t)q4.z, (int32_t)q4.w};
#pragma unroll
      for (int k = 0; k < 4; k++) {
        if (k >= nv) continue;
        const double x = (double)b.xs[m][k];
        double y;
        if (lossless) y = (double)qv[k];
        else y = (double)to_out<T>(dequant_rk(qv[k], Rq, eq));
        const double d = x - y;
        if (OP == P_STATS) {
          if (!A.curve) {
            t[S_X] += x;
            t[S_Y] += y;
            t[S_D] += d;
            const double ad = __builtin_fabs(d);
            dmax = ad > dmax ? ad : dmax;
          }
          t[S_XX] += x * x;
          t[S_YY] += y * y;
          t[S_DD] += d * d;
          t[S_DS] += d * (x + y);
        } else {
          const double ex = x - mx, ey = y - my, ed = d - md;
          t[S_XX] += ex * ex;  // slots of the centred sums S_CXX, S_CYY, S_CDD
          t[S_YY] += ey * ey;
          t[S_DD] += ed * ed;
        }
      }
    }
    if (++lcount == 64) flush();
  }
  flush();

  // ---- workgroup partial record (waves in order, then the record)
  const int nwv = wg_nwaves();
  if constexpr (L1 > L0) {
    const double tot = wave_totals<L1 - L0>(acc, lane);
    const int idx = wave_totals_index<L1 - L0>(lane);
    if (lane < 8 && idx < L1 - L0) s_red[wave][L0 + idx] = tot;
  }
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const double tt = __shfl_xor(dmax, o, 64);
    dmax = tt > dmax ? tt : dmax;
  }
  if (lane == 0) s_dm[wave] = __builtin_bit_cast(uint64_t, dmax);
  __syncthreads();
  const PParts P = pparts(A.parts, (int64_t)gridDim.y * A.nwg);
  const int64_t r = (int64_t)ci * A.nwg + blockIdx.x;
  if (tid < NL) {
    const int i = tid;
    if (i >= L0 && i < L1) {
      double tt = s_red[0][i];
      for (int w = 1; w < nwv; w++) tt += s_red[w][i];
      const int si = OP == P_CENTER ? i - S_XX + S_CXX : i;  // sum index of the slot
      P.s[(int64_t)si * P.R + r] = tt;
    }
  }
  if (tid == 0) {
    uint64_t dm = 0;
    for (int w = 0; w < nwv; w++) dm = s_dm[w] > dm ? s_dm[w] : dm;
    P.words[r] = wsum;
    P.dmax[r] = dm;
    P.nfit[r] = nfit;
#pragma unroll
    for (int t = 0; t < 8; t++) P.hist[(int64_t)t * P.R + r] = hcnt[t];
  }
}

template <typename K>
static hipError_t wprof_lds_attr(K kernel, size_t lds) {
  if (lds <= 65536) return hipSuccess;
  return hipFuncSetAttribute((const void*)kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
}

template <typename T, int NDIM, int OPK>
static hipError_t wprof_t(const ProfArgs& A, hipStream_t s) {
  const size_t lds = wide_lds_bytes(A.g);
  hipError_t e = wprof_lds_attr(k_wprofile<T, NDIM, OPK>, lds);
  if (e != hipSuccess) return e;
  const dim3 grid((unsigned)A.nwg, A.maxcodes), block(wide_threads(A.g.G));
  hipLaunchKernelGGL((k_wprofile<T, NDIM, OPK>), grid, block, lds, s, A);
  return hipGetLastError();
}

template <typename T, int NDIM>
static hipError_t wprof_op(const ProfArgs& A, hipStream_t s) {
  if (A.op == P_FITS) return wprof_t<T, NDIM, P_FITS>(A, s);
  if (A.op == P_STATS && A.curve) return wprof_t<T, NDIM, P_CURVE>(A, s);
  if (A.op == P_STATS) return wprof_t<T, NDIM, P_STATS>(A, s);
  return wprof_t<T, NDIM, P_CENTER>(A, s);
}

template <typename T>
static hipError_t wprof_nd(const ProfArgs& A, int ndim, hipStream_t s) {
  if (ndim == 1) return wprof_op<T, 1>(A, s);
  if (ndim == 2) return wprof_op<T, 2>(A, s);
  return wprof_op<T, 3>(A, s);
}

hipError_t launch_wide_profile(int dtype, int ndim, const ProfArgs& A, hipStream_t s) {
  switch (dtype) {
    case DT_I8: return wprof_nd<int8_t>(A, ndim, s);
    case DT_I16: return wprof_nd<int16_t>(A, ndim, s);
    case DT_I32: return wprof_nd<int32_t>(A, ndim, s);
    case DT_F32: return wprof_nd<float>(A, ndim, s);
    default: return wprof_nd<double>(A, ndim, s);
  }
}

}  // namespace apax
