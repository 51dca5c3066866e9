/*
 * apax_oracle.c -- plain, slow, single-threaded CPU reference of the APAX
 * numerical encoder, decoder and profiler (arXiv 1303.4994).
 *
 * TEST INFRASTRUCTURE ONLY: used by the tests, the smoke check and the
 * CPU-baseline leg of the benchmark to check the GPU library.  It shares no
 * code with the GPU path.  Build: gcc -O2 -std=c99 -ffp-contract=off
 * (no FMA contraction, no fast-math): every floating-point step below is a
 * single IEEE binary64 operation in round-to-nearest-even.
 *
 * Paper map (section numbers of the paper):
 *   Sec. 6, encoder block diagram  : blocks of 64..16384 samples (multiple of
 *        4), attenuator (a per-block floating-point gain under an adaptive
 *        loop aiming at a packet size or a correlation target), redundancy
 *        remover (keeps the filtered stream that needs the fewest bits),
 *        4-byte (ints) / 6-byte (floats) block header.
 *   Sec. 6, bit packer             : block floating point with one exponent
 *        per group of N = 4 samples; joint exponent encoding (JEE) of
 *        exponent differences: nine 4-bit tokens for two differences in
 *        [-1, 1], five 4-bit tokens for one difference in [-2, 2], an 8-bit
 *        token otherwise; the first exponent is sent absolutely.
 *   Sec. 5                         : derivatives against oversampling, block
 *        exponents against peak-to-average ratio, attenuation against
 *        over-cast (low-ENOB) data.
 *   Sec. 4, profiler               : correlation r = sum(xy)/sqrt(sum x^2 sum y^2)
 *        between input x and decoded y, recommended operating point at a
 *        correlation target, rate-correlation curve, summary metrics.
 * Where the paper is silent (bit order, token code values, header fields,
 * gain grid, fixed-rate search, N-d bricks, container) the reading of the
 * project design notes is followed; each such step says "reading".
 */
#include "apax_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* geometry and parameter validation (Sec. 6: block size 64..16384, mult. 4) */

typedef struct {
  int dtype, mode, ndim;
  int W;        /* bits of a quantized sample: 8/16/32 for ints, 32 for floats */
  int H;        /* block header bits: 32 for ints (4 B), 48 for floats (6 B)   */
  int esz;      /* bytes of one input sample                                   */
  int isint;
  int64_t n[3]; /* array extent, z y x (leading 1 for lower ndim)             */
  int64_t b[3]; /* brick extent, z y x                                         */
  int B, G;     /* samples and exponent groups per block                       */
  int N;        /* samples per exponent group: 4, or 8 with ORC_FLAG_GROUP8     */
  int64_t nb[3];
  int64_t nblocks;
  uint32_t mask;   /* effective stream mask for this mode */
  int budget;      /* fixed-rate words per block, 0 otherwise */
  int target;      /* adaptive rate: target words per block, 0 otherwise */
  int fk, fneg;    /* filter stream: stride (0: none) and sign (1: x[n] + x[n-k]) */
  int cmin, cmax;  /* admissible gain codes */
  int code;
} geom;

static const uint32_t ALLOWED[4] = {0, 0x87u, 0xAFu, 0xFFu};

static int64_t floordiv16(int64_t c) { return c >= 0 ? c / 16 : -((-c + 15) / 16); }

static int setup_geom_b(const orc_params* p, geom* g, int forced_budget) {
  memset(g, 0, sizeof(*g));
  if (!p || p->size != sizeof(orc_params)) return ORC_E_INVALID;
  if (p->dtype < ORC_I8 || p->dtype > ORC_F64) return ORC_E_INVALID;
  if (p->ndim < 1 || p->ndim > 3) return ORC_E_INVALID;
  if (p->mode > ORC_ADAPTIVE_RATE) return ORC_E_INVALID;
  if (p->flags & ~(ORC_FLAG_LAGGED | ORC_FILTER(31, 1) | ORC_FLAG_GROUP8)) return ORC_E_INVALID;
  if ((p->flags & ORC_FLAG_LAGGED) && p->mode != ORC_LOSSLESS) return ORC_E_INVALID;
  /* filter stream: 1-d only, stride 1..16, a sign only with a stride */
  g->fk = (int)ORC_FILTER_K(p->flags);
  g->fneg = (p->flags & ORC_FILTER_NEG) ? 1 : 0;
  if (g->fk > 16 || (g->fneg && !g->fk) || (g->fk && p->ndim != 1)) return ORC_E_INVALID;
  g->dtype = (int)p->dtype;
  g->mode = (int)p->mode;
  g->ndim = (int)p->ndim;
  static const int esz[6] = {0, 1, 2, 4, 4, 8};
  static const int wq[6] = {0, 8, 16, 32, 32, 32};
  g->esz = esz[g->dtype];
  g->W = wq[g->dtype];
  g->isint = g->dtype <= ORC_I32;
  g->H = g->isint ? 32 : 48;
  if (g->mode == ORC_LOSSLESS && !g->isint) return ORC_E_UNSUPPORTED;
  for (int i = 0; i < 3; i++) { g->n[i] = 1; g->b[i] = 1; }
  int off = 3 - g->ndim;
  int64_t B = 1;
  for (int i = 0; i < g->ndim; i++) {
    if (p->brick[i] < 1 || p->brick[i] > 16384) return ORC_E_INVALID;
    g->n[off + i] = (int64_t)p->dims[i];
    g->b[off + i] = p->brick[i];
    B *= p->brick[i];
  }
  if (B < 64 || B > 16384 || B % 4 != 0) return ORC_E_INVALID;
  g->N = (p->flags & ORC_FLAG_GROUP8) ? 8 : 4;
  if (g->b[2] % g->N != 0 || B % g->N != 0) return ORC_E_INVALID; /* reading: groups never straddle rows */
  for (int i = 0; i < 3; i++) {
    if (g->n[i] < 0 || g->n[i] > ((int64_t)1 << 40)) return ORC_E_INVALID;
  }
  g->B = (int)B;
  g->G = (int)(B / g->N);
  g->nblocks = 1;
  int64_t ns = 1, nbytes_in;
  for (int i = 0; i < 3; i++) {
    g->nb[i] = (g->n[i] + g->b[i] - 1) / g->b[i];
    /* counts that do not fit the index types are refused, not wrapped */
    if (__builtin_mul_overflow(g->nblocks, g->nb[i], &g->nblocks)) return ORC_E_UNSUPPORTED;
    if (__builtin_mul_overflow(ns, g->n[i], &ns)) return ORC_E_UNSUPPORTED;
  }
  if (__builtin_mul_overflow(ns, (int64_t)g->esz, &nbytes_in) || nbytes_in > ((int64_t)1 << 56))
    return ORC_E_UNSUPPORTED;
  if (g->nblocks > (int64_t)0x7FFFFFFF) return ORC_E_UNSUPPORTED;
  uint32_t allowed = ALLOWED[g->ndim] | (g->fk ? 0x08u : 0u);
  uint32_t m = p->stream_mask ? p->stream_mask : allowed;
  if (m & ~allowed) return ORC_E_INVALID;
  if (g->mode == ORC_FIXED_RATE)
    m = (m | 1u) & 0x7Fu;
  else
    m = m | 0x81u;
  g->mask = m;
  if (g->isint) { g->cmin = -512; g->cmax = 0; }
  else { g->cmin = -17120; g->cmax = 16383; }
  g->code = 0;
  if (g->mode != ORC_LOSSLESS) {
    if (p->code < g->cmin || p->code > g->cmax) return ORC_E_INVALID;
    g->code = p->code;
  }
  if (g->mode == ORC_FIXED_RATE) {
    double words;
    if (forced_budget >= 0) {
      words = forced_budget;
    } else {
      if (!(p->rate > 0.0) || !isfinite(p->rate)) return ORC_E_INVALID;
      /* budget: whole 32-bit words per block, header included (reading) */
      words = floor((double)g->B * 8.0 * g->esz / (p->rate * 32.0));
    }
    /* an all-zero block needs its header and ceil((G-1)/2) pair tokens */
    int min_words = (g->H + 4 * (g->G / 2) + 31) / 32;
    if (words < min_words || words > 65535.0) return ORC_E_INVALID;
    g->budget = (int)words;
  }
  if (g->mode == ORC_FIXED_QUALITY) {
    if (!(p->target_corr > 0.0 && p->target_corr <= 1.0)) return ORC_E_INVALID;
  }
  if (g->mode == ORC_ADAPTIVE_RATE) {
    /* target words per block, from the rate as in fixed rate (reading) */
    double words;
    if (forced_budget >= 0) {
      words = forced_budget;
    } else {
      if (!(p->rate > 0.0) || !isfinite(p->rate)) return ORC_E_INVALID;
      words = floor((double)g->B * 8.0 * g->esz / (p->rate * 32.0));
    }
    if (words < 1.0 || words > 65535.0) return ORC_E_INVALID;
    g->target = (int)words;
  }
  return ORC_OK;
}

static int setup_geom(const orc_params* p, geom* g) { return setup_geom_b(p, g, -1); }

/* ------------------------------------------------------------------------ */
/* samples */

static double xval(const void* x, int dtype, int64_t i) {
  switch (dtype) {
    case ORC_I8: return (double)((const int8_t*)x)[i];
    case ORC_I16: return (double)((const int16_t*)x)[i];
    case ORC_I32: return (double)((const int32_t*)x)[i];
    case ORC_F32: return (double)((const float*)x)[i];
    default: return ((const double*)x)[i];
  }
}

/* Array index of brick position p of block j, or -1 when the position lies
 * past the array edge ("absent"). Bricks in row-major brick order, samples
 * row-major inside a brick, x fastest (reading for N-d data). */
static int64_t sample_index(const geom* g, int64_t j, int p) {
  int64_t bx = j % g->nb[2];
  int64_t t = j / g->nb[2];
  int64_t by = t % g->nb[1];
  int64_t bz = t / g->nb[1];
  int64_t x = p % g->b[2];
  int64_t y = (p / g->b[2]) % g->b[1];
  int64_t z = p / (g->b[2] * g->b[1]);
  int64_t X = bx * g->b[2] + x, Y = by * g->b[1] + y, Z = bz * g->b[0] + z;
  if (X >= g->n[2] || Y >= g->n[1] || Z >= g->n[0]) return -1;
  return (Z * g->n[1] + Y) * g->n[2] + X;
}

/* ------------------------------------------------------------------------ */
/* attenuator (Sec. 6: multiply each sample by a per-block floating-point
 * value).  Reading: the value is taken from the grid
 * g(c) = (16 + f) * 2^(k - 4), c = 16 k + f, 0 <= f < 16 -- 16 steps per
 * octave, every g(c) exact in binary64; g(0) = 1. */

double orc_gain(int32_t c) {
  int64_t k = floordiv16(c);
  int64_t f = c - 16 * k;
  return ldexp((double)(16 + f), (int)(k - 4));
}

/* R[f] = 16 / (16 + f): the mantissa of 1/g(c) (reading, inverse attenuator). */
double orc_inv_gain_mantissa(int32_t f) { return 16.0 / (double)(16 + f); }

/* Largest code c in [cmin, cmax] with fl64(M * g(c)) <= lim.  M * g(c) is
 * non-decreasing in c (g increases, rounding is monotone), and the caller
 * guarantees the predicate holds at cmin, so bisection finds it. */
static int largest_code(double M, double lim, int cmin, int cmax) {
  if (M * orc_gain(cmax) <= lim) return cmax;
  int lo = cmin, hi = cmax;
  while (hi - lo > 1) {
    int mid = lo + ((hi - lo) >> 1);
    if (M * orc_gain(mid) <= lim) lo = mid; else hi = mid;
  }
  return lo;
}

/* Bracket of one block with maximum magnitude M: c_cap is the largest code
 * whose products stay within the 32-bit quantizer range (ints: 0, so the
 * attenuator never amplifies an integer); c_floor is the largest code at
 * which every sample rounds to zero (|x g| <= 1/2). */
static void bracket(const geom* g, double M, int* cf, int* cc) {
  *cc = g->isint ? 0 : largest_code(M, 2147483647.0, g->cmin, g->cmax);
  *cf = largest_code(M, 0.5, g->cmin, g->cmax);
}

static int clamp_code(int c, int cf, int cc) {
  if (c < cf) c = cf;
  if (c > cc) c = cc;
  return c;
}

/* Quantizer (reading): a = rint(fl64(x * g(c))), rint half-to-even. */
static int64_t quantize(double x, int c) { return (int64_t)rint(x * orc_gain(c)); }

/* Dequantizer (reading): y = ldexp(fl64(a * R[f]), -k). */
static double dequantize(int64_t a, int c) {
  int64_t k = floordiv16(c);
  int64_t f = c - 16 * k;
  return ldexp((double)a * orc_inv_gain_mantissa((int32_t)f), (int)(-k));
}

/* ------------------------------------------------------------------------ */
/* redundancy remover (Sec. 5 derivatives, Sec. 6 filtered streams) */

static int64_t wrapW(int64_t v, int W) {
  uint64_t m = (W >= 64) ? ~(uint64_t)0 : (((uint64_t)1 << W) - 1);
  uint64_t u = (uint64_t)v & m;
  if (W < 64 && ((u >> (W - 1)) & 1)) u |= ~m;
  return (int64_t)u;
}

/* One difference along an axis of the brick; the neighbour outside the
 * brick counts as 0 (reading). */
static void diff_axis(const int64_t* f, int64_t* o, const int64_t* b, int axis) {
  int64_t B = b[0] * b[1] * b[2];
  int64_t stride = axis == 2 ? 1 : (axis == 1 ? b[2] : b[2] * b[1]);
  for (int64_t p = 0; p < B; p++) {
    int64_t coord = axis == 2 ? p % b[2] : (axis == 1 ? (p / b[2]) % b[1] : p / (b[2] * b[1]));
    o[p] = f[p] - (coord > 0 ? f[p - stride] : 0);
  }
}

/* Filter stream of a 1-d block: v[p] = a[p] - sgn a[p - k] (0 before the
 * block's start). */
static void filter_block(const int64_t* a, int64_t* v, int64_t B, int k, int neg) {
  for (int64_t p = 0; p < B; p++) {
    int64_t prev = p >= k ? a[p - k] : 0;
    v[p] = neg ? a[p] + prev : a[p] - prev;
  }
}

/* Candidate stream s of a brick (reading): 0 samples, 1 dx, 2 dx dx, 3 dy
 * (1-d arrays with a filter: the filter stream), 4 dz, 5 dx dy, 6 dx dy dz,
 * all modulo 2^W. Stream 7 (verbatim) is not a transform. tmp must hold 2 B
 * values. */
static void make_stream(const int64_t* a, int64_t* v, int64_t* tmp, const int64_t* b, int W,
                        int s, int fk, int fneg) {
  int64_t B = b[0] * b[1] * b[2];
  int64_t* t1 = tmp;
  int64_t* t2 = tmp + B;
  switch (s) {
    case 1: diff_axis(a, v, b, 2); break;
    case 2: diff_axis(a, t1, b, 2); diff_axis(t1, v, b, 2); break;
    case 3:
      if (fk) filter_block(a, v, B, fk, fneg);
      else diff_axis(a, v, b, 1);
      break;
    case 4: diff_axis(a, v, b, 0); break;
    case 5: diff_axis(a, t1, b, 1); diff_axis(t1, v, b, 2); break;
    case 6: diff_axis(a, t1, b, 0); diff_axis(t1, t2, b, 1); diff_axis(t2, v, b, 2); break;
    default: memcpy(v, a, (size_t)B * sizeof(int64_t)); break;
  }
  for (int64_t p = 0; p < B; p++) v[p] = wrapW(v[p], W);
}

/* Inverse of one axis difference: running sum along the axis (mod 2^W). */
static void sum_axis(int64_t* f, const int64_t* b, int axis, int W) {
  int64_t B = b[0] * b[1] * b[2];
  int64_t stride = axis == 2 ? 1 : (axis == 1 ? b[2] : b[2] * b[1]);
  for (int64_t p = 0; p < B; p++) {
    int64_t coord = axis == 2 ? p % b[2] : (axis == 1 ? (p / b[2]) % b[1] : p / (b[2] * b[1]));
    if (coord > 0) f[p] = wrapW(f[p] + f[p - stride], W);
  }
}

/* Inverse of the filter: a[p] = v[p] + sgn a[p - k], in increasing p. */
static void unfilter_block(int64_t* v, int64_t B, int k, int neg, int W) {
  for (int64_t p = k; p < B; p++) v[p] = wrapW(neg ? v[p] - v[p - k] : v[p] + v[p - k], W);
}

static void unmake_stream(int64_t* v, const int64_t* b, int W, int s, int fk, int fneg) {
  if (s == 3 && fk) {
    unfilter_block(v, b[0] * b[1] * b[2], fk, fneg, W);
    return;
  }
  switch (s) {
    case 1: sum_axis(v, b, 2, W); break;
    case 2: sum_axis(v, b, 2, W); sum_axis(v, b, 2, W); break;
    case 3: sum_axis(v, b, 1, W); break;
    case 4: sum_axis(v, b, 0, W); break;
    case 5: sum_axis(v, b, 2, W); sum_axis(v, b, 1, W); break;
    case 6: sum_axis(v, b, 2, W); sum_axis(v, b, 1, W); sum_axis(v, b, 0, W); break;
    default: break;
  }
}

/* ------------------------------------------------------------------------ */
/* block floating point exponents (Sec. 5/6: one exponent per 4 samples) */

/* Minimal two's-complement width of one value (0 for 0). */
static int width_of(int64_t v) {
  if (v == 0) return 0;
  uint64_t m = v < 0 ? ~(uint64_t)v : (uint64_t)v;
  int n = 0;
  while (m) { n++; m >>= 1; }
  return n + 1;
}

/* Exponent code of a group of n samples: the width of its widest sample (0
 * if all are zero), saturated at 31 (reading: code 31 means 32 bits when
 * W = 32). */
static int group_eps(const int64_t* v, int n) {
  int w = 0;
  for (int k = 0; k < n; k++) {
    int t = width_of(v[k]);
    if (t > w) w = t;
  }
  return w > 31 ? 31 : w;
}

static int payload_width(int eps, int W) { return (W == 32 && eps == 31) ? 32 : eps; }

/* JEE, greedy left to right over i = 1..G-1 with d_i = eps_i - eps_{i-1}
 * (Sec. 6).  Reading of the code values: two differences (da, db) in
 * [-1, 1] -> 3 (da + 1) + (db + 1) in 0..8; one difference d in [-2, 2] ->
 * 11 + d in 9..13; otherwise the 8-bit token (14 + (eps >> 4), eps & 15).
 * Returns the number of 4-bit nibbles written. */
static int jee_tokens(const int* eps, int G, uint8_t* nib) {
  int n = 0;
  int i = 1;
  while (i <= G - 1) {
    int d = eps[i] - eps[i - 1];
    if (i + 1 <= G - 1 && d >= -1 && d <= 1) {
      int d2 = eps[i + 1] - eps[i];
      if (d2 >= -1 && d2 <= 1) {
        nib[n++] = (uint8_t)(3 * (d + 1) + (d2 + 1));
        i += 2;
        continue;
      }
    }
    if (d >= -2 && d <= 2) {
      nib[n++] = (uint8_t)(11 + d);
    } else {
      nib[n++] = (uint8_t)(14 + (eps[i] >> 4));
      nib[n++] = (uint8_t)(eps[i] & 15);
    }
    i += 1;
  }
  return n;
}

/* ------------------------------------------------------------------------ */
/* bit writer / reader: LSB-first inside little-endian 32-bit words (reading) */

typedef struct { uint32_t* w; int64_t cap_bits; int64_t pos; } bitw;

static void put_bits(bitw* bw, uint64_t v, int nbits) {
  for (int i = 0; i < nbits; i++) {
    if ((v >> i) & 1) {
      int64_t p = bw->pos + i;
      if (p < bw->cap_bits) bw->w[p >> 5] |= (uint32_t)1 << (p & 31);
    }
  }
  bw->pos += nbits;
}

typedef struct { const uint32_t* w; int64_t nbits; int64_t pos; int err; } bitr;

static uint64_t get_bits(bitr* br, int nbits) {
  uint64_t v = 0;
  for (int i = 0; i < nbits; i++) {
    int64_t p = br->pos + i;
    if (p >= br->nbits) { br->err = 1; return 0; }
    if ((br->w[p >> 5] >> (p & 31)) & 1) v |= (uint64_t)1 << i;
  }
  br->pos += nbits;
  return v;
}

static int64_t sext(uint64_t v, int nbits) {
  if (nbits == 0) return 0;
  if (nbits < 64 && ((v >> (nbits - 1)) & 1)) v |= ~(((uint64_t)1 << nbits) - 1);
  return (int64_t)v;
}

/* ------------------------------------------------------------------------ */
/* one block: scratch, costing, emission */

typedef struct {
  int64_t* a;    /* quantized samples (0 at absent positions) */
  int64_t* v;    /* stream values */
  int64_t* tmp;  /* 2B */
  int64_t* best; /* stream values of the chosen stream */
  double* x;     /* block samples (0 at absent positions) */
  uint8_t* valid;
  int* eps;
  int* beps;
  uint8_t* nib;
  uint8_t* bnib;
} scratch;

static int scratch_alloc(scratch* s, int B) {
  memset(s, 0, sizeof(*s));
  s->a = malloc(sizeof(int64_t) * B);
  s->v = malloc(sizeof(int64_t) * B);
  s->tmp = malloc(sizeof(int64_t) * 2 * B);
  s->best = malloc(sizeof(int64_t) * B);
  s->x = malloc(sizeof(double) * B);
  s->valid = malloc((size_t)B);
  s->eps = malloc(sizeof(int) * (B / 4));
  s->beps = malloc(sizeof(int) * (B / 4));
  s->nib = malloc((size_t)B);
  s->bnib = malloc((size_t)B);
  return (s->a && s->v && s->tmp && s->best && s->x && s->valid && s->eps && s->beps && s->nib &&
          s->bnib) ? ORC_OK : ORC_E_INVALID;
}

static void scratch_free(scratch* s) {
  free(s->a); free(s->v); free(s->tmp); free(s->best); free(s->x);
  free(s->valid); free(s->eps); free(s->beps); free(s->nib); free(s->bnib);
}

/* Gather block j: samples as doubles, validity, count and max magnitude. */
static int gather(const geom* g, const void* xin, int64_t j, scratch* s, double* M) {
  int nv = 0;
  double m = 0.0;
  for (int p = 0; p < g->B; p++) {
    int64_t idx = sample_index(g, j, p);
    s->valid[p] = idx >= 0;
    s->x[p] = idx >= 0 ? xval(xin, g->dtype, idx) : 0.0;
    if (idx >= 0) {
      nv++;
      double ax = fabs(s->x[p]);
      if (ax > m) m = ax;
    }
  }
  *M = m;
  return nv;
}

static void quantize_block(const geom* g, scratch* s, int c) {
  for (int p = 0; p < g->B; p++) {
    if (!s->valid[p]) s->a[p] = 0;
    else if (g->mode == ORC_LOSSLESS) s->a[p] = (int64_t)s->x[p];
    else s->a[p] = quantize(s->x[p], c);
  }
}

/* Size in bits of stream s for the current quantized block; leaves the
 * stream values in s->v, the exponents in s->eps and the tokens in s->nib. */
static int64_t cost_stream(const geom* g, scratch* s, int st, int* nnib) {
  if (st == 7) { *nnib = 0; return (int64_t)g->H + (int64_t)g->B * g->W; }
  make_stream(s->a, s->v, s->tmp, g->b, g->W, st, g->fk, g->fneg);
  for (int p = 0; p < g->B; p++)
    if (!s->valid[p]) s->v[p] = 0; /* absent positions carry 0 (reading) */
  int64_t bits = g->H;
  for (int i = 0; i < g->G; i++) {
    s->eps[i] = group_eps(s->v + g->N * i, g->N);
    bits += g->N * payload_width(s->eps[i], g->W);
  }
  *nnib = jee_tokens(s->eps, g->G, s->nib);
  return bits + 4 * (int64_t)(*nnib);
}

/* Best stream over a mask (fewest bits, ties to the lowest id, Sec. 6),
 * copying its values/exponents/tokens to the "best" slots. */
static int64_t best_stream(const geom* g, scratch* s, uint32_t mask, int* st_out, int* nnib_out) {
  int64_t best = -1;
  int bs = -1, bn = 0;
  for (int st = 0; st < 8; st++) {
    if (!((mask >> st) & 1)) continue;
    int nn;
    int64_t bits = cost_stream(g, s, st, &nn);
    if (best < 0 || bits < best) {
      best = bits; bs = st; bn = nn;
      if (st != 7) {
        memcpy(s->best, s->v, sizeof(int64_t) * g->B);
        memcpy(s->beps, s->eps, sizeof(int) * g->G);
        memcpy(s->bnib, s->nib, (size_t)nn);
      }
    }
  }
  *st_out = bs;
  *nnib_out = bn;
  return best;
}

/* Cost of one fixed stream at code c (re-quantizes the block). */
static int64_t cost_at(const geom* g, scratch* s, int st, int c, int* nn) {
  quantize_block(g, s, c);
  return cost_stream(g, s, st, nn);
}

/* Fixed-rate gain search ("cap-and-descend", reading of the adaptive loop of
 * Sec. 6 in per-block form): start at c = clamp(c_p); choose the stream with
 * the fewest bits there; if it fits the budget stop; else step down one
 * octave at a time (never below c_floor, where every sample is 0) until it
 * fits; then bisect between the last fitting and the last failing code. */
static int fixed_rate_search(const geom* g, scratch* s, int cp, int cf, int cc, uint32_t mask,
                             int* st_out) {
  int64_t budget_bits = (int64_t)g->budget * 32;
  int c = clamp_code(cp, cf, cc);
  quantize_block(g, s, c);
  int st, nn;
  int64_t bits = best_stream(g, s, mask & 0x7Fu, &st, &nn);
  *st_out = st;
  if (bits <= budget_bits) return c;
  int hi = c;
  for (;;) {
    c = c - 16 < cf ? cf : c - 16;
    if (cost_at(g, s, st, c, &nn) <= budget_bits) break;
    hi = c;
  }
  int lo = c;
  while (hi - lo > 1) {
    int mid = lo + ((hi - lo) >> 1);
    if (cost_at(g, s, st, mid, &nn) <= budget_bits) lo = mid; else hi = mid;
  }
  return lo;
}

/* Emit one block (reading of the layout): header | JEE tokens | payload,
 * LSB-first, padded with zeros to a word (variable modes) or to the budget
 * (fixed rate).  Header (ints, 32 bits): [0:2] stream, [3:7] first exponent,
 * [8:17] code (two's complement), [18:31] zero.  Floats (48 bits): [0:2]
 * stream, [3:7] first exponent, [8:23] code, [24:47] zero. */
static int64_t emit_block(const geom* g, scratch* s, int st, int c, int nnib, uint32_t* words,
                          int cap_words) {
  memset(words, 0, sizeof(uint32_t) * (size_t)cap_words);
  bitw bw = {words, (int64_t)cap_words * 32, 0};
  int eps0 = st == 7 ? 0 : s->beps[0];
  put_bits(&bw, (uint64_t)st, 3);
  put_bits(&bw, (uint64_t)eps0, 5);
  if (g->isint) {
    put_bits(&bw, (uint64_t)((uint32_t)c & 0x3FFu), 10);
    put_bits(&bw, 0, 14);
  } else {
    put_bits(&bw, (uint64_t)((uint32_t)c & 0xFFFFu), 16);
    put_bits(&bw, 0, 24);
  }
  if (st == 7) {
    for (int p = 0; p < g->B; p++) put_bits(&bw, (uint64_t)s->a[p], g->W);
  } else {
    for (int t = 0; t < nnib; t++) put_bits(&bw, s->bnib[t], 4);
    for (int i = 0; i < g->G; i++) {
      int pw = payload_width(s->beps[i], g->W);
      for (int k = 0; k < g->N; k++) put_bits(&bw, (uint64_t)s->best[g->N * i + k], pw);
    }
  }
  return bw.pos;
}

static int max_block_words(const geom* g) { return (g->H + g->B * g->W + 31) / 32; }

/* Operating-point rule for one block: 0 lossless, 1 fixed-rate search from
 * `code`, 2 fixed quality at clamp(code). */
typedef struct { int rule; int code; uint32_t mask; int lag_st; } oprule;  /* lag_st: stream to use (lagged), or -1 */

/* Analyse (and, if words != NULL, emit) block j.  Returns the number of
 * words; leaves the quantized block in s->a and its samples in s->x. */
static int do_block(const geom* g, const void* xin, int64_t j, const oprule* r, scratch* s,
                    uint32_t* words, int cap_words, int* st_out, int* cj_out, int64_t* bits_out,
                    int* nvalid) {
  double M;
  int nv = gather(g, xin, j, s, &M);
  if (nvalid) *nvalid = nv;
  int cf, cc;
  bracket(g, M, &cf, &cc);
  int c, st, nn;
  int64_t bits;
  if (r->rule == ORC_LOSSLESS && r->lag_st >= 0) {
    /* the block's own best stream is reported (for the next block); the
     * block is coded with the previous block's */
    c = 0;
    quantize_block(g, s, c);
    int own;
    best_stream(g, s, r->mask, &own, &nn);
    /* a lagged stream that would code the block above its verbatim size
     * gives way to verbatim (stream 7), so no block outgrows the bound */
    int use = r->lag_st;
    bits = cost_stream(g, s, use, &nn);
    if (use != 7 && bits > cost_stream(g, s, 7, &nn)) {
      use = 7;
      bits = cost_stream(g, s, use, &nn);
    } else {
      bits = cost_stream(g, s, use, &nn);  /* s->v, eps, nib of the stream used */
    }
    memcpy(s->best, s->v, sizeof(int64_t) * g->B);
    memcpy(s->beps, s->eps, sizeof(int) * g->G);
    memcpy(s->bnib, s->nib, (size_t)nn);
    int nw = (int)((bits + 31) / 32);
    if (words) {
      if (nw > cap_words) return -1;
      int64_t pos = emit_block(g, s, use, c, nn, words, nw);
      if (pos != bits) return -2;
    }
    *st_out = own;
    *cj_out = c;
    *bits_out = bits;
    return nw;
  } else if (r->rule == ORC_LOSSLESS) {
    c = 0;
    quantize_block(g, s, c);
    bits = best_stream(g, s, r->mask, &st, &nn);
  } else if (r->rule == ORC_FIXED_QUALITY) {
    c = clamp_code(r->code, cf, cc);
    quantize_block(g, s, c);
    bits = best_stream(g, s, r->mask, &st, &nn);
  } else {
    c = fixed_rate_search(g, s, r->code, cf, cc, r->mask, &st);
    quantize_block(g, s, c);
    /* refresh the chosen stream's values at the final code */
    bits = cost_stream(g, s, st, &nn);
    memcpy(s->best, s->v, sizeof(int64_t) * g->B);
    memcpy(s->beps, s->eps, sizeof(int) * g->G);
    memcpy(s->bnib, s->nib, (size_t)nn);
  }
  int nw = g->budget ? g->budget : (int)((bits + 31) / 32);
  if (words) {
    if (nw > cap_words) return -1;
    int64_t pos = emit_block(g, s, st, c, nn, words, nw);
    if (pos != bits) return -2; /* internal consistency: size formula == emitted bits */
  }
  *st_out = st;
  *cj_out = c;
  *bits_out = bits;
  return nw;
}

/* ------------------------------------------------------------------------ */
/* stream container (reading): 64-byte header, for variable-size modes an
 * index of uint16 block lengths (words) plus one uint64 word offset per 64
 * blocks, then the blocks from a 16-byte aligned offset. */

#define ORC_MAGIC 0x58415041u

static uint64_t area_offset(const geom* g) {
  if (g->mode == ORC_FIXED_RATE) return 64;
  uint64_t nb = (uint64_t)g->nblocks;
  uint64_t lens = (2 * nb + 7) / 8 * 8;
  uint64_t sbo = 8 * ((nb + 63) / 64);
  uint64_t o = 64 + lens + sbo;
  return (o + 15) / 16 * 16;
}

static void put16(uint8_t* b, uint16_t v) { b[0] = (uint8_t)v; b[1] = (uint8_t)(v >> 8); }
static void put32(uint8_t* b, uint32_t v) { for (int i = 0; i < 4; i++) b[i] = (uint8_t)(v >> (8 * i)); }
static void put64(uint8_t* b, uint64_t v) { for (int i = 0; i < 8; i++) b[i] = (uint8_t)(v >> (8 * i)); }
static uint16_t get16(const uint8_t* b) { return (uint16_t)(b[0] | (b[1] << 8)); }
static uint32_t get32(const uint8_t* b) { uint32_t v = 0; for (int i = 0; i < 4; i++) v |= (uint32_t)b[i] << (8 * i); return v; }
static uint64_t get64(const uint8_t* b) { uint64_t v = 0; for (int i = 0; i < 8; i++) v |= (uint64_t)b[i] << (8 * i); return v; }

int orc_encode_bound(const orc_params* p, uint64_t* bound) {
  geom g;
  int e = setup_geom(p, &g);
  if (e) return e;
  uint64_t per = g.budget ? (uint64_t)g.budget : (uint64_t)max_block_words(&g);
  *bound = area_offset(&g) + 4 * per * (uint64_t)g.nblocks;
  return ORC_OK;
}

static int check_finite(const geom* g, const void* x) {
  if (g->isint) return ORC_OK;
  uint64_t n = (uint64_t)(g->n[0] * g->n[1] * g->n[2]);
  for (uint64_t i = 0; i < n; i++)
    if (!isfinite(xval(x, g->dtype, (int64_t)i))) return ORC_E_NONFINITE;
  return ORC_OK;
}

static oprule rule_of(const geom* g) {
  oprule r;
  /* adaptive rate codes each block as fixed quality at its requested code */
  r.rule = g->mode == ORC_ADAPTIVE_RATE ? ORC_FIXED_QUALITY : g->mode;
  r.code = g->code;
  r.mask = g->mask;
  r.lag_st = -1;
  return r;
}

int orc_encode(const void* x, const orc_params* p, void* out, uint64_t cap, uint64_t* nbytes) {
  geom g;
  int e = setup_geom(p, &g);
  if (e) return e;
  uint64_t bound;
  orc_encode_bound(p, &bound);
  if (cap < bound) return ORC_E_CAPACITY;
  e = check_finite(&g, x);
  if (e) return e;
  uint8_t* o = (uint8_t*)out;
  uint64_t area = area_offset(&g);
  memset(o, 0, area);
  scratch s;
  if (scratch_alloc(&s, g.B)) { scratch_free(&s); return ORC_E_INVALID; }
  oprule r = rule_of(&g);
  const int lagged = (p->flags & ORC_FLAG_LAGGED) != 0;
  if (lagged) r.lag_st = 0;  /* block 0: stream 0 */
  /* adaptive rate: the controller's window and state (a requested code) */
  const int adapt = g.mode == ORC_ADAPTIVE_RATE;
  const int lo = g.code - ORC_ADAPT_HALF < g.cmin ? g.cmin : g.code - ORC_ADAPT_HALF;
  const int hi = g.code + ORC_ADAPT_HALF - 1 > g.cmax ? g.cmax : g.code + ORC_ADAPT_HALF - 1;
  int state = g.code;
  uint64_t wpos = 0;
  int cap_words = g.budget ? g.budget : max_block_words(&g);
  uint8_t* lens = o + 64;
  uint8_t* sbo = o + 64 + (2 * (uint64_t)g.nblocks + 7) / 8 * 8;
  for (int64_t j = 0; j < g.nblocks; j++) {
    uint32_t* w = (uint32_t*)(void*)(o + area + 4 * wpos);
    int st, cj;
    int64_t bits;
    if (adapt) r.code = state;
    int nw = do_block(&g, x, j, &r, &s, w, cap_words, &st, &cj, &bits, NULL);
    if (nw < 0) { scratch_free(&s); return ORC_E_INVALID; }
    if (lagged) r.lag_st = st;
    if (adapt) {
      /* feedback: one code step towards the target packet size */
      if (nw < g.target) state += 1;
      else if (nw > g.target) state -= 1;
      if (state < lo) state = lo;
      if (state > hi) state = hi;
    }
    if (g.mode != ORC_FIXED_RATE) {
      if (j % 64 == 0) put64(sbo + 8 * (j / 64), wpos);
      put16(lens + 2 * j, (uint16_t)nw);
    }
    wpos += (uint64_t)nw;
  }
  scratch_free(&s);
  put32(o + 0, ORC_MAGIC);
  put16(o + 4, 1);
  o[6] = (uint8_t)g.dtype;
  o[7] = (uint8_t)g.mode;
  o[8] = (uint8_t)(g.ndim | (g.N == 8 ? 0x10 : 0)); /* bit 4: groups of 8 */
  o[9] = (uint8_t)g.mask;
  put16(o + 10, (uint16_t)(adapt ? g.target : g.budget));
  put32(o + 12, (uint32_t)g.code);
  for (int i = 0; i < 3; i++) put64(o + 16 + 8 * i, i < (int)p->ndim ? p->dims[i] : 0);
  for (int i = 0; i < 3; i++) put16(o + 40 + 2 * i, (uint16_t)(i < (int)p->ndim ? p->brick[i] : 0));
  o[46] = (uint8_t)g.fk;  /* filter stream: stride and sign (0 0: none) */
  o[47] = (uint8_t)g.fneg;
  put64(o + 48, (uint64_t)g.nblocks);
  put64(o + 56, wpos);
  *nbytes = area + 4 * wpos;
  return ORC_OK;
}

/* Rebuild parameters from a stream header; validates every field. */
static int parse_header(const uint8_t* b, uint64_t nbytes, orc_params* p, geom* g,
                        uint64_t* payload_words) {
  if (nbytes < 64) return ORC_E_CORRUPT;
  if (get32(b) != ORC_MAGIC || get16(b + 4) != 1) return ORC_E_CORRUPT;
  memset(p, 0, sizeof(*p));
  p->size = sizeof(orc_params);
  p->dtype = b[6];
  p->mode = b[7];
  p->ndim = b[8] & 0x0F;
  if (b[8] & 0xE0) return ORC_E_CORRUPT;
  if (b[8] & 0x10) p->flags |= ORC_FLAG_GROUP8;
  p->stream_mask = b[9];
  if (p->ndim < 1 || p->ndim > 3) return ORC_E_CORRUPT;
  for (int i = 0; i < 3; i++) {
    uint64_t d = get64(b + 16 + 8 * i);
    uint16_t k = get16(b + 40 + 2 * i);
    if (i < (int)p->ndim) { p->dims[i] = d; p->brick[i] = k; }
    else if (d != 0 || k != 0) return ORC_E_CORRUPT;
  }
  if (b[46] > 16 || b[47] > 1 || (b[47] && !b[46])) return ORC_E_CORRUPT;
  if (b[46]) p->flags |= ORC_FILTER(b[46], b[47]);
  p->code = (int32_t)get32(b + 12);
  int budget = get16(b + 10);
  if (p->mode == ORC_FIXED_RATE || p->mode == ORC_ADAPTIVE_RATE) {
    uint32_t B = 1;
    for (int i = 0; i < (int)p->ndim; i++) B *= p->brick[i];
    static const int esz[6] = {0, 1, 2, 4, 4, 8};
    if (p->dtype < 1 || p->dtype > 5 || budget == 0) return ORC_E_CORRUPT;
    p->rate = (double)B * 8.0 * esz[p->dtype] / (32.0 * (double)budget); /* informative */
  } else {
    if (budget != 0) return ORC_E_CORRUPT;
    p->rate = 0.0;
  }
  p->target_corr = 0.5;
  int e = setup_geom_b(p, g, (p->mode == ORC_FIXED_RATE || p->mode == ORC_ADAPTIVE_RATE) ? budget : -1);
  if (e) return ORC_E_CORRUPT;
  if (g->mask != p->stream_mask) return ORC_E_CORRUPT;
  if (get64(b + 48) != (uint64_t)g->nblocks) return ORC_E_CORRUPT;
  *payload_words = get64(b + 56);
  if (g->mode == ORC_FIXED_RATE && *payload_words != (uint64_t)g->nblocks * (uint64_t)g->budget)
    return ORC_E_CORRUPT;
  return ORC_OK;
}

int orc_stream_info(const void* in, uint64_t nbytes, orc_params* p) {
  geom g;
  uint64_t pw;
  return parse_header((const uint8_t*)in, nbytes, p, &g, &pw);
}

/* Decode one block (inverse of emit_block) into s->a. */
static int decode_block(const geom* g, const uint32_t* w, int nwords, scratch* s, int* c_out) {
  bitr br = {w, (int64_t)nwords * 32, 0, 0};
  int st = (int)get_bits(&br, 3);
  int eps0 = (int)get_bits(&br, 5);
  int c;
  if (g->isint) {
    c = (int)sext(get_bits(&br, 10), 10);
    if (get_bits(&br, 14) != 0) return ORC_E_CORRUPT;
  } else {
    c = (int)sext(get_bits(&br, 16), 16);
    if (get_bits(&br, 24) != 0) return ORC_E_CORRUPT;
  }
  if (br.err) return ORC_E_CORRUPT;
  if (!((g->mask >> st) & 1)) return ORC_E_CORRUPT;
  if (g->mode == ORC_LOSSLESS ? c != 0 : (c < g->cmin || c > g->cmax)) return ORC_E_CORRUPT;
  int maxeps = g->W == 32 ? 31 : g->W;
  if (st == 7) {
    if (eps0 != 0) return ORC_E_CORRUPT;
    for (int p = 0; p < g->B; p++) s->a[p] = sext(get_bits(&br, g->W), g->W);
  } else {
    if (eps0 > maxeps) return ORC_E_CORRUPT;
    s->eps[0] = eps0;
    int i = 1;
    while (i <= g->G - 1) {
      int t = (int)get_bits(&br, 4);
      if (br.err) return ORC_E_CORRUPT;
      if (t <= 8) {
        if (i + 1 > g->G - 1) return ORC_E_CORRUPT;
        s->eps[i] = s->eps[i - 1] + (t / 3 - 1);
        s->eps[i + 1] = s->eps[i] + (t % 3 - 1);
        if (s->eps[i] < 0 || s->eps[i] > maxeps || s->eps[i + 1] < 0 || s->eps[i + 1] > maxeps)
          return ORC_E_CORRUPT;
        i += 2;
      } else if (t <= 13) {
        s->eps[i] = s->eps[i - 1] + (t - 11);
        if (s->eps[i] < 0 || s->eps[i] > maxeps) return ORC_E_CORRUPT;
        i += 1;
      } else {
        int lo = (int)get_bits(&br, 4);
        s->eps[i] = (t - 14) * 16 + lo;
        if (s->eps[i] > maxeps) return ORC_E_CORRUPT;
        i += 1;
      }
    }
    for (int gi = 0; gi < g->G; gi++) {
      int pw = payload_width(s->eps[gi], g->W);
      for (int k = 0; k < g->N; k++) s->v[g->N * gi + k] = sext(get_bits(&br, pw), pw);
    }
    if (br.err) return ORC_E_CORRUPT;
    unmake_stream(s->v, g->b, g->W, st, g->fk, g->fneg);
    memcpy(s->a, s->v, sizeof(int64_t) * g->B);
  }
  if (br.err) return ORC_E_CORRUPT;
  /* padding after the last used bit must be zero */
  while (br.pos < br.nbits)
    if (get_bits(&br, 1)) return ORC_E_CORRUPT;
  *c_out = c;
  return ORC_OK;
}

static void store_y(const geom* g, void* y, int64_t idx, int64_t a, int c) {
  if (g->mode == ORC_LOSSLESS) {
    switch (g->dtype) {
      case ORC_I8: ((int8_t*)y)[idx] = (int8_t)a; break;
      case ORC_I16: ((int16_t*)y)[idx] = (int16_t)a; break;
      default: ((int32_t*)y)[idx] = (int32_t)a; break;
    }
    return;
  }
  double d = dequantize(a, c);
  if (g->dtype == ORC_F32) { ((float*)y)[idx] = (float)d; return; }
  if (g->dtype == ORC_F64) { ((double*)y)[idx] = d; return; }
  double r = rint(d);
  double lo = g->dtype == ORC_I8 ? -128.0 : (g->dtype == ORC_I16 ? -32768.0 : -2147483648.0);
  double hi = g->dtype == ORC_I8 ? 127.0 : (g->dtype == ORC_I16 ? 32767.0 : 2147483647.0);
  if (r < lo) r = lo;
  if (r > hi) r = hi;
  switch (g->dtype) {
    case ORC_I8: ((int8_t*)y)[idx] = (int8_t)r; break;
    case ORC_I16: ((int16_t*)y)[idx] = (int16_t)r; break;
    default: ((int32_t*)y)[idx] = (int32_t)r; break;
  }
}

int orc_decode(const void* in, uint64_t nbytes, void* y, uint64_t cap_bytes) {
  const uint8_t* b = (const uint8_t*)in;
  orc_params p;
  geom g;
  uint64_t pwords;
  int e = parse_header(b, nbytes, &p, &g, &pwords);
  if (e) return e;
  uint64_t nsamp = (uint64_t)(g.n[0] * g.n[1] * g.n[2]);
  if (cap_bytes < nsamp * (uint64_t)g.esz) return ORC_E_CAPACITY;
  uint64_t area = area_offset(&g);
  if (nbytes < area + 4 * pwords) return ORC_E_CORRUPT;
  const uint8_t* lens = b + 64;
  const uint8_t* sbo = b + 64 + (2 * (uint64_t)g.nblocks + 7) / 8 * 8;
  scratch s;
  if (scratch_alloc(&s, g.B)) { scratch_free(&s); return ORC_E_INVALID; }
  uint64_t wpos = 0;
  int maxw = max_block_words(&g);
  for (int64_t j = 0; j < g.nblocks; j++) {
    int nw;
    if (g.mode == ORC_FIXED_RATE) {
      nw = g.budget;
    } else {
      if (j % 64 == 0 && get64(sbo + 8 * (j / 64)) != wpos) { scratch_free(&s); return ORC_E_CORRUPT; }
      nw = get16(lens + 2 * j);
      if (nw < 1 || nw > maxw) { scratch_free(&s); return ORC_E_CORRUPT; }
    }
    if (wpos + (uint64_t)nw > pwords) { scratch_free(&s); return ORC_E_CORRUPT; }
    const uint32_t* w = (const uint32_t*)(const void*)(b + area + 4 * wpos);
    int c;
    e = decode_block(&g, w, nw, &s, &c);
    if (e) { scratch_free(&s); return e; }
    for (int p2 = 0; p2 < g.B; p2++) {
      int64_t idx = sample_index(&g, j, p2);
      if (idx >= 0) store_y(&g, y, idx, s.a[p2], c);
    }
    wpos += (uint64_t)nw;
  }
  scratch_free(&s);
  if (wpos != pwords) return ORC_E_CORRUPT;
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* statistics (Sec. 4): fp64 with Neumaier compensated sums */

typedef struct { double s, c; } ksum;

static void kadd(ksum* k, double v) {
  double t = k->s + v;
  if (fabs(k->s) >= fabs(v)) k->c += (k->s - t) + v;
  else k->c += (v - t) + k->s;
  k->s = t;
}
static double kval(const ksum* k) { return k->s + k->c; }

typedef struct { ksum x, y, d, xx, yy, dd, ds; double maxd; uint64_t n; } acc;

static void acc_init(acc* a) { memset(a, 0, sizeof(*a)); }

static void acc_add(acc* a, double x, double y) {
  double d = x - y;
  kadd(&a->x, x);
  kadd(&a->y, y);
  kadd(&a->d, d);
  kadd(&a->xx, x * x);
  kadd(&a->yy, y * y);
  kadd(&a->dd, d * d);
  kadd(&a->ds, d * (x + y));
  if (fabs(d) > a->maxd) a->maxd = fabs(d);
  a->n++;
}

/* r in the cancellation-free form 1 - r = (Sdd - (|x| - |y|)^2) / (2 |x| |y|),
 * |x| - |y| = Sds / (|x| + |y|): algebraically the printed formula of Sec. 4. */
static void finish_r(double sxx, double syy, double sdd, double sds, double* r, double* omr) {
  if (sxx == 0.0 && syy == 0.0) { *r = 1.0; *omr = 0.0; return; }
  if (sxx == 0.0 || syy == 0.0) { *r = 0.0; *omr = 1.0; return; }
  double nx = sqrt(sxx), ny = sqrt(syy);
  double dn = sds / (nx + ny);
  *omr = (sdd - dn * dn) / (2.0 * nx * ny);
  *r = 1.0 - *omr;
}

static void finish_metrics(const acc* a, orc_metrics* m) {
  m->n = a->n;
  m->sum_x = kval(&a->x);
  m->sum_y = kval(&a->y);
  m->sum_d = kval(&a->d);
  m->sxx = kval(&a->xx);
  m->syy = kval(&a->yy);
  m->sdd = kval(&a->dd);
  m->sds = kval(&a->ds);
  m->max_abs_d = a->maxd;
  finish_r(m->sxx, m->syy, m->sdd, m->sds, &m->r, &m->one_minus_r);
  if (m->sdd == 0.0) { m->snr_db = INFINITY; m->rms_pct = 0.0; m->rms_db = -INFINITY; }
  else if (m->sxx == 0.0) { m->snr_db = -INFINITY; m->rms_pct = INFINITY; m->rms_db = INFINITY; }
  else {
    m->snr_db = 10.0 * log10(m->sxx / m->sdd);
    m->rms_pct = 100.0 * sqrt(m->sdd / m->sxx);
    m->rms_db = -m->snr_db;
  }
  double n = (double)(a->n ? a->n : 1);
  m->mean_x = m->sum_x / n;
  m->mean_y = m->sum_y / n;
  m->mean_d = m->sum_d / n;
}

int orc_stats(const double* x, const double* y, uint64_t n, orc_metrics* m) {
  acc a;
  acc_init(&a);
  for (uint64_t i = 0; i < n; i++) acc_add(&a, x[i], y[i]);
  memset(m, 0, sizeof(*m));
  finish_metrics(&a, m);
  ksum vx = {0, 0}, vy = {0, 0}, vd = {0, 0};
  for (uint64_t i = 0; i < n; i++) {
    double ex = x[i] - m->mean_x, ey = y[i] - m->mean_y, ed = (x[i] - y[i]) - m->mean_d;
    kadd(&vx, ex * ex); kadd(&vy, ey * ey); kadd(&vd, ed * ed);
  }
  double nn = (double)(n ? n : 1);
  m->std_x = sqrt(kval(&vx) / nn);
  m->std_y = sqrt(kval(&vy) / nn);
  m->std_d = sqrt(kval(&vd) / nn);
  return ORC_OK;
}

/* decoded value of a quantized sample, as the output dtype returns it */
static double yval(const geom* g, int64_t a, int c) {
  if (g->mode == ORC_LOSSLESS) return (double)a;
  double d = dequantize(a, c);
  if (g->dtype == ORC_F32) return (double)(float)d;
  if (g->dtype == ORC_F64) return d;
  double r = rint(d);
  double lo = g->dtype == ORC_I8 ? -128.0 : (g->dtype == ORC_I16 ? -32768.0 : -2147483648.0);
  double hi = g->dtype == ORC_I8 ? 127.0 : (g->dtype == ORC_I16 ? 32767.0 : 2147483647.0);
  return r < lo ? lo : (r > hi ? hi : r);
}

/* ------------------------------------------------------------------------ */
/* profiler (Sec. 4), reading of the procedure:
 *   1. one pass: N, max|x| -> whole-array bracket [c_floor, c_cap];
 *   2. operating point by bisection (mid = lo + ((hi - lo) >> 1)):
 *      fixed quality: smallest code with r >= target on the full array;
 *      fixed rate: largest code at which >= ceil(0.9 n_sub) subsample blocks
 *      fit the budget with their best stream;
 *   3. stream mask = {0, 7} + streams chosen by >= max(1, ceil(n_sub/100))
 *      subsample blocks at the chosen code;
 *   4. rate-correlation curve: 17 codes, quarter-octave (4-code) steps,
 *      +-2 octaves around the chosen code, on the subsample;
 *   5. metrics at the chosen operating point on the full array.
 * Subsample: blocks j = 0 mod 16, or all blocks when there are < 1024. */

static int in_sub(const geom* g, int64_t j) { return g->nblocks < 1024 ? 1 : (j % 16 == 0); }

typedef struct { const geom* g; const void* x; scratch* s; int* cf; int* cc; } pctx;

/* r over the full array with every block at clamp(c) (fixed quality) */
static double r_full(pctx* P, int c, acc* out) {
  const geom* g = P->g;
  acc a;
  acc_init(&a);
  for (int64_t j = 0; j < g->nblocks; j++) {
    double M;
    gather(g, P->x, j, P->s, &M);
    int cj = clamp_code(c, P->cf[j], P->cc[j]);
    quantize_block(g, P->s, cj);
    for (int p = 0; p < g->B; p++)
      if (P->s->valid[p]) acc_add(&a, P->s->x[p], yval(g, P->s->a[p], cj));
  }
  if (out) *out = a;
  double r, omr;
  finish_r(kval(&a.xx), kval(&a.yy), kval(&a.dd), kval(&a.ds), &r, &omr);
  return r;
}

/* number of subsample blocks whose best BFPE stream fits the budget at clamp(c) */
static int64_t fits_count(pctx* P, int c) {
  const geom* g = P->g;
  int64_t n = 0;
  for (int64_t j = 0; j < g->nblocks; j++) {
    if (!in_sub(g, j)) continue;
    double M;
    gather(g, P->x, j, P->s, &M);
    quantize_block(g, P->s, clamp_code(c, P->cf[j], P->cc[j]));
    int st, nn;
    int64_t bits = best_stream(g, P->s, g->mask & 0x7Fu, &st, &nn);
    if (bits <= (int64_t)g->budget * 32) n++;
  }
  return n;
}

int orc_profile(const void* x, const orc_params* p, orc_profile_result* res) {
  geom g;
  orc_params q = *p;
  if (q.mode == ORC_ADAPTIVE_RATE) return ORC_E_UNSUPPORTED; /* the loop sets its own codes */
  if (q.mode != ORC_LOSSLESS) q.code = 0; /* the profiler chooses the code */
  int e = setup_geom(&q, &g);
  if (e) return e;
  e = check_finite(&g, x);
  if (e) return e;
  memset(res, 0, sizeof(*res));
  res->size = sizeof(*res);
  scratch s;
  int* cf = malloc(sizeof(int) * (size_t)(g.nblocks ? g.nblocks : 1));
  int* cc = malloc(sizeof(int) * (size_t)(g.nblocks ? g.nblocks : 1));
  if (scratch_alloc(&s, g.B) || !cf || !cc) {
    scratch_free(&s); free(cf); free(cc);
    return ORC_E_INVALID;
  }
  /* 1. pass over the array */
  double Mall = 0.0;
  uint64_t n_sub = 0;
  for (int64_t j = 0; j < g.nblocks; j++) {
    double M;
    gather(&g, x, j, &s, &M);
    bracket(&g, M, &cf[j], &cc[j]);
    if (M > Mall) Mall = M;
    if (in_sub(&g, j)) n_sub++;
  }
  int CF, CC;
  bracket(&g, Mall, &CF, &CC);
  res->c_floor = CF;
  res->c_cap = CC;
  res->n_sub = (uint32_t)n_sub;
  pctx P = {&g, x, &s, cf, cc};

  /* 2. operating point */
  int code = 0;
  if (g.mode == ORC_FIXED_QUALITY) {
    double rt = p->target_corr;
    if (CF >= CC) {
      code = CC;
    } else {
      double r = r_full(&P, CC, NULL);
      res->n_probes++;
      if (fabs(r - rt) < 1e-11) res->flags |= ORC_NEAR_TIE;
      if (!(r >= rt)) {
        code = CC;
      } else {
        int lo = CF, hi = CC;
        while (hi - lo > 1) {
          int mid = lo + ((hi - lo) >> 1);
          r = r_full(&P, mid, NULL);
          res->n_probes++;
          if (fabs(r - rt) < 1e-11) res->flags |= ORC_NEAR_TIE;
          if (r >= rt) hi = mid; else lo = mid;
        }
        code = hi;
      }
    }
  } else if (g.mode == ORC_FIXED_RATE) {
    int64_t need = (int64_t)((9 * n_sub + 9) / 10);
    if (CF >= CC) {
      code = CC;
    } else {
      res->n_probes++;
      if (fits_count(&P, CC) >= need) {
        code = CC;
      } else {
        int lo = CF, hi = CC;
        while (hi - lo > 1) {
          int mid = lo + ((hi - lo) >> 1);
          res->n_probes++;
          if (fits_count(&P, mid) >= need) lo = mid; else hi = mid;
        }
        code = lo;
      }
    }
  }
  res->code = code;

  /* 3. stream mask from the subsample histogram at the chosen code */
  int64_t hist[8] = {0};
  for (int64_t j = 0; j < g.nblocks; j++) {
    if (!in_sub(&g, j)) continue;
    double M;
    gather(&g, x, j, &s, &M);
    int cj = g.mode == ORC_LOSSLESS ? 0 : clamp_code(code, cf[j], cc[j]);
    quantize_block(&g, &s, cj);
    int st, nn;
    uint32_t m = g.mode == ORC_FIXED_RATE ? (g.mask & 0x7Fu) : g.mask;
    best_stream(&g, &s, m, &st, &nn);
    hist[st]++;
  }
  int64_t thresh = (int64_t)((n_sub + 99) / 100);
  if (thresh < 1) thresh = 1;
  uint32_t mask = 0x81u;
  for (int st = 0; st < 8; st++)
    if (hist[st] >= thresh) mask |= 1u << st;
  mask &= (g.mask | 0x81u);
  res->stream_mask = mask;

  /* 4. rate-correlation curve on the subsample (variable-size encoding at
   *    each code with the pruned mask, verbatim allowed) */
  geom gc = g;
  gc.mode = ORC_FIXED_QUALITY;
  gc.budget = 0;
  gc.mask = mask | 0x81u;
  for (int t = 0; t < ORC_NCURVE; t++) {
    int ct = code + 4 * (t - ORC_NCURVE / 2);
    if (ct < g.cmin) ct = g.cmin;
    if (ct > g.cmax) ct = g.cmax;
    acc a;
    acc_init(&a);
    double in_bits = 0.0, out_bits = 0.0;
    oprule r = {ORC_FIXED_QUALITY, ct, gc.mask};
    for (int64_t j = 0; j < g.nblocks; j++) {
      if (!in_sub(&g, j)) continue;
      int st, cj, nv;
      int64_t bits;
      int nw = do_block(&gc, x, j, &r, &s, NULL, 0, &st, &cj, &bits, &nv);
      in_bits += (double)nv * 8.0 * g.esz;
      out_bits += 32.0 * nw;
      for (int p2 = 0; p2 < g.B; p2++)
        if (s.valid[p2]) acc_add(&a, s.x[p2], yval(&gc, s.a[p2], cj));
    }
    double rr, omr;
    finish_r(kval(&a.xx), kval(&a.yy), kval(&a.dd), kval(&a.ds), &rr, &omr);
    res->curve[t].code = ct;
    res->curve[t].ratio = out_bits > 0 ? in_bits / out_bits : 0.0;
    res->curve[t].r = rr;
  }

  /* 5. metrics at the operating point, full array */
  geom gm = g;
  gm.mask = g.mode == ORC_FIXED_RATE ? (mask & 0x7Fu) | 1u : (mask | 0x81u);
  gm.code = code;
  oprule r = rule_of(&gm);
  acc a;
  acc_init(&a);
  uint64_t words = 0;
  for (int64_t j = 0; j < g.nblocks; j++) {
    int st, cj, nv;
    int64_t bits;
    int nw = do_block(&gm, x, j, &r, &s, NULL, 0, &st, &cj, &bits, &nv);
    words += (uint64_t)nw;
    for (int p2 = 0; p2 < g.B; p2++)
      if (s.valid[p2]) acc_add(&a, s.x[p2], yval(&gm, s.a[p2], cj));
  }
  orc_metrics* m = &res->m;
  finish_metrics(&a, m);
  m->enc_bytes = area_offset(&g) + 4 * words;
  uint64_t nsamp = (uint64_t)(g.n[0] * g.n[1] * g.n[2]);
  m->ratio = m->enc_bytes ? (double)(nsamp * (uint64_t)g.esz) / (double)m->enc_bytes : 0.0;
  /* second pass for the population standard deviations */
  ksum vx = {0, 0}, vy = {0, 0}, vd = {0, 0};
  for (int64_t j = 0; j < g.nblocks; j++) {
    int st, cj, nv;
    int64_t bits;
    do_block(&gm, x, j, &r, &s, NULL, 0, &st, &cj, &bits, &nv);
    for (int p2 = 0; p2 < g.B; p2++) {
      if (!s.valid[p2]) continue;
      double xv = s.x[p2], yv = yval(&gm, s.a[p2], cj);
      double ex = xv - m->mean_x, ey = yv - m->mean_y, ed = (xv - yv) - m->mean_d;
      kadd(&vx, ex * ex); kadd(&vy, ey * ey); kadd(&vd, ed * ed);
    }
  }
  double nn = (double)(m->n ? m->n : 1);
  m->std_x = sqrt(kval(&vx) / nn);
  m->std_y = sqrt(kval(&vy) / nn);
  m->std_d = sqrt(kval(&vd) / nn);
  scratch_free(&s);
  free(cf);
  free(cc);
  return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* pieces exposed for pins */

/* r over the full array with every block at clamp(code) (the fixed-quality
 * predicate of the profiler's bisection) */
int orc_corr_at(const void* x, const orc_params* p, int32_t code, double* r) {
  geom g;
  orc_params q = *p;
  q.code = 0;
  q.mode = ORC_FIXED_QUALITY;
  int e = setup_geom(&q, &g);
  if (e) return e;
  scratch s;
  int* cf = malloc(sizeof(int) * (size_t)(g.nblocks ? g.nblocks : 1));
  int* cc = malloc(sizeof(int) * (size_t)(g.nblocks ? g.nblocks : 1));
  if (scratch_alloc(&s, g.B) || !cf || !cc) {
    scratch_free(&s); free(cf); free(cc);
    return ORC_E_INVALID;
  }
  for (int64_t j = 0; j < g.nblocks; j++) {
    double M;
    gather(&g, x, j, &s, &M);
    bracket(&g, M, &cf[j], &cc[j]);
  }
  pctx P = {&g, x, &s, cf, cc};
  *r = r_full(&P, code, NULL);
  scratch_free(&s);
  free(cf);
  free(cc);
  return ORC_OK;
}

int orc_block_bracket(const void* x, const orc_params* p, int64_t j, double* M, int32_t* c_floor,
                      int32_t* c_cap) {
  geom g;
  orc_params q = *p;
  q.code = 0;
  int e = setup_geom(&q, &g);
  if (e) return e;
  if (j < 0 || j >= g.nblocks) return ORC_E_INVALID;
  scratch s;
  if (scratch_alloc(&s, g.B)) { scratch_free(&s); return ORC_E_INVALID; }
  gather(&g, x, j, &s, M);
  int cf, cc;
  bracket(&g, *M, &cf, &cc);
  *c_floor = cf;
  *c_cap = cc;
  scratch_free(&s);
  return ORC_OK;
}

int orc_encode_block(const void* x, const orc_params* p, int64_t j, uint32_t* words,
                     int32_t cap_words, int32_t* nwords, int32_t* stream, int32_t* cj,
                     int32_t* used_bits) {
  geom g;
  int e = setup_geom(p, &g);
  if (e) return e;
  if (j < 0 || j >= g.nblocks) return ORC_E_INVALID;
  scratch s;
  if (scratch_alloc(&s, g.B)) { scratch_free(&s); return ORC_E_INVALID; }
  for (int p2 = 0; p2 < g.B; p2++) {
    int64_t idx = sample_index(&g, j, p2);
    if (idx >= 0 && !g.isint && !isfinite(xval(x, g.dtype, idx))) {
      scratch_free(&s);
      return ORC_E_NONFINITE;
    }
  }
  oprule r = rule_of(&g);
  int st, c;
  int64_t bits;
  int nw = do_block(&g, x, j, &r, &s, words, cap_words, &st, &c, &bits, NULL);
  scratch_free(&s);
  if (nw < 0) return ORC_E_CAPACITY;
  *nwords = nw;
  *stream = st;
  *cj = c;
  *used_bits = (int32_t)bits;
  return ORC_OK;
}

int orc_stream_values(const int64_t* a, const uint32_t* brick, int32_t W, int32_t s, int64_t* v) {
  int64_t b[3] = {brick[0], brick[1], brick[2]};
  int64_t B = b[0] * b[1] * b[2];
  if (s < 0 || s > 7 || B <= 0) return ORC_E_INVALID;
  int64_t* tmp = malloc(sizeof(int64_t) * 2 * (size_t)B);
  int64_t* aw = malloc(sizeof(int64_t) * (size_t)B);
  if (!tmp || !aw) { free(tmp); free(aw); return ORC_E_INVALID; }
  for (int64_t p = 0; p < B; p++) aw[p] = wrapW(a[p], W);
  make_stream(aw, v, tmp, b, W, s == 7 ? 0 : s, 0, 0);
  free(tmp);
  free(aw);
  return ORC_OK;
}

int orc_stream_values_f(const int64_t* a, const uint32_t* brick, int32_t W, int32_t s, int32_t fk,
                        int32_t fneg, int64_t* v) {
  int64_t b[3] = {brick[0], brick[1], brick[2]};
  int64_t B = b[0] * b[1] * b[2];
  if (s < 0 || s > 7 || B <= 0 || fk < 0 || fk > 16) return ORC_E_INVALID;
  int64_t* tmp = malloc(sizeof(int64_t) * 2 * (size_t)B);
  int64_t* aw = malloc(sizeof(int64_t) * (size_t)B);
  if (!tmp || !aw) { free(tmp); free(aw); return ORC_E_INVALID; }
  for (int64_t p = 0; p < B; p++) aw[p] = wrapW(a[p], W);
  make_stream(aw, v, tmp, b, W, s == 7 ? 0 : s, fk, fneg);
  free(tmp);
  free(aw);
  return ORC_OK;
}

int orc_stream_inverse(const int64_t* v, const uint32_t* brick, int32_t W, int32_t s, int32_t fk,
                       int32_t fneg, int64_t* a) {
  int64_t b[3] = {brick[0], brick[1], brick[2]};
  int64_t B = b[0] * b[1] * b[2];
  if (s < 0 || s > 7 || B <= 0 || fk < 0 || fk > 16) return ORC_E_INVALID;
  for (int64_t p = 0; p < B; p++) a[p] = wrapW(v[p], W);
  if (s != 7) unmake_stream(a, b, W, s, fk, fneg);
  return ORC_OK;
}

int orc_group_eps(const int64_t* v, int32_t G, int32_t W, int32_t* eps) {
  (void)W;
  for (int i = 0; i < G; i++) eps[i] = group_eps(v + 4 * i, 4);
  return ORC_OK;
}

int orc_group_eps_n(const int64_t* v, int32_t G, int32_t n, int32_t* eps) {
  if (n < 1) return ORC_E_INVALID;
  for (int i = 0; i < G; i++) eps[i] = group_eps(v + (int64_t)n * i, n);
  return ORC_OK;
}

int orc_jee_tokens(const int32_t* eps, int32_t G, uint8_t* nibbles, int32_t* n_nibbles) {
  int* e = malloc(sizeof(int) * (size_t)G);
  if (!e) return ORC_E_INVALID;
  for (int i = 0; i < G; i++) e[i] = eps[i];
  *n_nibbles = jee_tokens(e, G, nibbles);
  free(e);
  return ORC_OK;
}
