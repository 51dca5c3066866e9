/*
 * apax_oracle.h -- plain single-threaded CPU reference for the APAX numerical
 * encoder, decoder and profiler (A. Wegener, "Universal Numerical Encoder and
 * Profiler ...", arXiv 1303.4994).
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists so that tests, the smoke
 * check and the CPU-baseline leg of the benchmark can check the GPU library
 * against an independent, obviously-correct implementation.  It shares no
 * source, header, table or helper with the GPU path, and the GPU path never
 * loads it.
 *
 * Every array pointer here is HOST memory owned by the caller.  Integer
 * return values: 0 on success, a negative ORC_E_* code otherwise.
 *
 * The bitstream format this oracle writes is the reading of the paper frozen
 * in the project design notes (block header, JEE tokens, BFPE payload,
 * 64-byte stream header, block-length index); the comments in
 * apax_oracle.c cite the paper section each step follows.
 */
#ifndef APAX_ORACLE_H
#define APAX_ORACLE_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_I8 = 1, ORC_I16 = 2, ORC_I32 = 3, ORC_F32 = 4, ORC_F64 = 5 };
enum { ORC_LOSSLESS = 0, ORC_FIXED_RATE = 1, ORC_FIXED_QUALITY = 2, ORC_ADAPTIVE_RATE = 3 };

/* ORC_ADAPTIVE_RATE (Sec. 6, the attenuator under an adaptive loop that
 * converges to the desired packet size), reading: a target of
 * T = floor(B * 8 * esz / (rate * 32)) words per block (1..65535) and a start
 * code c0 (p->code).  The controller's state is a requested code in the
 * window [lo, hi] = [max(cmin, c0 - 32), min(cmax, c0 + 31)], starting at c0.
 * Blocks are visited in order; block j is coded as in fixed quality at
 * clamp(state, c_floor_j, c_cap_j) (best stream, verbatim allowed) and takes
 * n_j words; then the state steps by +1 if n_j < T, -1 if n_j > T, 0 if
 * equal, clamped to the window.  The stream container is the variable-size
 * one; its header carries T in the budget field and c0 in the code field. */
#define ORC_ADAPT_HALF 32
enum {
  ORC_OK = 0,
  ORC_E_INVALID = -1,
  ORC_E_UNSUPPORTED = -2,
  ORC_E_CAPACITY = -3,
  ORC_E_CORRUPT = -4,
  ORC_E_NONFINITE = -5
};
#define ORC_NEAR_TIE 1u
#define ORC_NCURVE 17

typedef struct {
  uint32_t size;        /* sizeof(orc_params) */
  uint32_t dtype;       /* ORC_I8 .. ORC_F64 */
  uint32_t ndim;        /* 1..3 */
  uint32_t mode;        /* ORC_LOSSLESS, ORC_FIXED_RATE, ORC_FIXED_QUALITY, ORC_ADAPTIVE_RATE */
  uint64_t dims[3];     /* slow -> fast, first ndim entries used */
  uint32_t brick[3];    /* slow -> fast, first ndim entries used */
  uint32_t stream_mask; /* bit s allows stream s; 0 = every stream of ndim */
  double rate;          /* fixed / adaptive rate: input bits per encoded bit */
  double target_corr;   /* fixed-quality: correlation target */
  int32_t code;         /* gain code (fixed-rate / adaptive start code, fixed-quality code) */
  uint32_t flags;       /* ORC_FLAG_LAGGED: lossless only */
} orc_params;

/* Lagged stream choice (Sec. 6, the streaming hardware's form): block j is
 * coded with the stream that was best for block j-1 (block 0: stream 0), or
 * verbatim where that stream would code it above the verbatim size; each
 * block's header still names the stream it uses, so decoding is unchanged. */
#define ORC_FLAG_LAGGED 1u

/* Filter stream (Sec. 5 oversampling / Sec. 6 redundancy remover: filtered
 * versions of the attenuated series, the signal monitor's centre frequency
 * telling which nearby samples of a modulated waveform are correlated),
 * reading: 1-d arrays only, stream id 3 (unused by 1-d derivatives) becomes
 * v[p] = a[p] - s a[p - k] inside the block (a[p - k] = 0 before the block's
 * start), k = 1..16 and s = +1 or -1 from p->flags = ORC_FILTER(k, s < 0);
 * the stream header records k and s (bytes 46, 47). */
/* Groups of 8 (Sec. 6: one exponent per group of N = 4 or 8 samples),
 * reading: p->flags |= ORC_FLAG_GROUP8 gives every exponent (and its JEE
 * position) 8 consecutive samples of a brick row; B and the brick's x extent
 * must be multiples of 8.  The stream header records it in bit 4 of the
 * ndim byte (byte 8). */
#define ORC_FLAG_GROUP8 0x4000u

#define ORC_FILTER(k, neg) ((((uint32_t)(k)) << 8) | ((neg) ? 0x2000u : 0u))
#define ORC_FILTER_K(flags) (((flags) >> 8) & 0x1Fu)
#define ORC_FILTER_NEG 0x2000u

typedef struct {
  double r, one_minus_r, snr_db, rms_pct, rms_db;
  double mean_x, mean_y, mean_d, std_x, std_y, std_d, max_abs_d;
  double sxx, syy, sdd, sds, sum_x, sum_y, sum_d;
  double ratio;
  uint64_t n, enc_bytes;
} orc_metrics;

typedef struct {
  int32_t code;
  int32_t pad;
  double ratio;
  double r;
} orc_curve_point;

typedef struct {
  uint32_t size;
  int32_t code;          /* recommended gain code (c* or c_p); 0 for lossless */
  uint32_t stream_mask;  /* pruned stream mask recommended to the encoder */
  uint32_t flags;        /* ORC_NEAR_TIE */
  int32_t c_floor, c_cap;/* whole-array bracket */
  uint32_t n_sub;        /* number of subsample blocks */
  uint32_t n_probes;     /* bisection probes taken */
  orc_curve_point curve[ORC_NCURVE];
  orc_metrics m;
} orc_profile_result;

/* whole-array calls */
int orc_encode_bound(const orc_params* p, uint64_t* bound);
int orc_encode(const void* x, const orc_params* p, void* out, uint64_t cap, uint64_t* nbytes);
int orc_decode(const void* in, uint64_t nbytes, void* y, uint64_t cap_bytes);
int orc_stream_info(const void* in, uint64_t nbytes, orc_params* p);
int orc_profile(const void* x, const orc_params* p, orc_profile_result* res);

/* pieces exposed for pins and for sampled comparisons at full size */
double orc_gain(int32_t c);
double orc_inv_gain_mantissa(int32_t f);
int orc_block_bracket(const void* x, const orc_params* p, int64_t j, double* M,
                      int32_t* c_floor, int32_t* c_cap);
int orc_encode_block(const void* x, const orc_params* p, int64_t j, uint32_t* words,
                     int32_t cap_words, int32_t* nwords, int32_t* stream, int32_t* cj,
                     int32_t* used_bits);
int orc_stream_values(const int64_t* a, const uint32_t* brick, int32_t W, int32_t s,
                      int64_t* v);
/* the same with a filter (fk = 0: none; fneg: s = -1) and the inverse */
int orc_stream_values_f(const int64_t* a, const uint32_t* brick, int32_t W, int32_t s, int32_t fk,
                        int32_t fneg, int64_t* v);
int orc_stream_inverse(const int64_t* v, const uint32_t* brick, int32_t W, int32_t s, int32_t fk,
                       int32_t fneg, int64_t* a);
int orc_group_eps(const int64_t* v, int32_t G, int32_t W, int32_t* eps);
/* exponents of G groups of n samples each */
int orc_group_eps_n(const int64_t* v, int32_t G, int32_t n, int32_t* eps);
int orc_jee_tokens(const int32_t* eps, int32_t G, uint8_t* nibbles, int32_t* n_nibbles);
int orc_stats(const double* x, const double* y, uint64_t n, orc_metrics* m);
int orc_corr_at(const void* x, const orc_params* p, int32_t code, double* r);

#ifdef __cplusplus
}
#endif
#endif
