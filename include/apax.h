/*
 * apax.h -- C ABI of libapax.so, the MI355X (gfx950) implementation of the
 * APAX numerical encoder, decoder and profiler (A. Wegener, arXiv 1303.4994).
 *
 * What the calls compute (paper sections):
 *   apax_profile  Sec. 4  profiler: recommended operating point (gain code) for a
 *                         correlation target (fixed quality) or a rate (fixed
 *                         rate), the rate-correlation curve (Window 1) and the
 *                         time-domain summary metrics (Window 2: r, SNR, RMS
 *                         residual in % and dB, means, standard deviations).
 *   apax_encode   Sec. 6  encoder: per-block attenuation, redundancy removal
 *                         (derivative streams, Sec. 5), block floating point with
 *                         one exponent per 4 samples, joint exponent encoding
 *                         (JEE) of exponent differences, 4-byte (ints) / 6-byte
 *                         (floats) block headers.
 *   apax_decode   Sec. 1/6 decoder: the inverse of every encoder stage.
 * The bit-level format (token codes, header fields, bit order, container) is
 * not given in the paper; the library implements the reading documented with
 * the project (LSB-first 32-bit words, [header][tokens][payload] per block,
 * 64-byte stream header, uint16 block-length index).
 *
 * Conventions for every call
 *   - Array, stream and workspace pointers are DEVICE pointers allocated and
 *     owned by the caller (hipMalloc / torch).  Result structs of
 *     apax_profile are HOST memory owned by the caller.
 *   - Work is enqueued on the caller's stream; apax_encode/apax_decode return
 *     before the GPU finishes.  apax_profile and apax_status synchronize the
 *     stream.
 *   - Return value: APAX_OK (0) or a negative APAX_E_* code.  Errors found on
 *     the host (bad parameters, too-small buffers) return before anything is
 *     enqueued.  Errors found on the device (non-finite input, corrupt
 *     stream) are recorded in a status word inside the workspace; read them
 *     with apax_status after the call completes.
 *   - Calls that share one workspace must not overlap in time.
 *   - Input arrays are C-contiguous (row-major, dims[ndim-1] fastest).
 */
#ifndef APAX_H
#define APAX_H
#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

/* dtypes (the integer and float types of the paper's Table 2) */
enum { APAX_I8 = 1, APAX_I16 = 2, APAX_I32 = 3, APAX_F32 = 4, APAX_F64 = 5 };
/* modes: lossless (integers only, unit gain), fixed rate (per-block word
 * budget, Sec. 6 "compressed packet size"), fixed quality (correlation
 * target), adaptive rate (Sec. 6: the attenuator's gain under a feedback loop
 * that converges to the desired packet size).
 * Adaptive rate: a target of T = floor(B * 8 * esz / (rate * 32)) words per
 * block (1..65535) and a start code c0 = p->code.  The controller's state is a
 * requested code in [max(cmin, c0 - APAX_ADAPT_HALF), min(cmax, c0 +
 * APAX_ADAPT_HALF - 1)], starting at c0; blocks are coded in order, block j
 * as in fixed quality at clamp(state, c_floor_j, c_cap_j) (best stream,
 * verbatim allowed) in n_j words, after which the state steps by +1 if
 * n_j < T, -1 if n_j > T, 0 if equal, clamped to the window.  The stream is
 * the variable-size container (its header holds T in the budget field and c0
 * in the code field) and decodes like any other.  The loop runs as a parallel
 * scan over per-block transition maps, exactly reproducing the sequential
 * order.  Not accepted by the profiler or APAX_CODE_PROFILED
 * (APAX_E_UNSUPPORTED): the loop sets its own codes.  Batches and the server
 * run such items as single calls. */
enum { APAX_LOSSLESS = 0, APAX_FIXED_RATE = 1, APAX_FIXED_QUALITY = 2, APAX_ADAPTIVE_RATE = 3 };
#define APAX_ADAPT_HALF 32
enum {
  APAX_OK = 0,
  APAX_E_INVALID = -1,     /* bad parameters */
  APAX_E_UNSUPPORTED = -2, /* valid request the library does not implement (lossless floats; the
                              profiler in adaptive rate; blocks above 256 samples or groups of 8 on a
                              device whose workgroups get too little LDS for them) */
  APAX_E_CAPACITY = -3,    /* output or workspace buffer too small */
  APAX_E_CORRUPT = -4,     /* stream fails validation */
  APAX_E_NONFINITE = -5,   /* NaN or Inf in the input */
  APAX_E_HIP = -6,         /* HIP runtime error */
  APAX_E_INTERNAL = -7     /* device-side safety limit hit (should not happen) */
};
#define APAX_NEAR_TIE 1u /* profile: a bisection probe was within 1e-11 of the target */
#define APAX_NCURVE 17
/* apax_params.code for apax_encode: take the code and stream mask
 * (intersected with p->stream_mask; lossless mode: the mask) from the
 * profile the workspace holds, on the device.  The stream header records the
 * adopted values.  A workspace without a profile result (or one for another
 * code range) makes the encode fall back to code 0 and the caller's mask and
 * report APAX_E_INVALID through apax_status.  Not accepted by batches. */
#define APAX_CODE_PROFILED ((int32_t)0x80000000)

typedef struct apax_params {
  uint32_t size;        /* = sizeof(apax_params) */
  uint32_t dtype;       /* APAX_I8 .. APAX_F64 */
  uint32_t ndim;        /* 1..3 */
  uint32_t mode;        /* APAX_LOSSLESS / APAX_FIXED_RATE / APAX_FIXED_QUALITY / APAX_ADAPTIVE_RATE */
  uint64_t dims[3];     /* array extent, slow -> fast; first ndim entries used */
  uint32_t brick[3];    /* block (brick) extent, slow -> fast; product B in
                           [64, 16384], B % 4 == 0 (Sec. 6), brick[ndim-1] % 4 == 0 */
  uint32_t stream_mask; /* bit s allows stream s (0 samples, 1 dx, 2 dx dx, 3 dy,
                           4 dz, 5 dx dy, 6 dx dy dz, 7 verbatim); 0 = all of ndim.
                           Variable modes always add streams 0 and 7; fixed rate
                           adds 0 and never uses 7. */
  double rate;          /* fixed rate: input bits per encoded bit (e.g. 4.0) */
  double target_corr;   /* fixed quality (profile): correlation target, e.g. 0.99999 */
  int32_t code;         /* gain code g(c) = (16+f) 2^(k-4), c = 16k+f: fixed-rate
                           start code / fixed-quality code (from apax_profile);
                           ignored in lossless mode.  ints: [-512, 0];
                           floats: [-17120, 16383] */
  uint32_t flags;       /* APAX_FLAG_LAGGED (lossless only) | APAX_FILTER(k, neg) (1-d) | APAX_FLAG_GROUP8 */
} apax_params;

/* apax_params.flags: the streaming hardware's lagged stream choice (Sec. 6):
 * block j is coded with the stream that was best for block j-1 (block 0:
 * stream 0), as an encoder that decides after the block has streamed out.
 * Lossless mode only; the stream format is unchanged (each block header
 * names its stream).  Batches and the server run such items as single calls. */
#define APAX_FLAG_LAGGED 1u

/* apax_params.flags: the filter stream (Sec. 5 oversampling, Sec. 6: the
 * redundancy remover's filtered versions of the series, the signal monitor's
 * centre frequency telling which nearby samples of a modulated waveform are
 * correlated).  1-d arrays only: stream id 3 (unused by 1-d derivatives)
 * becomes v[n] = a[n] - s a[n - k] inside the block (a before the block's
 * start counts as 0), k = 1..16, s = +1 or -1 (neg), typically the stride and
 * sign apax_signal_monitor reports; allowed in every mode and mixed with the
 * other streams by the usual fewest-bits choice.  The stream header records
 * k and s (bytes 46, 47), so decoding needs no parameter.  Other ndim, k > 16
 * or a sign without a stride: APAX_E_INVALID. */
/* apax_params.flags: groups of 8 samples per exponent (Sec. 6: one exponent
 * per group of N = 4 or 8 samples; default 4).  Every exponent and JEE
 * position then covers 8 consecutive samples of a brick row: the block size
 * and the brick's x extent must be multiples of 8 (else APAX_E_INVALID).  The
 * stream header records it in bit 4 of the ndim byte (byte 8).  Encoded and
 * decoded, and profiled, by the one-workgroup-per-block kernels; batches and
 * the server run such items as single calls. */
#define APAX_FLAG_GROUP8 0x4000u

#define APAX_FILTER(k, neg) ((((uint32_t)(k)) << 8) | ((neg) ? 0x2000u : 0u))
#define APAX_FILTER_NEG 0x2000u

typedef struct apax_metrics {
  double r, one_minus_r;   /* Sec. 4 correlation (uncentered, as printed) */
  double snr_db;           /* 10 log10(sum x^2 / sum d^2), d = x - y */
  double rms_pct, rms_db;  /* RMS residual relative to RMS(x), in % and dB */
  double mean_x, mean_y, mean_d, std_x, std_y, std_d, max_abs_d;
  double sxx, syy, sdd, sds, sum_x, sum_y, sum_d; /* the sums behind the above */
  double ratio;            /* input bytes / encoded bytes (whole stream) */
  uint64_t n, enc_bytes;
} apax_metrics;

typedef struct apax_curve_point {
  int32_t code;
  int32_t pad;
  double ratio;
  double r;
} apax_curve_point;

typedef struct apax_profile_result {
  uint32_t size;          /* = sizeof(apax_profile_result) */
  int32_t code;           /* recommended code (c* fixed quality, c_p fixed rate, 0 lossless) */
  uint32_t stream_mask;   /* recommended (pruned) stream mask */
  uint32_t flags;         /* APAX_NEAR_TIE */
  int32_t c_floor, c_cap; /* whole-array code bracket */
  uint32_t n_sub;         /* subsample blocks (j % 16 == 0, or all if < 1024 blocks) */
  uint32_t n_probes;      /* bisection probes */
  apax_curve_point curve[APAX_NCURVE]; /* rate-correlation curve, Sec. 4 Window 1 */
  apax_metrics m;         /* metrics at the recommended point, full array */
} apax_profile_result;

/* Upper bound of the encoded stream size in bytes (exact for fixed rate). */
int apax_encode_bound(const apax_params* p, uint64_t* bytes);

/* Workspace bytes needed by apax_profile / apax_encode / apax_decode for p
 * (the maximum over the three calls). */
int apax_workspace_size(const apax_params* p, uint64_t* bytes);

/* Sec. 4 profiler.  d_x: input array (p->dtype, p->dims).  Synchronous:
 * fills *h_out on return.  p->code is ignored.  Blocks of at most 256
 * samples (larger: APAX_E_UNSUPPORTED). */
int apax_profile(const void* d_x, const apax_params* p, apax_profile_result* h_out,
                 void* d_ws, uint64_t ws_bytes, hipStream_t stream);

/* The same profile, enqueued on `stream` without waiting: the result stays
 * in d_ws (device memory).  A later apax_encode of the same array with
 * p->code = APAX_CODE_PROFILED, the same workspace and stream adopts the
 * profile's code and stream mask on the device, so profile -> encode needs no
 * host round trip.  apax_profile_read reads the result when wanted. */
int apax_profile_async(const void* d_x, const apax_params* p, void* d_ws, uint64_t ws_bytes,
                       hipStream_t stream);

/* apax_profile_async that also records point_ready on `stream` as soon as
 * the operating point (code, stream mask) is final -- after the stream
 * histogram, before the curve and metrics passes.  Work that needs only the
 * operating point (an encode with APAX_CODE_PROFILED) can wait for that event
 * on another stream and overlap the rest of the profile. */
int apax_profile_async_point(const void* d_x, const apax_params* p, void* d_ws, uint64_t ws_bytes,
                             hipStream_t stream, hipEvent_t point_ready);

/* Profile and encode of one array in one launch sequence on `stream` (the
 * Sec. 4 profiler feeding the Sec. 6 encoder): the profile as
 * apax_profile_async, and the stream of d_x at the profiled operating point
 * (the bytes apax_encode writes with p->code = APAX_CODE_PROFILED) into
 * d_stream / *d_nbytes.  The encode is taken from the profile's metrics pass,
 * which already runs the encoder's per-block analysis at that point (fixed
 * rate: each block's gain search; every mode: each block's stream choice
 * and size).  Fixed rate: that pass also writes each block's words, and the
 * stream header is written before it.  Other modes: it records each block's
 * stream and size, and the encode only places, quantizes, forms that stream
 * and packs.  `encoded` (optional) is recorded
 * on `stream` as soon as the stream is complete, before the profile's
 * centred and curve passes, so a decode on another stream can overlap them.
 * p->code is ignored; d_ws holds the profile as after apax_profile_async.
 * The lagged choice, blocks of more than 256 samples and groups of 8 run the
 * plain encode after the profile (their passes record no per-block
 * choices). */
/* side (optional, else null): a second stream for two of the profile's
 * passes.  Then `forked` (an event the caller owns) is recorded on `stream`
 * at the end of the stream-histogram pass, `side` waits for it and runs the
 * curve pass beside the metrics pass; `forked` is recorded again at the end
 * of the metrics pass kernel and `side` then runs that pass's reduction
 * (the means) and the centred pass, while the encode (and whatever the
 * caller enqueues after it on `stream`, such as a decode of the stream) runs
 * on `stream`.  The profile
 * result is complete when both streams have reached the end of this call's
 * work: join them (wait on `side`) before apax_profile_read or another
 * profile in d_ws.  side == stream, or side without forked: APAX_E_INVALID.
 * The lagged choice, wide blocks and groups of 8 run everything on `stream`. */
int apax_profile_encode_async(const void* d_x, const apax_params* p, void* d_ws, uint64_t ws_bytes,
                              void* d_stream, uint64_t cap, uint64_t* d_nbytes, hipStream_t stream,
                              hipEvent_t encoded, hipStream_t side, hipEvent_t forked);

/* Copies the operating point of the profile in d_ws_from into d_ws_to
 * (enqueued on `stream`), so an encode with APAX_CODE_PROFILED can run on its
 * own workspace while d_ws_from goes on with the profile. */
int apax_adopt_point(const void* d_ws_from, void* d_ws_to, hipStream_t stream);

/* Instrumentation for benchmarks: apax_profile with HIP events recorded on
 * `stream` just before and after the main kernel of each pass; pass_ms[i]
 * (APAX_NPASS entries) receives that kernel's duration for pass i, or -1 if
 * the pass did not run (the one-workgroup reduction after each pass lies
 * outside the pair).  Synchronous, like apax_profile. */
enum {
  APAX_PASS_MAX = 0,      /* max |x| pass (P1) */
  APAX_PASS_PROBE0 = 1,   /* bisection probe launches 1..9 (P2) */
  APAX_PASS_HIST = 10,    /* stream histogram at the chosen code (P3) */
  APAX_PASS_CURVE = 11,   /* the 17-code curve (P3) */
  APAX_PASS_METRICS = 12, /* metrics at the operating point (P4) */
  APAX_PASS_CENTRED = 13, /* centred sums for the standard deviations (P4) */
  APAX_NPASS = 14
};
int apax_profile_timed(const void* d_x, const apax_params* p, apax_profile_result* h_out,
                       float* pass_ms, void* d_ws, uint64_t ws_bytes, hipStream_t stream);
/* Instrumentation for benchmarks: apax_profile_encode_async on one stream
 * (the profile of Sec. 4, then the encode of Sec. 5-6 at its operating
 * point into d_stream, cap bytes, *d_nbytes; the same bytes) with the pass
 * events of apax_profile_timed.  In fixed-rate mode the metrics pass writes
 * the stream's blocks itself, so pass_ms[APAX_PASS_METRICS] times that
 * kernel.  Synchronous.  The lagged choice, blocks of more than 256 samples,
 * groups of 8 and empty arrays: APAX_E_UNSUPPORTED. */
int apax_profile_encode_timed(const void* d_x, const apax_params* p, apax_profile_result* h_out,
                              float* pass_ms, void* d_ws, uint64_t ws_bytes, void* d_stream, uint64_t cap,
                              uint64_t* d_nbytes, hipStream_t stream);

/* Sec. 4 Window 4: the 2-sigma signal-to-residual margin of the operating
 * point of the profile that d_ws holds (run apax_profile / _async on d_x with
 * the same p first; fixed rate uses the per-block codes of its metrics pass).
 * With d = x - y, y the decoded array: the ceil(0.045 n)-th smallest of the
 * per-sample ratios |x| / |d| (binary64; d = 0 gives +inf) in *h_ratio, and
 * 20 log10 of it in *h_db (-inf for a zero ratio).  Exact (a digit-by-digit
 * selection on the ratio's bit pattern: three passes over d_x, then two over
 * the ratios that share the first 26 bits of the answer, kept in d_ws's
 * partial-record region, or two more passes over d_x when they do not fit).
 * Uses the profile's partial records (spent by then; the profile result is
 * kept).  Synchronous; NaN for an empty array. */
int apax_s2r_margin(const void* d_x, const apax_params* p, double* h_ratio, double* h_db, void* d_ws,
                    uint64_t ws_bytes, hipStream_t stream);

/* Decode-on-read consumer (the "time to results" use of Sec. 1, Fig. 1): the
 * dot product sum_i y_i w_i of the array y a stream decodes with the array
 * d_w (same dtype and shape), computed while decoding -- y is never written.
 * Arguments as apax_decode; the result (binary64, deterministic order: per
 * tile, then tiles in order) goes to the device double *d_out.  Enqueued on
 * `stream`; corrupt streams are reported through apax_status. */
int apax_decode_dot(const void* h_hdr, const void* d_stream, uint64_t nbytes, const void* d_w, double* d_out,
                    void* d_ws, uint64_t ws_bytes, hipStream_t stream);

/* The same consumer on an uncompressed array (the baseline of the above):
 * *d_out = sum_i x_i w_i over n samples of `dtype`, binary64.  d_ws: at
 * least APAX_DOT_WGS * 8 bytes.  Enqueued on `stream`. */
#define APAX_DOT_WGS 1024
int apax_dot(const void* d_x, const void* d_w, uint32_t dtype, uint64_t n, double* d_out, void* d_ws,
             uint64_t ws_bytes, hipStream_t stream);

/* Sec. 4 Windows 3-4, spectral metrics of an array x and its decoded array y
 * (same dtype and n; device).  The paper names them without an estimator;
 * this library reads them as a Welch power spectrum of the samples in memory
 * order: segments of 1024 samples, hop 512, periodic Hann window
 * sin^2(pi i / 1024), one-sided bins 1..512 (no DC), P = mean over segments
 * of |DFT|^2 (binary64).  For x, y and d = x - y: peak = max P, floor = the
 * 256th smallest bin (nearest-rank median); resid_mean = mean of P_d; all in
 * dB (10 log10 P; -inf for 0); dr = peak_x - floor_x, srr = peak_x -
 * resid_mean, fft_s2r_margin = floor_x - resid_mean.  n < 1024: NaN fields,
 * 0 segments.  d_ws: at least apax_spectral_workspace_bytes().  Synchronous. */
typedef struct apax_spectral {
  double peak_x, floor_x, peak_y, floor_y, peak_d, floor_d;
  double resid_mean, dr, srr, fft_s2r_margin;
  uint64_t segments;
} apax_spectral;
uint64_t apax_spectral_workspace_bytes(void);
int apax_spectral_metrics(const void* d_x, const void* d_y, uint32_t dtype, uint64_t n, apax_spectral* h_out,
                          void* d_ws, uint64_t ws_bytes, hipStream_t stream);

/* Sec. 6 signal monitor of an array x (device, n samples of `dtype`, in
 * memory order, binary64 arithmetic).  The paper names its outputs (center
 * frequency, SNR) and says the center frequency tells which nearby samples
 * are correlated; this library reads them as:
 *   acf[k] = (R[k] / (n - k)) / (R[0] / n), R[k] = sum_{i >= k} x_i x_(i-k),
 *            k = 0..16 (zero for lags >= n, all zero when R[0] = 0);
 *   peak_bin = the first largest bin b of the Welch spectrum above (1..512),
 *   center_freq = b / 1024 cycles per sample, peak_db and floor_db as above,
 *   snr_db = 10 log10(mean bin / floor bin);
 *   stride = the smallest k in 1..16 whose phase m = b k mod 1024 (in
 *   1/1024 turns) lies nearest a multiple of 512; sign = +1 when m is nearer
 *   0 mod 1024 (a quarter turn counts as +1), else -1: x_i - sign x_(i-k)
 *   cancels a tone at bin b;
 *   gain_db = 10 log10(sum_{i >= k} x_i^2 / sum_{i >= k} (x_i - sign
 *   x_(i-k))^2) at k = stride (+inf for a zero residual, NaN for zero x).
 * n < 1024: only acf (NaN fields, peak_bin = stride = sign = segments = 0).
 * d_ws: at least apax_spectral_workspace_bytes(), 16-byte aligned
 * (APAX_E_CAPACITY otherwise).  Synchronous. */
typedef struct apax_monitor {
  double acf[17];
  double center_freq, peak_db, floor_db, snr_db, gain_db;
  int32_t peak_bin, stride, sign, pad;
  uint64_t segments;
} apax_monitor;
int apax_signal_monitor(const void* d_x, uint32_t dtype, uint64_t n, apax_monitor* h_out, void* d_ws,
                        uint64_t ws_bytes, hipStream_t stream);

/* Waits for `stream`, then fills *h_out from the profile that d_ws holds
 * (p: the parameters that profile was called with).  Same errors as
 * apax_profile. */
int apax_profile_read(const apax_params* p, apax_profile_result* h_out, const void* d_ws,
                        hipStream_t stream);

/* Sec. 6 encoder.  Writes the whole stream (header, index, blocks) to
 * d_stream (cap bytes, >= apax_encode_bound) and its byte length to
 * *d_nbytes (device uint64).  Asynchronous.  Non-finite input sets
 * APAX_E_NONFINITE in the workspace status.  Every block size of Sec. 6
 * (64..16384 samples); blocks above 256 samples run one workgroup per block
 * with the block in LDS (up to about 120 KB of it per workgroup at 16384). */
int apax_encode(const void* d_x, const apax_params* p, void* d_stream, uint64_t cap,
                uint64_t* d_nbytes, void* d_ws, uint64_t ws_bytes, hipStream_t stream);

/* Scratch bytes the library holds on each GPU for apax_encode_noalloc. */
#define APAX_NOALLOC_SCRATCH_BYTES (8ull << 20)

/* apax_encode for callers that cannot allocate device memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the
 * same stream bytes and byte count as apax_encode with the same arguments,
 * but no workspace argument.  Its scratch (status word, one byte per block
 * for the chosen stream and 4 bytes per 64 blocks for their word count, one
 * int32 per block with APAX_FLAG_LAGGED) lives in a library-owned device
 * array of APAX_NOALLOC_SCRATCH_BYTES (8 MiB) per GPU, which the GPU holds
 * until the process ends; the call itself allocates nothing (no hipMalloc,
 * no library allocation).  An array whose scratch would exceed 8 MiB returns
 * APAX_E_CAPACITY before anything is enqueued (about 7.9 million blocks
 * without the lagged choice, 1.6 million with it).  APAX_CODE_PROFILED is not
 * accepted (APAX_E_INVALID): no profile writes that scratch.
 * d_status (device int32, may be NULL) receives APAX_OK, APAX_E_NONFINITE or
 * APAX_E_INTERNAL once the encode has run.  Every call on one GPU shares its
 * scratch and keeps the last call's contents: calls that overlap in time on
 * one GPU (two host threads, or two streams) race and give undefined streams.
 * Asynchronous, enqueued on `stream` on the current device. */
int apax_encode_noalloc(const void* d_x, const apax_params* p, void* d_stream, uint64_t cap,
                        uint64_t* d_nbytes, int32_t* d_status, hipStream_t stream);

/* Decoder.  h_hdr: host copy of the first 64 bytes of the stream (the
 * parameters are taken from it; apax_stream_info parses it); d_stream: the
 * whole stream on the device, nbytes long; d_y: output array (cap bytes).
 * Asynchronous.  A malformed stream sets APAX_E_CORRUPT in the workspace
 * status (output then unspecified). */
int apax_decode(const void* h_hdr, const void* d_stream, uint64_t nbytes, void* d_y,
                uint64_t cap, void* d_ws, uint64_t ws_bytes, hipStream_t stream);

/* Parse a 64-byte stream header (host memory) into parameters. */
int apax_stream_info(const void* h_hdr, uint64_t n, apax_params* out);

/* Length in bytes of the whole stream whose 64-byte header h_hdr holds (host
 * memory, n >= 64 readable bytes): the header, the block-length index of the
 * variable-size modes and the block area.  APAX_E_CORRUPT when the header is
 * not a valid stream header or its payload size exceeds the largest encoding
 * of its blocks (fixed rate: differs from nblocks * budget words). */
int apax_stream_size(const void* h_hdr, uint64_t n, uint64_t* nbytes);

/* Clear the workspace status word (enqueued on stream). */
int apax_status_clear(void* d_ws, hipStream_t stream);

/* Synchronize stream and return the workspace status (APAX_OK or the first
 * device-side error of the calls since the last clear). */
int apax_status(const void* d_ws, hipStream_t stream);

const char* apax_strerror(int code);

/* ------------------------------------------------------------------------
 * Batches: many arrays (any sizes, dtypes, modes, ndim) encoded or decoded by
 * one persistent kernel launch per block-shape class (one launch when every
 * item has the same ndim and a block of 129..256 samples), optionally
 * replayed as a hipGraph.  Each item's output is byte-identical to a
 * separate apax_encode / apax_decode call.  Items the shared launch does not
 * take (blocks of more than 256 samples, groups of 8, the lagged choice,
 * adaptive rate) run in the same batch run as single-array calls, each with
 * its own region of the batch workspace and its own status word.  Launch geometry (waves per
 * workgroup, persistent workgroups per CU, tiles taken per work-queue
 * ticket) never changes any output; an autotuner chooses it. */
enum { APAX_OP_ENCODE = 0, APAX_OP_DECODE = 1 };

typedef struct apax_batch_item {
  apax_params p;        /* encode: the array's parameters; decode: ignored (from h_hdr) */
  const void* d_in;     /* encode: input array; decode: input stream (device) */
  void* d_out;          /* encode: stream buffer; decode: output array (device) */
  uint64_t in_bytes;    /* decode: stream length in bytes */
  uint64_t cap;         /* bytes available at d_out */
  uint64_t* d_nbytes;   /* encode: device uint64 receiving the stream length */
  const void* h_hdr;    /* decode: host copy of the stream's 64-byte header */
} apax_batch_item;

typedef struct apax_tune {
  uint32_t waves_per_wg;     /* 2, 4 or 8 (0 = 4) */
  uint32_t wgs_per_cu;       /* persistent workgroups per compute unit (0 = 8) */
  uint32_t tiles_per_ticket; /* tiles taken per atomic ticket (0 = 4; encode uses at most 4) */
  uint32_t reserved;
} apax_tune;

typedef struct apax_batch apax_batch; /* opaque host-side plan */

/* Validate n host-side items and build a plan; *ws_bytes receives the
 * workspace size the plan needs.  Items are copied; their buffers must stay
 * valid while the plan is used.  Errors name the first bad item's code. */
int apax_batch_create(int op, const apax_batch_item* h_items, uint32_t n, const apax_tune* tune,
                      apax_batch** out, uint64_t* ws_bytes);
/* Copy the plan's descriptor tables into the workspace (asynchronous, from a
 * pinned staging buffer the plan owns) and clear the workspace status.  Each
 * item records its device-side errors in its own status word; apax_batch_run
 * ORs them into the workspace status read by apax_status. */
int apax_batch_upload(apax_batch* b, void* d_ws, uint64_t ws_bytes, hipStream_t stream);
/* Enqueue the whole batch (work-queue reset + persistent kernels). */
int apax_batch_run(apax_batch* b, hipStream_t stream);
/* Record apax_batch_run into a hipGraph (on a private capture stream). */
int apax_batch_capture(apax_batch* b);
/* Replay the captured graph on stream (apax_batch_run if none was captured). */
int apax_batch_launch(apax_batch* b, hipStream_t stream);
void apax_batch_destroy(apax_batch* b);

/* ------------------------------------------------------------------------
 * Serving: a request loop with continuous batching.  Requests (encode or
 * decode of one array, any size/dtype/mode) are submitted as they arrive and
 * wait in a FIFO.  apax_server_poll (non-blocking) retires the groups whose
 * GPU work has finished, then admits requests from the head of the FIFO onto
 * every free slot while the in-flight footprint (input bytes + output
 * capacity of each admitted request) stays within the HBM budget, and
 * launches each admitted group on the slot's own stream: requests of 16 MB
 * and more, and those no shared launch takes (blocks of more than 256
 * samples, groups of 8, the lagged choice, adaptive rate; their workspace
 * must fit the slot's, else APAX_E_CAPACITY at submit), as single
 * apax_encode / apax_decode calls (each with its own status word), the rest
 * as one persistent batch.  Groups on different slots
 * overlap on the device; a request that
 * arrives while others run is admitted as soon as a slot and budget free up.
 * Codec state stays on the device: each slot owns resident workspaces
 * (status words, work-queue tickets, look-back states, descriptor tables).
 * Every result is byte-identical to a separate apax_encode / apax_decode
 * call.  Buffers named by a request are owned by the caller and must stay
 * valid until its completion is returned.  One host thread drives a server. */
typedef struct apax_server apax_server;

typedef struct apax_request {
  int32_t op;            /* APAX_OP_ENCODE / APAX_OP_DECODE */
  uint32_t flags;        /* 0 or APAX_REQ_AFTER */
  apax_batch_item item;  /* as for a batch; a decode header is copied at submit */
  uint64_t tag;          /* caller's cookie, returned in the completion */
  hipStream_t after;     /* with APAX_REQ_AFTER: the request's kernels start only
                            after the work enqueued on this stream before the
                            submit call (inputs, output fills) has finished */
} apax_request;
/* apax_request.flags: order the request after the submitter's stream (an event
 * recorded on `after` at submit, waited on by the slot stream at launch).
 * Without it the caller must have completed the inputs before submitting. */
#define APAX_REQ_AFTER 1u

typedef struct apax_completion {
  uint64_t id, tag;
  int32_t status;        /* APAX_OK or the request's device-side error */
  uint32_t slot;
  double latency_s;      /* submit -> completion observed by apax_server_poll */
} apax_completion;

/* budget_bytes: HBM admission budget; n_slots (1..16) concurrent groups;
 * max_group requests per group; ws_bytes: resident workspace per slot and
 * direction (two per slot, counted against the budget).  Allocates device
 * and pinned host memory. */
int apax_server_create(uint64_t budget_bytes, uint32_t n_slots, uint32_t max_group, uint64_t ws_bytes,
                       const apax_tune* tune, apax_server** out);
/* Validate and enqueue; *id receives the request id.  APAX_E_CAPACITY when the
 * request alone exceeds the budget (nothing is enqueued then). */
int apax_server_submit(apax_server* s, const apax_request* req, uint64_t* id);
/* Retire, admit, launch; copy up to max_done completions to done[]. */
int apax_server_poll(apax_server* s, apax_completion* done, uint32_t max_done, uint32_t* n_done);
/* Queued requests, in-flight footprint bytes, groups launched so far. */
int apax_server_stats(const apax_server* s, uint64_t* queued, uint64_t* in_flight_bytes, uint64_t* groups);
/* Waits for in-flight work, then frees the server. */
void apax_server_destroy(apax_server* s);

#ifdef __cplusplus
}
#endif
#endif
