// kernels.h -- kernel argument blocks and launchers of libapax.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "codec.h"

namespace apax {

constexpr int WPG = 4;  // wavefronts per workgroup (one tile per workgroup)
constexpr int RUN = 4;  // encode: tiles per work-queue ticket in variable-size modes

struct EncArgs {
  const void* x;
  uint8_t* out_base;     // stream start (64-byte header)
  uint32_t* out_words;   // block area
  uint16_t* lens;        // block lengths (variable modes)
  uint64_t* sbo;         // superblock word offsets (variable modes)
  uint64_t* d_nbytes;
  uint32_t* status;
  uint32_t* ticket;
  uint64_t* tile_state;
  uint64_t area;         // byte offset of the block area
  int64_t ntiles;
  uint32_t hdr[16];      // stream header (payload words written on device)
  uint64_t zpad[4];      // byte ranges [0,1) and [2,3) of index padding to zero
  const int32_t* sel;    // {code, stream mask} a profile left in the workspace, or null
  const int32_t* lag;    // lagged stream choice: each block's own best stream, or null
  uint8_t* bst;          // variable-size modes, single array: each block's chosen stream
  uint32_t* ssum;        // variable-size modes, single array: words per superblock of 64 blocks
  const int32_t* bcode;  // adaptive rate: each block's requested code, or null
  Geo g;
};

// Operating point of an encode: the caller's code and stream mask, or, when
// `sel` is set, those a preceding profile of the same workspace chose on the
// device (its mask intersected with the caller's).  Returns false, keeping
// the caller's, when `sel` holds no profile result for this code range.
// `any`: 8 readable bytes, read instead of `sel` when it is null, so the
// loads carry no branch and their latency can overlap the block's.
__device__ __forceinline__ bool operating_point(const int32_t* sel, const void* any, int32_t cmin,
                                                int32_t cmax, int32_t ucode, uint32_t umask,
                                                int32_t& code, uint32_t& mask) {
  const int32_t* sp = sel ? sel : reinterpret_cast<const int32_t*>(any);
  const int32_t c = sp[0];
  const uint32_t m = (uint32_t)sp[1];
  const bool ok = !sel || (m != 0 && c >= cmin && c <= cmax);
  const bool use = sel && ok;
  code = use ? c : ucode;
  mask = use ? (m & umask) : umask;
  return ok;
}

// Stream of an array without blocks: the header alone.
struct HdrArgs {
  uint32_t* out;
  uint64_t* d_nbytes;
  uint64_t nbytes;
  uint32_t hdr[16];
  const int32_t* sel;  // as EncArgs::sel
  uint32_t* status;
  int32_t cmin, cmax, ucode;
  uint32_t umask;
};

struct DecArgs {
  const uint8_t* in;
  const uint32_t* words;
  const uint16_t* lens;
  const uint64_t* sbo;
  void* y;
  uint32_t* status;
  uint64_t payload_words;
  int64_t ntiles;
  uint32_t hdr[16];
  Geo g;
};

enum { P_STATS = 1, P_FITS = 2, P_CENTER = 3, P_CURVE = 4 /* P_STATS on the curve's sums only */,
       P_MENC = 5 /* fixed-rate P_STATS that also writes each block's encoded words */ };
enum { R_LOSSLESS = 0, R_RATE = 1, R_QUALITY = 2 };
enum { S_X = 0, S_Y, S_D, S_XX, S_YY, S_DD, S_DS, S_CXX, S_CYY, S_CDD, NSUM };
constexpr int MAXCODES = 17;
constexpr int NCURVE = 17;

// Device-resident profiler state (start of the workspace).  The control
// kernel (one thread) makes every decision of the profile on the device --
// bracket, bisection walk, stream mask, curve codes, means -- so a whole
// profile is one asynchronous launch sequence and one read-back.
struct PState {
  uint32_t status;          // device-side error bits (shared with encode/decode)
  uint32_t ticket;          // encode: dynamic tile ticket
  uint64_t maxbits[2];      // max|x|, max|d| (binary64 bits, non-negative)
  int32_t cf, cc, escale, code;      // whole-array bracket, statistics scale, result code
  int32_t lo, hi, done, n_probes;    // bisection state
  int32_t flags, ncodes, first;
  int32_t centred;  // 1: the centred sums came from the raw moments (no centred pass)
  uint32_t mask_probe, mask_out, need, pad1;
  int32_t sel[2];           // operating point for the encoder: code, encoder stream mask
  int32_t codes[MAXCODES];  // codes evaluated by the next probe launch
  int32_t probe[MAXCODES];  // codes of the last probe launch (tree order)
  uint32_t fits[MAXCODES];
  uint32_t hist[8];
  uint64_t words[MAXCODES];
  double mean[3];
  double sums[MAXCODES][NSUM];        // finalize output of the last stats launch
  double curve_sums[NCURVE][4];       // Sxx, Syy, Sdd, Sds of the curve codes
  uint64_t curve_words[NCURVE];
  int32_t curve_codes[NCURVE];
  int32_t pad2;
  double msums[NSUM];                 // metrics at the operating point
  uint64_t mwords;
  uint64_t sub_samples;               // samples in the subsample blocks (histogram pass)
  uint64_t s2r_prefix, s2r_rank;      // S2R margin selection: digits chosen, rank left
  int32_t s2r_level, pad3;
};

// Per-(code, workgroup) partial results of a profile pass, one array per
// field (record r = code * nwg + workgroup, R records), reduced in a fixed
// order by the one-workgroup reduce kernel that follows the pass.
struct PParts {
  double* s;          // [NSUM][R] binary64 sums
  uint64_t* words;    // [R] encoded words
  uint64_t* dmax;     // [R] max |d| (binary64 bits)
  uint32_t* nfit;     // [R] blocks that fit the budget
  uint32_t* hist;     // [8][R] blocks per chosen stream
  int64_t R;
};
// The fit counts come first, so a pass that writes only them (the fixed-rate
// probes, up to MAXCODES x 2048 records) needs 4 bytes per record.
__host__ __device__ inline PParts pparts(void* base, int64_t R) {
  PParts P;
  uint8_t* b = (uint8_t*)base;
  P.nfit = (uint32_t*)b;
  b += (4 * R + 7) / 8 * 8;
  P.s = (double*)b;
  b += 8 * NSUM * R;
  P.words = (uint64_t*)b;
  b += 8 * R;
  P.dmax = (uint64_t*)b;
  b += 8 * R;
  P.hist = (uint32_t*)b;
  P.R = R;
  return P;
}
constexpr int PPART_BYTES = 8 * NSUM + 8 + 8 + 4 + 4 * 8;  // per record

// control steps of the profile (run by the last workgroup of a launch)
enum { C_NONE = -1, C_INIT = 0, C_DECIDE = 1, C_MASK = 2, C_CURVE = 3, C_KEEP_CURVE = 4, C_MEANS = 5 };
struct CtlArgs {
  PState* st;
  int step, mode, isint, depth, cmin, cmax;
  uint32_t mask_user;         // effective user stream mask
  uint64_t nsub, nsamples;
  double target;
};

struct ProfArgs {
  const void* x;
  PState* st;
  void* parts;                // PParts of maxcodes * nwg records
  int32_t* cj;                // per-block codes (fixed rate): written by P_STATS, read by P_CENTER
  int64_t jstride;            // 1 (full array) or 16 (subsample)
  int64_t nbe;                // blocks visited
  int64_t ntiles;             // tiles of blocks to visit
  int64_t nwg;                // persistent workgroups per code
  int op, rule;
  int maxcodes;               // grid rows launched (rows >= st->ncodes idle)
  int store_cj, hist;         // P_STATS: store per-block codes; P_FITS: histogram streams
  int mask_sel;               // 0 st->mask_probe, 1 st->mask_out (+0x81), 2 metrics mask
  int final_code;             // evaluate st->code (one code) instead of st->codes[]
  int curve;                  // P_STATS: only the four sums of r and the word count
  // several codes per launch: a 1-D grid of nwg * maxcodes workgroups whose
  // ids are spread so the workgroups of every code that visit the same
  // tiles share an XCD (and its L2), which then fetches those tiles once
  int xcd_map;
  int probe_all;              // fixed-rate probes: every code tested on each tile (k_probe_all)
  // metrics pass of a profile that encodes next (else null): each block's
  // chosen stream, and in variable-size modes its length (into the stream's
  // index) and its superblock's word sum -- the encoder's first pass
  uint8_t* bst;
  uint16_t* lens;
  uint32_t* ssum;
  // fixed-rate metrics pass of a profile that encodes next (else null): the
  // stream's block area, each block's budget words written there by the pass
  // itself (the bytes the fixed-rate encode would write at the block's code
  // and stream)
  uint32_t* enc_words;
  CtlArgs C;                  // control step run by the reduce kernel (C.step, C_NONE: none)
  Geo g;
};
constexpr int PMAX_WGS = 1024;

// 2-sigma S2R margin passes (after a profile of the same array)
constexpr uint64_t S2R_HIST_BYTES = 8192 * 4;  // the selection's 8192 bins
struct S2RArgs {
  const void* x;
  PState* st;
  const int32_t* cj;  // fixed rate: per-block codes of the profile's metrics pass
  uint32_t* hist;     // 8192 bins
  uint64_t* ncand;    // keys that matched the level-2 prefix (all of them counted)
  uint64_t* cand;     // the first cand_cap of those keys
  uint64_t cand_cap;
  int64_t ntiles, nwg;
  int rule, pad;
  Geo g;
};
hipError_t launch_s2r(int dtype, int ndim, S2RArgs& A, uint64_t rank, hipStream_t s);



// ---- batches: many arrays, one persistent launch per (LPB, NDIM) class
struct BatchEnc {
  int32_t dtype, ndim;
  int64_t tile_start;  // first global tile of this item
  EncArgs a;           // per-item arguments (a.ntiles, a.tile_state for the batch tile size)
};
struct BatchDec {
  int32_t dtype, ndim;
  int64_t tile_start;
  DecArgs a;
};
struct BatchArgs {
  const void* items;       // BatchEnc* / BatchDec* (device)
  const int64_t* starts;   // tile_start of items 0..n-1 (device)
  uint32_t* ticket;        // work-queue counter (zeroed by the reset kernel)
  uint64_t* tile_state;    // look-back states of every tile of the class
  int64_t total_tiles;
  uint32_t n;
  uint32_t tiles_per_ticket;
  int32_t ldsw;            // LDS words per block slot: the class's largest block buffer
  int32_t pad;
};

int lpb_of(const Geo& g);
int64_t encode_tiles(const Geo& g);
int64_t encode_tiles_wp(const Geo& g, int wp);
hipError_t launch_encode_batch(int lpb, int ndim, int wp, const BatchArgs& B, int grid,
                               size_t lds, hipStream_t s);
hipError_t launch_decode_batch(int lpb, int ndim, int wp, const BatchArgs& B, int grid,
                               size_t lds, hipStream_t s);
hipError_t launch_batch_reset(uint32_t* ticket, uint64_t* tile_state, int64_t n, hipStream_t s);
hipError_t launch_encode(int dtype, int ndim, EncArgs& A, hipStream_t s);
// the encode of a profiled array in a variable-size mode from its metrics
// pass's per-block results: the lengths, streams and superblock sums it left
// (scan + emit).  Fixed rate: the metrics pass writes the blocks itself
// (ProfArgs::enc_words) and launch_encode_header the header
hipError_t launch_encode_profiled(int dtype, int ndim, EncArgs& A, const int32_t* cj, hipStream_t s);
// the stream header (and byte count) of a fixed-rate encode whose blocks a
// profile's metrics pass writes (ProfArgs::enc_words)
hipError_t launch_encode_header(const EncArgs& A, hipStream_t s);
// each block's own best stream into best[nblocks] (lossless; the lagged choice)
hipError_t launch_stream_choice(int dtype, int ndim, const EncArgs& A, int32_t* best, hipStream_t s);
hipError_t launch_decode(int dtype, int ndim, DecArgs& A, hipStream_t s);
// variable-size encodes: zero the superblock sums; their exclusive scan, the
// payload size in the stream header and the byte count
void launch_encode_reset(uint32_t* ssum, int64_t nsuper, hipStream_t s);
void launch_encode_scan(const EncArgs& A, int64_t nsuper, hipStream_t s);
// sum of n binary64 partials in index order into *out
void launch_dot_reduce(const double* partial, int64_t n, double* out, hipStream_t s);
// blocks of more than 256 samples (G > 64): one workgroup per block
hipError_t launch_wide_encode(int dtype, int ndim, EncArgs& A, hipStream_t s);
hipError_t launch_wide_choice(int dtype, int ndim, const EncArgs& A, int32_t* best, hipStream_t s);
hipError_t launch_wide_decode(int dtype, int ndim, DecArgs& A, hipStream_t s);
hipError_t launch_wide_table(int dtype, int ndim, const EncArgs& A, uint8_t* tab, hipStream_t s);
// adaptive rate: the controller's state of every block (the loop as a scan
// over per-block transition maps) as requested codes into bcode; `region`
// holds adapt_bytes(nblocks)
uint64_t adapt_bytes(int64_t nblocks);
hipError_t launch_adapt(int dtype, int ndim, const EncArgs& A, void* region, int32_t* bcode, hipStream_t s);
hipError_t launch_wide_decode_dot(int dtype, int ndim, DecArgs& A, const void* w, double* partial, double* out,
                                  hipStream_t s);
// decode-on-read dot product (partial: one double per tile) and the plain one
hipError_t launch_decode_dot(int dtype, int ndim, DecArgs& A, const void* w, double* partial, double* out,
                             hipStream_t s);
hipError_t launch_dot_plain(int dtype, const void* x, const void* w, int64_t n, double* partial, int nwg,
                            double* out, hipStream_t s);
int64_t prof_tiles(const Geo& g, int64_t nbe);
int64_t prof_wgs(int64_t ntiles, int ncodes);
// ev (optional): events recorded just before and just after the pass kernel
// (its one-workgroup reduce follows outside the pair)
// rs (with the event fork): run the pass's reduce kernel on stream rs, which
// waits for the pass kernel on s
hipError_t launch_profile(int dtype, int ndim, ProfArgs& A, hipStream_t s, hipEvent_t* ev = nullptr,
                          hipStream_t rs = nullptr, hipEvent_t fork = nullptr);
// the pass kernel for blocks of more than 64 groups or groups of 8 (A.nwg set)
hipError_t launch_wide_profile(int dtype, int ndim, const ProfArgs& A, hipStream_t s);
hipError_t launch_pmax(int dtype, const void* x, uint64_t n, void* parts, const CtlArgs& C,
                       hipStream_t s, hipEvent_t* ev = nullptr);
hipError_t launch_ctl(const CtlArgs& C, hipStream_t s);

}  // namespace apax
