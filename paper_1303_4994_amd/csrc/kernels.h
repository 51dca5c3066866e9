// kernels.h -- kernel argument blocks and launchers of libapax.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "codec.h"

namespace apax {

constexpr int WPG = 4;  // wavefronts per workgroup (one tile per workgroup)

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
  Geo g;
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

enum { P_MAX = 0, P_STATS = 1, P_FITS = 2, P_CENTER = 3 };
enum { R_LOSSLESS = 0, R_RATE = 1, R_QUALITY = 2 };
enum { S_X = 0, S_Y, S_D, S_XX, S_YY, S_DD, S_DS, S_CXX, S_CYY, S_CDD, NSUM };
constexpr int MAXCODES = 17;

struct ProfArgs {
  const void* x;
  float* partials;            // [ncodes][nwg][NSUM][2]
  int32_t* cj;                // per-block codes (fixed rate): written by P_STATS, read by P_CENTER
  unsigned long long* words;  // [ncodes] total block words
  unsigned int* fits;         // [ncodes]
  unsigned int* hist;         // [8]
  unsigned long long* maxbits;// [0] max|x|, [1] max|d| (binary64 bits, non-negative)
  uint32_t* status;
  int64_t jstride;            // 1 (full array) or 16 (subsample)
  int64_t nbe;                // blocks visited
  int64_t ntiles;             // tiles of blocks to visit
  int64_t nwg;                // persistent workgroups per code
  int op, rule;
  int store_cj, hist_code;    // P_STATS: store per-block codes; P_FITS: code index histogrammed
  uint32_t mask;
  int ncodes;
  int escale;                 // sums are scaled by 2^-escale (linear) or 2^-2escale (squares)
  int codes[MAXCODES];
  double mean_x, mean_y, mean_d;
  Geo g;
};

int64_t encode_tiles(const Geo& g);
hipError_t launch_encode(int dtype, int ndim, EncArgs& A, hipStream_t s);
hipError_t launch_decode(int dtype, int ndim, DecArgs& A, hipStream_t s);
int64_t prof_tiles(const Geo& g, int64_t nbe);
int64_t prof_wgs(int64_t ntiles);
hipError_t launch_profile(int dtype, int ndim, ProfArgs& A, hipStream_t s);
hipError_t launch_finalize(const float* partials, int64_t ntiles, int ncodes, double* out,
                           hipStream_t s);

}  // namespace apax
