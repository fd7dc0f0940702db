// Step 4 of Algorithm 1: the host-visible interface of the ZFP compressor
// kernels (compress.hip).
#pragma once

#include <hip/hip_runtime.h>

#include "szsel.h"

namespace szsel {

// Device-side totals of one compression.
struct ZcResult {
  uint64_t bits;         // stream length
  uint64_t maxerr_bits;  // largest absolute error, order-preserving bits
  uint64_t vmin_bits, vmax_bits;
  uint64_t nonfinite;    // nonzero when the field holds NaN or Inf
  double sse;
};

struct ZcArgs {
  const void *field;
  int64_t dims[3];
  int64_t nb[3];         // blocks per axis, ceil(dims / 4)
  int nd, dtype, minexp, pad;
  int64_t nblocks;
  uint32_t *counts;      // bits of each block
  uint64_t *offsets;     // bit offset of each block
  uint64_t *chunk;       // scan chunk totals
  double *bsse;          // squared error of each block
  double *red;           // two halves of red_half values (tree levels)
  int64_t red_half;
  uint64_t *stream;      // the output stream (stream_words words, zeroed here)
  int64_t stream_words;
  void *decoded;         // decompressed field, or nullptr
  ZcResult *res;
};

// Words a stream of nblocks blocks may need (a bound, plus the reader's
// spare word), and the workspace element counts.
size_t zc_stream_words(int64_t nblocks, int nd, int dtype);
size_t zc_red_half(int64_t nblocks);
size_t zc_chunks(int64_t nblocks);

hipError_t zc_launch(const ZcArgs &a, hipStream_t s);

// SZ compression of the whole field (quantize first, Lorenzo on the
// integers; see compress.hip).
constexpr int kSzCopies = 16;  // global histogram copies
struct SzResult {
  uint64_t escapes, code_bits, symbols, huff_ok;
  uint64_t maxerr_bits, vmin_bits, vmax_bits;
  uint64_t nonfinite;  // nonzero when the field holds NaN or Inf
  double sse, hsum;    // hsum: sum of h log2 h over the symbol counts
};

struct SzArgs {
  const void *field;
  int64_t dims[3];
  int nd, dtype;
  int64_t n;
  double delta, inv, eb;
  uint32_t *hist;      // kSzCopies x 65536 counts (zeroed here)
  uint32_t *hfinal;    // the 65536 symbol counts
  double *chunk_sse;   // squared-error sum of each chunk of points
  int64_t nchunks;
  double *red;
  int64_t red_half;
  void *decoded;       // decompressed field, or nullptr
  uint16_t *symbols;   // symbol of every point, or nullptr
  SzResult *res;
};
size_t sz4_chunks(int64_t n);
hipError_t sz4_launch(const SzArgs &a, hipStream_t s);

}  // namespace szsel
