/*
 * Plain CPU oracle for the sampling-based SZ-vs-ZFP rate-distortion selector of
 * Tao, Di, Liang, Chen, Cappello, "Optimizing Lossy Compression Rate-Distortion
 * from Automatic Online Selection between SZ and ZFP" (arXiv:1806.08901).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the benchmark's
 * CPU-baseline leg may load this library.  The product path (the HIP library in
 * paper_1806_08901_amd/) never calls, links or includes anything from here, and
 * this file includes nothing from there.
 *
 * Arithmetic conventions (all functions):
 *   - real arithmetic in IEEE binary64, round to nearest, no FMA contraction
 *     (built with -ffp-contract=off);
 *   - integer ZFP arithmetic is two's complement modulo 2^W (W = 32 for binary32
 *     fields, 64 for binary64 fields), right shift is floor division by 2;
 *   - every floating-point sum is the adjacent-pair tree over the sequence padded
 *     with +0.0 to a power of two (level l+1 element i = element 2i + element 2i+1).
 */
#ifndef SZSEL_ORACLE_H
#define SZSEL_ORACLE_H
#include <stdint.h>
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_F32 = 0, ORC_F64 = 1 };
enum { ORC_EB_ABS = 0, ORC_EB_REL = 1 };
enum { ORC_OP_SZ = 0, ORC_OP_ZFP = 1, ORC_OP_SELECT = 2, ORC_OP_FIXED_EB = 3 };
enum {
  ORC_FLAG_CONSTANT = 1, ORC_FLAG_NONFINITE = 2, ORC_FLAG_ZERO_MSE = 4,
  ORC_FLAG_EB_EXCEEDS = 8, ORC_FLAG_NO_BLOCKS = 16, ORC_FLAG_BAD_EB = 32
};

typedef struct {
  uint32_t flags;
  int32_t choice;            /* 0 = SZ, 1 = ZFP, -1 = not a selection */
  double vmin, vmax, vr, eb_abs;
  int32_t minexp, pad0;
  /* ZFP side (Section 5.2) */
  double zfp_bitrate, zfp_mse, zfp_psnr, zfp_nsb_mean, zfp_maxerr, zfp_sse;
  uint64_t zfp_bits, zfp_values, zfp_blocks, zfp_nsb_total;
  /* SZ side (Section 5.1) */
  double sz_delta, sz_inv_delta, sz_eb, sz_entropy, sz_bitrate;
  double sz_psnr_model, sz_psnr_measured, sz_mse, sz_maxerr, sz_sse;
  uint64_t sz_values, sz_unpredictable;
  /* selection (Algorithm 1) */
  double chosen_eb;
  /* exact Huffman cost of the code histogram (when requested) */
  uint64_t sz_huffman_bits;
  double sz_huffman_bitrate;
} orc_result;

/* Optional per-sample outputs; every pointer may be NULL. */
typedef struct {
  uint16_t *codes;     /* n_s quantization codes, sampled-block order then in-block row-major */
  uint32_t *zfp_bits;  /* bits of each sampled block */
  double *zfp_sse;     /* data-domain squared error of each sampled block */
  int32_t *zfp_emax;   /* block exponent (frexp convention), INT32_MIN for an empty block */
  double *sz_sse;      /* SZ squared error of each sampled block */
  uint32_t *hist;      /* 65536 code counts */
} orc_dump;

/* Whole estimator: range, sampling, ZFP side and/or SZ side, selection.
 * op: ORC_OP_SZ (delta = 2 eb_abs), ORC_OP_ZFP, ORC_OP_SELECT (Algorithm 1),
 * ORC_OP_FIXED_EB (both sides at the same eb_abs, pick the lower bit-rate).
 * huffman: 0 = no Huffman cost; 1 = also report the exact Huffman cost of
 * the code histogram; 2 = report it and select with it as BR_sz (in place of
 * entropy + offset).  Returns 0, or -1 on invalid arguments. */
int orc_run(int op, const void *field, const int64_t *dims, int ndims, int dtype,
            double eb, int eb_mode, const int32_t *stride, double sz_offset, int huffman,
            orc_result *out, orc_dump *dump);

/* Total bits of an optimal prefix code for the symbol counts hist[0..nbins)
 * (Huffman): the sum of the internal node weights of a tree built by
 * repeatedly merging the two lightest nodes.  A single symbol gets 1 bit per
 * occurrence; no symbol, 0. */
uint64_t orc_huffman_bits(const uint32_t *hist, int64_t nbins);

/* ---- pieces exposed for the pin tests ---- */
int orc_range(const void *field, int64_t n, int dtype, double *vmin, double *vmax);
int64_t orc_num_sampled_blocks(const int64_t *dims, int ndims, const int32_t *stride);
void orc_sampled_block_origin(const int64_t *dims, int ndims, const int32_t *stride,
                              int64_t j, int64_t *origin);
int orc_frexp_exponent(double m);
int orc_floor_log2(double tau);
int orc_precision(int emax, int minexp, int ndims, int W);
void orc_fwd_lift(int64_t *v, ptrdiff_t s, int W);
void orc_inv_lift(int64_t *v, ptrdiff_t s, int W);
void orc_fwd_xform(int64_t *c, int ndims, int W);
void orc_inv_xform(int64_t *c, int ndims, int W);
void orc_reorder_table(int ndims, int32_t *perm);
uint64_t orc_to_negabinary(int64_t c, int W);
int64_t orc_from_negabinary(uint64_t u, int W);
/* Emits the group-testing embedded code of planes W-1 .. W-prec of the 4^d
 * negabinary values u[].  Writes one byte (0/1) per bit into bits[] when it is
 * not NULL (cap bytes).  Returns the number of bits emitted. */
int64_t orc_encode_planes(const uint64_t *u, int size, int W, int prec,
                          uint8_t *bits, int64_t cap);
/* One ZFP block of 4^d values stored row-major.  Returns the block's bit count;
 * writes the decoded values (in the field dtype, widened to double) to xhat,
 * the block SSE to *sse and the significant-bit total to *nsb. */
uint32_t orc_zfp_block(const double *x, int ndims, int dtype, int minexp,
                       double *xhat, double *sse, uint64_t *nsb, int32_t *emax_out);
double orc_lorenzo(const void *field, const int64_t *dims, int ndims, int dtype,
                   const int64_t *p);
double orc_tree_sum(const double *a, int64_t n);
double orc_entropy(const uint32_t *hist, int64_t nbins, uint64_t n);

#ifdef __cplusplus
}
#endif
#endif
