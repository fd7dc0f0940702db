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
  ORC_FLAG_EB_EXCEEDS = 8, ORC_FLAG_NO_BLOCKS = 16, ORC_FLAG_BAD_EB = 32,
  ORC_FLAG_EC_SAMPLED = 128
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
  /* point sub-sampling of the ZFP side (when requested): sub-sampled points,
   * and twice the interpolated significant-bit total over all values of the
   * sampled blocks (an integer) */
  uint64_t zfp_ec_points, zfp_ec_nsb2;
} orc_result;

/* Optional per-sample outputs; every pointer may be NULL. */
typedef struct {
  uint16_t *codes;     /* n_s quantization codes, sampled-block order then in-block row-major */
  uint32_t *zfp_bits;  /* bits of each sampled block */
  double *zfp_sse;     /* data-domain squared error of each sampled block */
  int32_t *zfp_emax;   /* block exponent (frexp convention), INT32_MIN for an empty block */
  double *sz_sse;      /* SZ squared error of each sampled block */
  uint32_t *hist;      /* 65536 code counts */
  uint32_t *ec_nsb2;   /* sub-sampling: twice the interpolated significant bits of each block */
  double *ec_err;      /* sub-sampling: R slots per block (R = r rounded up to a power of two),
                          the scaled transform-domain error of each sampled point, 0 in the pads */
} orc_dump;

/* Whole estimator: range, sampling, ZFP side and/or SZ side, selection.
 * op: ORC_OP_SZ (delta = 2 eb_abs), ORC_OP_ZFP, ORC_OP_SELECT (Algorithm 1),
 * ORC_OP_FIXED_EB (both sides at the same eb_abs, pick the lower bit-rate).
 * huffman: 0 = no Huffman cost; 1 = also report the exact Huffman cost of
 * the code histogram; 2 = report it and select with it as BR_sz (in place of
 * entropy + offset).
 * ec_points: 0 = the exact ZFP estimate (coder bit count, decoded error);
 * otherwise the paper's point sub-sampling of Section 5.2 with ec_points
 * points per block (1 = the paper's 3, 9 or 16 for 1, 2 or 3 D; at most
 * 4^d): BR_zfp is the interpolated mean significant-bit count and MSE_zfp
 * the mean squared transform-domain truncation error of the sub-sampled
 * points.  ec_weight: 0 = those errors as the paper states them (its
 * Theorem 1 assumes a norm-preserving transform); 1 = each squared error
 * times the squared norm of its coefficient's data-domain image under ZFP's
 * inverse transform.  Returns 0, or -1 on invalid arguments. */
int orc_run(int op, const void *field, const int64_t *dims, int ndims, int dtype,
            double eb, int eb_mode, const int32_t *stride, double sz_offset, int huffman,
            int ec_points, int ec_weight, orc_result *out, orc_dump *dump);

/* Squared norm of the data-domain image of unit coefficient i (in-block
 * index) under ZFP's inverse transform: the product over the axes of
 * 4, 5, 4, 13/4 for frequencies 0..3. */
double orc_ec_gain(int i, int ndims);

/* The paper's sub-sample size for a rank (3, 9, 16) and the coding-order
 * positions of r points spread evenly over a block of `size` values. */
int orc_ec_default_points(int ndims);
void orc_ec_positions(int size, int r, int32_t *pos);
/* Sub-sampled estimate of one block: twice the interpolated significant-bit
 * total (nsb2), the significant bits of the r points (nsb_pts), and their
 * scaled truncation errors in err[0..R) (R = r rounded up to a power of two,
 * zeros past r) with their coefficients' gains (orc_ec_gain; 1 past r). */
void orc_zfp_block_ec(const double *x, int ndims, int dtype, int minexp, int r, uint64_t *nsb2,
                      uint64_t *nsb_pts, double *err, double *gain, int32_t *emax_out);

/* Total bits of an optimal prefix code for the symbol counts hist[0..nbins)
 * (Huffman): the sum of the internal node weights of a tree built by
 * repeatedly merging the two lightest nodes.  A single symbol gets 1 bit per
 * occurrence; no symbol, 0. */
uint64_t orc_huffman_bits(const uint32_t *hist, int64_t nbins);

/* Step 4 (Section 3): compressing the whole field with the compressor
 * Algorithm 1 selects. */
typedef struct {
  uint64_t bits, values, blocks;
  double bitrate, sse, mse, psnr, maxerr, vr, eb_abs;
  /* SZ only: values stored raw, distinct code symbols, bits of the optimal
   * prefix code of the symbols */
  uint64_t unpredictable, symbols, code_bits;
  double code_entropy;
} orc_step4;

/* ZFP fixed-accuracy compression of every block of the field at eb_abs
 * (partial blocks repeat the last value along each axis), one byte per
 * stream bit into bits[0..cap) (NULL: count only), then each block decoded
 * from the stream; decoded (N values, may be NULL) receives the
 * decompressed field.  SSE: pair tree over the blocks' 4^d slots (zeros at
 * padded positions).  Returns 0, -1 on bad arguments, -2 if a block does
 * not decode to the bits it was coded in. */
int orc_zfp_compress(const void *field, const int64_t *dims, int ndims, int dtype, double eb_abs,
                     uint8_t *bits, int64_t cap, double *decoded, orc_step4 *out);
int64_t orc_zfp_num_blocks(const int64_t *dims, int ndims);

/* SZ compression of the whole field at eb_abs with Lorenzo prediction from
 * decompressed values, made parallel by quantizing first: q = the nearest
 * multiple of 2 eb_abs in units (round half away from zero, 1/(2 eb_abs)
 * one IEEE division; 0 when |x| / (2 eb_abs) >= 2^50), code = q - L(q) with
 * L the Lorenzo predictor (Section 4.3 terms, integers, 0 outside the
 * field); symbol code + 32768, or 0 (escape, value stored in W bits) when
 * |code| >= 32768 or q 2 eb_abs rounded to the field's precision misses
 * eb_abs.  Decompressed value: q 2 eb_abs (rounded), or the stored value.
 * Size: optimal prefix-code bits of the symbols + W per escape + 32 per
 * distinct symbol (the code table).  SSE: pair tree in field order.
 * hist (65536, may be NULL) receives the symbol counts, symbols (N, may be
 * NULL) the symbol of every value, decoded (N, may be NULL) the
 * decompressed field. */
int orc_sz_compress(const void *field, const int64_t *dims, int ndims, int dtype, double eb_abs,
                    uint32_t *hist, uint16_t *symbols, double *decoded, orc_step4 *out);

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
