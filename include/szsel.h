/*
 * szsel: sampling-based SZ-vs-ZFP rate-distortion estimation and selection on
 * MI355X (gfx950), after Tao, Di, Liang, Chen, Cappello, "Optimizing Lossy
 * Compression Rate-Distortion from Automatic Online Selection between SZ and
 * ZFP" (arXiv:1806.08901).
 *
 * Every entry point below enqueues HIP kernels on the caller's stream; the
 * whole estimator runs on the GPU.  Plain C ABI: device or host pointers and
 * sizes only.
 *
 * Conventions shared by all entry points
 *   field   device pointer to a C-order array (dims[0] slowest), binary32
 *           (SZSEL_F32) or binary64 (SZSEL_F64).  Owned by the caller, who
 *           keeps it alive and unmodified until the stream work completes.
 *   dims    host array of ndims extents, each >= 1; ndims in {1, 2, 3}.
 *   eb      error bound: absolute (SZSEL_EB_ABS) or relative to the field's
 *           value range (SZSEL_EB_REL), Algorithm 1.  Must be > 0.
 *   stride  host array of ndims block strides, each >= 1: the 4^d block with
 *           block index b is sampled iff b_k mod stride[k] == 0 on every axis
 *           (Section 4.3: a fixed distance per dimension).  NULL means 1 on
 *           every axis (every block sampled).
 *   out     host memory for the result (szsel_result), written by an
 *           asynchronous device-to-host copy ordered on `stream`.  Read it
 *           only after synchronising the stream.  Pinned memory keeps the call
 *           fully asynchronous; pageable memory may make the copy synchronous.
 *   stream  a hipStream_t cast to void* (NULL = the null stream).
 *
 * Errors: argument and launch errors are returned synchronously as negative
 * SZSEL_E* codes, with text from szsel_last_error().  Conditions that depend
 * on the data (non-finite values, a constant field, ...) are reported in
 * szsel_result.flags.  No C++ exception crosses this interface.  A context is
 * not thread-safe; calls on one context that run on different streams are
 * ordered by the context itself (each call's workspace slot waits for the
 * previous use of that slot).
 */
#ifndef SZSEL_H
#define SZSEL_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct szsel_ctx szsel_ctx;

enum { SZSEL_F32 = 0, SZSEL_F64 = 1 };
enum { SZSEL_EB_ABS = 0, SZSEL_EB_REL = 1 };

/* What one request computes. */
enum {
  SZSEL_OP_SZ = 0,       /* SZ side only, bin width delta = 2 eb_abs (Section 5.1.4) */
  SZSEL_OP_ZFP = 1,      /* ZFP side only (Section 5.2) */
  SZSEL_OP_SELECT = 2,   /* Algorithm 1: ZFP first, SZ at the delta of equal PSNR */
  SZSEL_OP_FIXED_EB = 3  /* both sides at the same eb_abs, lower bit-rate wins
                            (the fixed-maximum-error criterion of Section 6.4) */
};

enum {
  SZSEL_OK = 0,
  SZSEL_EINVAL = -1,  /* bad argument */
  SZSEL_EDTYPE = -2,  /* unsupported dtype */
  SZSEL_ENOMEM = -3,  /* workspace would exceed the context's budget */
  SZSEL_EHIP = -4,    /* a HIP runtime call failed */
  SZSEL_EBUSY = -5    /* batch larger than the context supports */
};

/* Data-dependent conditions, OR-ed into szsel_result.flags. */
enum {
  SZSEL_FLAG_CONSTANT = 1,    /* value range is 0: nothing to estimate, choice = SZ */
  SZSEL_FLAG_NONFINITE = 2,   /* NaN or Inf in the field: nothing estimated, choice = -1 */
  SZSEL_FLAG_ZERO_MSE = 4,    /* ZFP reproduced the samples exactly: delta = 2 eb_abs */
  SZSEL_FLAG_EB_EXCEEDS = 8,  /* the SZ bound delta/2 is larger than eb_abs */
  SZSEL_FLAG_NO_BLOCKS = 16,  /* no full 4^d block: nothing estimated, choice = SZ */
  SZSEL_FLAG_BAD_EB = 32,     /* eb_rel * value range is 0 or not finite */
  SZSEL_FLAG_NO_HUFFMAN = 64, /* Huffman cost requested but not computed: the counts
                                 took more than 8192 distinct values during the
                                 construction (impossible with at most 2^25 sampled
                                 values), or 2^32 sampled values or more */
  SZSEL_FLAG_EC_SAMPLED = 128, /* the ZFP side is the point sub-sampling estimate
                                  (SZSEL_OPT_EC_SAMPLING) */
  SZSEL_FLAG_FAILED = 256     /* serving only: nothing estimated, the request could not
                                 be run (szsel_server_last_error says why); choice = -1 */
};

/* Result of one request.  Bit-rates are bits per value, PSNRs in dB, MSEs in
 * squared field units; *_sse are the raw sums the MSEs come from. */
typedef struct {
  uint32_t flags;
  int32_t choice;             /* 0 = SZ, 1 = ZFP (Algorithm 1's selection bit); -1 if not selecting */
  double vmin, vmax, vr, eb_abs;
  int32_t minexp, pad0;       /* floor(log2(eb_abs)): ZFP's lowest coded bit plane */
  /* ZFP side (Section 5.2): exact coder bits of the sampled blocks and the
   * data-domain error after decoding them */
  double zfp_bitrate, zfp_mse, zfp_psnr, zfp_nsb_mean, zfp_maxerr, zfp_sse;
  uint64_t zfp_bits, zfp_values, zfp_blocks, zfp_nsb_total;
  /* SZ side (Section 5.1): bin width, entropy of the Lorenzo/quantization
   * codes (Eq. 5), bit-rate = entropy + offset + escapes, PSNR model (Eq. 10)
   * and measured PSNR of the sampled points */
  double sz_delta, sz_inv_delta, sz_eb, sz_entropy, sz_bitrate;
  double sz_psnr_model, sz_psnr_measured, sz_mse, sz_maxerr, sz_sse;
  uint64_t sz_values, sz_unpredictable;
  double chosen_eb;           /* error bound handed to the chosen compressor */
  /* exact Huffman cost of the SZ code histogram (SZSEL_OPT_HUFFMAN): total
   * bits of an optimal prefix code for the codes, and that per value plus
   * W raw bits per unpredictable point; 0 when not requested */
  uint64_t sz_huffman_bits;
  double sz_huffman_bitrate;
  /* ZFP point sub-sampling (SZSEL_OPT_EC_SAMPLING): points sub-sampled, and
   * twice the interpolated significant-bit total of all values of the
   * sampled blocks (an integer); 0 otherwise */
  uint64_t zfp_ec_points, zfp_ec_nsb2;
} szsel_result;

/* One request of a batch (szsel_select_batch). */
typedef struct {
  const void *field;          /* device pointer, as above */
  int64_t dims[3];            /* first ndims entries used */
  int32_t ndims, dtype;
  double eb;
  int32_t eb_mode, op;        /* SZSEL_EB_*, SZSEL_OP_* */
  int32_t stride[3];          /* first ndims entries used; 0 means 1 */
  int32_t pad0;
} szsel_request;

/* Device buffers that receive per-sample values of the NEXT request (debug
 * and parity testing).  Any pointer may be NULL.  Sizes: codes n_s uint16
 * (sampled-block order, then in-block row-major); zfp_bits, zfp_emax,
 * zfp_sse, sz_sse one entry per sampled block; hist 65536 uint32. */
typedef struct {
  uint16_t *codes;
  uint32_t *zfp_bits;
  double *zfp_sse;
  int32_t *zfp_emax;
  double *sz_sse;
  uint32_t *hist;
} szsel_debug;

/* Creates a context on HIP device `hip_device`.  workspace_budget_bytes caps
 * the device memory the context may allocate (0 = 16 GiB; a request needs
 * about 4.8 MB plus 2 bytes per sampled value).  Returns SZSEL_OK and *ctx,
 * or a negative code. */
int szsel_create(szsel_ctx **ctx, int hip_device, size_t workspace_budget_bytes);

/* Waits for the context's outstanding work and frees its device memory. */
void szsel_destroy(szsel_ctx *ctx);

/* SZ-side estimate (Section 5.1; Eq. 5, 9, 10, 11 with delta = 2 eb_abs). */
int szsel_estimate_sz(szsel_ctx *ctx, const void *field, const int64_t *dims, int ndims, int dtype,
                      double eb, int eb_mode, const int32_t *stride, szsel_result *out,
                      void *stream);

/* ZFP-side estimate (Section 5.2: embedded-coding bit count and the PSNR of
 * the sampled blocks). */
int szsel_estimate_zfp(szsel_ctx *ctx, const void *field, const int64_t *dims, int ndims,
                       int dtype, double eb, int eb_mode, const int32_t *stride,
                       szsel_result *out, void *stream);

/* Algorithm 1: value range, block sampling, ZFP bit-rate and PSNR, the bin
 * width delta with PSNR_sz = PSNR_zfp (Eq. 10), SZ bit-rate from the code
 * histogram at delta, choice of the lower bit-rate (ties to ZFP). */
int szsel_select(szsel_ctx *ctx, const void *field, const int64_t *dims, int ndims, int dtype,
                 double eb, int eb_mode, const int32_t *stride, szsel_result *out, void *stream);

/* Fixed-maximum-error selection (Section 6.4): SZ at delta = 2 eb_abs against
 * ZFP at eb_abs, lower bit-rate wins. */
int szsel_select_fixed_eb(szsel_ctx *ctx, const void *field, const int64_t *dims, int ndims,
                          int dtype, double eb, int eb_mode, const int32_t *stride,
                          szsel_result *out, void *stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): the same
 * request and the same result as szsel_select, bit for bit, with the
 * request's workspace in a static device array of
 * SZSEL_NOALLOC_SCRATCH_BYTES that the library holds on every GPU it runs on
 * until the process ends (looked up and zeroed by szsel_create).  The call
 * enqueues kernels and the result's copy on `stream` and allocates nothing
 * (no hipMalloc, hipFree or allocating library routine; no event either).
 * `out` should be pinned host memory where the call is captured.
 * A request whose workspace would exceed the array (about 4.8 MB plus 2
 * bytes per sampled value) returns SZSEL_ENOMEM with the sizes in
 * szsel_last_error(); argument errors are those of szsel_select.
 * Every call on one GPU, from any context, uses that GPU's one array, which
 * keeps the last call's contents (the kernels leave what must start at zero
 * cleared): calls that may overlap on the device (on different streams, or
 * from different threads, without ordering between them) race and give
 * wrong results.  Issue them on one stream or synchronise between them. */
#define SZSEL_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
int szsel_select_noalloc(szsel_ctx *ctx, const void *field, const int64_t *dims, int ndims,
                         int dtype, double eb, int eb_mode, const int32_t *stride,
                         szsel_result *out, void *stream);

/* n <= 1024 requests of any shape, dtype, bound and op together: one launch
 * per pass covers every request (the ZFP and SZ passes one per class of
 * dtype, rank and alignment; the range, overflow and entropy passes one for
 * all), captured as a HIP graph and replayed while the batch shape repeats.
 * Requests on the same field (same pointer, dtype and dims) share one
 * value-range scan.  out[i] receives the result of reqs[i]; each equals what
 * the single-request entry point returns for the same request, bit for bit.
 * The context keeps 4 batch workspaces in rotation; a call that reuses one
 * first waits (on the host) for the batch that last used it.  Errors:
 * SZSEL_EINVAL (a request is invalid; the message names it), SZSEL_EBUSY
 * (n > 1024), SZSEL_ENOMEM (workspace beyond the budget). */
int szsel_select_batch(szsel_ctx *ctx, const szsel_request *reqs, int n, szsel_result *out,
                       void *stream);

/* Text of the last error on this context ("" if none). */
const char *szsel_last_error(const szsel_ctx *ctx);

/* Block strides that sample a fraction close to r_sp (0 < r_sp <= 1) of the
 * full 4^d blocks, with stride 1 on the fastest axis (Section 4.3, the default
 * rate being 5%).  Writes ndims strides; returns SZSEL_OK or SZSEL_EINVAL. */
int szsel_stride_for_rate(double r_sp, int ndims, const int64_t *dims, int32_t *stride_out);

/* Options.
 * SZSEL_OPT_SZ_OFFSET: bits per value added to the SZ entropy estimate
 *   (Section 6.2 sets it to 0.5; default 0.5).
 * SZSEL_OPT_PROFILE: nonzero records HIP events between the passes of every
 *   single-request call and around every launch of a batch (batches then
 *   launch without a graph); read with szsel_profile_read.
 * SZSEL_OPT_AUTOTUNE: nonzero lets szsel_select_batch time a few launch
 *   shapes (workgroups per request and pass, ZFP waves per launch class,
 *   request groups, stream lanes, how the counts are shared, overflow codes
 *   per slice of the overflow pass) the first
 *   time it sees a batch shape and keep the fastest; 0 (default) uses the
 *   fixed schedule.  The results do not depend on it.  The schedules are
 *   kept per device architecture and batch shape (request count, and per
 *   request dtype, rank, op, extents, strides, 16-byte alignment and which
 *   earlier request shares its field) and launch mode (graph or not: each
 *   candidate is timed the way the batch will run) for the process; when the
 *   environment variable SZSEL_TUNE_CACHE names a file, they are also read
 *   from it on first use and every newly tuned one is appended to it (one
 *   JSON object per line; lines written by another build of the library
 *   are ignored), so that later processes skip the tuning.
 * SZSEL_OPT_BATCH_GRAPH: nonzero (default) captures a batch's launches as a
 *   HIP graph and replays it while the batch shape repeats.
 * SZSEL_OPT_SZ_WGS, SZSEL_OPT_ZFP_CHUNK, SZSEL_OPT_RANGE_WGS: the schedule
 *   of single-request calls and of batches without autotuning (and the
 *   autotuner's starting point): SZ workgroups in quarters of the CU
 *   count (1..256, default 8), smallest ZFP chunk in sampled blocks (a
 *   power of two 16..65536, default 16; 3-D blocks without point
 *   sub-sampling take chunks from 16, other blocks from 64; above it the
 *   chunk aims at 64 one-wave ZFP workgroups per CU), range
 *   workgroups (scan chunks of
 *   a field) per CU (a multiple of 0.25 up to 64, default 1); 0 restores
 *   the default.  Results do not depend on them.
 * SZSEL_OPT_BATCH_SHARE: how a batch applies the SZ and range counts above
 *   (0..3, default 0): 0 gives them to every request; 1 makes the SZ count
 *   the whole batch's, dealt to its requests in proportion to their sampled
 *   blocks; 2 does that and deals the range count of the batch in
 *   proportion to the bytes of the fields (a field scanned once for all its
 *   requests counts once); 3 deals the SZ count as 1 does, but within each
 *   class of requests that share a launch (dtype, rank, alignment and point
 *   sub-sampling), each class getting the whole count.  In every mode a
 *   batch deals the ZFP waves within each class instead of aiming at them
 *   per request.  Many small fields favour 1 to 3, mixes of large and small
 *   ones 0; the autotuner tries all four.
 * SZSEL_OPT_BATCH_GROUPS: request groups of the batch schedule (1..8,
 *   default 1; 0 restores it): the requests are dealt to that many groups
 *   (requests on one field stay together); the groups' range scans run one
 *   after another on a side stream and group g's sampled passes start when
 *   its scans are done, so the scans of later groups overlap the sampled
 *   passes of earlier ones.
 * SZSEL_OPT_BATCH_LANES: stream lanes of a batch of one request group
 *   (1..3, default 2; 0 restores it).  1 runs every launch on the caller's
 *   stream.  2 and 3 run the passes after the range scans on two streams
 *   (the caller's and a side stream joined before the results are read),
 *   so that the passes of the two lanes overlap: 2 deals the launch
 *   classes (dtype, rank, alignment, point sub-sampling) to the lanes in
 *   turn, or, for a batch of one class, cuts the requests where half of the
 *   sampled work lies before them; 3 always makes that cut.
 * SZSEL_OPT_RANGE_GRID: workgroups of a batch's range-scan launch (0 =
 *   default, one per scan chunk; k = 1..64: k per CU, each looping over
 *   the launch's chunks, which leaves the other wave slots of every CU to
 *   the sampled passes that run beside the scans).
 * SZSEL_OPT_HUFFMAN: 0 (default) no Huffman cost; 1 also computes the exact
 *   Huffman cost of the SZ code histogram (the entropy-coding stage that the
 *   0.5 bits/value offset of Section 6.2 stands in for) into
 *   sz_huffman_bits / sz_huffman_bitrate; 2 computes it and selects with it
 *   as BR_sz in place of entropy + offset.  The minimum cost is unique, so
 *   the result does not depend on how the tree is built.
 * SZSEL_OPT_EC_SAMPLING: 0 (default) the exact ZFP estimate (coder bit count
 *   of every sampled block, error after decoding); 1 the paper's cheaper
 *   estimate (Section 5.2.1-5.2.2, Algorithm 1's pointwise sampling): 3, 9 or 16
 *   coefficients per 1-, 2- or 3-D block, spread evenly over the coding
 *   order (position round(k (4^d - 1)/(r - 1))); BR_zfp = the mean
 *   significant-bit count with the other positions interpolated linearly;
 *   MSE_zfp = the mean squared truncation error of the sampled coefficients
 *   scaled by 2^(emax - P); 2 as 1 with each squared error weighted by the
 *   squared norm of its coefficient's data-domain image under ZFP's inverse
 *   transform (products of 4, 5, 4, 13/4 per axis), which the paper's
 *   norm-preservation argument leaves out.  zfp_bits is then 0, zfp_nsb_total
 *   counts the sampled points only, zfp_bitrate = zfp_nsb_mean =
 *   zfp_ec_nsb2 / (2 zfp_values), zfp_mse = zfp_sse / zfp_ec_points, and the
 *   flag SZSEL_FLAG_EC_SAMPLED is set. */
enum { SZSEL_OPT_SZ_OFFSET = 1, SZSEL_OPT_PROFILE = 2, SZSEL_OPT_AUTOTUNE = 3,
       SZSEL_OPT_BATCH_GRAPH = 4, SZSEL_OPT_SZ_WGS = 5, SZSEL_OPT_ZFP_CHUNK = 6,
       SZSEL_OPT_RANGE_WGS = 7, SZSEL_OPT_BATCH_GROUPS = 8, SZSEL_OPT_HUFFMAN = 9,
       SZSEL_OPT_EC_SAMPLING = 10, SZSEL_OPT_BATCH_SHARE = 11, SZSEL_OPT_RANGE_GRID = 12,
       SZSEL_OPT_BATCH_LANES = 13 };
int szsel_set_option(szsel_ctx *ctx, int option, double value);

/* ---------------------------------------------------------------------
 * Step 4 (Section 3; the compression that ends Algorithm 1): compressing the whole field with the
 * chosen compressor, for the true bit-rate and PSNR behind an estimate.
 * --------------------------------------------------------------------- */
typedef struct {
  uint64_t bits;              /* compressed size in bits */
  uint64_t values, blocks;    /* values of the field, 4^d blocks coded */
  double bitrate;             /* bits / values */
  double sse, mse, psnr, maxerr;  /* decompressed field against the input; PSNR with VR below */
  double vr, eb_abs;          /* value range of the field, the bound used */
  /* SZ only: values stored raw (escapes), distinct code symbols, bits of the
   * optimal prefix code of the symbols, their entropy in bits per value */
  uint64_t unpredictable, symbols, code_bits;
  double code_entropy;
  uint32_t flags;             /* SZSEL_FLAG_NO_HUFFMAN: code_bits not computed;
                                 SZSEL_FLAG_NONFINITE: the field holds NaN or Inf
                                 (the stream and totals are then meaningless) */
  int32_t pad;
} szsel_compressed;

/* Bytes of stream buffer szsel_zfp_compress needs for a field (a bound on
 * the stream plus two spare words); 0 for invalid arguments. */
size_t szsel_zfp_stream_bytes(const int64_t *dims, int ndims, int dtype);

/* ZFP fixed-accuracy compression at eb_abs of every 4^d block of the field
 * (Section 4.2 transform, Section 5.2 embedded coding; the same blocks the
 * estimator samples, padded at the upper faces by repeating the last value
 * along each axis), and its decompression.  Stream format: bit i is bit
 * (i mod 64) of 64-bit word i/64; blocks in row-major block order; a block
 * is one 0 bit (all zero or no plane kept), or a 1, E = 8/11 bits of
 * emax + 2^(E-1) - 1 (lowest first; emax at least the smallest normal
 * exponent) and the group-testing code of planes W-1 .. W-prec, prec =
 * emax - floor(log2 eb_abs) + 2(d+1) clamped to [0, W].  On whole blocks the
 * stream holds exactly the bits the estimator counts at stride 1.
 *   field        device pointer, C order, dims[0..ndims) slowest first
 *   stream_buf   device buffer (8-byte aligned) of stream_bytes >=
 *                szsel_zfp_stream_bytes(); receives the stream
 *   decoded      device buffer of the field's size and dtype for the
 *                decompressed field, or NULL
 *   out          host; filled when the call returns (the call waits for the
 *                work it queued on `stream`)
 * Returns SZSEL_OK or a negative code (szsel_last_error). */
int szsel_zfp_compress(szsel_ctx *ctx, const void *field, const int64_t *dims, int ndims, int dtype,
                       double eb_abs, void *stream_buf, size_t stream_bytes, void *decoded,
                       szsel_compressed *out, void *stream);

/* SZ compression at eb_abs of the whole field: Lorenzo prediction
 * (Section 4.3) from the decompressed values and linear-scaling
 * quantization (Section 5.1) with bins of 2 eb_abs, made parallel by
 * quantizing first: q = the nearest integer to x / (2 eb_abs) (halves away
 * from zero, 1/(2 eb_abs) one IEEE division; 0 when that is 2^50 or more),
 * so the decompressed neighbours are q 2 eb_abs exactly and the prediction
 * is the integer Lorenzo sum of their q (0 outside the field); code =
 * q - prediction.  A value is an escape, stored in W bits, when |code| >=
 * 32768 or q 2 eb_abs in the field's precision misses it by more than
 * eb_abs; its symbol is 0, otherwise code + 32768.  Decompressed value:
 * q 2 eb_abs, or the stored value.  bits = optimal prefix-code bits of the
 * symbols + W per escape + 32 per distinct symbol (the code table); when
 * the optimal code cannot be computed (SZSEL_FLAG_NO_HUFFMAN: more than
 * 16,384 distinct weights during the construction, impossible for fields of
 * at most 2^27 values; or 2^32 values or more), bits is 0 and bitrate uses
 * the symbols' entropy instead.  The squared errors are summed
 * by the pair tree in field order.
 *   symbols  device buffer of N uint16 for the symbols, or NULL
 *   decoded  device buffer of the field's size and dtype, or NULL
 * The call waits for the work it queued on `stream`. */
int szsel_sz_compress(szsel_ctx *ctx, const void *field, const int64_t *dims, int ndims, int dtype,
                      double eb_abs, void *symbols, void *decoded, szsel_compressed *out, void *stream);

/* Phase timers: synchronises the recorded events and returns, per phase
 * (0 = range pass, 1 = ZFP pass, 2 = SZ pass, 3 = overflow count, 4 =
 * entropy and selection, with the Huffman pass when it runs), the summed GPU
 * milliseconds in ms[5] and the number of timed calls (single requests) or
 * launches (batches: one launch per pass and request class) in calls[5];
 * then clears them. */
int szsel_profile_read(szsel_ctx *ctx, double *ms, uint64_t *calls);

/* The same split by field dtype: entry 2 * phase + dtype (SZSEL_F32 = 0,
 * SZSEL_F64 = 1) of ms[10] and calls[10] (a batched launch that serves both
 * dtypes counts under its first request's); clears the timers too. */
int szsel_profile_read_split(szsel_ctx *ctx, double *ms, uint64_t *calls);

/* Arms per-sample dumps for the next single-request call (NULL disarms). */
int szsel_set_debug(szsel_ctx *ctx, const szsel_debug *dump);

/* ---------------------------------------------------------------------
 * Serving: continuous batching of snapshots (not a step of the paper's
 * method; it runs the method online on snapshots as a simulation produces
 * them, the in-situ setting of Section 3).
 *
 * The caller owns a device pool (pool, pool_bytes; 256-byte aligned).  A
 * snapshot is admitted by reserving its bytes in the pool
 * (szsel_server_reserve: first fit over 256-byte granules; SZSEL_EBUSY while
 * the pool lacks room, SZSEL_ENOMEM if it never can).  The producer writes
 * the snapshot's fields into the reservation, then submits its requests
 * (every field must lie inside the reservation; producer_stream, if not
 * NULL, is the stream the producer wrote on, and the estimation waits for
 * it).  szsel_server_submit checks every request as the single-request
 * calls do and rejects the whole snapshot synchronously when one is
 * invalid (SZSEL_EINVAL / SZSEL_EDTYPE; nothing is queued, the reservation
 * stays and can be cancelled) or needs more workspace than one lane has
 * (SZSEL_ENOMEM).  Submitted requests wait in one FIFO; each of `lanes`
 * lanes (a stream with its own batch workspace of at most
 * lane_workspace_bytes, 0 = 4 GiB, of which the fixed workspace of up to 64
 * requests within half the budget and a quarter of the budget of variable
 * workspace are allocated at creation, so that serving rarely allocates)
 * takes up to 64 waiting requests, from any
 * number of snapshots and as many as its workspace holds, as one batch
 * whenever it is free, so work that arrives while other work runs starts on
 * the next free lane and overlaps it.  A batch that fails to launch is put
 * back in the queue and retried in halves; a request that fails alone
 * completes with SZSEL_FLAG_FAILED (for tests, the environment variable
 * SZSEL_SERVER_FAIL_BATCHES = k, read at creation, makes the server's first
 * k batches fail before they launch).  szsel_server_progress
 * retires finished lanes (writing results to each snapshot's `out`, which
 * must stay valid until the snapshot completes), releases completed
 * snapshots' reservations and dispatches waiting requests; with wait != 0
 * it first blocks until a busy lane finishes.  It returns the number of
 * snapshots completed by the call, or a negative code.  Results are the
 * same, bit for bit, as the single-request calls'.  Single-threaded: all
 * calls from one host thread.  With ctx == NULL only the admission calls
 * (reserve, cancel, stats) work: bookkeeping without a device. */
typedef struct szsel_server szsel_server;
int szsel_server_create(szsel_server **srv, szsel_ctx *ctx, void *pool, size_t pool_bytes, int lanes,
                        size_t lane_workspace_bytes);
void szsel_server_destroy(szsel_server *srv);
int szsel_server_reserve(szsel_server *srv, size_t bytes, void **dev_ptr, uint64_t *ticket);
/* Releases a reservation that was not submitted. */
int szsel_server_cancel(szsel_server *srv, uint64_t ticket);
int szsel_server_submit(szsel_server *srv, uint64_t ticket, const szsel_request *reqs, int n,
                        szsel_result *out, void *producer_stream);
int szsel_server_progress(szsel_server *srv, int wait);
/* 1 (and *latency_ms = submit-to-completion time) once the snapshot is
 * complete, after which the ticket is forgotten; 0 while it is not. */
int szsel_server_status(szsel_server *srv, uint64_t ticket, double *latency_ms);
/* stats[8]: batches launched, requests in them, snapshots completed,
 * requests waiting, busy lanes, pool bytes reserved, pool bytes, largest
 * free range. */
int szsel_server_stats(const szsel_server *srv, uint64_t *stats);
const char *szsel_server_last_error(const szsel_server *srv);

#ifdef __cplusplus
}
#endif
#endif /* SZSEL_H */
