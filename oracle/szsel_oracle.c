/*
 * Plain CPU oracle for the sampling-based SZ-vs-ZFP rate-distortion selector
 * (arXiv:1806.08901, Algorithm 1 with Sections 4 and 5).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the
 * benchmark's CPU-baseline leg, never by the product library.  It shares no
 * code, header, table or constant with the HIP path.
 *
 * Everything here is written for clarity, not speed: one loop per step, in the
 * order the method states it, FP64 throughout, built with -ffp-contract=off.
 * Where the paper leaves a convention open (ZFP internals, rounding, borders,
 * reduction order) the reading used is stated at the function that applies it.
 */
#include "szsel_oracle.h"

#include <float.h>
#include <limits.h>
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define NBINS 65536
#define RADIUS 32768

/* ------------------------------------------------------------------ */
/* Reductions                                                          */
/* ------------------------------------------------------------------ */

/* Adjacent-pair tree over a[0..n) padded with +0.0 to a power of two.
 * This fixes the association of every floating-point sum in the oracle. */
double orc_tree_sum(const double *a, int64_t n) {
  if (n <= 0) return 0.0;
  int64_t p = 1;
  while (p < n) p *= 2;
  double *buf = (double *)malloc((size_t)p * sizeof(double));
  for (int64_t i = 0; i < p; i++) buf[i] = i < n ? a[i] : 0.0;
  while (p > 1) {
    for (int64_t i = 0; i < p / 2; i++) buf[i] = buf[2 * i] + buf[2 * i + 1];
    p /= 2;
  }
  double s = buf[0];
  free(buf);
  return s;
}

/* ------------------------------------------------------------------ */
/* Field access                                                        */
/* ------------------------------------------------------------------ */

static double load(const void *field, int dtype, int64_t i) {
  return dtype == ORC_F32 ? (double)((const float *)field)[i] : ((const double *)field)[i];
}

/* Round a binary64 value to the field's precision (round to nearest even). */
static double to_dtype(double v, int dtype) {
  return dtype == ORC_F32 ? (double)(float)v : v;
}

static int64_t prod(const int64_t *dims, int nd) {
  int64_t n = 1;
  for (int k = 0; k < nd; k++) n *= dims[k];
  return n;
}

/* Value range over ALL values of the field (Algorithm 1's error bound; the value
 * range VR appears in the PSNR definition, Eq. 8).  Returns 1 when any value
 * is NaN or infinite, 0 otherwise. */
int orc_range(const void *field, int64_t n, int dtype, double *vmin, double *vmax) {
  double lo = INFINITY, hi = -INFINITY;
  for (int64_t i = 0; i < n; i++) {
    double v = load(field, dtype, i);
    if (!isfinite(v)) return 1;
    if (v < lo) lo = v;
    if (v > hi) hi = v;
  }
  *vmin = lo;
  *vmax = hi;
  return 0;
}

/* ------------------------------------------------------------------ */
/* Block sampling (Section 4.3; Algorithm 1)                          */
/* ------------------------------------------------------------------ */

/* Reading: the field is cut into full 4^d blocks (floor(n_k/4) per axis) and
 * block b is sampled iff b_k mod stride_k == 0 on every axis; sampled blocks
 * are enumerated row-major (last axis fastest), which fixes every reduction
 * order below. */
int64_t orc_num_sampled_blocks(const int64_t *dims, int nd, const int32_t *stride) {
  int64_t c = 1;
  for (int k = 0; k < nd; k++) {
    int64_t nb = dims[k] / 4;
    c *= (nb + stride[k] - 1) / stride[k];
  }
  return c;
}

void orc_sampled_block_origin(const int64_t *dims, int nd, const int32_t *stride,
                              int64_t j, int64_t *origin) {
  for (int k = nd - 1; k >= 0; k--) {
    int64_t nb = dims[k] / 4;
    int64_t ns = (nb + stride[k] - 1) / stride[k];
    int64_t jk = j % ns;
    j /= ns;
    origin[k] = 4 * jk * stride[k];
  }
}

/* Linear index of in-block point i (row-major over the block, last axis
 * fastest) of the block at origin[]. */
static int64_t block_point_index(const int64_t *dims, int nd, const int64_t *origin, int i,
                                 int64_t *pt) {
  int64_t lin = 0;
  for (int k = 0; k < nd; k++) {
    int shift = 2 * (nd - 1 - k);
    int off = (i >> shift) & 3;
    pt[k] = origin[k] + off;
    lin = lin * dims[k] + pt[k];
  }
  return lin;
}

/* ------------------------------------------------------------------ */
/* ZFP side (Stage I block transform, Section 4.2; embedded coding,    */
/* Section 5.2).  The paper names ZFP's steps without defining them;   */
/* the steps below follow ZFP's published fixed-accuracy design.       */
/* ------------------------------------------------------------------ */

/* Exponent e with m in [2^(e-1), 2^e) for m > 0 (the frexp convention). */
int orc_frexp_exponent(double m) {
  int e;
  (void)frexp(m, &e);
  return e;
}

/* floor(log2(tau)) for tau > 0, which is the smallest coded bit plane of the
 * fixed-accuracy mode. */
int orc_floor_log2(double tau) { return orc_frexp_exponent(tau) - 1; }

/* Number of coded bit planes of a block with exponent emax at tolerance
 * 2^minexp: emax - minexp + 2(d+1), clamped to [0, W]. */
int orc_precision(int emax, int minexp, int nd, int W) {
  long p = (long)emax - (long)minexp + 2L * (nd + 1);
  if (p < 0) p = 0;
  if (p > W) p = W;
  return (int)p;
}

/* Two's complement wrap of v to W bits (W = 32 or 64), sign-extended. */
static int64_t wrap(uint64_t v, int W) {
  return W == 64 ? (int64_t)v : (int64_t)(int32_t)(uint32_t)v;
}
static int64_t add(int64_t a, int64_t b, int W) { return wrap((uint64_t)a + (uint64_t)b, W); }
static int64_t sub(int64_t a, int64_t b, int W) { return wrap((uint64_t)a - (uint64_t)b, W); }
static int64_t half(int64_t a) { return a >> 1; } /* floor(a / 2) */

/* Forward 4-point decorrelating transform as integer lifting.  On inputs that
 * are multiples of 16 it equals the matrix
 *     (1/16) [[ 4, 4, 4, 4], [ 5, 1,-1,-5], [-4, 4, 4,-4], [-2, 6,-6, 2]]
 * exactly (ZFP's published non-orthogonal transform); elsewhere each halving
 * rounds toward minus infinity.  Factorisation: average/difference the outer
 * pair and the inner pair, then the two averages and the two differences,
 * then two shears between the last two outputs. */
void orc_fwd_lift(int64_t *v, ptrdiff_t s, int W) {
  int64_t x0 = v[0], x1 = v[s], x2 = v[2 * s], x3 = v[3 * s];
  int64_t a = half(add(x0, x3, W)), p = sub(x0, a, W); /* (x0+x3)/2, (x0-x3)/2 */
  int64_t b = half(add(x1, x2, W)), q = sub(x1, b, W); /* (x1+x2)/2, (x1-x2)/2 */
  int64_t y0 = half(add(a, b, W)), y2 = sub(b, y0, W);
  int64_t u = half(add(p, q, W)), w = sub(p, u, W);
  int64_t y3 = sub(half(u), w, W);
  int64_t y1 = sub(u, half(y3), W);
  v[0] = y0;
  v[s] = y1;
  v[2 * s] = y2;
  v[3 * s] = y3;
}

/* Inverse lifting: undoes every step of orc_fwd_lift in reverse order, so
 * that fwd(inv(y)) == y; inv(fwd(x)) differs from x by the discarded low bits. */
void orc_inv_lift(int64_t *v, ptrdiff_t s, int W) {
  int64_t y0 = v[0], y1 = v[s], y2 = v[2 * s], y3 = v[3 * s];
  int64_t u = add(y1, half(y3), W);
  int64_t w = sub(half(u), y3, W);
  int64_t p = add(u, w, W), q = sub(u, w, W);
  int64_t b = add(y0, y2, W), a = sub(y0, y2, W);
  v[0] = add(a, p, W);
  v[3 * s] = sub(a, p, W);
  v[s] = add(b, q, W);
  v[2 * s] = sub(b, q, W);
}

/* Separable block transform (Section 4.2: the 1-D transform is applied along
 * each of the d axes of the 4^d block in turn).  Axis order: fastest first. */
void orc_fwd_xform(int64_t *c, int nd, int W) {
  int size = 1 << (2 * nd);
  for (int a = 0; a < nd; a++) {
    int s = 1 << (2 * a);
    for (int i = 0; i < size; i++)
      if (((i / s) & 3) == 0) orc_fwd_lift(c + i, s, W);
  }
}

void orc_inv_xform(int64_t *c, int nd, int W) {
  int size = 1 << (2 * nd);
  for (int a = nd - 1; a >= 0; a--) {
    int s = 1 << (2 * a);
    for (int i = 0; i < size; i++)
      if (((i / s) & 3) == 0) orc_inv_lift(c + i, s, W);
  }
}

/* Coefficient order for the embedded coder: ascending total sequency
 * (sum of the per-axis frequencies), ties by the sum of squared frequencies,
 * then by the slowest axis' frequency, ..., then the fastest.  perm[r] is the
 * in-block index of the coefficient coded at position r. */
static int reorder_less(int i, int j, int nd) {
  int fi[3] = {0, 0, 0}, fj[3] = {0, 0, 0};
  for (int a = 0; a < nd; a++) {
    fi[a] = (i >> (2 * a)) & 3; /* a = 0: fastest axis */
    fj[a] = (j >> (2 * a)) & 3;
  }
  int si = fi[0] + fi[1] + fi[2], sj = fj[0] + fj[1] + fj[2];
  if (si != sj) return si < sj;
  int qi = fi[0] * fi[0] + fi[1] * fi[1] + fi[2] * fi[2];
  int qj = fj[0] * fj[0] + fj[1] * fj[1] + fj[2] * fj[2];
  if (qi != qj) return qi < qj;
  for (int a = nd - 1; a >= 0; a--)
    if (fi[a] != fj[a]) return fi[a] < fj[a];
  return 0;
}

void orc_reorder_table(int nd, int32_t *perm) {
  int size = 1 << (2 * nd);
  for (int i = 0; i < size; i++) perm[i] = i;
  for (int i = 1; i < size; i++) { /* insertion sort by the key above */
    int v = perm[i], k = i - 1;
    while (k >= 0 && reorder_less(v, perm[k], nd)) {
      perm[k + 1] = perm[k];
      k--;
    }
    perm[k + 1] = v;
  }
}

static uint64_t nb_mask(int W) { return W == 64 ? 0xAAAAAAAAAAAAAAAAull : 0xAAAAAAAAull; }
static uint64_t low_bits(int W) { return W == 64 ? ~0ull : 0xFFFFFFFFull; }

/* Negabinary (base -2) digits of c as a W-bit word: u = (c + M) xor M. */
uint64_t orc_to_negabinary(int64_t c, int W) {
  uint64_t m = nb_mask(W);
  return (((uint64_t)c + m) ^ m) & low_bits(W);
}

int64_t orc_from_negabinary(uint64_t u, int W) {
  uint64_t m = nb_mask(W);
  return wrap((u ^ m) - m, W);
}

static int msb64(uint64_t v) { /* index of the highest set bit, -1 for 0 */
  int k = -1;
  while (v) {
    k++;
    v >>= 1;
  }
  return k;
}

/* Group-testing embedded coding of bit planes W-1 down to W-prec (Section 5.2,
 * "group-testing-based EC").  Per plane: the bits of the n values already
 * known to be significant are sent verbatim; then, while values remain, one
 * bit tells whether any remaining value has a 1 in this plane; if so the
 * remaining bits are sent one by one up to and including that 1 (the bit of
 * the last value is implied, not sent), and all values up to it become
 * significant. */
int64_t orc_encode_planes(const uint64_t *u, int size, int W, int prec, uint8_t *bits,
                          int64_t cap) {
  int64_t nbits = 0;
#define EMIT(b)                                          \
  do {                                                   \
    if (bits && nbits < cap) bits[nbits] = (uint8_t)(b); \
    nbits++;                                             \
  } while (0)
  int n = 0;
  for (int k = W - 1; k >= W - prec; k--) {
    int plane[64];
    for (int i = 0; i < size; i++) plane[i] = (int)((u[i] >> k) & 1u);
    for (int i = 0; i < n; i++) EMIT(plane[i]);
    int pos = n;
    while (pos < size) {
      int any = 0;
      for (int j = pos; j < size; j++) any |= plane[j];
      EMIT(any);
      if (!any) break;
      while (pos < size - 1) {
        EMIT(plane[pos]);
        if (plane[pos]) break;
        pos++;
      }
      pos++; /* the 1 just sent, or implied at the last position */
      n = pos;
    }
  }
#undef EMIT
  return nbits;
}

/* One 4^d block through block-floating-point conversion, forward transform,
 * reordering, negabinary, embedded coding of the planes that the
 * fixed-accuracy mode keeps, and the matching decode.
 *   - empty block (all values zero) or zero coded planes: 1 bit, decodes to 0;
 *   - otherwise 1 + E header bits (E = 8 for binary32, 11 for binary64) plus
 *     the coder's bits.
 * The error is measured in the data domain after decoding (the paper measures
 * it in the transform domain, which equals the data-domain error only for an
 * orthogonal transform; ZFP's transform is not orthogonal). */
uint32_t orc_zfp_block(const double *x, int nd, int dtype, int minexp, double *xhat,
                       double *sse, uint64_t *nsb, int32_t *emax_out) {
  const int W = dtype == ORC_F32 ? 32 : 64;
  const int P = W - 2;
  const int E = dtype == ORC_F32 ? 8 : 11;
  const int size = 1 << (2 * nd);
  double err2[64];
  double m = 0.0;
  for (int i = 0; i < size; i++)
    if (fabs(x[i]) > m) m = fabs(x[i]);
  *nsb = 0;
  if (m == 0.0) {
    for (int i = 0; i < size; i++) {
      xhat[i] = 0.0;
      err2[i] = x[i] * x[i];
    }
    *sse = orc_tree_sum(err2, size);
    *emax_out = INT32_MIN;
    return 1;
  }
  const int emax = orc_frexp_exponent(m);
  *emax_out = emax;
  const int prec = orc_precision(emax, minexp, nd, W);
  if (prec == 0) {
    for (int i = 0; i < size; i++) {
      xhat[i] = 0.0;
      err2[i] = x[i] * x[i];
    }
    *sse = orc_tree_sum(err2, size);
    return 1;
  }
  /* block-floating-point: common exponent emax, P-bit signed integers */
  int64_t c[64];
  for (int i = 0; i < size; i++) c[i] = (int64_t)trunc(ldexp(x[i], P - emax));
  orc_fwd_xform(c, nd, W);
  int32_t perm[64];
  orc_reorder_table(nd, perm);
  uint64_t u[64];
  for (int r = 0; r < size; r++) u[r] = orc_to_negabinary(c[perm[r]], W);
  int64_t coder = orc_encode_planes(u, size, W, prec, NULL, 0);
  /* significant bits of each value within the coded planes (Section 5.2.1) */
  const int kmin = W - prec;
  uint64_t nsum = 0;
  for (int r = 0; r < size; r++) {
    int ms = msb64(u[r]);
    if (ms >= kmin) nsum += (uint64_t)(ms - kmin + 1);
  }
  *nsb = nsum;
  /* decode: drop the planes below kmin and invert every step */
  uint64_t keep = kmin == 0 ? low_bits(W) : (low_bits(W) & ~((1ull << kmin) - 1ull));
  int64_t d[64];
  for (int r = 0; r < size; r++) d[perm[r]] = orc_from_negabinary(u[r] & keep, W);
  orc_inv_xform(d, nd, W);
  for (int i = 0; i < size; i++) {
    xhat[i] = to_dtype(ldexp((double)d[i], emax - P), dtype);
    double e = x[i] - xhat[i];
    err2[i] = e * e;
  }
  *sse = orc_tree_sum(err2, size);
  return (uint32_t)(1 + E + coder);
}

/* ------------------------------------------------------------------ */
/* ZFP side by point sub-sampling (Sections 5.2.1, 5.2.2)              */
/* ------------------------------------------------------------------ */

int orc_ec_default_points(int nd) { return nd == 1 ? 3 : (nd == 2 ? 9 : 16); }

/* k-th of r positions: round(k (size - 1) / (r - 1)), halves rounded up. */
void orc_ec_positions(int size, int r, int32_t *pos) {
  for (int k = 0; k < r; k++)
    pos[k] = (int32_t)((2L * k * (size - 1) + (r - 1)) / (2L * (r - 1)));
}

/* The paper's estimate for one block: transform the block as ZFP does, take
 * r coefficients spread over the coding order, count each one's significant
 * bits within the coded planes (its top set bit down to the last coded
 * plane), fill the other positions by linear interpolation between the
 * neighbouring samples and sum; and take each sampled coefficient's
 * truncation error (the value of the digits below the last coded plane),
 * scaled by the block's exponent to the data's units.
 * The interpolated sum over a gap between samples at positions a < b with
 * counts va, vb is (b - a - 1)(va + vb)/2, so twice the block's total is an
 * integer. */
/* Squared norm of the data-domain image of a unit coefficient with
 * frequency f along one axis: the columns of the inverse of ZFP's transform
 * matrix (1/16)[[4,4,4,4],[5,1,-1,-5],[-4,4,4,-4],[-2,6,-6,2]] are
 * (1/4)(4,4,4,4), (1/4)(6,2,-2,-6), (1/4)(-4,4,4,-4), (1/4)(-1,5,-5,1). */
static const double kInvColNorm2[4] = {4.0, 5.0, 4.0, 3.25};

double orc_ec_gain(int i, int nd) {
  double g = 1.0;
  for (int a = 0; a < nd; a++) g *= kInvColNorm2[(i >> (2 * a)) & 3];
  return g;
}

void orc_zfp_block_ec(const double *x, int nd, int dtype, int minexp, int r, uint64_t *nsb2,
                      uint64_t *nsb_pts, double *err, double *gain, int32_t *emax_out) {
  const int W = dtype == ORC_F32 ? 32 : 64;
  const int P = W - 2;
  const int size = 1 << (2 * nd);
  int R = 1;
  while (R < r) R *= 2;
  int32_t perm[64], pos[64];
  orc_reorder_table(nd, perm);
  orc_ec_positions(size, r, pos);
  for (int k = 0; k < R; k++) {
    err[k] = 0.0;
    gain[k] = k < r ? orc_ec_gain(perm[pos[k]], nd) : 1.0;
  }
  *nsb2 = 0;
  *nsb_pts = 0;
  double m = 0.0;
  for (int i = 0; i < size; i++)
    if (fabs(x[i]) > m) m = fabs(x[i]);
  if (m == 0.0) { /* every coefficient is 0: no bits, no error */
    *emax_out = INT32_MIN;
    return;
  }
  const int emax = orc_frexp_exponent(m);
  *emax_out = emax;
  const int prec = orc_precision(emax, minexp, nd, W);
  int64_t c[64];
  for (int i = 0; i < size; i++) c[i] = (int64_t)trunc(ldexp(x[i], P - emax));
  orc_fwd_xform(c, nd, W);
  const int kmin = W - prec;
  const uint64_t keep = kmin >= W ? 0ull : (low_bits(W) & ~((1ull << kmin) - 1ull));
  uint64_t v[64];
  for (int k = 0; k < r; k++) {
    const int64_t coef = c[perm[pos[k]]];
    const uint64_t u = orc_to_negabinary(coef, W);
    const int ms = msb64(u);
    v[k] = ms >= kmin ? (uint64_t)(ms - kmin + 1) : 0;
    *nsb_pts += v[k];
    const int64_t kept = orc_from_negabinary(u & keep, W);
    err[k] = ldexp((double)sub(coef, kept, W), emax - P);
  }
  uint64_t twice = 0;
  for (int k = 0; k < r; k++) twice += 2 * v[k];
  for (int k = 0; k + 1 < r; k++) twice += (uint64_t)(pos[k + 1] - pos[k] - 1) * (v[k] + v[k + 1]);
  *nsb2 = twice;
}

/* ------------------------------------------------------------------ */
/* SZ side (prediction-based transform, Section 4.1; linear-scaling     */
/* quantization, Section 5.1)                                           */
/* ------------------------------------------------------------------ */

/* Lorenzo prediction from the ORIGINAL neighbours (Section 4.3): the sum over
 * the non-empty subsets S of the axes of (-1)^(|S|+1) X[p - e_S], with X = 0
 * outside the field (so borders fall back to the lower-order predictor).
 * Terms are added in a fixed order: |S| = 1 by axis (slowest axis first),
 * then |S| = 2 in lexicographic order, then |S| = 3. */
double orc_lorenzo(const void *field, const int64_t *dims, int nd, int dtype,
                   const int64_t *p) {
  int order[7], cnt = 0;
  for (int sz = 1; sz <= nd; sz++) { /* subsets as bit masks, axis 0 = bit 0 */
    if (sz == 1)
      for (int a = 0; a < nd; a++) order[cnt++] = 1 << a;
    else if (sz == 2)
      for (int a = 0; a < nd; a++)
        for (int b = a + 1; b < nd; b++) order[cnt++] = (1 << a) | (1 << b);
    else
      order[cnt++] = 7;
  }
  double acc = 0.0;
  for (int t = 0; t < cnt; t++) {
    int S = order[t], card = 0, inside = 1;
    int64_t lin = 0;
    for (int k = 0; k < nd; k++) {
      int64_t c = p[k];
      if (S & (1 << k)) {
        c -= 1;
        card++;
      }
      if (c < 0) inside = 0;
      lin = lin * dims[k] + c;
    }
    double v = inside ? load(field, dtype, lin) : 0.0;
    if (t == 0)
      acc = v;
    else if (card & 1)
      acc = acc + v;
    else
      acc = acc - v;
  }
  return acc;
}

/* Shannon entropy of the code histogram (Eq. 5 with P_i = h_i / n):
 * H = log2(n) - (1/n) sum_i h_i log2 h_i, with 0 log 0 = 0. */
double orc_entropy(const uint32_t *hist, int64_t nbins, uint64_t n) {
  if (n == 0) return 0.0;
  double *t = (double *)malloc((size_t)nbins * sizeof(double));
  for (int64_t i = 0; i < nbins; i++) {
    double h = (double)hist[i];
    t[i] = hist[i] ? h * log2(h) : 0.0;
  }
  double s = orc_tree_sum(t, nbins);
  free(t);
  return log2((double)n) - s / (double)n;
}

/* Exact cost of the entropy-coding stage that the +0.5 bits/value offset of
 * Section 6.2 stands in for: the code histogram is Huffman coded (Section
 * 3's Stage III), and an optimal prefix code spends sum_i h_i L_i bits, which
 * equals the sum of the internal node weights of the Huffman tree.  The
 * minimum is unique even though the tree is not.  Binary min-heap of 64-bit
 * node weights. */
static void heap_push(uint64_t *h, int64_t *n, uint64_t v) {
  int64_t i = (*n)++;
  h[i] = v;
  while (i > 0) {
    int64_t p = (i - 1) / 2;
    if (h[p] <= h[i]) break;
    uint64_t t = h[p];
    h[p] = h[i];
    h[i] = t;
    i = p;
  }
}

static uint64_t heap_pop(uint64_t *h, int64_t *n) {
  uint64_t top = h[0];
  h[0] = h[--(*n)];
  int64_t i = 0;
  for (;;) {
    int64_t l = 2 * i + 1, r = l + 1, m = i;
    if (l < *n && h[l] < h[m]) m = l;
    if (r < *n && h[r] < h[m]) m = r;
    if (m == i) break;
    uint64_t t = h[m];
    h[m] = h[i];
    h[i] = t;
    i = m;
  }
  return top;
}

uint64_t orc_huffman_bits(const uint32_t *hist, int64_t nbins) {
  uint64_t *h = (uint64_t *)malloc((size_t)(nbins > 0 ? nbins : 1) * sizeof(uint64_t));
  int64_t n = 0;
  uint64_t total = 0;
  for (int64_t i = 0; i < nbins; i++)
    if (hist[i]) {
      heap_push(h, &n, hist[i]);
      total += hist[i];
    }
  uint64_t cost = 0;
  if (n == 1) cost = total; /* one symbol: 1 bit each */
  while (n > 1) {
    uint64_t a = heap_pop(h, &n), b = heap_pop(h, &n);
    cost += a + b;
    heap_push(h, &n, a + b);
  }
  free(h);
  return cost;
}

/* ------------------------------------------------------------------ */
/* The estimator (Algorithm 1)                                          */
/* ------------------------------------------------------------------ */

int orc_run(int op, const void *field, const int64_t *dims, int nd, int dtype, double eb,
            int eb_mode, const int32_t *stride, double sz_offset, int huffman, int ec_points,
            int ec_weight, orc_result *out, orc_dump *dump) {
  if (!out || !field || !dims || !stride) return -1;
  if (nd < 1 || nd > 3 || (dtype != ORC_F32 && dtype != ORC_F64)) return -1;
  if (op < ORC_OP_SZ || op > ORC_OP_FIXED_EB) return -1;
  if (ec_points < 0 || ec_points > (1 << (2 * nd))) return -1;
  const int ec_r = ec_points == 1 ? orc_ec_default_points(nd) : ec_points;
  if (huffman < 0 || huffman > 2) return -1;
  if (!(eb > 0.0) || !isfinite(eb) || (eb_mode != ORC_EB_ABS && eb_mode != ORC_EB_REL)) return -1;
  for (int k = 0; k < nd; k++)
    if (dims[k] < 1 || stride[k] < 1) return -1;
  memset(out, 0, sizeof(*out));
  const int selecting = op == ORC_OP_SELECT || op == ORC_OP_FIXED_EB;
  out->choice = -1;
  const int W = dtype == ORC_F32 ? 32 : 64;
  const int size = 1 << (2 * nd);
  const int64_t N = prod(dims, nd);

  /* error bound from the value range of the whole field */
  double vmin = 0.0, vmax = 0.0;
  if (orc_range(field, N, dtype, &vmin, &vmax)) {
    out->flags |= ORC_FLAG_NONFINITE;
    return 0;
  }
  out->vmin = vmin;
  out->vmax = vmax;
  const double vr = vmax - vmin;
  out->vr = vr;
  const double eb_abs = eb_mode == ORC_EB_REL ? eb * vr : eb;
  out->eb_abs = eb_abs;
  if (vr == 0.0) { /* constant field: nothing to estimate; SZ by convention */
    out->flags |= ORC_FLAG_CONSTANT;
    if (selecting) out->choice = 0;
    return 0;
  }
  if (!(eb_abs > 0.0) || !isfinite(eb_abs)) { /* eb_rel * VR left the binary64 range */
    out->flags |= ORC_FLAG_BAD_EB;
    if (selecting) out->choice = 0;
    return 0;
  }
  /* blockwise sampling */
  const int64_t nblk = orc_num_sampled_blocks(dims, nd, stride);
  if (nblk == 0) {
    out->flags |= ORC_FLAG_NO_BLOCKS;
    if (selecting) out->choice = 0;
    return 0;
  }
  const int64_t nvals = nblk * size;
  const int minexp = orc_floor_log2(eb_abs);
  out->minexp = minexp;

  double *err2 = (double *)malloc((size_t)nvals * sizeof(double));
  int64_t origin[3], pt[3];
  double x[64], xh[64];

  /* ZFP bit-rate and PSNR on the sampled blocks */
  double br_zfp = 0.0, mse_zfp = 0.0;
  if (op != ORC_OP_SZ && ec_r) {
    /* as Algorithm 1 states it: point sub-sampling of the
     * sampled blocks, interpolated mean significant-bit count, MSE of the
     * sub-sampled points' transform-domain errors */
    int R = 1;
    while (R < ec_r) R *= 2;
    double *e2 = (double *)malloc((size_t)nblk * R * sizeof(double));
    uint64_t twice_total = 0, pts_total = 0;
    double maxerr = 0.0, err[64], gain[64];
    for (int64_t j = 0; j < nblk; j++) {
      orc_sampled_block_origin(dims, nd, stride, j, origin);
      for (int i = 0; i < size; i++)
        x[i] = load(field, dtype, block_point_index(dims, nd, origin, i, pt));
      uint64_t twice, pts;
      int32_t emax;
      orc_zfp_block_ec(x, nd, dtype, minexp, ec_r, &twice, &pts, err, gain, &emax);
      twice_total += twice;
      pts_total += pts;
      for (int k = 0; k < R; k++) {
        e2[j * R + k] = ec_weight ? (err[k] * err[k]) * gain[k] : err[k] * err[k];
        if (fabs(err[k]) > maxerr) maxerr = fabs(err[k]);
        if (dump && dump->ec_err) dump->ec_err[j * R + k] = err[k];
      }
      if (dump && dump->ec_nsb2) dump->ec_nsb2[j] = (uint32_t)twice;
      if (dump && dump->zfp_emax) dump->zfp_emax[j] = emax;
    }
    const int64_t npts = nblk * ec_r;
    const double sse = orc_tree_sum(e2, nblk * R);
    free(e2);
    mse_zfp = sse / (double)npts;
    br_zfp = (double)twice_total / (double)(2 * nvals);
    out->flags |= ORC_FLAG_EC_SAMPLED;
    out->zfp_sse = sse;
    out->zfp_mse = mse_zfp;
    out->zfp_bits = 0;
    out->zfp_values = (uint64_t)nvals;
    out->zfp_blocks = (uint64_t)nblk;
    out->zfp_nsb_total = pts_total;
    out->zfp_nsb_mean = br_zfp;
    out->zfp_bitrate = br_zfp;
    out->zfp_maxerr = maxerr;
    out->zfp_psnr = mse_zfp > 0.0 ? 20.0 * log10(vr) - 10.0 * log10(mse_zfp) : INFINITY;
    out->zfp_ec_points = (uint64_t)npts;
    out->zfp_ec_nsb2 = twice_total;
  } else if (op != ORC_OP_SZ) {
    uint64_t bits_total = 0, nsb_total = 0;
    double maxerr = 0.0;
    for (int64_t j = 0; j < nblk; j++) {
      orc_sampled_block_origin(dims, nd, stride, j, origin);
      for (int i = 0; i < size; i++)
        x[i] = load(field, dtype, block_point_index(dims, nd, origin, i, pt));
      double bsse;
      uint64_t bnsb;
      int32_t emax;
      uint32_t bits = orc_zfp_block(x, nd, dtype, minexp, xh, &bsse, &bnsb, &emax);
      bits_total += bits;
      nsb_total += bnsb;
      for (int i = 0; i < size; i++) {
        double e = x[i] - xh[i];
        err2[j * size + i] = e * e;
        if (fabs(e) > maxerr) maxerr = fabs(e);
      }
      if (dump && dump->zfp_bits) dump->zfp_bits[j] = bits;
      if (dump && dump->zfp_sse) dump->zfp_sse[j] = bsse;
      if (dump && dump->zfp_emax) dump->zfp_emax[j] = emax;
    }
    double sse = orc_tree_sum(err2, nvals);
    mse_zfp = sse / (double)nvals;
    br_zfp = (double)bits_total / (double)nvals;
    out->zfp_sse = sse;
    out->zfp_mse = mse_zfp;
    out->zfp_bits = bits_total;
    out->zfp_values = (uint64_t)nvals;
    out->zfp_blocks = (uint64_t)nblk;
    out->zfp_nsb_total = nsb_total;
    out->zfp_nsb_mean = (double)nsb_total / (double)nvals;
    out->zfp_bitrate = br_zfp;
    out->zfp_maxerr = maxerr;
    out->zfp_psnr = mse_zfp > 0.0 ? 20.0 * log10(vr) - 10.0 * log10(mse_zfp) : INFINITY;
  }

  if (op != ORC_OP_ZFP) {
    /* bin size delta.  Selection: the delta whose uniform-error PSNR
     * (Eq. 10) equals PSNR_zfp, i.e. delta = sqrt(12 MSE_zfp).  Otherwise SZ's
     * own rule delta = 2 eb_abs (Section 5.1.4). */
    double delta = 2.0 * eb_abs;
    if (op == ORC_OP_SELECT) {
      if (mse_zfp > 0.0)
        delta = sqrt(12.0 * mse_zfp);
      else
        out->flags |= ORC_FLAG_ZERO_MSE;
    }
    const double inv = 1.0 / delta;
    const double eb_sz = 0.5 * delta;
    uint32_t *hist = (uint32_t *)calloc(NBINS, sizeof(uint32_t));
    uint64_t unpred = 0;
    double maxerr = 0.0;
    /* quantization codes of all points of the sampled blocks */
    for (int64_t j = 0; j < nblk; j++) {
      orc_sampled_block_origin(dims, nd, stride, j, origin);
      for (int i = 0; i < size; i++) {
        int64_t lin = block_point_index(dims, nd, origin, i, pt);
        double xv = load(field, dtype, lin);
        double pred = orc_lorenzo(field, dims, nd, dtype, pt);
        double d = xv - pred;
        int code = 0;
        double e2 = 0.0;
        double t = fabs(d) * inv + 0.5; /* round half away from zero */
        if (t < (double)RADIUS) {
          int64_t q = (int64_t)floor(t);
          if (d < 0.0) q = -q;
          double recon = to_dtype(pred + (double)q * delta, dtype);
          double e = xv - recon;
          if (fabs(e) <= eb_sz) { /* reconstruction stays within the bound */
            code = (int)q + RADIUS;
            e2 = e * e;
            if (fabs(e) > maxerr) maxerr = fabs(e);
          }
        }
        if (code == 0) unpred++;
        hist[code]++;
        err2[j * size + i] = e2;
        if (dump && dump->codes) dump->codes[j * size + i] = (uint16_t)code;
      }
      if (dump && dump->sz_sse) dump->sz_sse[j] = orc_tree_sum(err2 + j * size, size);
    }
    double sse = orc_tree_sum(err2, nvals);
    double H = orc_entropy(hist, NBINS, (uint64_t)nvals);
    double br = H + sz_offset;
    br = br + ((double)unpred * (double)W) / (double)nvals;
    out->sz_delta = delta;
    out->sz_inv_delta = inv;
    out->sz_eb = eb_sz;
    out->sz_entropy = H;
    out->sz_bitrate = br;
    out->sz_sse = sse;
    out->sz_mse = sse / (double)nvals;
    out->sz_maxerr = maxerr;
    out->sz_values = (uint64_t)nvals;
    out->sz_unpredictable = unpred;
    out->sz_psnr_model = 20.0 * log10(vr / delta) + 10.0 * log10(12.0);
    out->sz_psnr_measured =
        out->sz_mse > 0.0 ? 20.0 * log10(vr) - 10.0 * log10(out->sz_mse) : INFINITY;
    double br_sel = br; /* hist[0] counts the unpredictable points (code 0) */
    if (huffman) {
      const uint64_t hb = orc_huffman_bits(hist, NBINS);
      double hbr = (double)hb / (double)nvals;
      hbr = hbr + ((double)unpred * (double)W) / (double)nvals;
      out->sz_huffman_bits = hb;
      out->sz_huffman_bitrate = hbr;
      if (huffman == 2) br_sel = hbr;
    }
    if (dump && dump->hist) memcpy(dump->hist, hist, NBINS * sizeof(uint32_t));
    free(hist);

    /* selection: the lower estimated bit-rate wins; ties go to ZFP */
    if (selecting) {
      out->choice = br_sel < br_zfp ? 0 : 1;
      out->chosen_eb = out->choice == 0 ? eb_sz : eb_abs;
      if (eb_sz > eb_abs) out->flags |= ORC_FLAG_EB_EXCEEDS;
    }
  }
  free(err2);
  return 0;
}

/* ------------------------------------------------------------------ */
/* Step 4 (Section 3; Algorithm 1's ZFP branch): ZFP compression of    */
/* the whole field at eb_abs, and its decompression                    */
/* ------------------------------------------------------------------ */

/* Stream: the bits in order, bit i in bit (i mod 64) of 64-bit word i/64
 * (here one byte per bit).  Blocks in row-major block order over
 * ceil(n_k / 4) blocks per axis; a block's positions past the field's
 * upper faces repeat the field's last value along that axis.  A block:
 * one bit (0: coded as zero, when all values are 0 or no plane is kept;
 * 1: coded), then E bits of emax + 2^(E-1) - 1 (lowest bit first; emax
 * is at least 2 - 2^(E-1), ZFP's smallest normal exponent), then the
 * group-testing code of planes W-1 .. W-prec. */

static void put_bits(uint8_t *bits, int64_t cap, int64_t *pos, uint64_t v, int n) {
  for (int b = 0; b < n; b++) {
    if (bits && *pos < cap) bits[*pos] = (uint8_t)((v >> b) & 1u);
    (*pos)++;
  }
}

static int get_bit(const uint8_t *bits, int64_t nbits, int64_t *pos) {
  int b = *pos < nbits ? bits[*pos] : 0;
  (*pos)++;
  return b;
}

/* Gathers block (row-major block index jb) with edge repetition. */
static void gather_block(const void *field, const int64_t *dims, int nd, int dtype, int64_t jb,
                         double *x, int64_t *lin, int *valid) {
  int64_t nb[3], bo[3];
  for (int k = 0; k < nd; k++) nb[k] = (dims[k] + 3) / 4;
  int64_t rem = jb;
  for (int k = nd - 1; k >= 0; k--) {
    bo[k] = 4 * (rem % nb[k]);
    rem /= nb[k];
  }
  const int size = 1 << (2 * nd);
  for (int i = 0; i < size; i++) {
    int64_t l = 0;
    int ok = 1;
    for (int k = 0; k < nd; k++) {
      int off = (i >> (2 * (nd - 1 - k))) & 3;
      int64_t p = bo[k] + off;
      if (p >= dims[k]) {
        p = dims[k] - 1;
        ok = 0;
      }
      l = l * dims[k] + p;
    }
    x[i] = load(field, dtype, l);
    lin[i] = l;
    valid[i] = ok;
  }
}

int64_t orc_zfp_num_blocks(const int64_t *dims, int nd) {
  int64_t n = 1;
  for (int k = 0; k < nd; k++) n *= (dims[k] + 3) / 4;
  return n;
}

/* Encodes one gathered block; returns the number of bits. */
static int64_t zfp_encode_block(const double *x, int nd, int dtype, int minexp, uint8_t *bits,
                                int64_t cap, int64_t pos0) {
  const int W = dtype == ORC_F32 ? 32 : 64;
  const int P = W - 2;
  const int E = dtype == ORC_F32 ? 8 : 11;
  const int bias = (1 << (E - 1)) - 1;
  const int size = 1 << (2 * nd);
  int64_t pos = pos0;
  double m = 0.0;
  for (int i = 0; i < size; i++)
    if (fabs(x[i]) > m) m = fabs(x[i]);
  int emax = m > 0.0 ? orc_frexp_exponent(m) : 0;
  if (emax < 1 - bias) emax = 1 - bias;
  const int prec = m > 0.0 ? orc_precision(emax, minexp, nd, W) : 0;
  if (prec == 0) {
    put_bits(bits, cap, &pos, 0, 1);
    return pos - pos0;
  }
  put_bits(bits, cap, &pos, 1, 1);
  put_bits(bits, cap, &pos, (uint64_t)(emax + bias), E);
  int64_t c[64];
  for (int i = 0; i < size; i++) c[i] = (int64_t)trunc(ldexp(x[i], P - emax));
  orc_fwd_xform(c, nd, W);
  int32_t perm[64];
  orc_reorder_table(nd, perm);
  uint64_t u[64];
  for (int r = 0; r < size; r++) u[r] = orc_to_negabinary(c[perm[r]], W);
  int64_t nb = orc_encode_planes(u, size, W, prec, bits ? bits + pos : NULL,
                                 bits ? (cap > pos ? cap - pos : 0) : 0);
  return pos + nb - pos0;
}

/* Decodes one block from the stream at *pos (advanced past it). */
static void zfp_decode_block(const uint8_t *bits, int64_t nbits, int64_t *pos, int nd, int dtype,
                             int minexp, double *xhat) {
  const int W = dtype == ORC_F32 ? 32 : 64;
  const int P = W - 2;
  const int E = dtype == ORC_F32 ? 8 : 11;
  const int bias = (1 << (E - 1)) - 1;
  const int size = 1 << (2 * nd);
  for (int i = 0; i < size; i++) xhat[i] = 0.0;
  if (!get_bit(bits, nbits, pos)) return;
  uint64_t e = 0;
  for (int b = 0; b < E; b++) e |= (uint64_t)get_bit(bits, nbits, pos) << b;
  const int emax = (int)e - bias;
  const int prec = orc_precision(emax, minexp, nd, W);
  uint64_t u[64] = {0};
  int n = 0;
  for (int k = W - 1; k >= W - prec; k--) {
    const uint64_t one = 1ull << k;
    for (int i = 0; i < n; i++)
      if (get_bit(bits, nbits, pos)) u[i] |= one;
    int p = n;
    while (p < size) {
      if (!get_bit(bits, nbits, pos)) break; /* no further value gains this plane */
      while (p < size - 1 && !get_bit(bits, nbits, pos)) p++;
      u[p] |= one; /* read as 1, or implied at the last position */
      p++;
      n = p;
    }
  }
  int32_t perm[64];
  orc_reorder_table(nd, perm);
  int64_t d[64];
  for (int r = 0; r < size; r++) d[perm[r]] = orc_from_negabinary(u[r], W);
  orc_inv_xform(d, nd, W);
  for (int i = 0; i < size; i++) xhat[i] = to_dtype(ldexp((double)d[i], emax - P), dtype);
}

int orc_zfp_compress(const void *field, const int64_t *dims, int nd, int dtype, double eb_abs,
                     uint8_t *bits, int64_t cap, double *decoded, orc_step4 *out) {
  if (!field || !dims || !out || nd < 1 || nd > 3) return -1;
  if (dtype != ORC_F32 && dtype != ORC_F64) return -1;
  if (!(eb_abs > 0.0) || !isfinite(eb_abs)) return -1;
  for (int k = 0; k < nd; k++)
    if (dims[k] < 1) return -1;
  memset(out, 0, sizeof(*out));
  const int64_t N = prod(dims, nd);
  double vmin, vmax;
  if (orc_range(field, N, dtype, &vmin, &vmax)) return -1;
  const int minexp = orc_floor_log2(eb_abs);
  const int size = 1 << (2 * nd);
  const int64_t nblocks = orc_zfp_num_blocks(dims, nd);
  double *e2 = (double *)calloc((size_t)nblocks * size, sizeof(double));
  double x[64], xh[64];
  int64_t lin[64];
  int valid[64];
  int64_t pos = 0;
  double maxerr = 0.0;
  for (int64_t jb = 0; jb < nblocks; jb++) {
    gather_block(field, dims, nd, dtype, jb, x, lin, valid);
    const int64_t start = pos;
    pos += zfp_encode_block(x, nd, dtype, minexp, bits, cap, pos);
    if (bits && pos <= cap) { /* decode from the stream itself */
      int64_t rp = start;
      zfp_decode_block(bits, pos, &rp, nd, dtype, minexp, xh);
      if (rp != pos) {
        free(e2);
        return -2; /* the decoder read a different number of bits */
      }
      for (int i = 0; i < size; i++)
        if (valid[i]) {
          const double e = x[i] - xh[i];
          e2[jb * size + i] = e * e;
          if (fabs(e) > maxerr) maxerr = fabs(e);
          if (decoded) decoded[lin[i]] = xh[i];
        }
    }
  }
  out->bits = (uint64_t)pos;
  out->values = (uint64_t)N;
  out->blocks = (uint64_t)nblocks;
  out->bitrate = (double)pos / (double)N;
  out->vr = vmax - vmin;
  out->eb_abs = eb_abs;
  if (bits && pos <= cap) {
    out->sse = orc_tree_sum(e2, nblocks * size);
    out->mse = out->sse / (double)N;
    out->maxerr = maxerr;
    out->psnr = out->mse > 0.0 ? 20.0 * log10(out->vr) - 10.0 * log10(out->mse) : INFINITY;
  }
  free(e2);
  return 0;
}

/* ------------------------------------------------------------------ */
/* Step 4, SZ: compression of the whole field (quantize first, then    */
/* Lorenzo on the integers)                                            */
/* ------------------------------------------------------------------ */

static int64_t prequant(double x, double inv) {
  const double t = fabs(x) * inv + 0.5;
  if (!(t < 1125899906842624.0)) return 0; /* 2^50 */
  const int64_t q = (int64_t)floor(t);
  return x < 0.0 ? -q : q;
}

int orc_sz_compress(const void *field, const int64_t *dims, int nd, int dtype, double eb_abs,
                    uint32_t *hist_out, uint16_t *symbols, double *decoded, orc_step4 *out) {
  if (!field || !dims || !out || nd < 1 || nd > 3) return -1;
  if (dtype != ORC_F32 && dtype != ORC_F64) return -1;
  if (!(eb_abs > 0.0) || !isfinite(eb_abs)) return -1;
  for (int k = 0; k < nd; k++)
    if (dims[k] < 1) return -1;
  memset(out, 0, sizeof(*out));
  const int W = dtype == ORC_F32 ? 32 : 64;
  const int64_t N = prod(dims, nd);
  double vmin, vmax;
  if (orc_range(field, N, dtype, &vmin, &vmax)) return -1;
  const double delta = 2.0 * eb_abs;
  const double inv = 1.0 / delta;
  int64_t *q = (int64_t *)malloc((size_t)N * sizeof(int64_t));
  for (int64_t i = 0; i < N; i++) q[i] = prequant(load(field, dtype, i), inv);
  uint32_t *hist = (uint32_t *)calloc(NBINS, sizeof(uint32_t));
  double *e2 = (double *)malloc((size_t)N * sizeof(double));
  uint64_t esc = 0;
  double maxerr = 0.0;
  int64_t p[3] = {0, 0, 0};
  for (int64_t i = 0; i < N; i++) {
    /* coordinates of point i */
    int64_t rem = i;
    for (int k = nd - 1; k >= 0; k--) {
      p[k] = rem % dims[k];
      rem /= dims[k];
    }
    /* Lorenzo on the integers: the sum over the nonempty subsets S of the
     * axes of (-1)^(|S|+1) q[p - e_S], 0 outside */
    int64_t pred = 0;
    for (int S = 1; S < (1 << nd); S++) {
      int card = 0, inside = 1;
      int64_t lin = 0;
      for (int k = 0; k < nd; k++) {
        int64_t c = p[k];
        if (S & (1 << k)) {
          c -= 1;
          card++;
        }
        if (c < 0) inside = 0;
        lin = lin * dims[k] + c;
      }
      if (!inside) continue;
      pred = (card & 1) ? pred + q[lin] : pred - q[lin];
    }
    const double x = load(field, dtype, i);
    const int64_t code = q[i] - pred;
    const double recon = to_dtype((double)q[i] * delta, dtype);
    int sym = 0;
    double xh = x;
    if (code > -RADIUS && code < RADIUS && fabs(x - recon) <= eb_abs) {
      sym = (int)code + RADIUS;
      xh = recon;
    } else {
      esc++;
    }
    hist[sym]++;
    if (symbols) symbols[i] = (uint16_t)sym;
    const double e = x - xh;
    e2[i] = e * e;
    if (fabs(e) > maxerr) maxerr = fabs(e);
    if (decoded) decoded[i] = xh;
  }
  uint64_t nsym = 0;
  for (int b = 0; b < NBINS; b++) nsym += hist[b] ? 1 : 0;
  const uint64_t code_bits = orc_huffman_bits(hist, NBINS);
  out->code_bits = code_bits;
  out->code_entropy = orc_entropy(hist, NBINS, (uint64_t)N);
  out->symbols = nsym;
  out->unpredictable = esc;
  out->bits = code_bits + (uint64_t)W * esc + 32ull * nsym;
  out->values = (uint64_t)N;
  out->bitrate = (double)out->bits / (double)N;
  out->sse = orc_tree_sum(e2, N);
  out->mse = out->sse / (double)N;
  out->maxerr = maxerr;
  out->vr = vmax - vmin;
  out->eb_abs = eb_abs;
  out->psnr = out->mse > 0.0 ? 20.0 * log10(out->vr) - 10.0 * log10(out->mse) : INFINITY;
  if (hist_out) memcpy(hist_out, hist, NBINS * sizeof(uint32_t));
  free(q);
  free(hist);
  free(e2);
  return 0;
}
