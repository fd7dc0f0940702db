// The estimator's device work, shared by the per-request kernels and the
// batched kernels:
//   * range pass: min/max/non-finite over all N values, one contiguous chunk
//     per workgroup (Algorithm 1's error bound);
//   * ZFP pass: every sampled block through block-floating-point, transform,
//     reorder, negabinary, embedded-coding count and decode (Sections 4.2, 5.2);
//   * SZ pass: Lorenzo prediction, quantization codes and their histogram
//     (Sections 4.1, 5.1);
// each followed by a finalizer run by the last workgroup to finish.
//
// Every workgroup of the ZFP and SZ passes owns an aligned, power-of-two
// chunk of consecutive sampled blocks and reduces it to one partial, so the
// partial sums are exact subtrees of the adjacent-pair tree over all blocks.
#pragma once

#include "device.hpp"

namespace szsel {

constexpr int kHistWin = 4096;    // LDS histogram window around the zero code
constexpr int kOvfMaxRegions = kMaxParts / kOvfSlices + 1;  // SZ workgroups per overflow slice
constexpr int kHistLo = kRadius - kHistWin / 2;

template <int D> struct Order {
  static constexpr OrderTable<D> table{};
};

// LDS of one workgroup: per-block values of the current tile, and the
// binary-counter stack that folds tile sums into the workgroup's subtree.
struct TileLds {
  double sse[kMaxTile];
  double red[kWaves];
  double stk[24];
  int sp;
  uint32_t pushes;
  int last, last2;
};

__device__ inline bool skip_request(const ReqState *st) {
  return (get_u32(&st->flags) & kSkipFlags) != 0;
}

// Partial result of a workgroup or a completion group: s is summed by the
// adjacent-pair tree (or, for the range pass, minimised), m maximised, a and
// b summed as integers.
struct Part {
  double s, m;
  uint64_t a, b;
};

template <bool MINMAX>
__device__ inline Part part_identity() {
  Part v;
  v.s = MINMAX ? INFINITY : 0.0;
  v.m = MINMAX ? -INFINITY : 0.0;
  v.a = 0;
  v.b = 0;
  return v;
}

__device__ inline void part_store(const Parts &p, int i, const Part &v) {
  put_f64(p.sse + i, v.s);
  put_f64(p.err + i, v.m);
  put_u64(p.a + i, v.a);
  put_u64(p.b + i, v.b);
}

__device__ inline Part part_load(const Parts &p, int i) {
  Part v;
  v.s = get_f64(p.sse + i);
  v.m = get_f64(p.err + i);
  v.a = get_u64(p.a + i);
  v.b = get_u64(p.b + i);
  return v;
}

// Left-to-right combination of two adjacent partials.
template <bool MINMAX>
__device__ inline Part part_combine(const Part &x, const Part &y) {
  Part v;
  v.s = MINMAX ? fmin(x.s, y.s) : x.s + y.s;
  v.m = fmax(x.m, y.m);
  v.a = x.a + y.a;
  v.b = x.b + y.b;
  return v;
}

// Combination of the 64 lanes' partials in lane order (the xor butterfly
// associates like the adjacent-pair tree); the result is in every lane.
template <bool MINMAX>
__device__ inline Part part_wave(Part v) {
  v.s = MINMAX ? group_min<kWave>(v.s) : group_tree_sum<kWave>(v.s);
  v.m = group_max<kWave>(v.m);
  v.a = group_isum<kWave>(v.a);
  v.b = group_isum<kWave>(v.b);
  return v;
}

// Completion of a pass of n <= kMaxParts workgroups, each of which has
// stored its partial at its index of `p`.  The workgroups count in groups of
// kGroup; the last workgroup of a group combines the group's partials
// (an aligned subtree) into gp[g] and counts on the top counter; the last
// group combines the group partials.  Agent-scope atomics only, no fences:
// every thread first waits for its own memory operations.  Returns true in
// every thread of the workgroup that holds the pass totals (in wave 0).
template <bool MINMAX>
__device__ inline bool pass_complete(const Parts &p, const Parts &gp, PassSync *sy, int w, int n,
                                     TileLds &L, Part &tot) {
  const int g = w / kGroup;
  const int ng = (n + kGroup - 1) / kGroup;
  const int gs = min(kGroup, n - g * kGroup);
  wait_memory();
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t old = __hip_atomic_fetch_add(&sy->group[g].v, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    L.last = old == (uint32_t)gs - 1;
    if (L.last) put_u32(&sy->group[g].v, 0);
  }
  __syncthreads();
  if (!L.last) return false;
  if (threadIdx.x < kWave) {
    const int lane = threadIdx.x;
    const Part v = part_wave<MINMAX>(lane < gs ? part_load(p, g * kGroup + lane) : part_identity<MINMAX>());
    if (lane == 0) part_store(gp, g, v);
    wait_memory();
    if (lane == 0) {
      const uint32_t old = __hip_atomic_fetch_add(&sy->top.v, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      L.last2 = old == (uint32_t)ng - 1;
      if (L.last2) put_u32(&sy->top.v, 0);
    }
  }
  __syncthreads();
  if (!L.last2) return false;
  if (threadIdx.x < kWave) {
    const int lane = threadIdx.x;
    const Part x = 2 * lane < ng ? part_load(gp, 2 * lane) : part_identity<MINMAX>();
    const Part y = 2 * lane + 1 < ng ? part_load(gp, 2 * lane + 1) : part_identity<MINMAX>();
    tot = part_wave<MINMAX>(part_combine<MINMAX>(x, y));
  }
  return true;
}

// ===========================================================================
// Value range (Algorithm 1's error bound)
// ===========================================================================

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
template <typename T> struct Vec16;
template <> struct Vec16<float> { using V = f32x4; static constexpr int N = 4; };
template <> struct Vec16<double> { using V = f64x2; static constexpr int N = 2; };

// Running min, max and the largest magnitude bit pattern (high word for
// binary64): a value is NaN or infinite iff its magnitude bits reach the
// all-ones exponent, so one integer max per value replaces a compare.
template <typename T>
struct RangeAcc {
  T lo, hi;
  uint32_t amax;
  __device__ RangeAcc() : lo(INFINITY), hi(-INFINITY), amax(0u) {}
  __device__ void add(T v) {
    lo = fmin(lo, v);
    hi = fmax(hi, v);
    if constexpr (sizeof(T) == 4)
      amax = max(amax, __float_as_uint(v) & 0x7fffffffu);
    else
      amax = max(amax, (uint32_t)((uint64_t)__double_as_longlong(v) >> 32) & 0x7fffffffu);
  }
};

// Scans values [beg, end) with the threads of one workgroup: 16-byte
// non-temporal loads, 8 per thread in flight, unaligned head/tail singly.
template <typename T>
__device__ inline void range_scan(const global_t<T> *x, int64_t beg, int64_t end, RangeAcc<T> &acc) {
  using V = typename Vec16<T>::V;
  constexpr int VN = Vec16<T>::N;
  constexpr int U = 8;
  const int64_t lane = threadIdx.x;
  const uintptr_t a = (uintptr_t)(x + beg);
  int64_t head = (int64_t)(((16 - (a & 15)) & 15) / sizeof(T));
  if (head > end - beg) head = end - beg;
  const int64_t nvec = (end - beg - head) / VN;
  const global_t<V> *xv = (const global_t<V> *)(x + beg + head);
  int64_t i = lane;
  for (; i + (U - 1) * kThreads < nvec; i += U * kThreads) {
    V v[U];
#pragma unroll
    for (int k = 0; k < U; k++) v[k] = __builtin_nontemporal_load(xv + i + k * kThreads);
    // all U loads are issued before the first is used (the scheduler would
    // otherwise interleave them with the reductions and keep fewer in flight)
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int k = 0; k < U; k++) {
#pragma unroll
      for (int e = 0; e < VN; e++) acc.add(v[k][e]);
    }
  }
  for (; i < nvec; i += kThreads) {
    const V v = __builtin_nontemporal_load(xv + i);
#pragma unroll
    for (int e = 0; e < VN; e++) acc.add(v[e]);
  }
  const int64_t tail0 = beg + head + nvec * VN;
  if (lane < head) acc.add(x[beg + lane]);
  if (lane < end - tail0) acc.add(x[tail0 + lane]);
}

// Workgroup min/max/amax; every thread returns the workgroup's values.
template <typename T>
__device__ inline void range_reduce_wg(RangeAcc<T> acc, double &lo, double &hi, uint32_t &amax) {
  lo = (double)acc.lo;
  hi = (double)acc.hi;
  amax = acc.amax;
#pragma unroll
  for (int s = 1; s < kWave; s <<= 1) {
    lo = fmin(lo, __shfl_xor(lo, s));
    hi = fmax(hi, __shfl_xor(hi, s));
    amax = max(amax, (uint32_t)__shfl_xor((int)amax, s));
  }
  __shared__ double s_lo[kWaves], s_hi[kWaves];
  __shared__ uint32_t s_am[kWaves];
  const int w = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0) {
    s_lo[w] = lo;
    s_hi[w] = hi;
    s_am[w] = amax;
  }
  __syncthreads();
  lo = fmin(fmin(s_lo[0], s_lo[1]), fmin(s_lo[2], s_lo[3]));
  hi = fmax(fmax(s_hi[0], s_hi[1]), fmax(s_hi[2], s_hi[3]));
  amax = max(max(s_am[0], s_am[1]), max(s_am[2], s_am[3]));
  __syncthreads();
}

// Turns the min/max of the whole field into the request's state and the
// first part of its result (called by one thread).
__device__ inline void range_finalize_one(const ReqDesc &r, double lo, double hi, bool bad) {
  ReqState *st = r.st;
  szsel_result *res = r.res;
  uint64_t *w = (uint64_t *)res;
  for (size_t k = 0; k < sizeof(szsel_result) / 8; k++) put_u64(w + k, 0);
  const bool selecting = r.op == SZSEL_OP_SELECT || r.op == SZSEL_OP_FIXED_EB;
  int32_t choice = -1;
  uint32_t flags = 0;
  double vr = 0.0, eb_abs = 0.0;
  int minexp = 0;
  if (bad) {
    flags = SZSEL_FLAG_NONFINITE;
    lo = hi = 0.0;
  } else {
    vr = hi - lo;
    eb_abs = r.eb_mode == SZSEL_EB_REL ? r.eb * vr : r.eb;
    if (vr == 0.0)
      flags = SZSEL_FLAG_CONSTANT;
    else if (!(eb_abs > 0.0) || !isfinite(eb_abs))
      flags = SZSEL_FLAG_BAD_EB;
    else if (r.nblk == 0)
      flags = SZSEL_FLAG_NO_BLOCKS;
    else
      minexp = floor_log2_bits(eb_abs);
    if (flags && selecting) choice = 0;
  }
  put_f64(&res->vmin, lo);
  put_f64(&res->vmax, hi);
  put_f64(&res->vr, vr);
  put_f64(&res->eb_abs, eb_abs);
  put_u64((uint64_t *)&res->flags, (uint64_t)flags | ((uint64_t)(uint32_t)choice << 32));
  put_u64((uint64_t *)&res->minexp, (uint64_t)(uint32_t)minexp);
  put_u64(&st->code_chunks, 0);
  put_f64(&st->vmin, lo);
  put_f64(&st->vmax, hi);
  put_f64(&st->vr, vr);
  put_f64(&st->eb_abs, eb_abs);
  put_i32(&st->minexp, minexp);
  // SZ's own bin width (Section 5.1.4: delta = 2 eb_abs) unless Algorithm 1
  // derives it from the ZFP estimate later.
  const double delta = 2.0 * eb_abs;
  put_f64(&st->delta, delta);
  put_f64(&st->inv, 1.0 / delta);
  put_f64(&st->eb_sz, 0.5 * delta);
  put_u32(&st->flags, flags);
}

// Whole range pass of workgroup `w` of `nwg`: scan, partial, and (last
// workgroup) the finalizer.
template <typename T>
__device__ inline void range_wg(const ReqDesc &r, int w, TileLds &L) {
  RangeAcc<T> acc;
  const int64_t beg = (int64_t)w * r.rchunk;
  const int64_t end = min(r.n, beg + r.rchunk);
  if (beg < end) range_scan<T>(to_global((const T *)r.field), beg, end, acc);
  double lo, hi;
  uint32_t amax;
  range_reduce_wg<T>(acc, lo, hi, amax);
  if (threadIdx.x == 0) {
    Part v;
    v.s = lo;
    v.m = hi;
    v.a = amax >= (sizeof(T) == 4 ? 0x7f800000u : 0x7ff00000u) ? 1u : 0u;
    v.b = 0;
    part_store(r.rp, w, v);
  }
  Part tot;
  if (!pass_complete<true>(r.rp, r.grp[kPassRange], r.sync + kPassRange, w, r.nrange, L, tot)) return;
  // this request and, in a batch, the requests on the same field that
  // follow it in the table (one scan serves them all)
  if (threadIdx.x == 0)
    for (int d = 0; d <= r.nshare; d++) range_finalize_one((&r)[d], tot.s, tot.m, tot.a != 0);
}

// ===========================================================================
// ZFP side (Sections 4.2 and 5.2): one lane per sampled block
// ===========================================================================

// Forward 4-point lift in place: average/difference the outer pair (x0, x3)
// and the inner pair (x1, x2), then the two averages and the two
// differences, then two shears between the last two outputs.  On multiples
// of 16 it equals (1/16)[[4,4,4,4],[5,1,-1,-5],[-4,4,4,-4],[-2,6,-6,2]].
template <typename I>
__device__ inline void fwd_lift4(I &x0, I &x1, I &x2, I &x3) {
  const I s03 = wadd(x0, x3) >> 1, d03 = wsub(x0, s03);
  const I s12 = wadd(x1, x2) >> 1, d12 = wsub(x1, s12);
  const I y0 = wadd(s03, s12) >> 1;
  const I y2 = wsub(s12, y0);
  const I dm = wadd(d03, d12) >> 1;
  const I dd = wsub(d03, dm);
  const I y3 = wsub(dm >> 1, dd);
  const I y1 = wsub(dm, y3 >> 1);
  x0 = y0;
  x1 = y1;
  x2 = y2;
  x3 = y3;
}

// Inverse lift: undoes each forward step in reverse order.
template <typename I>
__device__ inline void inv_lift4(I &y0, I &y1, I &y2, I &y3) {
  const I dm = wadd(y1, y3 >> 1);
  const I dd = wsub(dm >> 1, y3);
  const I d03 = wadd(dm, dd), d12 = wsub(dm, dd);
  const I s12 = wadd(y0, y2), s03 = wsub(y0, y2);
  y0 = wadd(s03, d03);
  y1 = wadd(s12, d12);
  y2 = wsub(s12, d12);
  y3 = wsub(s03, d03);
}

// Separable block transform (Section 4.2): the 4-point lift along every
// line of the block, fastest axis first; the inverse runs the axes in the
// opposite order.
template <int D, typename I>
__device__ inline void fwd_xform(I (&c)[1 << (2 * D)]) {
  constexpr int BS = 1 << (2 * D);
#pragma unroll
  for (int a = 0; a < D; a++) {
    const int s = 1 << (2 * a);
#pragma unroll
    for (int i = 0; i < BS; i++)
      if (((i >> (2 * a)) & 3) == 0) fwd_lift4(c[i], c[i + s], c[i + 2 * s], c[i + 3 * s]);
  }
}

template <int D, typename I>
__device__ inline void inv_xform(I (&c)[1 << (2 * D)]) {
  constexpr int BS = 1 << (2 * D);
#pragma unroll
  for (int a = D - 1; a >= 0; a--) {
    const int s = 1 << (2 * a);
#pragma unroll
    for (int i = 0; i < BS; i++)
      if (((i >> (2 * a)) & 3) == 0) inv_lift4(c[i], c[i + s], c[i + 2 * s], c[i + 3 * s]);
  }
}

// Values of sampled block j in in-block row-major order.  Rows of 4 values
// are read as 16-byte vectors when the request's rows are 16-byte aligned.
// A j past the last block reads block 0 (its results are discarded).
template <typename T, int D, bool VEC>
__device__ inline void load_block_row(const ReqDesc &r, const global_t<T> *p, int q, T (&x)[1 << (2 * D)]) {
  int64_t off = 0;
  if constexpr (D == 2) off = (int64_t)q * r.dims[1];
  if constexpr (D == 3) off = ((int64_t)(q >> 2) * r.dims[1] + (q & 3)) * r.dims[2];
  const global_t<T> *row = p + off;
  if constexpr (VEC) {
    if constexpr (sizeof(T) == 4) {
      const f32x4 v = *(const global_t<f32x4> *)row;
      x[4 * q] = v[0];
      x[4 * q + 1] = v[1];
      x[4 * q + 2] = v[2];
      x[4 * q + 3] = v[3];
    } else {
      const f64x2 a = *(const global_t<f64x2> *)row, b = *(const global_t<f64x2> *)(row + 2);
      x[4 * q] = a[0];
      x[4 * q + 1] = a[1];
      x[4 * q + 2] = b[0];
      x[4 * q + 3] = b[1];
    }
  } else {
#pragma unroll
    for (int e = 0; e < 4; e++) x[4 * q + e] = row[e];
  }
}

template <typename T, int D, bool VEC>
__device__ inline void load_block(const ReqDesc &r, int64_t j, T (&x)[1 << (2 * D)]) {
  int64_t o[3];
  const global_t<T> *p = to_global((const T *)r.field) + block_base<D>(r, j < r.nblk ? (uint32_t)j : 0u, o);
#pragma unroll
  for (int q = 0; q < (1 << (2 * D)) / 4; q++) load_block_row<T, D, VEC>(r, p, q, x);
}

// Rows [q0, q0 + n) of block j again, at an address made opaque and
// dependent on `after` by an empty asm, so that the read is neither merged
// with the first one nor issued before `after` is known.
template <typename T, int D, bool VEC>
__device__ inline void load_rows_of_block(const ReqDesc &r, int64_t j, T (&x)[1 << (2 * D)], int q0,
                                          int n, uint32_t after) {
  int64_t o[3];
  const global_t<T> *p = to_global((const T *)r.field) + block_base<D>(r, j < r.nblk ? (uint32_t)j : 0u, o);
  asm volatile("" : "+v"(p) : "v"(after));
#pragma unroll
  for (int q = 0; q < (1 << (2 * D)) / 4; q++)
    if (q >= q0 && q < q0 + n) load_block_row<T, D, VEC>(r, p, q, x);
}

// 2^e as a binary32 value, -126 <= e <= 127.
__device__ inline float pow2f(int e) { return __uint_as_float((uint32_t)(e + 127) << 23); }

// Block-floating-point integer trunc(x 2^(P - emax)).  Binary32: two exact
// power-of-two scalings (s1 = 2^min(P - emax, 127), s2 = the rest, >= 1)
// and a truncating conversion.  A product can only be inexact when it falls
// below the normal range, and then the result is below 1 and truncates to 0
// either way.  Binary64: from the bits.
template <typename T>
__device__ inline typename Prec<T>::I bfp_value(T x, int emax, float s1, float s2) {
  if constexpr (sizeof(T) == 4)
    return (int32_t)((x * s1) * s2);
  else
    return bfp_int<T>(x, emax);
}

// Occupancy of the SZ kernels: waves per SIMD (the register budget that
// keeps their state out of scratch memory; one more wave would spill).
template <typename T, int D>
constexpr int kSzWavesPerSimd = D == 3 ? (sizeof(T) == 8 ? 3 : 4) : (sizeof(T) == 8 ? 4 : 5);

// Occupancy of the ZFP kernels: waves per SIMD (one block per lane; 3-D
// blocks of the exact estimate: one block per quad of lanes).
template <typename T, int D, bool EC>
constexpr int kZfpWavesPerSimd = (D == 3 && !EC) ? (sizeof(T) == 8 ? 4 : 5)
                                                 : ((sizeof(T) == 8 && D == 3) ? 1 : 2);

// Results of one block: coder bits (headers included), significant bits,
// data-domain squared error (adjacent-pair tree in in-block order), largest
// absolute error, block exponent (INT32_MIN for an all-zero block).
struct ZfpLane {
  uint32_t bits, nsb;
  double sse, maxerr;
  int emax;
};

// Point sub-sampling of the ZFP side (Sections 5.2.1, 5.2.2): kPts of the
// 4^D coefficients at coding positions round(k (4^D - 1) / (kPts - 1)),
// halves up, and for each the squared norm of its data-domain image under
// the inverse transform (per axis 4, 5, 4, 13/4 for frequencies 0..3: the
// column norms of the inverse of (1/16)[[4,4,4,4],[5,1,-1,-5],[-4,4,4,-4],
// [-2,6,-6,2]]).
template <int D> struct EcTable {
  static constexpr int kSize = 1 << (2 * D);
  static constexpr int kPts = D == 1 ? 3 : (D == 2 ? 9 : 16);
  static constexpr int kSlots = D == 1 ? 4 : 16;  // kPts rounded up to a power of two
  int pos[kPts];      // coding positions sampled
  int coef[kPts];     // in-block coefficient coded there
  double gain[kPts];  // its squared data-domain norm
  constexpr EcTable() : pos(), coef(), gain() {
    const double g1[4] = {4.0, 5.0, 4.0, 3.25};
    for (int k = 0; k < kPts; k++) {
      pos[k] = (2 * k * (kSize - 1) + (kPts - 1)) / (2 * (kPts - 1));
      coef[k] = Order<D>::table.perm[pos[k]];
      double g = 1.0;
      for (int a = 0; a < D; a++) g *= g1[(coef[k] >> (2 * a)) & 3];
      gain[k] = g;
    }
  }
};
template <int D> struct Ec {
  static constexpr EcTable<D> table{};
};

// The sub-sampled estimate of one block from its negabinary coefficients:
// significant bits of each sampled coefficient within the coded planes, the
// other positions filled by linear interpolation (a gap of g positions
// between counts va and vb adds g (va + vb) / 2, so twice the block's total
// is an integer: `bits`), and each sampled coefficient's truncation error
// (the value of its digits below the last coded plane) scaled by
// 2^(emax - P), squared, optionally weighted by its gain, and summed by the
// pair tree over kSlots slots (zeros past kPts).
template <typename T, int D>
__device__ inline ZfpLane zfp_block_ec(const typename Prec<T>::I *c, int prec, int emax, bool empty,
                                       bool weighted) {
  using Q = Prec<T>;
  using U = typename Q::U;
  using I = typename Q::I;
  using E = Ec<D>;
  constexpr int NP = EcTable<D>::kPts, R = EcTable<D>::kSlots;
  constexpr int W = Q::W;
  const int kmin = W - prec;
  const U keep = kmin >= W ? U(0) : (~U(0) << kmin);
  uint32_t v[NP];
  double sq[R];
  double mx = 0.0;
  uint32_t pts = 0;
#pragma unroll
  for (int k = 0; k < NP; k++) {
    const U u = (U)c[E::table.coef[k]];
    const int m = u ? W - clz_u(u) : 0;
    v[k] = m > kmin ? (uint32_t)(m - kmin) : 0u;
    pts += v[k];
    const I e = (I)((((U)(u & ~keep)) ^ Q::NB) - Q::NB);
    const double es = ldexp((double)e, emax - Q::P);
    mx = fmax(mx, fabs(es));
    double s2 = es * es;
    if (weighted) s2 = s2 * E::table.gain[k];
    sq[k] = s2;
  }
#pragma unroll
  for (int k = NP; k < R; k++) sq[k] = 0.0;
#pragma unroll
  for (int w = R; w > 1; w >>= 1) {
#pragma unroll
    for (int k = 0; k < w / 2; k++) sq[k] = sq[2 * k] + sq[2 * k + 1];
  }
  uint32_t twice = 0;
#pragma unroll
  for (int k = 0; k < NP; k++) twice += 2u * v[k];
#pragma unroll
  for (int k = 0; k + 1 < NP; k++) twice += (uint32_t)(E::table.pos[k + 1] - E::table.pos[k] - 1) * (v[k] + v[k + 1]);
  ZfpLane out;
  out.emax = empty ? INT32_MIN : emax;
  out.bits = twice;
  out.nsb = pts;
  out.sse = sq[0];
  out.maxerr = mx;
  return out;
}

template <typename T, int D, bool VEC, bool EC>
__device__ inline ZfpLane zfp_block_lane(const ReqDesc &r, int64_t j, const int32_t *minexp_p) {
  using Q = Prec<T>;
  using U = typename Q::U;
  using I = typename Q::I;
  constexpr int BS = 1 << (2 * D);
  constexpr int W = Q::W;
  // binary32 blocks stay in registers for the error; binary64 blocks are
  // read again (L2 hits) rather than kept beside their 64-bit coefficients
  constexpr bool kKeep = sizeof(T) == 4;
  T x[BS];
  load_block<T, D, VEC>(r, j, x);
  const int minexp = get_i32(minexp_p);  // read while the block is in flight

  // block-floating-point: common exponent of the largest magnitude
  U mmax = 0;
#pragma unroll
  for (int i = 0; i < BS; i++) {
    const U m = Q::bits(x[i]) & ~(U(1) << (W - 1));
    mmax = m > mmax ? m : mmax;
  }
  const bool empty = mmax == 0;
  const int emax = empty ? 0 : frexp_exponent_bits<T>(mmax);
  int prec = emax - minexp + 2 * (D + 1);
  prec = empty ? 0 : (prec < 0 ? 0 : (prec > W ? W : prec));
  I c[BS];
  const int sh = Q::P - emax;  // in [-98, 179] for binary32
  const float s1 = pow2f(sh < 127 ? sh : 127), s2 = pow2f(sh < 127 ? 0 : sh - 127);
#pragma unroll
  for (int i = 0; i < BS; i++) c[i] = bfp_value<T>(x[i], emax, s1, s2);

  // decorrelating transform, then negabinary digits (in place; the
  // sequency order only decides the order in which the count reads them)
  fwd_xform<D>(c);
#pragma unroll
  for (int i = 0; i < BS; i++) c[i] = (I)(((U)c[i] + Q::NB) ^ Q::NB);
  if constexpr (EC) return zfp_block_ec<T, D>(c, prec, emax, empty, r.ec == 2);

  // Group-testing embedded coding of planes W-1 .. kmin, counted without
  // running the coder.  With msb_k the highest set bit of the coefficient
  // at coding position k (-1 for 0) and M_k = max_{k' >= k} msb_k', the
  // coder emits
  //     sum_k max(0, M_k - kmin + 1)            verbatim bits of significant values
  //   + W - max(kmin, msb_last + 1)             group tests that find nothing
  //   + #{k : msb_k = M_k >= kmin}              group tests that find a 1
  //   - [msb_last >= kmin]                      the implied final 1
  // bits, because a plane's test finds exactly the coefficients whose msb is
  // that plane and that no later coefficient exceeds.  Below, m = msb + 1
  // clamped at kmin, so that every term is a plain sum or maximum.
  const int kmin = W - prec;
  int run = kmin;  // max of the clamped m over the later positions
  uint32_t verb = 0, found = 0, sig = 0;
  int m_last = 0;
#pragma unroll
  for (int k = BS - 1; k >= 0; k--) {
    const U u = (U)c[Order<D>::table.perm[k]];
    const int m = u ? W - clz_u(u) : 0;
    if (k == BS - 1) m_last = m;
    const int mc = m > kmin ? m : kmin;
    found += (mc > kmin && mc >= run) ? 1u : 0u;
    run = mc > run ? mc : run;
    verb += (uint32_t)(run - kmin);
    sig += (uint32_t)(mc - kmin);
  }
  ZfpLane out;
  out.emax = empty ? INT32_MIN : emax;
  out.bits = prec == 0 ? 1u
                       : (uint32_t)(1 + Q::E + W - (m_last > kmin ? m_last : kmin) -
                                    (m_last > kmin ? 1 : 0)) + verb + found;
  out.nsb = prec == 0 ? 0u : sig;  // significant bits (Section 5.2.1)

  // decode at the cut-off: drop planes below kmin, invert every step
  const U keep = kmin >= W ? U(0) : (~U(0) << kmin);
#pragma unroll
  for (int i = 0; i < BS; i++) c[i] = (I)((((U)c[i] & keep) ^ Q::NB) - Q::NB);
  inv_xform<D>(c);

  // data-domain error of the decoded block; squared errors summed by the
  // adjacent-pair tree in in-block order (a binary counter over the values).
  // Binary64 blocks are read again in chunks of kChunk rows, each chunk's
  // address depending on the previous chunk's result, so that at most one
  // chunk is live beside the 64-bit coefficients.
  constexpr int kRows = BS / 4;
  constexpr int kChunk = kKeep ? kRows : (kRows > 4 ? 4 : kRows);
  double stk[2 * D];
  double maxerr = 0.0, sse = 0.0;
  uint32_t after = (uint32_t)c[BS - 1];
#pragma unroll
  for (int q0 = 0; q0 < kRows; q0 += kChunk) {
    if constexpr (!kKeep) load_rows_of_block<T, D, VEC>(r, j, x, q0, kChunk, after);
#pragma unroll
    for (int i = 4 * q0; i < 4 * (q0 + kChunk); i++) {
      T xh = (T)ldexp((double)c[i], emax - Q::P);
      if (prec == 0) xh = (T)0;
      // an empty asm makes x[i] opaque here, so that its widening to
      // binary64 is not hoisted up to the load (64 live doubles would spill)
      T xi = x[i];
      asm volatile("" : "+v"(xi));
      const double e = (double)xi - (double)xh;
      maxerr = fmax(maxerr, fabs(e));
      double v = e * e;
#pragma unroll
      for (int l = 0; l < 2 * D; l++) {
        if ((i >> l) & 1) {
          v = stk[l] + v;
        } else {
          stk[l] = v;
          break;
        }
      }
      if (i == BS - 1) sse = v;
      if ((i & 3) == 3) __builtin_amdgcn_sched_barrier(0);
    }
    after = (uint32_t)__double_as_longlong(maxerr);
  }
  out.sse = sse;
  out.maxerr = maxerr;
  return out;
}

// Adjacent-pair tree over the tile's per-block SSE values in LDS (wave 0);
// the result is valid on thread 0.
__device__ inline double tile_sse(const TileLds &L, int tile) {
  double sse = 0.0;
  if (threadIdx.x < kWave) {
    const int lane = threadIdx.x;
    const int c = tile > kWave ? tile / kWave : 1;
    double v = 0.0;
    if (c == 1) {
      if (lane < tile) v = L.sse[lane];
    } else if (c == 2) {
      v = L.sse[2 * lane] + L.sse[2 * lane + 1];
    } else {
      const int k = 4 * lane;
      v = (L.sse[k] + L.sse[k + 1]) + (L.sse[k + 2] + L.sse[k + 3]);
    }
    sse = group_tree_first<kWave>(v);
  }
  return sse;
}

// Workgroup accumulators.  The SSE subtrees of the tiles are folded on
// thread 0 with a binary counter, which associates exactly like the
// adjacent-pair tree over the workgroup's aligned chunk.  Integer counts and
// the maximum error are order-free: each lane accumulates its own and the
// workgroup reduces them once at the end.
struct LaneAcc {
  uint32_t a, b;
  double maxerr;
  uint64_t chunks;  // SZ: the entropy pass's 1024-bin chunks this lane's codes fell in
  __device__ LaneAcc() : a(0u), b(0u), maxerr(0.0), chunks(0) {}
};

__device__ inline void wg_acc_reset(TileLds &L) {
  if (threadIdx.x == 0) {
    L.sp = 0;
    L.pushes = 0;
  }
}

__device__ inline void wg_acc_push(TileLds &L, double sse) {
  if (threadIdx.x == 0) {
    double v = sse;
    for (uint32_t m = L.pushes; m & 1; m >>= 1) v = L.stk[--L.sp] + v;
    L.stk[L.sp++] = v;
    L.pushes++;
  }
}

__device__ inline void wg_acc_store(TileLds &L, const LaneAcc &acc, const Parts &p, int w) {
  uint64_t a = group_isum<kWave>((uint64_t)acc.a);
  uint64_t b = group_isum<kWave>((uint64_t)acc.b);
  double m = group_max<kWave>(acc.maxerr);
  __shared__ uint64_t s_a[kWaves], s_b[kWaves];
  __shared__ double s_m[kWaves];
  const int wv = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0) {
    s_a[wv] = a;
    s_b[wv] = b;
    s_m[wv] = m;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    put_f64(p.sse + w, L.stk[0]);
    put_f64(p.err + w, fmax(fmax(s_m[0], s_m[1]), fmax(s_m[2], s_m[3])));
    put_u64(p.a + w, s_a[0] + s_a[1] + s_a[2] + s_a[3]);
    put_u64(p.b + w, s_b[0] + s_b[1] + s_b[2] + s_b[3]);
  }
}

// ZFP totals, PSNR_zfp and (for Algorithm 1) the SZ bin width delta whose
// uniform-error PSNR equals PSNR_zfp (Eq. 10 inverted: delta = sqrt(12 MSE)).
// With EC the totals are the sub-sampled ones: `bits` is twice the
// interpolated significant-bit total, `nsb` the sampled points' bits, `sse`
// over the sampled points.
template <typename T, int D, bool EC>
__device__ inline void zfp_finalize(const ReqDesc &r, const Part &tot) {
  const double sse = tot.s, maxerr = tot.m;
  const uint64_t bits = tot.a, nsb = tot.b;
  if (threadIdx.x == 0) {
    constexpr int BS = 1 << (2 * D);
    ReqState *st = r.st;
    szsel_result *res = r.res;
    const uint64_t nvals = (uint64_t)(r.nblk * BS);
    const double nv = (double)nvals;
    const double vr = get_f64(&st->vr);
    double mse;
    if constexpr (EC) {
      const uint64_t npts = (uint64_t)r.nblk * EcTable<D>::kPts;
      mse = sse / (double)npts;
      const double br = (double)bits / (double)(2 * nvals);
      put_u64(&res->zfp_bits, 0);
      put_u64(&res->zfp_ec_points, npts);
      put_u64(&res->zfp_ec_nsb2, bits);
      put_f64(&res->zfp_nsb_mean, br);
      put_f64(&res->zfp_bitrate, br);
      const uint64_t fc = get_u64((uint64_t *)&res->flags);
      put_u64((uint64_t *)&res->flags, fc | SZSEL_FLAG_EC_SAMPLED);
    } else {
      mse = sse / nv;
      put_u64(&res->zfp_bits, bits);
      put_f64(&res->zfp_nsb_mean, (double)nsb / nv);
      put_f64(&res->zfp_bitrate, (double)bits / nv);
    }
    put_f64(&res->zfp_sse, sse);
    put_f64(&res->zfp_mse, mse);
    put_u64(&res->zfp_values, nvals);
    put_u64(&res->zfp_blocks, (uint64_t)r.nblk);
    put_u64(&res->zfp_nsb_total, nsb);
    put_f64(&res->zfp_maxerr, maxerr);
    put_f64(&res->zfp_psnr, mse > 0.0 ? 20.0 * log10(vr) - 10.0 * log10(mse) : INFINITY);
    if (r.op == SZSEL_OP_SELECT) {
      double delta;
      if (mse > 0.0) {
        delta = sqrt(12.0 * mse);
      } else {
        delta = 2.0 * get_f64(&st->eb_abs);
        const uint64_t fc = get_u64((uint64_t *)&res->flags);
        put_u64((uint64_t *)&res->flags, fc | SZSEL_FLAG_ZERO_MSE);
      }
      put_f64(&st->delta, delta);
      put_f64(&st->inv, 1.0 / delta);
      put_f64(&st->eb_sz, 0.5 * delta);
    }
  }
}

// ===========================================================================
// ZFP side for 3-D blocks, four lanes per block
// ===========================================================================
// A 3-D block's 64 values and coefficients spread over a quad of lanes, 16
// per lane, so that a binary64 block (64 64-bit coefficients) fits in a
// quarter of the registers it needs in one lane.  Two layouts:
//   row layout:    lane q of the quad holds the rows (z, y = q), z = 0..3;
//   column layout: lane q holds the values (z, y, x = q), z, y = 0..3.
// The x lifts run in row layout and the y and z lifts in column layout; a
// 4 x 4 transpose within the quad (two DPP exchange stages) switches between
// them.  The coder count needs the coefficients in coding order: every lane
// writes the bit lengths of its 16 coefficients to LDS at their coding
// positions, and lane q scans positions 16q .. 16q + 15, starting from the
// largest bit length after them (a suffix maximum over the quad).

// Coding positions of lane q's coefficients in column layout, coefficient
// t = 4 z + y at index 16 z + 4 y + q, one byte each, four to a word.
struct QuadPositions {
  uint32_t w[4][4];  // [q][t / 4]
  constexpr QuadPositions() : w() {
    for (int q = 0; q < 4; q++)
      for (int t = 0; t < 16; t++)
        w[q][t >> 2] |= (uint32_t)Order<3>::table.inv[16 * (t >> 2) + 4 * (t & 3) + q] << (8 * (t & 3));
  }
};
struct QuadPos {
  static constexpr QuadPositions table{};
};

constexpr int kQuadBlocks = kWave / 4;  // blocks per wave and round
constexpr int kQuadLds = 80;            // LDS bytes per block (64 used; the padding spreads banks)

// Value of lane q ^ 1 (XOR1) or q ^ 2 of the quad.
template <int CTRL, typename V>
__device__ inline V quad_get(V v) {
  if constexpr (std::is_same<V, double>::value) {
    return dpp<CTRL>(v);
  } else {
    using UV = typename std::conditional<sizeof(V) == 8, uint64_t, uint32_t>::type;
    return (V)dpp<CTRL>((UV)v);
  }
}

// 4 x 4 transpose within the quad: lane q's a[k] becomes lane k's a[q].
// Stage one exchanges with lane q ^ 2 the elements whose bit 1 differs
// from q's, stage two with lane q ^ 1 those whose bit 0 differs.
template <typename V>
__device__ inline void quad_transpose(V (&a)[4], int q) {
  const bool h = (q & 2) != 0, l = (q & 1) != 0;
#pragma unroll
  for (int k = 0; k < 2; k++) {
    const V got = quad_get<kDppQuadXor2>(h ? a[k] : a[k + 2]);
    a[k] = h ? got : a[k];
    a[k + 2] = h ? a[k + 2] : got;
  }
#pragma unroll
  for (int k = 0; k < 4; k += 2) {
    const V got = quad_get<kDppQuadXor1>(l ? a[k] : a[k + 1]);
    a[k] = l ? got : a[k];
    a[k + 1] = l ? a[k + 1] : got;
  }
}

// Sum over the quad, in every lane of it: (v0 + v1) + (v2 + v3), the
// adjacent-pair association (the two orders of a sum are the same).
template <typename V>
__device__ inline V quad_sum(V v) {
  v = v + quad_get<kDppQuadXor1>(v);
  return v + quad_get<kDppQuadXor2>(v);
}

template <typename V>
__device__ inline V quad_max(V v) {
  V o = quad_get<kDppQuadXor1>(v);
  v = o > v ? o : v;
  o = quad_get<kDppQuadXor2>(v);
  return o > v ? o : v;
}

// Row (z, y) of block j, 4 values from `p` (the row's first element).
template <typename T, bool VEC>
__device__ inline void load_row4(const global_t<T> *p, T (&x)[4]) {
  if constexpr (VEC) {
    if constexpr (sizeof(T) == 4) {
      const f32x4 v = *(const global_t<f32x4> *)p;
      x[0] = v[0];
      x[1] = v[1];
      x[2] = v[2];
      x[3] = v[3];
    } else {
      const f64x2 a = *(const global_t<f64x2> *)p, b = *(const global_t<f64x2> *)(p + 2);
      x[0] = a[0];
      x[1] = a[1];
      x[2] = b[0];
      x[3] = b[1];
    }
  } else {
#pragma unroll
    for (int e = 0; e < 4; e++) x[e] = p[e];
  }
}

// The exact ZFP estimate of 3-D block j by quad lane q (same results as
// zfp_block_lane<T, 3, VEC, false>, in every lane of the quad).  `pos` are
// the lane's coding positions (QuadPositions), `sb` the block's LDS bytes.
template <typename T, bool VEC>
__device__ inline ZfpLane zfp_block_quad(const ReqDesc &r, int64_t j, int q, const int32_t *minexp_p,
                                         const uint32_t (&pos)[4], uint8_t *sb) {
  using Q = Prec<T>;
  using U = typename Q::U;
  using I = typename Q::I;
  constexpr int W = Q::W;
  // row layout: x[z][.] = row (z, y = q)
  T x[4][4];
  {
    int64_t o[3];
    const global_t<T> *p = to_global((const T *)r.field) + block_base<3>(r, j < r.nblk ? (uint32_t)j : 0u, o);
    const int64_t sz = r.dims[1] * r.dims[2], sy = r.dims[2];
#pragma unroll
    for (int z = 0; z < 4; z++) load_row4<T, VEC>(p + z * sz + q * sy, x[z]);
  }
  const int minexp = get_i32(minexp_p);  // read while the rows are in flight

  // block-floating-point: common exponent of the largest magnitude
  U mmax = 0;
#pragma unroll
  for (int z = 0; z < 4; z++)
#pragma unroll
    for (int e = 0; e < 4; e++) {
      const U m = Q::bits(x[z][e]) & ~(U(1) << (W - 1));
      mmax = m > mmax ? m : mmax;
    }
  mmax = quad_max(mmax);
  const bool empty = mmax == 0;
  const int emax = empty ? 0 : frexp_exponent_bits<T>(mmax);
  int prec = emax - minexp + 8;  // 2 (d + 1), d = 3
  prec = empty ? 0 : (prec < 0 ? 0 : (prec > W ? W : prec));
  const int sh = Q::P - emax;
  const float s1 = pow2f(sh < 127 ? sh : 127), s2 = pow2f(sh < 127 ? 0 : sh - 127);
  I c[4][4];
#pragma unroll
  for (int z = 0; z < 4; z++)
#pragma unroll
    for (int e = 0; e < 4; e++) c[z][e] = bfp_value<T>(x[z][e], emax, s1, s2);

  // forward transform, fastest axis first: x in row layout, then y and z
  // in column layout (c[z][y] = coefficient (z, y, x = q)); negabinary
#pragma unroll
  for (int z = 0; z < 4; z++) fwd_lift4(c[z][0], c[z][1], c[z][2], c[z][3]);
#pragma unroll
  for (int z = 0; z < 4; z++) quad_transpose(c[z], q);
#pragma unroll
  for (int z = 0; z < 4; z++) fwd_lift4(c[z][0], c[z][1], c[z][2], c[z][3]);
#pragma unroll
  for (int y = 0; y < 4; y++) fwd_lift4(c[0][y], c[1][y], c[2][y], c[3][y]);
#pragma unroll
  for (int z = 0; z < 4; z++)
#pragma unroll
    for (int y = 0; y < 4; y++) c[z][y] = (I)(((U)c[z][y] + Q::NB) ^ Q::NB);

  // bit lengths in coding order through LDS; lane q takes positions
  // 16q .. 16q + 15 (see zfp_block_lane for the count itself)
#pragma unroll
  for (int t = 0; t < 16; t++) {
    const U u = (U)c[t >> 2][t & 3];
    const int m = u ? W - clz_u(u) : 0;
    sb[(pos[t >> 2] >> (8 * (t & 3))) & 0xffu] = (uint8_t)m;
  }
  __syncthreads();
  const uint4 mv = *(const uint4 *)(sb + 16 * q);
  __syncthreads();
  const uint32_t mw[4] = {mv.x, mv.y, mv.z, mv.w};
  int lmax = 0;
#pragma unroll
  for (int t = 0; t < 16; t++) {
    const int m = (int)((mw[t >> 2] >> (8 * (t & 3))) & 0xffu);
    lmax = m > lmax ? m : lmax;
  }
  // largest bit length at the positions after the lane's 16.  Every lane
  // evaluates each cross-lane read (a lane left out of one would hand its
  // readers 0), and only then does lane 3 take 0.
  int after = max(lmax, (int)dpp<kDppQuad1233>((uint32_t)lmax));
  after = max(after, (int)dpp<kDppQuad2323>((uint32_t)after));
  const int later = (int)dpp<kDppQuad1233>((uint32_t)after);
  after = q == 3 ? 0 : later;
  const int kmin = W - prec;
  int run = after > kmin ? after : kmin;
  uint32_t verb = 0, found = 0, sig = 0;
#pragma unroll
  for (int t = 15; t >= 0; t--) {
    const int m = (int)((mw[t >> 2] >> (8 * (t & 3))) & 0xffu);
    const int mc = m > kmin ? m : kmin;
    found += (mc > kmin && mc >= run) ? 1u : 0u;
    run = mc > run ? mc : run;
    verb += (uint32_t)(run - kmin);
    sig += (uint32_t)(mc - kmin);
  }
  verb = quad_sum(verb);
  found = quad_sum(found);
  sig = quad_sum(sig);
  const int m_last = (int)dpp<kDppQuadBcast3>((mw[3] >> 24) & 0xffu);  // position 63
  ZfpLane out;
  out.emax = empty ? INT32_MIN : emax;
  out.bits = prec == 0 ? 1u
                       : (uint32_t)(1 + Q::E + W - (m_last > kmin ? m_last : kmin) -
                                    (m_last > kmin ? 1 : 0)) + verb + found;
  out.nsb = prec == 0 ? 0u : sig;

  // decode at the cut-off: drop planes below kmin, invert every step
  const U keep = kmin >= W ? U(0) : (~U(0) << kmin);
#pragma unroll
  for (int z = 0; z < 4; z++)
#pragma unroll
    for (int y = 0; y < 4; y++) c[z][y] = (I)((((U)c[z][y] & keep) ^ Q::NB) - Q::NB);
#pragma unroll
  for (int y = 0; y < 4; y++) inv_lift4(c[0][y], c[1][y], c[2][y], c[3][y]);
#pragma unroll
  for (int z = 0; z < 4; z++) inv_lift4(c[z][0], c[z][1], c[z][2], c[z][3]);
#pragma unroll
  for (int z = 0; z < 4; z++) quad_transpose(c[z], q);
#pragma unroll
  for (int z = 0; z < 4; z++) inv_lift4(c[z][0], c[z][1], c[z][2], c[z][3]);

  // data-domain error: the adjacent-pair tree in in-block row-major order
  // is, per z, the rows' pair trees (in the lane), then rows y = 0..3
  // across the quad, then the four z planes
  double plane[4];
  double maxerr = 0.0;
#pragma unroll
  for (int z = 0; z < 4; z++) {
    double e2[4];
#pragma unroll
    for (int e = 0; e < 4; e++) {
      T xh = (T)ldexp((double)c[z][e], emax - Q::P);
      if (prec == 0) xh = (T)0;
      const double d = (double)x[z][e] - (double)xh;
      maxerr = fmax(maxerr, fabs(d));
      e2[e] = d * d;
    }
    plane[z] = quad_sum((e2[0] + e2[1]) + (e2[2] + e2[3]));
  }
  out.sse = (plane[0] + plane[1]) + (plane[2] + plane[3]);
  out.maxerr = quad_max(maxerr);
  return out;
}

// Whole ZFP pass of workgroup w (one wave) for 3-D blocks: rounds of 16
// consecutive sampled blocks of its aligned chunk, one block per quad; the
// round sums (wave butterfly over the quads' first lanes, zero elsewhere)
// are folded with the binary counter as in zfp_wg.
template <typename T, bool VEC>
__device__ inline bool zfp_wg_quad(const ReqDesc &r, int w, TileLds &L) {
  __shared__ __align__(16) uint8_t s_msb[kQuadBlocks * kQuadLds];
  const int lane = threadIdx.x, q = lane & 3, b = lane >> 2;
  uint32_t pos[4];
#pragma unroll
  for (int k = 0; k < 4; k++)
    pos[k] = q == 0 ? QuadPos::table.w[0][k]
                    : (q == 1 ? QuadPos::table.w[1][k] : (q == 2 ? QuadPos::table.w[2][k] : QuadPos::table.w[3][k]));
  uint8_t *sb = s_msb + b * kQuadLds;
  const int rounds = r.zblk / kQuadBlocks;
  uint32_t bits = 0, nsb = 0;
  double maxerr = 0.0;
  wg_acc_reset(L);
  for (int k = 0; k < rounds; k++) {
    const int64_t base = (int64_t)w * r.zblk + (int64_t)k * kQuadBlocks;
    if (base >= r.nblk) {
      wg_acc_push(L, 0.0);
      continue;
    }
    const int64_t j = base + b;
    const bool active = j < r.nblk;
    const ZfpLane z = zfp_block_quad<T, VEC>(r, j, q, &r.st->minexp, pos, sb);
    double s = 0.0;
    if (active && q == 0) {
      bits += z.bits;
      nsb += z.nsb;
      maxerr = fmax(maxerr, z.maxerr);
      s = z.sse;
      if (r.dbg_zbits) r.dbg_zbits[j] = z.bits;
      if (r.dbg_zsse) r.dbg_zsse[j] = z.sse;
      if (r.dbg_zemax) r.dbg_zemax[j] = z.emax;
    }
    wg_acc_push(L, group_tree_first<kWave>(s));
  }
  Part v;
  v.s = 0.0;
  v.m = maxerr;
  v.a = bits;
  v.b = nsb;
  v = part_wave<false>(v);
  if (lane == 0) {
    v.s = L.stk[0];
    part_store(r.zp, w, v);
  }
  Part tot;
  if (!pass_complete<false>(r.zp, r.grp[kPassZfp], r.sync + kPassZfp, w, r.nzfp, L, tot)) return false;
  zfp_finalize<T, 3, false>(r, tot);
  return true;
}

// Whole ZFP pass of workgroup w (one wave): rounds of 64 consecutive
// sampled blocks of its aligned chunk, one block per lane; the round sums
// (wave butterfly) are folded with the binary counter.  Returns true in the
// workgroup that ran the finalizer.
template <typename T, int D, bool VEC, bool EC>
__device__ inline bool zfp_wg(const ReqDesc &r, int w, TileLds &L) {
  if constexpr (D == 3 && !EC) return zfp_wg_quad<T, VEC>(r, w, L);
  const int lane = threadIdx.x;
  const int rounds = r.zblk / kWave;
  uint32_t bits = 0, nsb = 0;
  double maxerr = 0.0;
  wg_acc_reset(L);
  for (int k = 0; k < rounds; k++) {
    const int64_t base = (int64_t)w * r.zblk + (int64_t)k * kWave;
    if (base >= r.nblk) {
      wg_acc_push(L, 0.0);
      continue;
    }
    const int64_t j = base + lane;
    const bool active = j < r.nblk;
    const ZfpLane z = zfp_block_lane<T, D, VEC, EC>(r, j, &r.st->minexp);
    double s = 0.0;
    if (active) {
      bits += z.bits;
      nsb += z.nsb;
      maxerr = fmax(maxerr, z.maxerr);
      s = z.sse;
      if (r.dbg_zbits) r.dbg_zbits[j] = z.bits;
      if (r.dbg_zsse) r.dbg_zsse[j] = z.sse;
      if (r.dbg_zemax) r.dbg_zemax[j] = z.emax;
    }
    wg_acc_push(L, group_tree_first<kWave>(s));
  }
  Part v;
  v.s = 0.0;
  v.m = maxerr;
  v.a = bits;
  v.b = nsb;
  v = part_wave<false>(v);
  if (lane == 0) {
    v.s = L.stk[0];
    part_store(r.zp, w, v);
  }
  Part tot;
  if (!pass_complete<false>(r.zp, r.grp[kPassZfp], r.sync + kPassZfp, w, r.nzfp, L, tot)) return false;
  zfp_finalize<T, D, EC>(r, tot);
  return true;
}

// ===========================================================================
// SZ side (Sections 4.1, 5.1): Lorenzo prediction from the original values,
// linear-scaling quantization, code histogram
// ===========================================================================

// SZ side, one lane per R consecutive rows of 4 points along the fastest
// axis (R = 2 in 2-D and 3-D, 1 in 1-D): 4^(D-1) / R lanes per sampled
// block.  A lane reads the rows its points' Lorenzo stencils touch, each
// with the value before it (x - 1): in 3-D the rows y0 - 1 .. y0 + R - 1 of
// its slice z and of slice z - 1, in 2-D the rows y0 - 1 .. y0 + R - 1, in
// 1-D its row; a row serves every point of the lane whose stencil touches
// it, so two rows per lane need 6 rows (3-D) instead of 8.  Values outside
// the field are 0 (the lower-order predictor at borders).
template <int D>
struct SzLayout {
  static constexpr int R = D == 1 ? 1 : 2;         // rows per lane
  static constexpr int ROWS = 1 << (2 * (D - 1));  // rows per block
  static constexpr int LPB = ROWS / R;             // lanes per block
  static constexpr int BPW = kWave / LPB;          // blocks per wave
  static constexpr int NY = D == 1 ? 1 : R + 1;    // rows along y: y0 - 1 .. y0 + R - 1
  static constexpr int NZ = D == 3 ? 2 : 1;        // along z: z - 1, z
  static constexpr int NP = 4 * R;                 // points per lane
};

template <typename T, int D>
struct Rows {
  using Lay = SzLayout<D>;
  static constexpr int NR = Lay::NZ * Lay::NY;
  static constexpr uint32_t kAll = (2u << NR) - 1u;  // every row and x - 1 inside the field
  T v[Lay::NZ][Lay::NY][5];  // [slice][row][x + 1]
  uint32_t keep;             // bit zi * NY + yi: row inside the field; bit NR: x - 1 is
  // own row dy of the lane (0 .. R - 1)
  __device__ static constexpr int own(int dy) { return D == 1 ? 0 : dy + 1; }
};

// Reads one row of 4 values and the value before it.  Nothing is done with
// the values here, so that the loads stay in flight until the round that
// uses them (rows_mask zeroes what lies outside the field).
template <typename T, bool VEC>
__device__ inline void load_row(const global_t<T> *p, T (&out)[5], bool left) {
  if constexpr (VEC) {
    if constexpr (sizeof(T) == 4) {
      const f32x4 v = *(const global_t<f32x4> *)p;
      out[1] = v[0];
      out[2] = v[1];
      out[3] = v[2];
      out[4] = v[3];
    } else {
      const f64x2 a = *(const global_t<f64x2> *)p, b = *(const global_t<f64x2> *)(p + 2);
      out[1] = a[0];
      out[2] = a[1];
      out[3] = b[0];
      out[4] = b[1];
    }
  } else {
#pragma unroll
    for (int e = 0; e < 4; e++) out[1 + e] = p[e];
  }
  out[0] = p[left ? -1 : 0];
}

// Rows of lane row group q of sampled block j (all zero past the last
// block): q = z * (4 / R) + h in 3-D, q = h in 2-D; the lane's first own row
// is y0 = R h.
template <typename T, int D, bool VEC>
__device__ inline Rows<T, D> load_rows(const ReqDesc &r, int64_t j, int q) {
  using Lay = SzLayout<D>;
  Rows<T, D> s;
  const bool in = j < r.nblk;
  int64_t o[3] = {0, 0, 0};
  // a block past the end reads block 0 (always present) and is masked out
  const int64_t base = block_base<D>(r, in ? (uint32_t)j : 0u, o);
  const global_t<T> *x = to_global((const T *)r.field);
  int64_t own = 0, sy = 0, sz = 0;
  bool yprev = false, zprev = false;  // row y0 - 1 / slice z - 1 inside the field
  if constexpr (D == 2) {
    const int y0 = Lay::R * q;
    sy = r.dims[1];
    own = (int64_t)y0 * sy;
    yprev = o[0] + y0 > 0;
  } else if constexpr (D == 3) {
    const int z = q / (4 / Lay::R), y0 = Lay::R * (q % (4 / Lay::R));
    sz = r.dims[1] * r.dims[2];
    sy = r.dims[2];
    own = (int64_t)z * sz + (int64_t)y0 * sy;
    zprev = o[0] + z > 0;
    yprev = o[1] + y0 > 0;
  }
  const bool left = o[D - 1] > 0;
  const global_t<T> *row = x + base + own;
  uint32_t keep = (in && left) ? (1u << Rows<T, D>::NR) : 0u;
#pragma unroll
  for (int zi = 0; zi < Lay::NZ; zi++) {
#pragma unroll
    for (int yi = 0; yi < Lay::NY; yi++) {
      const int dz = zi - (Lay::NZ - 1), dy = D == 1 ? 0 : yi - 1;
      const bool own_row = dz == 0 && dy >= 0;  // inside block j (block 0 when !in)
      const bool ok = in && (own_row || ((dz == 0 || zprev) && (dy >= 0 || yprev)));
      keep |= ok ? (1u << (zi * Lay::NY + yi)) : 0u;
      // a missing neighbour row is read from the lane's own row and zeroed
      // later; own rows are read from their address unconditionally (were
      // they selected by `in`, the compiler could copy one row's values into
      // another behind a branch, which waits for the loads at once)
      load_row<T, VEC>(own_row || ok ? row + dz * sz + dy * sy : row, s.v[zi][yi], left);
    }
  }
  s.keep = keep;
  return s;
}

// Zeroes the stencil values that lie outside the field (or past the last
// block): the lower-order predictor at borders.
template <typename T, int D>
__device__ inline void rows_mask(Rows<T, D> &s) {
  using Lay = SzLayout<D>;
  const bool left = (s.keep >> Rows<T, D>::NR) & 1u;
#pragma unroll
  for (int zi = 0; zi < Lay::NZ; zi++)
#pragma unroll
    for (int yi = 0; yi < Lay::NY; yi++) {
      const bool ok = (s.keep >> (zi * Lay::NY + yi)) & 1u;
#pragma unroll
      for (int e = 0; e < 5; e++) s.v[zi][yi][e] = (ok && (e > 0 || left)) ? s.v[zi][yi][e] : (T)0;
    }
}

// Lorenzo prediction of point xi of the lane's own row dy (Section 4.1,
// from the original neighbours as Section 4.3 prescribes): the sum over
// non-empty axis subsets S of (-1)^(|S|+1) X[p - e_S], in FP64, terms in the
// order single axes (slowest first), pairs in lexicographic order, the
// triple.
template <typename T, int D>
__device__ inline double lorenzo_row(const Rows<T, D> &s, int dy, int xi) {
  const int c = xi + 1;
  if constexpr (D == 1) {
    return (double)s.v[0][0][c - 1];
  } else if constexpr (D == 2) {
    // {y}, {x}, {y,x}
    return ((double)s.v[0][dy][c] + (double)s.v[0][dy + 1][c - 1]) - (double)s.v[0][dy][c - 1];
  } else {
    // {z}, {y}, {x}, {z,y}, {z,x}, {y,x}, {z,y,x}; slice 0 is z - 1, row dy
    // is y - 1 of own row dy
    return (((((double)s.v[0][dy + 1][c] + (double)s.v[1][dy][c]) + (double)s.v[1][dy + 1][c - 1]) -
             (double)s.v[0][dy][c]) - (double)s.v[0][dy + 1][c - 1]) - (double)s.v[1][dy][c - 1] +
           (double)s.v[0][dy][c - 1];
  }
}

// Quantization code of one point (0 = unpredictable) and its error (0 for an
// unpredictable point).  Round half away from zero; the point is
// unpredictable when |q| >= 32768 or when the reconstruction, rounded to the
// field precision, misses the bound delta/2.
template <typename T>
__device__ inline int quantize(T xv, double pred, double delta, double inv, double ebsz, double &e,
                               bool active = true) {
  // branch-free: every lane computes the reconstruction and the tests only
  // select the results.  |q| = floor(t) carries the sign of d as a double
  // (exact: |q| <= 32768), so the reconstruction needs no integer round
  // trip; a t out of range (or NaN) computes with |q| = 32768 and is
  // rejected by `in`.  A q of -0 where the code is 0 changes at most the
  // sign of a zero error.
  const double xd = (double)xv;
  const double d = xd - pred;
  const double t = fabs(d) * inv + 0.5;
  const bool in = t < (double)kRadius;
  const double q = copysign(floor(fmin(t, (double)kRadius)), d);
  const T recon = (T)(pred + q * delta);
  const double err = xd - (double)recon;
  const bool ok = active && in && fabs(err) <= ebsz;  // (an inactive lane counts nothing)
  e = ok ? err : 0.0;
  return ok ? (int)q + kRadius : 0;
}

// Histogram update for the N codes of a lane (code 0 = unpredictable, not
// counted here).  Codes in the LDS window: when all N are equal (the common
// case on smooth data) one atomic adds N, else one atomic per code; the LDS
// serialises lanes that hit one bin, off the vector pipeline.  Codes outside
// the window are appended to the workgroup's overflow region, numbered by
// one LDS atomic per wave (the wave's first such lane reserves room for all),
// and their 1024-bin chunks are added to `chunks` (those of window codes are
// taken from the window at the hand-over).
template <int N>
__device__ inline void hist_add(const int (&code)[N], bool active, uint32_t *s_hist, global_t<uint16_t> *region,
                                uint32_t *s_n, uint64_t &chunks) {
  bool out[N];
  bool anyout = false;
  bool same = true;
#pragma unroll
  for (int k = 0; k < N; k++) {
    const int wi = code[k] - kHistLo;
    out[k] = active && code[k] != 0 && (wi < 0 || wi >= kHistWin);
    anyout = anyout || out[k];
    same = same && code[k] == code[0];
  }
  if (active) {
    const int w0 = code[0] - kHistLo;
    if (same && code[0] != 0 && !out[0]) {
      atomicAdd(&s_hist[w0], (uint32_t)N);
    } else if (!same) {
#pragma unroll
      for (int k = 0; k < N; k++)
        if (code[k] != 0 && !out[k]) atomicAdd(&s_hist[code[k] - kHistLo], 1u);
    }
  }
  if (__ballot(anyout)) {
    const int lane = threadIdx.x & (kWave - 1);
    uint32_t mine = 0;
#pragma unroll
    for (int k = 0; k < N; k++) mine += (uint32_t)out[k];
    // exclusive prefix of the lanes' counts and the wave's total, one bit
    // of the counts (at most N) at a time: a ballot of the bit, the lanes
    // below that have it (mbcnt) and its population count
    uint32_t below = 0, total = 0;
#pragma unroll
    for (int b = 0; (1 << b) <= N; b++) {
      const uint64_t m = __ballot((mine >> b) & 1u);
      below += __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u)) << b;
      total += (uint32_t)__popcll(m) << b;
    }
    uint32_t base = 0;
    if (lane == 0) base = atomicAdd(s_n, total);
    base = (uint32_t)__builtin_amdgcn_readfirstlane((int)base) + below;
#pragma unroll
    for (int k = 0; k < N; k++)
      if (out[k]) {
        region[base++] = (uint16_t)code[k];
        chunks |= 1ull << (code[k] >> 10);
      }
  }
}

// One round of the SZ side on the rows `sc` of block j (tile slot jl).
template <typename T, int D>
__device__ inline void sz_round(const ReqDesc &r, Rows<T, D> &sc, int64_t j, int jl, int q, double delta,
                                double inv, double ebsz, TileLds &L, uint32_t *s_hist, global_t<uint16_t> *region,
                                uint32_t *s_n, LaneAcc &acc) {
  using Lay = SzLayout<D>;
  constexpr int BS = 1 << (2 * D), LPB = Lay::LPB, R = Lay::R, NP = Lay::NP;
  const bool active = j < r.nblk;
  // only rows at the field's low faces (or past the last block) need
  // zeroing; most waves have none
  if (__ballot(sc.keep != Rows<T, D>::kAll)) rows_mask<T, D>(sc);
  // the points' predictions and codes first (independent chains the
  // compiler can interleave), then their histogram updates; a lane past the
  // last block gets code 0 and no error
  double e2[NP];
  int code[NP];
#pragma unroll
  for (int dy = 0; dy < R; dy++) {
#pragma unroll
    for (int xi = 0; xi < 4; xi++) {
      const int k = 4 * dy + xi;
      double e;
      code[k] = quantize<T>(sc.v[Lay::NZ - 1][Rows<T, D>::own(dy)][xi + 1], lorenzo_row<T, D>(sc, dy, xi),
                            delta, inv, ebsz, e, active);
      acc.maxerr = fmax(acc.maxerr, fabs(e));
      e2[k] = e * e;
    }
  }
  // (unpredictable points are counted at the hand-over, as the points no
  // bin received)
  hist_add<NP>(code, active, s_hist, region, s_n, acc.chunks);
  if (r.dbg_codes && active) {
#pragma unroll
    for (int k = 0; k < NP; k++) r.dbg_codes[j * BS + q * NP + k] = (uint16_t)code[k];
  }
  // pair tree over the lane's points, then across the block's lanes
#pragma unroll
  for (int w = NP; w > 1; w >>= 1) {
#pragma unroll
    for (int k = 0; k < w / 2; k++) e2[k] = e2[2 * k] + e2[2 * k + 1];
  }
  double bsse = e2[0];
  if constexpr (LPB > 1) bsse = group_tree_first<LPB>(bsse);
  if (q == 0) {
    L.sse[jl] = bsse;
    if (active && r.dbg_ssse) r.dbg_ssse[j] = bsse;
  }
}

// One tile of the SZ side (tile blocks starting at `base`): each round the
// 4 waves take 4 BPW consecutive blocks; the next round's rows are loaded
// while the current round is processed.  Per-block squared errors: the lane's 4 R points (consecutive
// in the block's row-major order) by the pair tree, then the block's lanes
// in order by the butterfly, i.e. the adjacent-pair tree in in-block
// row-major order.
template <typename T, int D, bool VEC>
__device__ inline void sz_tile(const ReqDesc &r, int64_t base, int tile, double delta, double inv,
                               double ebsz, TileLds &L, uint32_t *s_hist, global_t<uint16_t> *region,
                               uint32_t *s_n, LaneAcc &acc) {
  using Lay = SzLayout<D>;
  constexpr int LPB = Lay::LPB, BPW = Lay::BPW;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int q = lane & (LPB - 1), bw = lane / LPB;
  const int rounds = tile / (kWaves * BPW);  // a power of two
  const int j0 = wave * BPW + bw;            // tile slot of round 0
  Rows<T, D> sn = load_rows<T, D, VEC>(r, base + j0, q);
  for (int rd = 0; rd < rounds; rd++) {
    const int jl = rd * kWaves * BPW + j0;
    Rows<T, D> sc = sn;
    if (rd + 1 < rounds) sn = load_rows<T, D, VEC>(r, base + jl + kWaves * BPW, q);
    sz_round<T, D>(r, sc, base + jl, jl, q, delta, inv, ebsz, L, s_hist, region, s_n, acc);
  }
  __syncthreads();
  wg_acc_push(L, tile_sse(L, tile));
  __syncthreads();
}

__device__ inline void hist_clear(uint32_t *s_hist) {
  for (int b = threadIdx.x; b < kHistWin; b += kThreads) s_hist[b] = 0;
}

__device__ inline void hist_flush(uint32_t *s_hist, uint32_t *g) {
  for (int b = threadIdx.x; b < kHistWin; b += kThreads) {
    const uint32_t v = s_hist[b];
    if (v) {
      atomicAdd(&g[kHistLo + b], v);
      s_hist[b] = 0;
    }
  }
}

// Hands the workgroup's LDS window to the global histogram.  A narrow
// window (few distinct codes) is added bin by bin with global atomics.  A
// wide one, where one global atomic per distinct code would cost more than
// counting its points again, is written back as codes into the
// workgroup's overflow region (each thread expands 16 consecutive bins at
// the offset an exclusive scan of the bin counts gives it), and the
// overflow pass counts them in LDS.  `points` is the workgroup's number of
// sampled points; the region holds that many codes.  Adds the 1024-bin
// chunks of the window's nonzero bins to `chunks` and returns, in every
// thread, the number of codes the workgroup counted (window bins plus the
// codes already in the region), i.e. its predictable points.
__device__ inline uint32_t hist_hand_over(uint32_t *s_hist, uint32_t *g, global_t<uint16_t> *region, uint32_t *s_n,
                                          uint32_t points, uint64_t &chunks) {
  constexpr int kPer = kHistWin / kThreads;  // 16 bins per thread
  __shared__ uint32_t s_distinct, s_wave[kWaves];
  const int t = threadIdx.x;
  // a thread's 16 bins are visited starting at a lane-dependent one, so
  // that one read of the wave touches distinct LDS banks
  const int skew = t >> 2;
  uint32_t nz = 0, sum = 0;
#pragma unroll
  for (int k = 0; k < kPer; k++) {
    const uint32_t v = s_hist[t * kPer + ((k + skew) & (kPer - 1))];
    nz += v ? 1u : 0u;
    sum += v;
  }
  if (nz) chunks |= 1ull << ((kHistLo + t * kPer) >> 10);
  const uint32_t wnz = group_isum<kWave>(nz);
  // inclusive scan of the per-thread sums within the wave (Hillis-Steele)
  uint32_t inc = sum;
  const int lane = t & (kWave - 1), wv = t / kWave;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const uint32_t o = __shfl_up(inc, d);
    if (lane >= d) inc += o;
  }
  if (lane == kWave - 1) s_wave[wv] = inc;
  if (t == 0) s_distinct = 0;
  __syncthreads();
  uint32_t counted = *s_n;
#pragma unroll
  for (int q = 0; q < kWaves; q++) counted += s_wave[q];
  if (lane == 0) atomicAdd(&s_distinct, wnz);
  __syncthreads();
  if (s_distinct * 4u <= points) {
    hist_flush(s_hist, g);
    return counted;
  }
  uint32_t base = *s_n + inc - sum;
  for (int q = 0; q < wv; q++) base += s_wave[q];
  for (int k = 0; k < kPer; k++) {
    const int b = t * kPer + ((k + skew) & (kPer - 1));
    const uint32_t v = s_hist[b];
    for (uint32_t c = 0; c < v; c++) region[base + c] = (uint16_t)(kHistLo + b);
    base += v;
    s_hist[b] = 0;
  }
  __syncthreads();
  if (t == kThreads - 1) *s_n = base;
  __syncthreads();
  return counted;
}

// SZ totals of the request (last SZ workgroup): squared-error tree over the
// workgroups' subtrees, maximum error, unpredictable count.
__device__ inline void sz_finalize(const ReqDesc &r, const Part &tot) {
  if (threadIdx.x == 0) {
    // slices of the overflow count: about r.ovf_per_slice codes each, and
    // few enough SZ workgroups per slice for the overflow pass's LDS tables
    const uint64_t per = (uint64_t)r.ovf_per_slice;
    const uint64_t want = (tot.b + per - 1) / per;
    const uint64_t least = ((uint64_t)r.nsz + kOvfMaxRegions - 1) / kOvfMaxRegions;
    uint64_t sl = want > least ? want : least;
    sl = sl < 1 ? 1 : (sl > (uint64_t)kOvfSlices ? (uint64_t)kOvfSlices : sl);
    put_u32(&r.st->ovf_slices, tot.b ? (uint32_t)sl : 0u);
    put_u64(&r.st->ovf_count, tot.b);
    put_f64(&r.st->sz_sse, tot.s);
    put_f64(&r.st->sz_maxerr, tot.m);
    put_u64(&r.st->sz_unpred, tot.a);
  }
}

// Overflow pass, workgroup (p, q) of kOvfSlices x kOvfRanges: for p below
// the request's slice count S, counts, in LDS, the overflow codes of SZ
// workgroups [p n/S, (p+1) n/S) that lie in code range q, and adds the
// nonzero ones to the request's overflow counts (one global atomic per
// nonzero bin; the entropy pass reads and clears them).  The occupied
// 16-byte vectors (8 codes) of the
// slice's regions are numbered through an LDS prefix sum of the regions'
// vector counts, so the work follows the number of overflow codes; 4
// vectors are in flight per thread.
__device__ inline void ovf_wg(const ReqDesc &r, int g, uint32_t *s_cnt) {
  const int BS = 1 << (2 * r.nd);  // (any rank: one launch serves them all)
  const int p = g / kOvfRanges, q = g % kOvfRanges;
  const int S = (int)get_u32(&r.st->ovf_slices);  // 0 when there is no overflow code
  if (p >= S) return;
  __shared__ uint32_t s_n[kOvfMaxRegions], s_pre[kOvfMaxRegions + 1];
  const int w0 = (int)(((int64_t)r.nsz * p) / S);
  const int w1 = (int)(((int64_t)r.nsz * (p + 1)) / S);
  const int nreg = w1 - w0;
  for (int b = threadIdx.x; b < kOvfBins; b += kOvfThreads) s_cnt[b] = 0;
  for (int k = threadIdx.x; k < nreg; k += kOvfThreads) s_n[k] = (uint32_t)get_u64(r.sp.b + w0 + k);
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t acc = 0;
    for (int k = 0; k < nreg; k++) {
      s_pre[k] = acc;
      acc += (s_n[k] + 7) / 8;
    }
    s_pre[nreg] = acc;
  }
  __syncthreads();
  const int lo = q * kOvfBins;
  const int64_t cap = (int64_t)r.sblk * BS;  // codes per region (a multiple of 64)
  const uint32_t nv = s_pre[nreg];
  auto count = [&](uint4 v, int valid) {
    const uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
    for (int e = 0; e < 8; e++) {
      const int c = (int)((w[e >> 1] >> (16 * (e & 1))) & 0xffffu) - lo;
      if (e < valid && c >= 0 && c < kOvfBins) atomicAdd(&s_cnt[c], 1u);
    }
  };
  for (uint32_t k0 = threadIdx.x; k0 < nv; k0 += 4 * kOvfThreads) {
    uint4 v[4];
    int valid[4];
#pragma unroll
    for (int u = 0; u < 4; u++) {
      const uint32_t k = k0 + (uint32_t)u * kOvfThreads;
      valid[u] = 0;
      v[u] = make_uint4(0, 0, 0, 0);
      if (k < nv) {
        int lo_i = 0, hi_i = nreg - 1;  // last region with s_pre <= k
        while (lo_i < hi_i) {
          const int mid = (lo_i + hi_i + 1) >> 1;
          if (s_pre[mid] <= k) lo_i = mid; else hi_i = mid - 1;
        }
        const int64_t off = (int64_t)(k - s_pre[lo_i]) * 8;
        v[u] = load_u4(to_global(r.ovf) + (size_t)(w0 + lo_i) * cap + off);
        valid[u] = (int)min<int64_t>(8, (int64_t)s_n[lo_i] - off);
      }
    }
#pragma unroll
    for (int u = 0; u < 4; u++) count(v[u], valid[u]);
  }
  __syncthreads();
  uint32_t *out = r.ovf_hist + lo;
  for (int b = threadIdx.x; b < kOvfBins; b += kOvfThreads) {
    const uint32_t v = s_cnt[b];
    if (v) atomicAdd(&out[b], v);
  }
}

// Chunks of 1,024 bins the entropy pass works on: those some code fell in
// (chunk 0 always: it holds the unpredictable count), or all 64 when the
// final counts are wanted (Huffman cost, debug dump), since the others'
// final counts must then be written as zeros.
__device__ inline uint64_t ent_chunks(const ReqDesc &r) {
  return (r.huff || r.dbg_hist) ? ~0ull : (get_u64(&r.st->code_chunks) | 1ull);
}

// Entropy pass, chunk c (one of `chunks`): the adjacent-pair subtree of
// h log2 h over bins [1024c, 1024c+1024) (4 consecutive bins per thread),
// clearing the bins for the next request.  The chunks' workgroups count on
// one counter; the last one folds the 64 chunk subtrees (0 for a chunk
// without codes, whose h log2 h terms are all 0) by the wave butterfly, the
// same tree as the completion of the other passes, and finishes the
// request:
// entropy (Eq. 5 with P_i = h_i/n), SZ bit-rate (entropy + offset + W escape
// bits per unpredictable point, Section 6.2), both PSNRs and the selection
// of Algorithm 1 (lower bit-rate wins, ties go to ZFP).
__device__ inline void ent_wg(const ReqDesc &r, int c, uint64_t chunks, TileLds &L) {
  // (any dtype and rank: one launch serves them all)
  const int BS = 1 << (2 * r.nd);
  const double W = r.dtype == SZSEL_F32 ? (double)Prec<float>::W : (double)Prec<double>::W;
  const int t = threadIdx.x;
  const uint64_t unpred = get_u64(&r.st->sz_unpred);
  const int S = (int)get_u32(&r.st->ovf_slices);
  const int nhc = r.nhc;
  static_assert(kEntPerThread == 4, "four bins per thread, one 16-byte vector");
  const int bin0 = c * kEntChunk + t * kEntPerThread;
  static_assert(kEntChunk == 1024 && kEntWgs == 64, "one code-chunk bit per entropy workgroup");
  // the SZ workgroups' counts, spread over nhc copies so that no bin takes
  // more than about 128 workgroups' atomics; every copy's four bins are one
  // 16-byte load, all issued before any is used
  uint4 hc[kHistCopies];
#pragma unroll
  for (int q = 0; q < kHistCopies; q++)
    hc[q] = q < nhc ? load_u4(to_global(r.hist) + (size_t)q * kBins + bin0) : make_uint4(0, 0, 0, 0);
  uint32_t h[4] = {0, 0, 0, 0};
#pragma unroll
  for (int q = 0; q < kHistCopies; q++) {
    h[0] += hc[q].x;
    h[1] += hc[q].y;
    h[2] += hc[q].z;
    h[3] += hc[q].w;
  }
  // the overflow pass's counts
  const uint4 o = S > 0 ? load_u4(to_global(r.ovf_hist) + bin0) : make_uint4(0, 0, 0, 0);
  h[0] += o.x;
  h[1] += o.y;
  h[2] += o.z;
  h[3] += o.w;
  if (bin0 == 0) h[0] = (uint32_t)unpred;  // code 0: the unpredictable points
  if (r.huff) *(uint4 *)(r.hfinal + bin0) = make_uint4(h[0], h[1], h[2], h[3]);
  if (r.dbg_hist) {
#pragma unroll
    for (int k = 0; k < kEntPerThread; k++) r.dbg_hist[bin0 + k] = h[k];
  }
#pragma unroll
  for (int q = 0; q < kHistCopies; q++)
    if (q < nhc && (hc[q].x | hc[q].y | hc[q].z | hc[q].w))
      zero_u4(to_global(r.hist) + (size_t)q * kBins + bin0);
  if (o.x | o.y | o.z | o.w) zero_u4(to_global(r.ovf_hist) + bin0);
  double hv[kEntPerThread];
#pragma unroll
  for (int k = 0; k < kEntPerThread; k++) {
    const double hd = (double)h[k];
    hv[k] = h[k] ? hd * log2(hd) : 0.0;
  }
  // the thread's 4 consecutive bins, then the wave butterfly, then the
  // fixed combine of the 4 waves: the chunk's aligned subtree
  double v = (hv[0] + hv[1]) + (hv[2] + hv[3]);
  v = group_tree_sum<kWave>(v);
  const int w = t / kWave;
  if ((t & (kWave - 1)) == 0) L.red[w] = v;
  __syncthreads();
  if (t == 0) {
    Part pc = part_identity<false>();
    pc.s = (L.red[0] + L.red[1]) + (L.red[2] + L.red[3]);
    part_store(r.ep, c, pc);
  }
  wait_memory();
  __syncthreads();
  if (t == 0) {
    PassSync *sy = r.sync + kPassEnt;
    const uint32_t old = __hip_atomic_fetch_add(&sy->top.v, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    L.last = old == (uint32_t)__popcll(chunks) - 1u;
    if (L.last) put_u32(&sy->top.v, 0);
  }
  __syncthreads();
  if (!L.last) return;
  Part tot;
  if (t < kWave) tot = part_wave<false>(((chunks >> t) & 1u) ? part_load(r.ep, t) : part_identity<false>());
  if (t == 0) {
    const double s = tot.s;
    ReqState *st = r.st;
    szsel_result *res = r.res;
    const double nv = (double)(r.nblk * BS);
    const double sse = get_f64(&st->sz_sse);
    const double H = log2(nv) - s / nv;
    double br = H + r.sz_offset;
    br = br + ((double)unpred * W) / nv;
    const double delta = get_f64(&st->delta);
    const double eb_sz = get_f64(&st->eb_sz);
    const double eb_abs = get_f64(&st->eb_abs);
    const double vr = get_f64(&st->vr);
    const double mse = sse / nv;
    put_f64(&res->sz_delta, delta);
    put_f64(&res->sz_inv_delta, get_f64(&st->inv));
    put_f64(&res->sz_eb, eb_sz);
    put_f64(&res->sz_entropy, H);
    put_f64(&res->sz_bitrate, br);
    put_f64(&res->sz_sse, sse);
    put_f64(&res->sz_mse, mse);
    put_f64(&res->sz_maxerr, get_f64(&st->sz_maxerr));
    put_u64(&res->sz_values, (uint64_t)(r.nblk * BS));
    put_u64(&res->sz_unpredictable, unpred);
    put_f64(&res->sz_psnr_model, 20.0 * log10(vr / delta) + 10.0 * log10(12.0));
    put_f64(&res->sz_psnr_measured, mse > 0.0 ? 20.0 * log10(vr) - 10.0 * log10(mse) : INFINITY);
    if ((r.op == SZSEL_OP_SELECT || r.op == SZSEL_OP_FIXED_EB) && r.huff != 2) {
      const double br_zfp = get_f64(&res->zfp_bitrate);
      const int32_t choice = br < br_zfp ? 0 : 1;
      uint32_t flags = (uint32_t)get_u64((uint64_t *)&res->flags);
      if (eb_sz > eb_abs) flags |= SZSEL_FLAG_EB_EXCEEDS;
      put_u64((uint64_t *)&res->flags, (uint64_t)flags | ((uint64_t)(uint32_t)choice << 32));
      put_f64(&res->chosen_eb, choice == 0 ? eb_sz : eb_abs);
    }
  }
}

// ===========================================================================
// Exact Huffman cost of the code histogram (one workgroup per request)
// ===========================================================================

// The optimal prefix code's total length sum_i h_i L_i is the sum of the
// internal node weights of a Huffman tree; that minimum is unique, so any
// order of merging that a Huffman construction may take gives the same cost.
//
// The items (nonzero bin counts, then merged nodes) are kept as a sorted
// list of runs of equal weight.  One round: with s the sum of the two
// lightest items, every item of weight <= s is paired with its neighbour in
// sorted order, all pairs at once.  That is what the one-pair-at-a-time
// construction does too: every node formed weighs >= s, so items <= s stay
// the lightest until they are paired up.  An odd item out stays.  Within a
// run of m equal weights w the pairs form a run of (m - o) / 2 nodes of
// weight 2w (o = 1 when the run's first item pairs with the previous run's
// last); a run ending on an odd item pairs it with the next run's first.
// The new runs, sorted by construction, are merged into the rest of the
// list (equal weights combined).  The lightest weight at least doubles
// every two rounds, so a total below 2^32 needs fewer than 70 rounds; the
// list holds distinct weights whose sum is the total, so at most
// sqrt(2 total) runs: 8192 suffice for 2^25 sampled values.  Once at most
// 64 items are left, one wave merges them one pair at a time in registers.
// CAP: runs the list holds (a total of t values needs at most sqrt(2 t)).
// LDSB: the second pair of arrays (a round's new runs, and first the tally
// of small counts and the large counts) in LDS too; otherwise the caller
// passes global buffers of CAP entries for them (a list of 16,384 runs,
// enough for 2^27 values, fills 128 KiB of LDS by itself).
template <int CAP, bool LDSB>
struct HuffLdsT {
  uint32_t aw[CAP], am[CAP];  // the list: weights (ascending, distinct), multiplicities
  uint32_t bw[LDSB ? CAP : 1], bm[LDSB ? CAP : 1];
  uint32_t slots[2][2 * (kHuffThreads / kWave)];
  uint64_t red[kHuffThreads / kWave];
  uint32_t nbig, leaves, has_left, left_w;
  static constexpr int kCap = CAP;
  static constexpr bool kLdsB = LDSB;
};
using HuffLds = HuffLdsT<kHuffCap, true>;
static_assert(kHuffCap % kHuffThreads == 0 && kHuffSmall <= kHuffCap, "Huffman pass layout");

// Inclusive prefix sum over the 64 lanes of a wave: shifts of 1, 2, 4, 8
// within rows of 16 lanes (row_shr), then the row ends carried into the
// later rows (row_bcast:15 into rows 1 and 3, row_bcast:31 into rows 2 and
// 3).  Lanes without a source add 0.
__device__ inline uint32_t wave_incl_scan(uint32_t v) {
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xf, 0xf, false);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xf, 0xf, false);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xf, 0xf, false);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xf, 0xf, false);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xa, 0xf, false);
  v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xc, 0xf, false);
  return v;
}

// Exclusive prefixes (pa, pb) of a and b over the workgroup in thread
// order, and their totals; one barrier.  Consecutive calls use different
// slot arrays unless a barrier separates them.
__device__ inline void huff_scan2(uint32_t a, uint32_t b, uint32_t *slots, uint32_t &pa, uint32_t &pb,
                                  uint32_t &ta, uint32_t &tb) {
  constexpr int NW = kHuffThreads / kWave;
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  const uint32_t ia = wave_incl_scan(a), ib = wave_incl_scan(b);
  if (lane == kWave - 1) {
    slots[w] = ia;
    slots[NW + w] = ib;
  }
  __syncthreads();
  uint32_t sa = 0, sb = 0, xa = 0, xb = 0;
#pragma unroll
  for (int q = 0; q < NW; q++) {
    const uint32_t x = slots[q], y = slots[NW + q];
    sa += q < w ? x : 0u;
    sb += q < w ? y : 0u;
    xa += x;
    xb += y;
  }
  ta = xa;
  tb = xb;
  pa = sa + ia - a;
  pb = sb + ib - b;
}

// First index in [lo, hi) of the ascending array a whose value is >= x.
__device__ inline uint32_t huff_lower_bound(const uint32_t *a, uint32_t lo, uint32_t hi, uint32_t x) {
  while (lo < hi) {
    const uint32_t mid = (lo + hi) >> 1;
    if (a[mid] < x)
      lo = mid + 1;
    else
      hi = mid;
  }
  return lo;
}

// One merge round over the list (aw, am)[0, n) holding `items` items.
// Returns false when the new list would not fit.
template <typename Lds>
__device__ inline bool huff_round(Lds &S, uint32_t *bw, uint32_t *bm, uint32_t &n, uint32_t &items,
                                  uint64_t &cost) {
  constexpr int NT = kHuffThreads;
  constexpr int kPer = Lds::kCap / NT;  // list runs per thread at most
  const int t = threadIdx.x;
  const uint32_t w0 = S.aw[0], m0 = S.am[0];
  // s: the two lightest items' sum (at most the total: 32 bits)
  const uint32_t sv = m0 >= 2 ? 2u * w0 : w0 + S.aw[1];
  const uint64_t sv2 = 2ull * sv;
  if (t == 0) S.has_left = 0;
  // M = the runs of weight <= s (a prefix); the band = the runs <= 2s,
  // beyond which no new node reaches
  const uint32_t per = (n + NT - 1) / NT, i0 = t * per;
  uint32_t w[kPer], m[kPer];
  uint32_t cntM = 0, msumM = 0, cntB = 0;
#pragma unroll
  for (int j = 0; j < kPer; j++) {
    const uint32_t i = i0 + j;
    w[j] = 0;
    m[j] = 0;
    if ((uint32_t)j < per && i < n) {
      w[j] = S.aw[i];
      m[j] = S.am[i];
      if (w[j] <= sv) {
        cntM++;
        msumM += m[j];
      }
      if ((uint64_t)w[j] <= sv2) cntB++;
    }
  }
  uint32_t pm, pc, tm, tc;
  huff_scan2(msumM, cntM | (cntB << 16), S.slots[0], pm, pc, tm, tc);
  const uint32_t k = tc & 0xFFFFu, k2 = tc >> 16;
  // pair up M; a new run whose weight is already in the band joins that run
  uint32_t par = pm & 1u;
  uint32_t emit = 0, ecount = 0, made = 0;  // bit 2j: element j's run of pairs kept, bit 2j+1: its cross pair
#pragma unroll
  for (int j = 0; j < kPer; j++) {
    const uint32_t i = i0 + j;
    if ((uint32_t)j < per && i < k) {
      const uint32_t e = m[j] - par;
      const uint32_t pairs = e >> 1, odd = e & 1u;
      if (pairs) {
        const uint32_t x = 2u * w[j];
        cost += (uint64_t)x * pairs;
        made += pairs;
        const uint32_t f = huff_lower_bound(S.aw, k, k2, x);
        if (f < k2 && S.aw[f] == x) {
          atomicAdd(&S.am[f], pairs);
        } else {
          emit |= 1u << (2 * j);
          ecount++;
        }
      }
      if (odd && i + 1 < k) {
        const uint32_t x = w[j] + S.aw[i + 1];
        cost += x;
        made++;
        const uint32_t f = huff_lower_bound(S.aw, k, k2, x);
        if (f < k2 && S.aw[f] == x) {
          atomicAdd(&S.am[f], 1u);
        } else {
          emit |= 2u << (2 * j);
          ecount++;
        }
      } else if (odd) {
        S.has_left = 1;  // the odd item out
        S.left_w = w[j];
      }
      par = odd;
    }
  }
  uint32_t epos, pmade, a, tmade;
  huff_scan2(ecount, made, S.slots[1], epos, pmade, a, tmade);
  // new list: [odd item] + merge(new runs, rest); checked before any write
  const uint32_t has_left = S.has_left, left_w = S.left_w;
  const bool left_sep = has_left && left_w != sv;  // an odd item of weight s joins the first new run
  const uint32_t off = left_sep ? 1u : 0u;
  const uint32_t rest = n - k, n2 = off + a + rest;
  if (n2 > (uint32_t)Lds::kCap) return false;
  {
    uint32_t par2 = pm & 1u;
#pragma unroll
    for (int j = 0; j < kPer; j++) {
      const uint32_t i = i0 + j;
      if ((uint32_t)j < per && i < k) {
        const uint32_t e = m[j] - par2;
        if (emit & (1u << (2 * j))) {
          bw[epos] = 2u * w[j];
          bm[epos] = e >> 1;
          epos++;
        }
        if (emit & (2u << (2 * j))) {
          bw[epos] = w[j] + S.aw[i + 1];
          bm[epos] = 1;
          epos++;
        }
        par2 = e & 1u;
      }
    }
  }
  __syncthreads();
  // positions in the new list, all read before any thread writes it
  const uint32_t U = a + rest, uper = (U + NT - 1) / NT, u0 = t * uper;
  uint32_t pw[kPer], pq[kPer], pp[kPer];
#pragma unroll
  for (int j = 0; j < kPer; j++) {
    const uint32_t u = u0 + j;
    pp[j] = 0xFFFFFFFFu;
    pw[j] = 0;
    pq[j] = 0;
    if ((uint32_t)j < uper && u < U) {
      if (u < a) {
        pw[j] = bw[u];
        pq[j] = bm[u] + ((u == 0 && has_left && !left_sep) ? 1u : 0u);
        pp[j] = off + u + (huff_lower_bound(S.aw, k, k2, pw[j]) - k);
      } else {
        const uint32_t q = u - a;
        pw[j] = S.aw[k + q];
        pq[j] = S.am[k + q];
        pp[j] = off + q + (k + q < k2 ? huff_lower_bound(bw, 0, a, pw[j]) : a);
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int j = 0; j < kPer; j++)
    if (pp[j] != 0xFFFFFFFFu) {
      S.aw[pp[j]] = pw[j];
      S.am[pp[j]] = pq[j];
    }
  if (t == 0 && left_sep) {
    S.aw[0] = left_w;
    S.am[0] = 1;
  }
  __syncthreads();
  n = n2;
  items -= tmade;
  return true;
}

// At most 64 items (n runs) left: wave 0 places them in its lanes,
// ascending, and merges them one pair at a time, the leaves and the nodes
// made so far (ascending by construction) as two queues in registers.
template <typename Lds>
__device__ inline void huff_tail(Lds &S, uint32_t *bw, uint32_t n, uint32_t items, uint64_t &cost) {
  const int lane = threadIdx.x;
  uint32_t w = 0, m = 0;
  if ((uint32_t)lane < n) {
    w = S.aw[lane];
    m = S.am[lane];
  }
  const uint32_t pre = wave_incl_scan(m) - m;
  for (uint32_t q = 0; q < m; q++) bw[pre + q] = w;
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  const uint32_t leaf = (uint32_t)lane < items ? bw[lane] : 0xFFFFFFFFu;
  uint32_t node = 0xFFFFFFFFu;
  uint32_t li = 0, qh = 0, qt = 0;
  uint64_t c = 0;
  for (uint32_t step = 1; step < items; step++) {
    uint32_t lw = li < items ? (uint32_t)__builtin_amdgcn_readlane((int)leaf, (int)li) : 0xFFFFFFFFu;
    uint32_t qw = qh < qt ? (uint32_t)__builtin_amdgcn_readlane((int)node, (int)qh) : 0xFFFFFFFFu;
    uint32_t x;
    if (lw <= qw) {
      x = lw;
      li++;
      lw = li < items ? (uint32_t)__builtin_amdgcn_readlane((int)leaf, (int)li) : 0xFFFFFFFFu;
    } else {
      x = qw;
      qh++;
      qw = qh < qt ? (uint32_t)__builtin_amdgcn_readlane((int)node, (int)qh) : 0xFFFFFFFFu;
    }
    uint32_t y;
    if (lw <= qw) {
      y = lw;
      li++;
    } else {
      y = qw;
      qh++;
    }
    node = (uint32_t)lane == qt ? x + y : node;
    qt++;
    c += (uint64_t)x + y;
  }
  if (lane == 0) cost += c;
}

// Optimal prefix-code bits of the 65,536 counts hist (which sum to nv),
// by the whole workgroup; valid on thread 0, which returns true when it was
// computed (false: more distinct weights than the pass holds, or nv >=
// 2^32).  S.leaves holds the number of nonzero counts afterwards.  (bw, bm):
// S.bw and S.bm, or global buffers of CAP entries each.
template <typename Lds>
__device__ inline bool huff_cost(const uint32_t *hist, uint64_t nv, Lds &S, uint32_t *bw, uint32_t *bm,
                                 uint64_t &total_out) {
  constexpr int NT = kHuffThreads;
  constexpr int CAP = Lds::kCap;
  // the tally of small counts and the large counts are built and the large
  // counts sorted in LDS: in (bw, bm) when those are in LDS, else in the
  // list's arrays (unused until the list is built), then handed to (bw, bm)
  constexpr bool kLdsB = Lds::kLdsB;
  uint32_t *tw = kLdsB ? bw : S.aw;
  uint32_t *tb = kLdsB ? bm : S.am;
  constexpr int kSmallPer = kHuffSmall / NT;
  constexpr int kLoads = kBins / 4 / NT;
  const int t = threadIdx.x;
  // every node weighs at most the total: 32-bit weights
  bool ok = nv < (1ull << 32);
  uint64_t cost = 0;  // this thread's share of the internal node weights

  // ---- tally of the final counts (left in hfinal by the entropy pass) ----
  if (ok) {
#pragma unroll
    for (int k = 0; k < kSmallPer; k++) tw[t * kSmallPer + k] = 0;
    if (t == 0) {
      S.nbig = 0;
      S.leaves = 0;
    }
    __syncthreads();
    uint4 v[kLoads];
#pragma unroll
    for (int q = 0; q < kLoads; q++) v[q] = ((const uint4 *)hist)[t + q * NT];
    uint32_t leaves = 0;
#pragma unroll
    for (int q = 0; q < kLoads; q++) {
      const uint32_t c4[4] = {v[q].x, v[q].y, v[q].z, v[q].w};
#pragma unroll
      for (int k = 0; k < 4; k++) {
        const uint32_t c = c4[k];
        if (!c) continue;
        leaves++;
        if (c < (uint32_t)kHuffSmall) {
          atomicAdd(&tw[c], 1u);
        } else {
          const uint32_t i = atomicAdd(&S.nbig, 1u);
          if (i < (uint32_t)CAP) tb[i] = c;
        }
      }
    }
    leaves = group_isum<kWave>(leaves);
    if ((t & (kWave - 1)) == 0) atomicAdd(&S.leaves, leaves);
    __syncthreads();
    ok = S.nbig <= (uint32_t)CAP;
  }

  // ---- the initial list: runs of the small counts, then of the sorted large ones ----
  uint32_t n = 0;
  if (ok) {
    const uint32_t nbig = S.nbig;
    uint32_t P = 1;
    while (P < nbig) P <<= 1;
    for (uint32_t i = nbig + t; i < P; i += NT) tb[i] = 0xFFFFFFFFu;
    __syncthreads();
    for (uint32_t k = 2; k <= P; k <<= 1) {
      for (uint32_t j = k >> 1; j > 0; j >>= 1) {
        for (uint32_t i = t; i < P; i += NT) {
          const uint32_t l = i ^ j;
          if (l > i) {
            const uint32_t x = tb[i], y = tb[l];
            if ((i & k) == 0 ? x > y : x < y) {
              tb[i] = y;
              tb[l] = x;
            }
          }
        }
        __syncthreads();
      }
    }
    if constexpr (!kLdsB) {  // hand the tally and the sorted large counts over
      for (uint32_t i = t; i < (uint32_t)kHuffSmall; i += NT) bw[i] = tw[i];
      for (uint32_t i = t; i < nbig; i += NT) bm[i] = tb[i];
      __syncthreads();
    }
    uint32_t mult[kSmallPer];
    uint32_t occ = 0;
#pragma unroll
    for (int k = 0; k < kSmallPer; k++) {
      mult[k] = bw[t * kSmallPer + k];
      occ += mult[k] ? 1u : 0u;
    }
    const uint32_t bper = (nbig + NT - 1) / NT, b0 = t * bper;
    uint32_t starts = 0;
    for (uint32_t j = 0; j < bper; j++) {
      const uint32_t i = b0 + j;
      if (i < nbig && (i == 0 || bm[i] != bm[i - 1])) starts++;
    }
    uint32_t po, ps, nsmall, nbruns;
    huff_scan2(occ, starts, S.slots[0], po, ps, nsmall, nbruns);
    n = nsmall + nbruns;
    ok = n <= (uint32_t)CAP;
    if (ok) {
      uint32_t pos = po;
#pragma unroll
      for (int k = 0; k < kSmallPer; k++)
        if (mult[k]) {
          S.aw[pos] = (uint32_t)(t * kSmallPer + k);
          S.am[pos] = mult[k];
          pos++;
        }
      pos = nsmall + ps;
      for (uint32_t j = 0; j < bper; j++) {
        const uint32_t i = b0 + j;
        if (i < nbig && (i == 0 || bm[i] != bm[i - 1])) {
          S.aw[pos] = bm[i];
          S.am[pos] = 0;
          pos++;
        }
      }
      __syncthreads();
      // each large count adds one to its run (the last run started at or before it)
      uint32_t c = ps;
      for (uint32_t j = 0; j < bper; j++) {
        const uint32_t i = b0 + j;
        if (i < nbig) {
          if (i == 0 || bm[i] != bm[i - 1]) c++;
          atomicAdd(&S.am[nsmall + c - 1], 1u);
        }
      }
    }
    __syncthreads();
  }

  // ---- merge rounds, then the last items one pair at a time ----
  if (ok) {
    uint32_t items = S.leaves;
    int rounds = 0;
    while (ok && items > (uint32_t)kWave) {
      ok = huff_round(S, bw, bm, n, items, cost) && ++rounds <= kHuffMaxRounds;
    }
    if (ok && t < kWave) huff_tail(S, bw, n, items, cost);
  }

  // ---- total ----
  __syncthreads();  // a round left early may still have readers of the scan slots
  cost = group_isum<kWave>(cost);
  if ((t & (kWave - 1)) == 0) S.red[t / kWave] = cost;
  __syncthreads();
  uint64_t total = 0;
#pragma unroll
  for (int q = 0; q < NT / kWave; q++) total += S.red[q];
  if (ok && S.leaves == 1) total = nv;  // one symbol: 1 bit each
  total_out = total;
  return ok;
}

template <typename T, int D>
__device__ inline void huff_wg(const ReqDesc &r, HuffLds &S) {
  constexpr int BS = 1 << (2 * D);
  const uint64_t nv = (uint64_t)r.nblk * BS;
  uint64_t total;
  const bool ok = huff_cost(r.hfinal, nv, S, S.bw, S.bm, total);
  if (threadIdx.x != 0) return;
  ReqState *st = r.st;
  szsel_result *res = r.res;
  const uint64_t unpred = get_u64(&st->sz_unpred);
  double hbr = (double)total / (double)nv;
  hbr = hbr + ((double)unpred * (double)Prec<T>::W) / (double)nv;
  const uint64_t fc = get_u64((uint64_t *)&res->flags);
  uint32_t flags = (uint32_t)fc;
  uint32_t choice = (uint32_t)(fc >> 32);
  if (ok) {
    put_u64(&res->sz_huffman_bits, total);
    put_f64(&res->sz_huffman_bitrate, hbr);
  } else {
    flags |= SZSEL_FLAG_NO_HUFFMAN;
  }
  if (r.huff == 2 && (r.op == SZSEL_OP_SELECT || r.op == SZSEL_OP_FIXED_EB)) {
    // select with the Huffman bit-rate (with entropy + offset when it is missing)
    const double br = ok ? hbr : get_f64(&res->sz_bitrate);
    const double br_zfp = get_f64(&res->zfp_bitrate);
    const double eb_sz = get_f64(&st->eb_sz), eb_abs = get_f64(&st->eb_abs);
    choice = br < br_zfp ? 0u : 1u;
    if (eb_sz > eb_abs) flags |= SZSEL_FLAG_EB_EXCEEDS;
    put_f64(&res->chosen_eb, choice == 0 ? eb_sz : eb_abs);
  }
  put_u64((uint64_t *)&res->flags, (uint64_t)flags | ((uint64_t)choice << 32));
}

// Whole SZ pass of workgroup w (LDS window cleared on entry, flushed once at
// the end).  Returns true in the workgroup that ran the finalizer.
template <typename T, int D, bool VEC>
__device__ inline bool sz_wg(const ReqDesc &r, int w, TileLds &L, uint32_t *s_hist) {
  const double delta = get_f64(&r.st->delta);
  const double inv = get_f64(&r.st->inv);
  const double ebsz = get_f64(&r.st->eb_sz);
  const int tile = r.sblk < kMaxTile ? r.sblk : kMaxTile;
  const int ntile = r.sblk / tile;
  constexpr int BS = 1 << (2 * D);
  LaneAcc acc;
  __shared__ uint32_t s_n;
  global_t<uint16_t> *region = to_global(r.ovf) + (size_t)w * r.sblk * BS;
  hist_clear(s_hist);
  wg_acc_reset(L);
  if (threadIdx.x == 0) s_n = 0;
  __syncthreads();
  for (int k = 0; k < ntile; k++) {
    const int64_t base = (int64_t)w * r.sblk + (int64_t)k * tile;
    if (base < r.nblk)
      sz_tile<T, D, VEC>(r, base, tile, delta, inv, ebsz, L, s_hist, region, &s_n, acc);
    else
      wg_acc_push(L, 0.0);
  }
  __syncthreads();
  const int64_t nb = max<int64_t>(0, min<int64_t>((int64_t)r.sblk, r.nblk - (int64_t)w * r.sblk));
  const uint32_t points = (uint32_t)(nb * BS);
  const uint32_t counted =
      hist_hand_over(s_hist, r.hist + (size_t)(w & (r.nhc - 1)) * kBins, region, &s_n, points, acc.chunks);
  __syncthreads();
  // the chunks the codes fell in, for the entropy pass to skip empty ones:
  // one OR per wave, only when it adds a bit (most waves add none)
  uint64_t ch = acc.chunks;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) ch |= __shfl_xor(ch, d);
  if ((threadIdx.x & (kWave - 1)) == 0 && (ch & ~get_u64(&r.st->code_chunks)))
    __hip_atomic_fetch_or(&r.st->code_chunks, ch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (threadIdx.x == 0) {
    acc.a = points - counted;  // unpredictable points of this workgroup
    acc.b = s_n;               // overflow codes of this workgroup (summed below)
  }
  wg_acc_store(L, acc, r.sp, w);
  Part tot;
  if (!pass_complete<false>(r.sp, r.grp[kPassSz], r.sync + kPassSz, w, r.nsz, L, tot)) return false;
  sz_finalize(r, tot);
  return true;
}

}  // namespace szsel
