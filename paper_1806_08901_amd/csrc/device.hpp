// Device-side building blocks of the estimator (gfx950, wave64).
//
// Numerics contract (matches the CPU oracle, which shares none of this code):
//   * binary64 for all real arithmetic, round to nearest, no contraction
//     (the library is built with -ffp-contract=off);
//   * every floating-point sum is the adjacent-pair tree over the padded
//     power-of-two sequence; a wave computes it with the xor butterfly
//     (distances 1, 2, 4, ...), which associates exactly like that tree;
//   * integer ZFP arithmetic wraps modulo 2^W; >> on signed values is floor(x/2).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "szsel.h"

namespace szsel {

constexpr int kWave = 64;
constexpr int kThreads = 256;          // every kernel runs 4 waves per workgroup
constexpr int kWaves = kThreads / kWave;
constexpr int kBins = 65536;           // 65,535 symmetric bins plus the escape code 0
constexpr int kRadius = 32768;
constexpr int kMaxTile = 256;          // sampled blocks per tile

// Flags that stop the estimation after the range pass.
constexpr uint32_t kSkipFlags = SZSEL_FLAG_CONSTANT | SZSEL_FLAG_NONFINITE |
                                SZSEL_FLAG_NO_BLOCKS | SZSEL_FLAG_BAD_EB;

// Per-request state shared by the kernels of one request (device memory).
struct alignas(64) ReqState {
  double vmin, vmax, vr, eb_abs;
  double delta, inv, eb_sz;
  int32_t minexp;
  uint32_t flags;
  uint32_t range_done, zfp_done, sz_done;  // last-workgroup counters, reset by their finalizers
  uint32_t pad;
};

struct RangePart {
  double lo, hi;
  uint32_t bad, pad0;
  uint64_t pad1;
};

struct TilePart {
  double sse, maxerr;
  uint64_t bits;  // ZFP: coder bits of the tile; SZ: unused
  uint64_t cnt;   // ZFP: significant bits; SZ: unpredictable points
};

// Everything a kernel needs about one request (passed by value).
struct ReqDesc {
  const void *field;
  int64_t dims[3];
  int64_t n;      // number of values
  int64_t nblk;   // number of sampled blocks
  uint32_t nsel[3];
  int32_t stride[3];
  int32_t nd, dtype, op, eb_mode;
  double eb, sz_offset;
  int32_t tile;    // sampled blocks per tile (power of two, >= one round of 4 waves)
  int32_t ntiles;
  int32_t nrange;  // workgroups of the range pass
  int32_t nsz;     // workgroups of the SZ pass
  int32_t nzfp;    // workgroups of the ZFP pass
  int32_t pad0;
  ReqState *st;
  RangePart *rpart;
  TilePart *zpart;
  TilePart *spart;
  uint32_t *hist;
  szsel_result *res;
  uint16_t *dbg_codes;
  uint32_t *dbg_zbits;
  double *dbg_zsse;
  int32_t *dbg_zemax;
  double *dbg_ssse;
  uint32_t *dbg_hist;
};

// ---------------------------------------------------------------------------
// Type traits of the two field precisions
// ---------------------------------------------------------------------------
template <typename T> struct Prec;
template <> struct Prec<float> {
  using U = uint32_t;
  using I = int32_t;
  static constexpr int W = 32, P = 30, E = 8, MANT = 23, BIAS = 127;
  static constexpr U NB = 0xAAAAAAAAu;
  __device__ static U bits(float v) { return __float_as_uint(v); }
};
template <> struct Prec<double> {
  using U = uint64_t;
  using I = int64_t;
  static constexpr int W = 64, P = 62, E = 11, MANT = 52, BIAS = 1023;
  static constexpr U NB = 0xAAAAAAAAAAAAAAAAull;
  __device__ static U bits(double v) { return (U)__double_as_longlong(v); }
};

__device__ inline int clz_u(uint32_t v) { return __clz((int)v); }
__device__ inline int clz_u(uint64_t v) { return __clzll((long long)v); }

// Exponent e with m in [2^(e-1), 2^e), read from the bits of a positive
// magnitude m of the field type (normal or subnormal).
template <typename T>
__device__ inline int frexp_exponent_bits(typename Prec<T>::U m) {
  using Q = Prec<T>;
  const int eb = (int)(m >> Q::MANT);
  if (eb) return eb - (Q::BIAS - 1);
  const int msb = Q::W - 1 - clz_u(m);
  return msb - (Q::BIAS - 2 + Q::MANT);
}

// floor(log2(t)) of a positive finite binary64 value, from its bits.
__device__ inline int floor_log2_bits(double t) {
  const uint64_t b = (uint64_t)__double_as_longlong(t);
  const int eb = (int)((b >> 52) & 0x7ff);
  if (eb) return eb - 1023;
  const int msb = 63 - __clzll((long long)(b & 0xFFFFFFFFFFFFFull));
  return msb - 1074;
}

// Block-floating-point integer trunc(x * 2^(P - emax)), computed on the bits:
// the significand shifted by the distance between its LSB weight and the
// block's scale.  |x| < 2^emax guarantees the result fits in P bits.
template <typename T>
__device__ inline typename Prec<T>::I bfp_int(T x, int emax) {
  using Q = Prec<T>;
  using U = typename Q::U;
  using I = typename Q::I;
  const U b = Q::bits(x);
  const int eb = (int)((b >> Q::MANT) & ((1u << (Q::W - 1 - Q::MANT)) - 1));
  const U frac = b & ((U(1) << Q::MANT) - 1);
  const U mant = eb ? (frac | (U(1) << Q::MANT)) : frac;
  const int elsb = (eb ? eb : 1) - Q::BIAS - Q::MANT;
  const int sh = elsb + Q::P - emax;
  U mag;
  if (sh >= 0)
    mag = mant << sh;
  else
    mag = (-sh < Q::W) ? (mant >> (-sh)) : U(0);
  const U sgn = b >> (Q::W - 1);
  return sgn ? (I)(U(0) - mag) : (I)mag;
}

// ---------------------------------------------------------------------------
// Wraparound integer lifting (the decorrelating transform)
// ---------------------------------------------------------------------------
template <typename I> __device__ inline I wadd(I a, I b) {
  using U = typename std::make_unsigned<I>::type;
  return (I)((U)a + (U)b);
}
template <typename I> __device__ inline I wsub(I a, I b) {
  using U = typename std::make_unsigned<I>::type;
  return (I)((U)a - (U)b);
}

// Forward 4-point lift; equals (1/16)[[4,4,4,4],[5,1,-1,-5],[-4,4,4,-4],[-2,6,-6,2]]
// on multiples of 16.  Returns output number `which`.
template <typename I>
__device__ inline I fwd_lift_pick(I x0, I x1, I x2, I x3, int which) {
  const I s03 = wadd(x0, x3) >> 1, d03 = wsub(x0, s03);
  const I s12 = wadd(x1, x2) >> 1, d12 = wsub(x1, s12);
  const I y0 = wadd(s03, s12) >> 1;
  const I y2 = wsub(s12, y0);
  const I dm = wadd(d03, d12) >> 1;
  const I dd = wsub(d03, dm);
  const I y3 = wsub(dm >> 1, dd);
  const I y1 = wsub(dm, y3 >> 1);
  return which == 0 ? y0 : which == 1 ? y1 : which == 2 ? y2 : y3;
}

// Inverse lift (undoes each forward step in reverse order).
template <typename I>
__device__ inline I inv_lift_pick(I y0, I y1, I y2, I y3, int which) {
  const I dm = wadd(y1, y3 >> 1);
  const I dd = wsub(dm >> 1, y3);
  const I d03 = wadd(dm, dd), d12 = wsub(dm, dd);
  const I s12 = wadd(y0, y2), s03 = wsub(y0, y2);
  switch (which) {
    case 0: return wadd(s03, d03);
    case 1: return wadd(s12, d12);
    case 2: return wsub(s12, d12);
    default: return wsub(s03, d03);
  }
}

// ---------------------------------------------------------------------------
// Coefficient order: rank of each coefficient under the key (total sequency,
// sum of squared frequencies, slowest-axis frequency, ..., fastest).
// ---------------------------------------------------------------------------
template <int D> constexpr int seq_key(int i) {
  int f0 = i & 3, f1 = D > 1 ? (i >> 2) & 3 : 0, f2 = D > 2 ? (i >> 4) & 3 : 0;
  int s = f0 + f1 + f2, q = f0 * f0 + f1 * f1 + f2 * f2;
  return (s << 12) | (q << 6) | (f2 << 4) | (f1 << 2) | f0;
}

template <int D> struct OrderTable {
  int perm[1 << (2 * D)];     // perm[r]  = coefficient coded at position r
  int inv[1 << (2 * D)];      // inv[i]   = position of coefficient i
  constexpr OrderTable() : perm(), inv() {
    constexpr int n = 1 << (2 * D);
    for (int i = 0; i < n; i++) {
      int rank = 0;
      for (int j = 0; j < n; j++)
        if (seq_key<D>(j) < seq_key<D>(i)) rank++;
      inv[i] = rank;
      perm[rank] = i;
    }
  }
};

// ---------------------------------------------------------------------------
// Wave / workgroup reductions
// ---------------------------------------------------------------------------

// Adjacent-pair tree over the WIDTH consecutive lanes of each aligned group.
template <int WIDTH>
__device__ inline double group_tree_sum(double v) {
#pragma unroll
  for (int s = 1; s < WIDTH; s <<= 1) v = v + __shfl_xor(v, s);
  return v;
}

template <int WIDTH, typename V>
__device__ inline V group_max(V v) {
#pragma unroll
  for (int s = 1; s < WIDTH; s <<= 1) {
    V o = __shfl_xor(v, s);
    v = o > v ? o : v;
  }
  return v;
}

template <int WIDTH, typename V>
__device__ inline V group_isum(V v) {
#pragma unroll
  for (int s = 1; s < WIDTH; s <<= 1) v += __shfl_xor(v, s);
  return v;
}

// Adjacent-pair tree over a[0..n) padded with +0.0, computed by the whole
// workgroup (kThreads threads).  Thread t reduces the aligned chunk
// [t*C, (t+1)*C) with a binary-counter pass (which associates like the tree),
// then the wave butterfly and the fixed combine of the 4 wave results.
// Every thread returns the total.  `sh` is kWaves doubles of LDS.
__device__ inline double wg_tree_sum(const double *a, int64_t n, double *sh) {
  int64_t p = 1;
  while (p < n) p <<= 1;
  const int64_t chunk = p > kThreads ? p / kThreads : 1;
  const int t = threadIdx.x;
  double stk[40];
  int sp = 0;
  const int64_t beg = (int64_t)t * chunk;
  for (int64_t k = 0; k < chunk; k++) {
    const int64_t idx = beg + k;
    double v = idx < n ? a[idx] : 0.0;
    for (int64_t m = k; m & 1; m >>= 1) v = stk[--sp] + v;
    stk[sp++] = v;
  }
  double v = stk[0];
  v = group_tree_sum<kWave>(v);
  const int w = t / kWave;
  __syncthreads();
  if ((t & (kWave - 1)) == 0) sh[w] = v;
  __syncthreads();
  const double r = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  __syncthreads();
  return r;
}

// ---------------------------------------------------------------------------
// Sampled-block addressing
// ---------------------------------------------------------------------------
template <int D>
__device__ inline void block_origin(const ReqDesc &r, uint32_t j, int64_t o[3]) {
  // row-major over the sampled-block lattice, last axis fastest
#pragma unroll
  for (int k = D - 1; k >= 0; k--) {
    const uint32_t ns = r.nsel[k];
    const uint32_t q = j / ns;
    const uint32_t jk = j - q * ns;
    j = q;
    o[k] = 4 * (int64_t)jk * r.stride[k];
  }
}

// Point coordinates of in-block index i (row-major, last axis fastest).
template <int D>
__device__ inline void point_coords(const int64_t o[3], int i, int64_t p[3]) {
#pragma unroll
  for (int k = 0; k < D; k++) p[k] = o[k] + ((i >> (2 * (D - 1 - k))) & 3);
}

template <int D>
__device__ inline int64_t linear_index(const ReqDesc &r, const int64_t p[3]) {
  int64_t lin = p[0];
#pragma unroll
  for (int k = 1; k < D; k++) lin = lin * r.dims[k] + p[k];
  return lin;
}

}  // namespace szsel
