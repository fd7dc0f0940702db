// The estimator's per-tile work and per-request finalizers, shared by the
// plain per-request kernels and the persistent batch kernel.
//
// Section references are to arXiv:1806.08901.
#pragma once

#include <type_traits>

#include "device.hpp"

namespace szsel {

constexpr int kHistWin = 8192;    // LDS histogram window around the zero code
constexpr int kHistLo = kRadius - kHistWin / 2;

template <int D> struct Order {
  static constexpr OrderTable<D> table{};
};

// LDS scratch of one workgroup for a tile.
struct TileLds {
  double sse[kMaxTile];
  double err[kMaxTile];
  uint32_t a[kMaxTile];   // ZFP: bits; SZ: unpredictable count
  uint32_t b[kMaxTile];   // ZFP: significant bits
  double red[kWaves];
};

__device__ inline bool skip_request(const ReqState *st) {
  return (__atomic_load_n(&st->flags, __ATOMIC_RELAXED) & kSkipFlags) != 0;
}

// ===========================================================================
// Value range (Algorithm 1, line 2): min/max over ALL values, non-finite scan
// ===========================================================================

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x2 __attribute__((ext_vector_type(2)));
template <typename T> struct Vec16;
template <> struct Vec16<float> { using V = f32x4; static constexpr int N = 4; };
template <> struct Vec16<double> { using V = f64x2; static constexpr int N = 2; };

template <typename T>
__device__ inline bool nonfinite(T v) {
  using Q = Prec<T>;
  const auto b = Q::bits(v);
  constexpr int EBITS = Q::W - 1 - Q::MANT;
  return ((b >> Q::MANT) & ((1u << EBITS) - 1)) == ((1u << EBITS) - 1);
}

template <typename T>
struct RangeAcc {
  T lo, hi;
  bool bad;
  __device__ RangeAcc() : lo(INFINITY), hi(-INFINITY), bad(false) {}
  __device__ void add(T v) {
    lo = fmin(lo, v);
    hi = fmax(hi, v);
    bad |= nonfinite(v);
  }
};

// Scans values [beg, end) of the field: vector part with 16-byte loads, the
// unaligned head/tail element by element.  `lane0`/`nlanes` index the threads
// taking part.
template <typename T>
__device__ inline void range_scan(const T *x, int64_t beg, int64_t end, int64_t lane0,
                                  int64_t nlanes, RangeAcc<T> &acc) {
  using V = typename Vec16<T>::V;
  constexpr int VN = Vec16<T>::N;
  const uintptr_t a = (uintptr_t)(x + beg);
  int64_t head = (int64_t)(((16 - (a & 15)) & 15) / sizeof(T));
  if (head > end - beg) head = end - beg;
  const int64_t nvec = (end - beg - head) / VN;
  const V *xv = (const V *)(x + beg + head);
  int64_t i = lane0;
  for (; i + 3 * nlanes < nvec; i += 4 * nlanes) {
    const V v0 = __builtin_nontemporal_load(xv + i);
    const V v1 = __builtin_nontemporal_load(xv + i + nlanes);
    const V v2 = __builtin_nontemporal_load(xv + i + 2 * nlanes);
    const V v3 = __builtin_nontemporal_load(xv + i + 3 * nlanes);
    if constexpr (VN == 4) {
      acc.add(v0.x); acc.add(v0.y); acc.add(v0.z); acc.add(v0.w);
      acc.add(v1.x); acc.add(v1.y); acc.add(v1.z); acc.add(v1.w);
      acc.add(v2.x); acc.add(v2.y); acc.add(v2.z); acc.add(v2.w);
      acc.add(v3.x); acc.add(v3.y); acc.add(v3.z); acc.add(v3.w);
    } else {
      acc.add(v0.x); acc.add(v0.y); acc.add(v1.x); acc.add(v1.y);
      acc.add(v2.x); acc.add(v2.y); acc.add(v3.x); acc.add(v3.y);
    }
  }
  for (; i < nvec; i += nlanes) {
    const V v = __builtin_nontemporal_load(xv + i);
    if constexpr (VN == 4) {
      acc.add(v.x); acc.add(v.y); acc.add(v.z); acc.add(v.w);
    } else {
      acc.add(v.x); acc.add(v.y);
    }
  }
  const int64_t tail0 = beg + head + nvec * VN;
  if (lane0 < head) acc.add(x[beg + lane0]);
  if (lane0 < end - tail0) acc.add(x[tail0 + lane0]);
}

// Workgroup reduction of the accumulators; thread 0 gets the result.
template <typename T>
__device__ inline RangePart range_reduce_wg(RangeAcc<T> acc, double *sh_lo, double *sh_hi,
                                            uint32_t *sh_bad) {
  double lo = (double)acc.lo, hi = (double)acc.hi;
  uint32_t bad = acc.bad ? 1u : 0u;
#pragma unroll
  for (int s = 1; s < kWave; s <<= 1) {
    lo = fmin(lo, __shfl_xor(lo, s));
    hi = fmax(hi, __shfl_xor(hi, s));
    bad |= (uint32_t)__shfl_xor((int)bad, s);
  }
  const int w = threadIdx.x / kWave;
  if ((threadIdx.x & (kWave - 1)) == 0) {
    sh_lo[w] = lo;
    sh_hi[w] = hi;
    sh_bad[w] = bad;
  }
  __syncthreads();
  RangePart p{};
  if (threadIdx.x == 0) {
    p.lo = sh_lo[0];
    p.hi = sh_hi[0];
    p.bad = sh_bad[0];
    for (int k = 1; k < kWaves; k++) {
      p.lo = fmin(p.lo, sh_lo[k]);
      p.hi = fmax(p.hi, sh_hi[k]);
      p.bad |= sh_bad[k];
    }
  }
  __syncthreads();
  return p;
}

__device__ inline void zero_result(szsel_result *res) {
  uint64_t *w = (uint64_t *)res;
  for (size_t k = 0; k < sizeof(szsel_result) / 8; k++) w[k] = 0;
}

// Turns the min/max of the whole field into the request's state and the
// first part of its result (called by one thread).
__device__ inline void range_finalize_one(const ReqDesc &r, double lo, double hi, bool bad) {
  ReqState *st = r.st;
  szsel_result *res = r.res;
  zero_result(res);
  const bool selecting = r.op == SZSEL_OP_SELECT || r.op == SZSEL_OP_FIXED_EB;
  res->choice = -1;
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
    if (flags && selecting) res->choice = 0;
  }
  res->vmin = lo;
  res->vmax = hi;
  res->vr = vr;
  res->eb_abs = eb_abs;
  res->minexp = minexp;
  res->flags = flags;
  st->vmin = lo;
  st->vmax = hi;
  st->vr = vr;
  st->eb_abs = eb_abs;
  st->minexp = minexp;
  // SZ's own bin width (Section 5.1.4: delta = 2 eb_abs) unless Algorithm 1
  // derives it from the ZFP estimate later.
  const double delta = 2.0 * eb_abs;
  st->delta = delta;
  st->inv = 1.0 / delta;
  st->eb_sz = 0.5 * delta;
  __atomic_store_n(&st->flags, flags, __ATOMIC_RELAXED);
}

// ===========================================================================
// ZFP side (Sections 4.2 and 5.2) on one wave-group of 4^D lanes per block
// ===========================================================================

template <typename T, int D>
struct ZfpBlockOut {
  uint32_t bits, nsb;
  double sse, maxerr;
  int emax;
};

template <typename T, int D>
__device__ inline ZfpBlockOut<T, D> zfp_block(T xv, int minexp, int perm_i, int inv_i, int lane) {
  using Q = Prec<T>;
  using U = typename Q::U;
  using I = typename Q::I;
  constexpr int BS = 1 << (2 * D);
  constexpr int W = Q::W;
  const int i = lane & (BS - 1);
  const int gbase = lane - i;

  // block-floating-point: common exponent of the largest magnitude
  const U mag = Q::bits(xv) & ~(U(1) << (W - 1));
  const U mmax = group_max<BS>(mag);
  const bool empty = mmax == 0;
  const int emax = empty ? 0 : frexp_exponent_bits<T>(mmax);
  int prec = emax - minexp + 2 * (D + 1);
  prec = empty ? 0 : (prec < 0 ? 0 : (prec > W ? W : prec));
  I c = bfp_int<T>(xv, emax);

  // separable forward transform, fastest axis first
#pragma unroll
  for (int a = 0; a < D; a++) {
    const int s = 1 << (2 * a);
    const int coord = (i >> (2 * a)) & 3;
    const int lb = gbase + i - coord * s;
    const I v0 = __shfl(c, lb), v1 = __shfl(c, lb + s), v2 = __shfl(c, lb + 2 * s),
            v3 = __shfl(c, lb + 3 * s);
    c = fwd_lift_pick(v0, v1, v2, v3, coord);
  }
  // sequency order, then negabinary digits
  c = __shfl(c, gbase + perm_i);
  const U u = ((U)c + Q::NB) ^ Q::NB;

  // group-testing embedded coding of planes W-1 .. kmin.  Per plane the cost
  // follows from the plane mask alone: with n values already significant,
  // m ones at positions >= n and the highest one at p, the plane costs
  // n + [n < BS] bits if m == 0, else p + 1 + m + (p < BS-1 ? 1 : -1), and
  // afterwards n = p + 1.
  const int kmin = W - prec;
  int kstop = kmin;
  if constexpr (D < 3) {
#pragma unroll
    for (int s = BS; s < kWave; s <<= 1) kstop = min(kstop, __shfl_xor(kstop, s));
  } else {
    kstop = __builtin_amdgcn_readfirstlane(kstop);
  }
  const int sh = (D < 3) ? gbase : 0;
  constexpr uint64_t bmask = BS == 64 ? ~0ull : ((1ull << (BS & 63)) - 1ull);
  uint64_t acc = 0;
  uint32_t cost = 0;
  for (int k = W - 1; k >= kstop; --k) {
    const uint64_t all = __ballot((int)((u >> k) & 1));
    if (k >= kmin) {
      const uint64_t m = (all >> sh) & bmask;
      const int n = acc ? 64 - __clzll((long long)acc) : 0;
      const uint64_t rest = n < 64 ? (m >> n) : 0ull;
      if (rest == 0) {
        cost += (uint32_t)(n + (n < BS ? 1 : 0));
      } else {
        const int p = 63 - __clzll((long long)m);
        cost += (uint32_t)(p + 1 + __popcll(rest) + (p < BS - 1 ? 1 : -1));
      }
      acc |= m;
    }
  }
  ZfpBlockOut<T, D> out;
  out.emax = empty ? INT32_MIN : emax;
  out.bits = prec == 0 ? 1u : (uint32_t)(1 + Q::E) + cost;

  // significant bits within the coded planes (Section 5.2.1)
  const int msb = u ? (W - 1 - clz_u(u)) : -1;
  const uint32_t nsb = (prec > 0 && msb >= kmin) ? (uint32_t)(msb - kmin + 1) : 0u;
  out.nsb = group_isum<BS>(nsb);

  // decode at the cutoff: drop planes below kmin, invert every step
  U keep;
  if (kmin >= W)
    keep = 0;
  else if (kmin == 0)
    keep = ~U(0);
  else
    keep = ~((U(1) << kmin) - 1);
  I d = (I)(((u & keep) ^ Q::NB) - Q::NB);
  d = __shfl(d, gbase + inv_i);
#pragma unroll
  for (int a = D - 1; a >= 0; a--) {
    const int s = 1 << (2 * a);
    const int coord = (i >> (2 * a)) & 3;
    const int lb = gbase + i - coord * s;
    const I v0 = __shfl(d, lb), v1 = __shfl(d, lb + s), v2 = __shfl(d, lb + 2 * s),
            v3 = __shfl(d, lb + 3 * s);
    d = inv_lift_pick(v0, v1, v2, v3, coord);
  }
  T xh = (T)ldexp((double)d, emax - Q::P);
  if (prec == 0) xh = (T)0;
  const double e = (double)xv - (double)xh;
  out.sse = group_tree_sum<BS>(e * e);
  out.maxerr = group_max<BS>(fabs(e));
  return out;
}

// Reduces the tile's per-block values in LDS (adjacent tree for the SSE).
// Returns on thread 0: sse, maxerr, sum a, sum b.
__device__ inline void tile_reduce(TileLds &L, int tile, double &sse, double &maxerr,
                                   uint64_t &sa, uint64_t &sb) {
  // wave 0: each lane folds its aligned group of tile/64 entries
  if (threadIdx.x < kWave) {
    const int lane = threadIdx.x;
    const int c = tile > kWave ? tile / kWave : 1;
    double v = 0.0, m = 0.0;
    uint64_t a = 0, b = 0;
    if (c == 1) {
      if (lane < tile) {
        v = L.sse[lane];
        m = L.err[lane];
        a = L.a[lane];
        b = L.b[lane];
      }
    } else if (c == 2) {
      v = L.sse[2 * lane] + L.sse[2 * lane + 1];
      m = fmax(L.err[2 * lane], L.err[2 * lane + 1]);
      a = (uint64_t)L.a[2 * lane] + L.a[2 * lane + 1];
      b = (uint64_t)L.b[2 * lane] + L.b[2 * lane + 1];
    } else {
      const int k = 4 * lane;
      v = (L.sse[k] + L.sse[k + 1]) + (L.sse[k + 2] + L.sse[k + 3]);
      m = fmax(fmax(L.err[k], L.err[k + 1]), fmax(L.err[k + 2], L.err[k + 3]));
      a = (uint64_t)L.a[k] + L.a[k + 1] + L.a[k + 2] + L.a[k + 3];
      b = (uint64_t)L.b[k] + L.b[k + 1] + L.b[k + 2] + L.b[k + 3];
    }
    v = group_tree_sum<kWave>(v);
    m = group_max<kWave>(m);
    a = group_isum<kWave>(a);
    b = group_isum<kWave>(b);
    sse = v;
    maxerr = m;
    sa = a;
    sb = b;
  }
}

// One tile of sampled blocks through the ZFP side; writes zpart[t].
template <typename T, int D>
__device__ inline void zfp_tile(const ReqDesc &r, int t, int minexp, TileLds &L) {
  constexpr int BS = 1 << (2 * D), BPW = kWave / BS;
  const T *x = (const T *)r.field;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int i = lane & (BS - 1), bw = lane / BS;
  const int perm_i = Order<D>::table.perm[i];
  const int inv_i = Order<D>::table.inv[i];
  const int rounds = r.tile / (kWaves * BPW);
  const int64_t base = (int64_t)t * r.tile;
  for (int rd = 0; rd < rounds; rd++) {
    const int jl = (rd * kWaves + wave) * BPW + bw;
    const int64_t j = base + jl;
    const bool active = j < r.nblk;
    T xv = (T)0;
    if (active) {
      int64_t o[3], p[3];
      block_origin<D>(r, (uint32_t)j, o);
      point_coords<D>(o, i, p);
      xv = x[linear_index<D>(r, p)];
    }
    const ZfpBlockOut<T, D> z = zfp_block<T, D>(xv, minexp, perm_i, inv_i, lane);
    if (i == 0) {
      L.sse[jl] = active ? z.sse : 0.0;
      L.err[jl] = active ? z.maxerr : 0.0;
      L.a[jl] = active ? z.bits : 0u;
      L.b[jl] = active ? z.nsb : 0u;
      if (active && r.dbg_zbits) r.dbg_zbits[j] = z.bits;
      if (active && r.dbg_zsse) r.dbg_zsse[j] = z.sse;
      if (active && r.dbg_zemax) r.dbg_zemax[j] = z.emax;
    }
  }
  __syncthreads();
  double sse, maxerr;
  uint64_t sa, sb;
  tile_reduce(L, r.tile, sse, maxerr, sa, sb);
  if (threadIdx.x == 0) {
    TilePart p;
    p.sse = sse;
    p.maxerr = maxerr;
    p.bits = sa;
    p.cnt = sb;
    r.zpart[t] = p;
  }
  __syncthreads();
}

// Sum of the tiles' partials: SSE by the adjacent tree, integers exactly.
__device__ inline void tiles_total(const TilePart *part, int ntiles, double *sh, double &sse,
                                   double &maxerr, uint64_t &bits, uint64_t &cnt) {
  int64_t p = 1;
  while (p < ntiles) p <<= 1;
  const int64_t chunk = p > kThreads ? p / kThreads : 1;
  const int t = threadIdx.x;
  double stk[40];
  int sp = 0;
  double m = 0.0;
  uint64_t b = 0, c = 0;
  const int64_t beg = (int64_t)t * chunk;
  for (int64_t k = 0; k < chunk; k++) {
    const int64_t idx = beg + k;
    double v = 0.0;
    if (idx < ntiles) {
      const TilePart tp = part[idx];
      v = tp.sse;
      m = fmax(m, tp.maxerr);
      b += tp.bits;
      c += tp.cnt;
    }
    for (int64_t q = k; q & 1; q >>= 1) v = stk[--sp] + v;
    stk[sp++] = v;
  }
  double v = group_tree_sum<kWave>(stk[0]);
  m = group_max<kWave>(m);
  b = group_isum<kWave>(b);
  c = group_isum<kWave>(c);
  __shared__ double s_m[kWaves];
  __shared__ uint64_t s_b[kWaves], s_c[kWaves];
  const int w = t / kWave;
  if ((t & (kWave - 1)) == 0) {
    sh[w] = v;
    s_m[w] = m;
    s_b[w] = b;
    s_c[w] = c;
  }
  __syncthreads();
  sse = (sh[0] + sh[1]) + (sh[2] + sh[3]);
  maxerr = fmax(fmax(s_m[0], s_m[1]), fmax(s_m[2], s_m[3]));
  bits = s_b[0] + s_b[1] + s_b[2] + s_b[3];
  cnt = s_c[0] + s_c[1] + s_c[2] + s_c[3];
  __syncthreads();
}

// ZFP totals, PSNR_zfp and (for Algorithm 1) the SZ bin width delta whose
// uniform-error PSNR equals PSNR_zfp (Eq. 10 inverted: delta = sqrt(12 MSE)).
template <typename T, int D>
__device__ inline void zfp_finalize(const ReqDesc &r, double *sh) {
  double sse, maxerr;
  uint64_t bits, nsb;
  tiles_total(r.zpart, r.ntiles, sh, sse, maxerr, bits, nsb);
  if (threadIdx.x == 0) {
    constexpr int BS = 1 << (2 * D);
    ReqState *st = r.st;
    szsel_result *res = r.res;
    const double nv = (double)(r.nblk * BS);
    const double mse = sse / nv;
    res->zfp_sse = sse;
    res->zfp_mse = mse;
    res->zfp_bits = bits;
    res->zfp_values = (uint64_t)(r.nblk * BS);
    res->zfp_blocks = (uint64_t)r.nblk;
    res->zfp_nsb_total = nsb;
    res->zfp_nsb_mean = (double)nsb / nv;
    res->zfp_bitrate = (double)bits / nv;
    res->zfp_maxerr = maxerr;
    res->zfp_psnr = mse > 0.0 ? 20.0 * log10(st->vr) - 10.0 * log10(mse) : INFINITY;
    if (r.op == SZSEL_OP_SELECT) {
      double delta;
      if (mse > 0.0) {
        delta = sqrt(12.0 * mse);
      } else {
        delta = 2.0 * st->eb_abs;
        res->flags |= SZSEL_FLAG_ZERO_MSE;
      }
      st->delta = delta;
      st->inv = 1.0 / delta;
      st->eb_sz = 0.5 * delta;
    }
    st->zfp_done = 0;
  }
}

// ===========================================================================
// SZ side (Sections 4.1, 5.1): Lorenzo prediction from the original values,
// linear-scaling quantization, code histogram
// ===========================================================================

template <typename T, int D>
__device__ inline double lorenzo_pred(const T *x, const ReqDesc &r, const int64_t p[3]) {
  // terms: single axes (slowest first), then pairs in lexicographic order,
  // then the triple; values outside the field are 0
  if constexpr (D == 1) {
    return p[0] > 0 ? (double)x[p[0] - 1] : 0.0;
  } else if constexpr (D == 2) {
    const int64_t nx = r.dims[1];
    const int64_t c = p[0] * nx + p[1];
    const bool y = p[0] > 0, xo = p[1] > 0;
    const double v0 = y ? (double)x[c - nx] : 0.0;
    const double v1 = xo ? (double)x[c - 1] : 0.0;
    const double v01 = (y && xo) ? (double)x[c - nx - 1] : 0.0;
    return (v0 + v1) - v01;
  } else {
    const int64_t ny = r.dims[1], nx = r.dims[2];
    const int64_t sz = ny * nx;
    const int64_t c = (p[0] * ny + p[1]) * nx + p[2];
    const bool z = p[0] > 0, y = p[1] > 0, xo = p[2] > 0;
    const double v0 = z ? (double)x[c - sz] : 0.0;
    const double v1 = y ? (double)x[c - nx] : 0.0;
    const double v2 = xo ? (double)x[c - 1] : 0.0;
    const double v01 = (z && y) ? (double)x[c - sz - nx] : 0.0;
    const double v02 = (z && xo) ? (double)x[c - sz - 1] : 0.0;
    const double v12 = (y && xo) ? (double)x[c - nx - 1] : 0.0;
    const double v012 = (z && y && xo) ? (double)x[c - sz - nx - 1] : 0.0;
    return (((((v0 + v1) + v2) - v01) - v02) - v12) + v012;
  }
}

// Quantization code of one point (0 = unpredictable), its squared error and
// absolute error.  Round half away from zero; the point is unpredictable when
// |q| >= 32768 or when the reconstruction, rounded to the field precision,
// misses the bound delta/2.
template <typename T>
__device__ inline int quantize(T xv, double pred, double delta, double inv, double ebsz,
                               double &e2, double &ae) {
  const double xd = (double)xv;
  const double d = xd - pred;
  const double t = fabs(d) * inv + 0.5;
  e2 = 0.0;
  ae = 0.0;
  if (t < (double)kRadius) {
    int q = (int)floor(t);
    if (d < 0.0) q = -q;
    const T recon = (T)(pred + (double)q * delta);
    const double e = xd - (double)recon;
    if (fabs(e) <= ebsz) {
      e2 = e * e;
      ae = fabs(e);
      return q + kRadius;
    }
  }
  return 0;
}

// One tile of sampled blocks through the SZ side.  Codes go to the LDS
// window s_hist (or straight to the global histogram outside it); the caller
// flushes s_hist.  Writes spart[t].
template <typename T, int D>
__device__ inline void sz_tile(const ReqDesc &r, int t, double delta, double inv, double ebsz,
                               TileLds &L, uint32_t *s_hist) {
  constexpr int BS = 1 << (2 * D), BPW = kWave / BS;
  const T *x = (const T *)r.field;
  const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
  const int i = lane & (BS - 1), bw = lane / BS;
  const int rounds = r.tile / (kWaves * BPW);
  const int64_t base = (int64_t)t * r.tile;
  for (int rd = 0; rd < rounds; rd++) {
    const int jl = (rd * kWaves + wave) * BPW + bw;
    const int64_t j = base + jl;
    const bool active = j < r.nblk;
    int code = 0;
    double e2 = 0.0, ae = 0.0;
    if (active) {
      int64_t o[3], p[3];
      block_origin<D>(r, (uint32_t)j, o);
      point_coords<D>(o, i, p);
      const T xv = x[linear_index<D>(r, p)];
      const double pred = lorenzo_pred<T, D>(x, r, p);
      code = quantize<T>(xv, pred, delta, inv, ebsz, e2, ae);
      if (code) {
        const int w = code - kHistLo;
        if (w >= 0 && w < kHistWin)
          atomicAdd(&s_hist[w], 1u);
        else
          atomicAdd(&r.hist[code], 1u);
      }
      if (r.dbg_codes) r.dbg_codes[j * BS + i] = (uint16_t)code;
    }
    const double bsse = group_tree_sum<BS>(e2);
    const double berr = group_max<BS>(ae);
    const uint32_t unp = group_isum<BS>((uint32_t)(active && code == 0));
    if (i == 0) {
      L.sse[jl] = bsse;
      L.err[jl] = berr;
      L.a[jl] = unp;
      L.b[jl] = 0;
      if (active && r.dbg_ssse) r.dbg_ssse[j] = bsse;
    }
  }
  __syncthreads();
  double sse, maxerr;
  uint64_t sa, sb;
  tile_reduce(L, r.tile, sse, maxerr, sa, sb);
  if (threadIdx.x == 0) {
    TilePart p;
    p.sse = sse;
    p.maxerr = maxerr;
    p.bits = 0;
    p.cnt = sa;
    r.spart[t] = p;
  }
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

// Entropy of the code histogram (Eq. 5 with P_i = h_i/n), the SZ bit-rate
// (entropy + offset + W escape bits per unpredictable point, Section 6.2),
// both PSNRs, and the selection of Algorithm 1 (lower bit-rate, ties to ZFP).
// Leaves the global histogram zeroed for the next request.
template <typename T, int D>
__device__ inline void sz_finalize(const ReqDesc &r, double *sh) {
  constexpr int BS = 1 << (2 * D);
  double sse, maxerr;
  uint64_t dummy, unpred;
  tiles_total(r.spart, r.ntiles, sh, sse, maxerr, dummy, unpred);
  const double nv = (double)(r.nblk * BS);
  // sum over the 65536 bins of h log2 h, adjacent tree: thread t folds the
  // aligned chunk of 256 bins with a binary-counter pass
  constexpr int chunk = kBins / kThreads;
  const int t = threadIdx.x;
  double stk[12];
  int sp = 0;
  for (int k = 0; k < chunk; k++) {
    const int idx = t * chunk + k;
    const uint32_t h = idx == 0 ? (uint32_t)unpred : r.hist[idx];
    if (r.dbg_hist) r.dbg_hist[idx] = h;
    double v = 0.0;
    if (h) {
      const double hd = (double)h;
      v = hd * log2(hd);
      r.hist[idx] = 0;
    }
    for (int q = k; q & 1; q >>= 1) v = stk[--sp] + v;
    stk[sp++] = v;
  }
  double s = group_tree_sum<kWave>(stk[0]);
  const int w = t / kWave;
  __syncthreads();
  if ((t & (kWave - 1)) == 0) sh[w] = s;
  __syncthreads();
  if (t == 0) {
    s = (sh[0] + sh[1]) + (sh[2] + sh[3]);
    ReqState *st = r.st;
    szsel_result *res = r.res;
    const double H = log2(nv) - s / nv;
    double br = H + r.sz_offset;
    br = br + ((double)unpred * (double)Prec<T>::W) / nv;
    const double delta = st->delta;
    res->sz_delta = delta;
    res->sz_inv_delta = st->inv;
    res->sz_eb = st->eb_sz;
    res->sz_entropy = H;
    res->sz_bitrate = br;
    res->sz_sse = sse;
    res->sz_mse = sse / nv;
    res->sz_maxerr = maxerr;
    res->sz_values = (uint64_t)(r.nblk * BS);
    res->sz_unpredictable = unpred;
    res->sz_psnr_model = 20.0 * log10(st->vr / delta) + 10.0 * log10(12.0);
    res->sz_psnr_measured =
        res->sz_mse > 0.0 ? 20.0 * log10(st->vr) - 10.0 * log10(res->sz_mse) : INFINITY;
    if (r.op == SZSEL_OP_SELECT || r.op == SZSEL_OP_FIXED_EB) {
      res->choice = br < res->zfp_bitrate ? 0 : 1;
      res->chosen_eb = res->choice == 0 ? st->eb_sz : st->eb_abs;
      if (st->eb_sz > st->eb_abs) res->flags |= SZSEL_FLAG_EB_EXCEEDS;
    }
    st->sz_done = 0;
  }
  __syncthreads();
}

// Last-workgroup detection: returns true in every thread of the workgroup
// that completes `counter` to `total`.
__device__ inline bool last_to_finish(uint32_t *counter, uint32_t total, int *s_flag) {
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) *s_flag = atomicAdd(counter, 1u) == total - 1;
  __syncthreads();
  const bool last = *s_flag != 0;
  if (last) __threadfence();
  return last;
}

}  // namespace szsel
