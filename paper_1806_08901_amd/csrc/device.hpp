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

#include <type_traits>

#include "szsel.h"

namespace szsel {

constexpr int kWave = 64;
constexpr int kThreads = 256;          // every kernel runs 4 waves per workgroup
constexpr int kWaves = kThreads / kWave;
constexpr int kBins = 65536;           // 65,535 symmetric bins plus the escape code 0
constexpr int kRadius = 32768;
constexpr int kMaxTile = 256;          // sampled blocks per tile
constexpr int kMaxParts = 8192;        // workgroups of one pass (partials per pass)
constexpr int kEntPerThread = 4;       // histogram bins per thread of the entropy pass
constexpr int kEntChunk = kThreads * kEntPerThread;  // bins per workgroup of the entropy pass
constexpr int kEntWgs = 65536 / kEntChunk;
constexpr int kOvfSlices = 64;         // overflow count: slices of the SZ workgroups ...
constexpr int kOvfRanges = 4;          // ... times code ranges of 16384 bins
constexpr int kOvfBins = kBins / kOvfRanges;
constexpr int kOvfThreads = 1024;      // threads of an overflow-pass workgroup (its LDS counts are 64 KiB)
constexpr int kHistCopies = 16;        // most global histogram copies (SZ workgroup w adds to copy w mod nhc)
constexpr int kOvfPerSlice = 65536;    // overflow codes per slice of the overflow count (default)
constexpr int kMaxBatch = 1024;        // requests per batch
constexpr int kGroup = 64;             // workgroups per completion group
constexpr int kMaxGroups = kMaxParts / kGroup;
enum { kPassRange = 0, kPassZfp = 1, kPassSz = 2, kPassEnt = 3, kPasses = 4 };
constexpr int kHuffThreads = 1024;     // threads of the Huffman pass (one workgroup per request)
constexpr int kHuffSmall = 8192;       // counts below this are tallied by value
constexpr int kHuffCap = 8192;         // runs of distinct weights held at once (and large counts)
constexpr int kHuffMaxRounds = 256;    // bound on the merge rounds (about 2 log2(total) are needed)

// Flags that stop the estimation after the range pass.
constexpr uint32_t kSkipFlags = SZSEL_FLAG_CONSTANT | SZSEL_FLAG_NONFINITE |
                                SZSEL_FLAG_NO_BLOCKS | SZSEL_FLAG_BAD_EB;

// A pointer into global memory.  The batched kernels read their buffers'
// addresses from the request table in memory, so the compiler cannot tell
// their address space and emits flat memory instructions; a flat access
// counts against the LDS counter as well, so every wait for an LDS result
// (the SZ histogram's atomics, a barrier) would also wait for the row loads
// prefetched for the next round.  Every buffer the kernels touch is device
// memory, so the hot paths read and write it through pointers typed as
// global, which lets the compiler use global loads and stores.
template <typename T>
using global_t = __attribute__((address_space(1))) T;
template <typename T>
__device__ __forceinline__ global_t<T> *to_global(T *p) {
  return (global_t<T> *)p;
}

// 16-byte vector load from / zero store to global memory at a 16-byte
// aligned address.
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
template <typename P>
__device__ __forceinline__ uint4 load_u4(const global_t<P> *p) {
  const u32x4 v = *(const global_t<u32x4> *)p;
  return make_uint4(v[0], v[1], v[2], v[3]);
}
template <typename P>
__device__ __forceinline__ void zero_u4(global_t<P> *p) {
  *(global_t<u32x4> *)p = u32x4{0u, 0u, 0u, 0u};
}

// ---------------------------------------------------------------------------
// Cross-workgroup communication.  MI355X has 8 XCDs whose L2 caches are not
// coherent with each other; an agent-scope fence makes the whole L2 write
// back and costs ~0.2 us per workgroup, serialised.  Everything one
// workgroup hands to another (partials, counters, per-request state) is
// therefore accessed only through agent-scope atomics, which bypass the
// non-coherent caches, and a workgroup waits for its own memory operations
// to complete before it bumps a completion counter.
// ---------------------------------------------------------------------------
__device__ inline void put_u64(uint64_t *p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline uint64_t get_u64(const uint64_t *p) {
  return __hip_atomic_load(const_cast<uint64_t *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void put_u32(uint32_t *p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline uint32_t get_u32(const uint32_t *p) {
  return __hip_atomic_load(const_cast<uint32_t *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void put_f64(double *p, double v) {
  put_u64((uint64_t *)p, (uint64_t)__double_as_longlong(v));
}
__device__ inline double get_f64(const double *p) {
  return __longlong_as_double((long long)get_u64((const uint64_t *)p));
}
__device__ inline void put_i32(int32_t *p, int32_t v) { put_u32((uint32_t *)p, (uint32_t)v); }
__device__ inline int32_t get_i32(const int32_t *p) { return (int32_t)get_u32((const uint32_t *)p); }

// Blocks until every memory operation this thread issued has completed.
__device__ inline void wait_memory() { __builtin_amdgcn_s_waitcnt(0); }

// Per-request state shared by the kernels of one request (device memory).
struct alignas(64) ReqState {
  double vmin, vmax, vr, eb_abs;
  double delta, inv, eb_sz;
  double sz_sse, sz_maxerr;  // SZ totals handed from the SZ pass to the entropy pass
  uint64_t sz_unpred;
  uint64_t ovf_count;        // codes in the overflow regions (set by the SZ finalizer)
  int32_t minexp;
  uint32_t flags;
  uint32_t ovf_slices;       // slices the overflow pass counts them in (set by the SZ finalizer)
  uint64_t code_chunks;      // bit c: some code fell in bins [1024 c, 1024 c + 1024)
};

// Completion counters of one pass.  Atomics on one address (one 128-byte
// line) serialise at about 11 ns each on this part, so thousands of
// workgroups counting on a single word would take tens of microseconds:
// workgroups count in groups of kGroup, each group on its own line, and the
// last workgroup of each group counts on `top`.  Every counter is reset by
// the workgroup that completes it.
struct alignas(128) LineCtr {
  uint32_t v;
};
struct PassSync {
  LineCtr top;
  LineCtr group[kMaxGroups];
};

// One entry per workgroup (or completion group) of a pass, structure of
// arrays.
struct Parts {
  double *sse;   // ZFP/SZ: squared-error subtree; range: min; entropy: h log2 h subtree
  double *err;   // ZFP/SZ: max |error|;            range: max
  uint64_t *a;   // ZFP: coder bits; SZ: unpredictable points; range: non-finite flag
  uint64_t *b;   // ZFP: significant bits; SZ: overflow codes
};

// Everything a kernel needs about one request (passed by value).
struct ReqDesc {
  const void *field;
  int64_t dims[3];
  int64_t n;       // number of values
  int64_t nblk;    // number of sampled blocks
  uint32_t nsel[3];
  uint32_t dmul[3];    // nsel[k] division by multiply-shift (Granlund-Montgomery)
  uint32_t dsh[3];     // shift pair: (sh1) | (sh2 << 8)
  int32_t stride[3];
  int64_t nboff[7];    // element offsets of the Lorenzo neighbours, in predictor term order
  int32_t nd, dtype, op, eb_mode;
  double eb, sz_offset;
  int32_t zblk;    // sampled blocks per ZFP workgroup (power of two, >= 64: one per lane)
  int32_t nzfp;    // ZFP workgroups = ceil(nblk / zblk)
  int32_t sblk;    // sampled blocks per SZ workgroup (power of two)
  int32_t nsz;     // SZ workgroups
  int64_t rchunk;  // values per range workgroup (multiple of 16 bytes)
  int32_t nrange;  // range workgroups
  int32_t vec;     // 1: every row of 4 values starts 16-byte aligned (vector loads)
  int32_t nshare;  // batches: requests right after this one in the table that share its range scan
  int32_t nhc;     // global histogram copies in use (power of two <= kHistCopies)
  int32_t huff;    // 0 no Huffman cost, 1 report it, 2 report and select with it
  int32_t ec;      // ZFP side: 0 exact, 1 point sub-sampling, 2 sub-sampling with gain weights
  int32_t ovf_per_slice;  // overflow codes per slice of the overflow pass (>= 1)
  int32_t pad0;
  ReqState *st;
  PassSync *sync;  // kPasses completion trees
  Parts rp, zp, sp;
  Parts ep;        // entropy pass: one h log2 h subtree per 256-bin chunk (sse slot)
  Parts grp[kPasses];  // per pass, the partials of its completion groups
  uint16_t *ovf;       // per SZ workgroup, sblk * 4^d codes that fell outside its LDS window
  uint32_t *ovf_hist;  // 65536-bin counts of the overflow codes (added to by the overflow
                       // pass, read and cleared by the entropy pass)
  uint32_t *hist;      // kHistCopies x 65536 counts, left zeroed by the entropy pass
  uint32_t *hfinal;    // the final 65536 counts, for the Huffman pass
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
__device__ inline V group_min(V v) {
#pragma unroll
  for (int s = 1; s < WIDTH; s <<= 1) {
    V o = __shfl_xor(v, s);
    v = o < v ? o : v;
  }
  return v;
}

template <int WIDTH, typename V>
__device__ inline V group_isum(V v) {
#pragma unroll
  for (int s = 1; s < WIDTH; s <<= 1) v += __shfl_xor(v, s);
  return v;
}

// ---------------------------------------------------------------------------
// Cross-lane moves without the LDS crossbar: DPP within rows of 16 lanes.
// Lane maps (checked on the device): quad_perm picks within each aligned
// group of 4 lanes, row_shl:s reads lane i+s of the same row.
// ---------------------------------------------------------------------------
constexpr int kDppQuad1233 = 0xF9;   // quad_perm [1,2,3,3]: shift down 1 in a quad
constexpr int kDppQuad2323 = 0xEE;   // quad_perm [2,3,2,3]: shift down 2 in a quad
constexpr int kDppQuadXor1 = 0xB1;   // quad_perm [1,0,3,2]: lane q reads lane q ^ 1
constexpr int kDppQuadXor2 = 0x4E;   // quad_perm [2,3,0,1]: lane q reads lane q ^ 2
constexpr int kDppQuadBcast3 = 0xFF; // quad_perm [3,3,3,3]: every lane reads the quad's last
constexpr int kDppRowShl1 = 0x101, kDppRowShl2 = 0x102, kDppRowShl4 = 0x104, kDppRowShl8 = 0x108;

// Lanes whose source lies outside the row read 0 (bound_ctrl); every use
// below either never reads such lanes or is neutral to 0.
template <int CTRL>
__device__ inline uint32_t dpp(uint32_t v) {
  return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, CTRL, 0xf, 0xf, true);
}
template <int CTRL>
__device__ inline uint64_t dpp(uint64_t v) {
  return (uint64_t)dpp<CTRL>((uint32_t)v) | ((uint64_t)dpp<CTRL>((uint32_t)(v >> 32)) << 32);
}
template <int CTRL>
__device__ inline double dpp(double v) {
  return __longlong_as_double((long long)dpp<CTRL>((uint64_t)__double_as_longlong(v)));
}

// Adjacent-pair tree over each aligned group of W lanes (the association of
// the tree over the group's values in lane order).  The result is valid in
// the group's first lane (in every lane for W = 64).
template <int W>
__device__ inline double group_tree_first(double v) {
  static_assert(W == 2 || W == 4 || W == 8 || W == 16 || W == 64, "group of 2, 4, 8, 16 or 64 lanes");
  if constexpr (W == 4) {
    v = v + dpp<kDppQuad1233>(v);
    v = v + dpp<kDppQuad2323>(v);
    return v;
  } else {
    v = v + dpp<kDppRowShl1>(v);
    if constexpr (W >= 8) {
      v = v + dpp<kDppRowShl2>(v);
      v = v + dpp<kDppRowShl4>(v);
    }
    if constexpr (W >= 16) v = v + dpp<kDppRowShl8>(v);
    if constexpr (W == 64) {
      const uint64_t b = (uint64_t)__double_as_longlong(v);
      auto rd = [&](int l) {
        const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, l);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), l);
        return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
      };
      v = (rd(0) + rd(16)) + (rd(32) + rd(48));
    }
    return v;
  }
}

// Sampled blocks one wave of the SZ pass takes per round: one lane per two
// rows of 4 points in 2-D and 3-D (8 and 2 lanes per block), one lane per
// block in 1-D.
__host__ __device__ constexpr int sz_blocks_per_wave(int nd) { return nd == 1 ? 64 : (nd == 2 ? 32 : 8); }

// ---------------------------------------------------------------------------
// Sampled-block addressing
// ---------------------------------------------------------------------------
// n / d for the divisor whose (multiplier, shifts) the host precomputed:
// t = mulhi(m, n), q = (t + ((n - t) >> sh1)) >> sh2.
__device__ inline uint32_t fast_div(uint32_t n, uint32_t m, uint32_t sh) {
  const uint32_t t = __umulhi(m, n);
  return (t + ((n - t) >> (sh & 0xff))) >> (sh >> 8);
}

template <int D>
__device__ inline void block_origin(const ReqDesc &r, uint32_t j, int64_t o[3]) {
  // row-major over the sampled-block lattice, last axis fastest
#pragma unroll
  for (int k = D - 1; k >= 0; k--) {
    const uint32_t q = k > 0 ? fast_div(j, r.dmul[k], r.dsh[k]) : 0u;
    const uint32_t jk = j - q * r.nsel[k];
    j = q;
    o[k] = 4 * (int64_t)jk * r.stride[k];
  }
}

// Linear index of the first point of sampled block j, and its coordinates.
template <int D>
__device__ inline int64_t block_base(const ReqDesc &r, uint32_t j, int64_t o[3]) {
  block_origin<D>(r, j, o);
  int64_t lin = o[0];
#pragma unroll
  for (int k = 1; k < D; k++) lin = lin * r.dims[k] + o[k];
  return lin;
}

// Offset of in-block point i from the block's first point.
template <int D>
__device__ inline int64_t point_offset(const ReqDesc &r, int i) {
  if constexpr (D == 1) return i;
  else if constexpr (D == 2) return (int64_t)(i >> 2) * r.dims[1] + (i & 3);
  else return ((int64_t)(i >> 4) * r.dims[1] + ((i >> 2) & 3)) * r.dims[2] + (i & 3);
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
