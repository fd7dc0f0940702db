// Step 4 (Section 3; Algorithm 1's ZFP branch) for ZFP: fixed-accuracy compression
// of every block of the whole field at eb_abs into one bit stream, and the
// decompression that gives the true bit-rate and PSNR.
//
// Stream: bit i is bit (i mod 64) of 64-bit word i / 64.  Blocks follow in
// row-major block order over ceil(n_k / 4) blocks per axis; positions past
// the field's upper faces repeat the field's last value along that axis.
// A block is one bit (0: coded as zero, when all values are 0 or no plane
// is kept), or a 1, E bits of emax + 2^(E-1) - 1 (lowest first; emax at
// least 2 - 2^(E-1), the smallest normal exponent), and the group-testing
// code of planes W-1 .. W-prec, the coder whose bits the estimator counts.
//
// Passes (one block per lane): count each block's bits by running the
// coder without writing; exclusive scan of the counts (block offsets);
// emit every block at its offset (64-bit words, OR-ed in because a word
// can hold the end of one block and the start of the next); decode every
// block from the stream, write the decompressed field and the block's
// squared error; pair-tree sum of the block errors.
#include "compress.hpp"
#include "estimator.hpp"

namespace szsel {

namespace {

constexpr int kZcThreads = 64;     // one wave, one block per lane
constexpr int kScanThreads = 1024;
constexpr int kScanPer = 8;        // counts per thread in the scan
constexpr int kScanChunk = kScanThreads * kScanPer;
constexpr int kRedThreads = 1024;  // the tree reduction: 2 values per thread
constexpr int kRedChunk = 2 * kRedThreads;

// Origin of block jb (row-major over the block grid) and its values, with
// positions past the upper faces repeating the last value along that axis.
template <typename T, int D>
__device__ inline void zc_gather(const ZcArgs &a, int64_t jb, T (&x)[1 << (2 * D)], int64_t (&org)[3]) {
  constexpr int BS = 1 << (2 * D);
  int64_t rem = jb;
#pragma unroll
  for (int k = D - 1; k >= 0; k--) {
    org[k] = 4 * (rem % a.nb[k]);
    rem /= a.nb[k];
  }
  const T *f = (const T *)a.field;
#pragma unroll
  for (int i = 0; i < BS; i++) {
    int64_t lin = 0;
#pragma unroll
    for (int k = 0; k < D; k++) {
      const int off = (i >> (2 * (D - 1 - k))) & 3;
      int64_t p = org[k] + off;
      p = p < a.dims[k] ? p : a.dims[k] - 1;
      lin = lin * a.dims[k] + p;
    }
    x[i] = f[lin];
  }
}

// Block-floating-point exponent of the block (clamped to the smallest
// normal exponent), its coded planes, and its negabinary coefficients in
// coding order.  Returns false for a block coded as zero.
template <typename T, int D>
__device__ inline bool zc_coefficients(const T (&x)[1 << (2 * D)], int minexp, int &emax, int &prec,
                                       typename Prec<T>::U (&u)[1 << (2 * D)]) {
  using Q = Prec<T>;
  using U = typename Q::U;
  using I = typename Q::I;
  constexpr int BS = 1 << (2 * D);
  constexpr int W = Q::W;
  constexpr int kMinExp = 2 - (1 << (Q::E - 1));
  constexpr int kMaxExp = 1 << (Q::E - 1);  // largest finite exponent (NaN / Inf blocks are clamped)
  U mmax = 0;
#pragma unroll
  for (int i = 0; i < BS; i++) {
    const U m = Q::bits(x[i]) & ~(U(1) << (W - 1));
    mmax = m > mmax ? m : mmax;
  }
  if (mmax == 0) {
    emax = 0;
    prec = 0;
    return false;
  }
  emax = frexp_exponent_bits<T>(mmax);
  emax = emax < kMinExp ? kMinExp : (emax > kMaxExp ? kMaxExp : emax);
  prec = emax - minexp + 2 * (D + 1);
  prec = prec < 0 ? 0 : (prec > W ? W : prec);
  if (prec == 0) return false;
  I c[BS];
  const int sh = Q::P - emax;
  const float s1 = pow2f(sh < 127 ? sh : 127), s2 = pow2f(sh < 127 ? 0 : sh - 127);
#pragma unroll
  for (int i = 0; i < BS; i++) c[i] = bfp_value<T>(x[i], emax, s1, s2);
  fwd_xform<D>(c);
#pragma unroll
  for (int r = 0; r < BS; r++) u[r] = ((U)c[Order<D>::table.perm[r]] + Q::NB) ^ Q::NB;
  return true;
}

// Appends bits to the stream through a 64-bit accumulator; every word is
// OR-ed in (the first and last words of a block are shared with its
// neighbours; the stream starts zeroed).  With out == nullptr it counts.
struct BitWriter {
  uint64_t *out;
  uint64_t wi;    // word the accumulator belongs to
  uint64_t acc;
  int fill;       // bits in the accumulator
  uint64_t count;
  __device__ BitWriter(uint64_t *o, uint64_t bitpos) : out(o), wi(bitpos >> 6), acc(0), fill((int)(bitpos & 63)), count(0) {}
  // n in [0, 64], v < 2^n
  __device__ void put(uint64_t v, int n) {
    count += (uint64_t)n;
    if (!out || n == 0) return;
    acc |= v << fill;  // fill < 64
    if (fill + n >= 64) {
      atomicOr((unsigned long long *)(out + wi), (unsigned long long)acc);
      wi++;
      acc = fill ? (v >> (64 - fill)) : 0;
      fill = fill + n - 64;
    } else {
      fill += n;
    }
  }
  __device__ void flush() {
    if (out && fill > 0) atomicOr((unsigned long long *)(out + wi), (unsigned long long)acc);
  }
};

__device__ inline uint64_t low_mask(int n) { return n >= 64 ? ~0ull : ((1ull << n) - 1); }

// Group-testing code of planes W-1 .. W-prec of the coefficients u (coding
// order): per plane, the bits of the values already significant verbatim,
// then tests "is any later value 1 in this plane?" each followed by the
// plane's bits up to and including the next 1 (the last position's 1 is
// implied).
template <typename U, int BS>
__device__ inline void zc_encode_planes(const U (&u)[BS], int W, int prec, BitWriter &bw) {
  int n = 0;
  for (int k = W - 1; k >= W - prec; k--) {
    uint64_t pm = 0;
#pragma unroll
    for (int r = 0; r < BS; r++) pm |= (uint64_t)((u[r] >> k) & 1u) << r;
    bw.put(pm & low_mask(n), n);
    int p = n;
    while (p < BS) {
      const uint64_t rest = pm >> p;
      bw.put(rest ? 1u : 0u, 1);
      if (!rest) break;
      const int z = __builtin_ctzll(rest);
      if (p + z < BS - 1) {
        bw.put(1ull << z, z + 1);  // z zeros, then the 1
        p += z + 1;
      } else {
        bw.put(0, BS - 1 - p);     // zeros up to the last position, whose 1 is implied
        p = BS;
      }
      n = p;
    }
  }
}

template <typename T, int D>
__device__ inline void zc_encode_block(const ZcArgs &a, int64_t jb, BitWriter &bw) {
  using Q = Prec<T>;
  using U = typename Q::U;
  constexpr int BS = 1 << (2 * D);
  T x[BS];
  int64_t org[3];
  zc_gather<T, D>(a, jb, x, org);
  U u[BS];
  int emax, prec;
  if (!zc_coefficients<T, D>(x, a.minexp, emax, prec, u)) {
    bw.put(0, 1);
    return;
  }
  bw.put(1, 1);
  bw.put((uint64_t)(emax + (1 << (Q::E - 1)) - 1), Q::E);
  zc_encode_planes<U, BS>(u, Q::W, prec, bw);
}

template <typename T, int D>
__global__ __launch_bounds__(kZcThreads, 1) void k_zc_count(ZcArgs a) {
  const int64_t jb = (int64_t)blockIdx.x * kZcThreads + threadIdx.x;
  if (jb >= a.nblocks) return;
  BitWriter bw(nullptr, 0);
  zc_encode_block<T, D>(a, jb, bw);
  a.counts[jb] = (uint32_t)bw.count;
}

template <typename T, int D>
__global__ __launch_bounds__(kZcThreads, 1) void k_zc_emit(ZcArgs a) {
  const int64_t jb = (int64_t)blockIdx.x * kZcThreads + threadIdx.x;
  if (jb >= a.nblocks) return;
  BitWriter bw(a.stream, a.offsets[jb]);
  zc_encode_block<T, D>(a, jb, bw);
  bw.flush();
}

// Reads the stream from bit position bp; peek() returns the next 64 bits
// (the stream buffer has two spare words past the longest stream).
struct BitReader {
  const uint64_t *in;
  uint64_t bp;
  __device__ uint64_t peek() const {
    const uint64_t w = bp >> 6;
    const int s = (int)(bp & 63);
    const uint64_t lo = in[w];
    return s ? (lo >> s) | (in[w + 1] << (64 - s)) : lo;
  }
  __device__ uint64_t get(int n) {
    const uint64_t v = n ? peek() & low_mask(n) : 0;
    bp += (uint64_t)n;
    return v;
  }
};

// Decodes block jb; writes its values where the field is, and returns the
// pair-tree sum of its squared errors (zeros at padded positions).
template <typename T, int D>
__device__ inline double zc_decode_block(const ZcArgs &a, int64_t jb, double &maxerr, double &vmin,
                                         double &vmax, bool &bad) {
  using Q = Prec<T>;
  using U = typename Q::U;
  using I = typename Q::I;
  constexpr int BS = 1 << (2 * D);
  constexpr int W = Q::W;
  T x[BS];
  int64_t org[3];
  zc_gather<T, D>(a, jb, x, org);
  BitReader br{a.stream, a.offsets[jb]};
  T xh[BS];
#pragma unroll
  for (int i = 0; i < BS; i++) xh[i] = (T)0;
  if (br.get(1)) {
    const int emax = (int)br.get(Q::E) - ((1 << (Q::E - 1)) - 1);
    int prec = emax - a.minexp + 2 * (D + 1);
    prec = prec < 0 ? 0 : (prec > W ? W : prec);
    U u[BS];
#pragma unroll
    for (int r = 0; r < BS; r++) u[r] = 0;
    int n = 0;
    for (int k = W - 1; k >= W - prec; k--) {
      uint64_t pm = br.get(n);
      int p = n;
      while (p < BS && br.get(1)) {
        const uint64_t ahead = br.peek() & low_mask(BS - 1 - p);
        if (ahead) {
          const int z = __builtin_ctzll(ahead);
          br.bp += (uint64_t)(z + 1);
          p += z;
        } else {
          br.bp += (uint64_t)(BS - 1 - p);
          p = BS - 1;
        }
        pm |= 1ull << p;
        p++;
        n = p;
      }
#pragma unroll
      for (int r = 0; r < BS; r++) u[r] |= (U)((pm >> r) & 1u) << k;
    }
    I c[BS];
#pragma unroll
    for (int r = 0; r < BS; r++) c[Order<D>::table.perm[r]] = (I)((u[r] ^ Q::NB) - Q::NB);
    inv_xform<D>(c);
#pragma unroll
    for (int i = 0; i < BS; i++) xh[i] = (T)ldexp((double)c[i], emax - Q::P);
  }
  // errors where the field is; the pair tree over the block's slots
  double e2[BS];
#pragma unroll
  for (int i = 0; i < BS; i++) {
    int64_t lin = 0;
    bool inside = true;
#pragma unroll
    for (int k = 0; k < D; k++) {
      const int off = (i >> (2 * (D - 1 - k))) & 3;
      const int64_t p = org[k] + off;
      inside = inside && p < a.dims[k];
      lin = lin * a.dims[k] + (p < a.dims[k] ? p : a.dims[k] - 1);
    }
    e2[i] = 0.0;
    if (inside) {
      const double e = (double)x[i] - (double)xh[i];
      e2[i] = e * e;
      maxerr = fmax(maxerr, fabs(e));
      vmin = fmin(vmin, (double)x[i]);
      vmax = fmax(vmax, (double)x[i]);
      bad = bad || !isfinite((double)x[i]);
      if (a.decoded) ((T *)a.decoded)[lin] = xh[i];
    }
  }
#pragma unroll
  for (int w = BS; w > 1; w >>= 1) {
#pragma unroll
    for (int i = 0; i < w / 2; i++) e2[i] = e2[2 * i] + e2[2 * i + 1];
  }
  return e2[0];
}

// Order-preserving map of a binary64 value onto unsigned integers (for
// atomic min / max).
__device__ inline uint64_t ordered_bits(double v) {
  const uint64_t b = (uint64_t)__double_as_longlong(v);
  return (b >> 63) ? ~b : (b | (1ull << 63));
}

template <typename T, int D>
__global__ __launch_bounds__(kZcThreads, 1) void k_zc_decode(ZcArgs a) {
  const int64_t jb = (int64_t)blockIdx.x * kZcThreads + threadIdx.x;
  double maxerr = 0.0, vmin = INFINITY, vmax = -INFINITY;
  bool bad = false;
  if (jb < a.nblocks) a.bsse[jb] = zc_decode_block<T, D>(a, jb, maxerr, vmin, vmax, bad);
  maxerr = group_max<kWave>(maxerr);
  vmin = group_min<kWave>(vmin);
  vmax = group_max<kWave>(vmax);
  const bool any_bad = __ballot(bad) != 0;
  if (threadIdx.x == 0) {
    if (any_bad) atomicOr((unsigned long long *)&a.res->nonfinite, 1ull);
    atomicMax((unsigned long long *)&a.res->maxerr_bits, (unsigned long long)ordered_bits(maxerr));
    atomicMin((unsigned long long *)&a.res->vmin_bits, (unsigned long long)ordered_bits(vmin));
    atomicMax((unsigned long long *)&a.res->vmax_bits, (unsigned long long)ordered_bits(vmax));
  }
}

// Exclusive scan of the block counts: each chunk of kScanChunk counts in
// one workgroup (thread-sequential runs of kScanPer, then the workgroup's
// prefix), chunk totals scanned by one workgroup, then added back.
__device__ inline uint64_t block_exscan_u64(uint64_t v, uint64_t *slots, uint64_t &total) {
  constexpr int NW = kScanThreads / kWave;
  const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
  uint64_t inc = v;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const uint64_t o = __shfl_up(inc, d);
    if (lane >= d) inc += o;
  }
  if (lane == kWave - 1) slots[w] = inc;
  __syncthreads();
  uint64_t pre = 0, tot = 0;
#pragma unroll
  for (int q = 0; q < NW; q++) {
    const uint64_t x = slots[q];
    pre += q < w ? x : 0;
    tot += x;
  }
  total = tot;
  return pre + inc - v;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_chunks(ZcArgs a) {
  __shared__ uint64_t slots[kScanThreads / kWave];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanPer;
  uint32_t v[kScanPer];
  uint64_t sum = 0;
#pragma unroll
  for (int k = 0; k < kScanPer; k++) {
    v[k] = base + k < a.nblocks ? a.counts[base + k] : 0u;
    sum += v[k];
  }
  uint64_t total;
  uint64_t pre = block_exscan_u64(sum, slots, total);
#pragma unroll
  for (int k = 0; k < kScanPer; k++) {
    if (base + k < a.nblocks) a.offsets[base + k] = pre;
    pre += v[k];
  }
  if (threadIdx.x == 0) a.chunk[blockIdx.x] = total;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_totals(ZcArgs a, int64_t nchunks) {
  __shared__ uint64_t slots[kScanThreads / kWave];
  uint64_t carry = 0;
  for (int64_t b0 = 0; b0 < nchunks; b0 += kScanThreads) {
    const int64_t i = b0 + threadIdx.x;
    const uint64_t v = i < nchunks ? a.chunk[i] : 0;
    uint64_t total;
    const uint64_t pre = block_exscan_u64(v, slots, total);
    if (i < nchunks) a.chunk[i] = carry + pre;
    carry += total;
    __syncthreads();
  }
  if (threadIdx.x == 0) a.res->bits = carry;
}

__global__ __launch_bounds__(kScanThreads) void k_scan_add(ZcArgs a) {
  const uint64_t add = a.chunk[blockIdx.x];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk;
  for (int k = threadIdx.x; k < kScanChunk; k += kScanThreads)
    if (base + k < a.nblocks) a.offsets[base + k] += add;
}

// One level of the pair-tree sum: aligned groups of kRedChunk values (zeros
// past n) to one value each.
__global__ __launch_bounds__(kRedThreads) void k_tree_level(const double *in, int64_t n, double *out) {
  __shared__ double s[kRedThreads];
  const int64_t i = (int64_t)blockIdx.x * kRedChunk + 2 * threadIdx.x;
  const double a0 = i < n ? in[i] : 0.0, a1 = i + 1 < n ? in[i + 1] : 0.0;
  s[threadIdx.x] = a0 + a1;
  __syncthreads();
  // each level reads all its pairs before any is overwritten: the slots a
  // level writes are read by other waves in the same level
  for (int w = kRedThreads / 2; w > 0; w >>= 1) {
    double v = 0.0;
    if ((int)threadIdx.x < w) v = s[2 * threadIdx.x] + s[2 * threadIdx.x + 1];
    __syncthreads();
    if ((int)threadIdx.x < w) s[threadIdx.x] = v;
    __syncthreads();
  }
  if (threadIdx.x == 0) out[blockIdx.x] = s[0];
}

__global__ void k_fill_u64(uint64_t *p, int64_t n, uint64_t v) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

template <typename T, int D>
hipError_t zc_typed(const ZcArgs &a, hipStream_t s) {
  const dim3 g((unsigned)((a.nblocks + kZcThreads - 1) / kZcThreads));
  hipLaunchKernelGGL((k_zc_count<T, D>), g, dim3(kZcThreads), 0, s, a);
  const int64_t nchunks = (a.nblocks + kScanChunk - 1) / kScanChunk;
  hipLaunchKernelGGL(k_scan_chunks, dim3((unsigned)nchunks), dim3(kScanThreads), 0, s, a);
  hipLaunchKernelGGL(k_scan_totals, dim3(1), dim3(kScanThreads), 0, s, a, nchunks);
  hipLaunchKernelGGL(k_scan_add, dim3((unsigned)nchunks), dim3(kScanThreads), 0, s, a);
  hipLaunchKernelGGL((k_zc_emit<T, D>), g, dim3(kZcThreads), 0, s, a);
  hipLaunchKernelGGL((k_zc_decode<T, D>), g, dim3(kZcThreads), 0, s, a);
  // pair tree over the block errors, level by level (ping-pong in `red`)
  const double *in = a.bsse;
  int64_t n = a.nblocks;
  double *bufs[2] = {a.red, a.red + a.red_half};
  int k = 0;
  do {
    const int64_t m = (n + kRedChunk - 1) / kRedChunk;
    hipLaunchKernelGGL(k_tree_level, dim3((unsigned)m), dim3(kRedThreads), 0, s, in, n, bufs[k]);
    in = bufs[k];
    k ^= 1;
    n = m;
  } while (n > 1);
  return hipMemcpyAsync(&a.res->sse, in, sizeof(double), hipMemcpyDeviceToDevice, s);
}

}  // namespace

size_t zc_stream_words(int64_t nblocks, int nd, int dtype) {
  const int W = dtype == SZSEL_F32 ? 32 : 64, E = dtype == SZSEL_F32 ? 8 : 11;
  const int BS = 1 << (2 * nd);
  // per block: flag, exponent, and per plane at most n verbatim bits plus
  // one test and one bit per remaining position
  const uint64_t per_block = 1 + (uint64_t)E + (uint64_t)W * (2 * (uint64_t)BS + 1);
  return (size_t)((nblocks * per_block + 63) / 64 + 2);  // spare words for the reader's look-ahead
}

size_t zc_red_half(int64_t nblocks) { return (size_t)((nblocks + kRedChunk - 1) / kRedChunk) + 1; }
size_t zc_chunks(int64_t nblocks) { return (size_t)((nblocks + kScanChunk - 1) / kScanChunk) + 1; }

hipError_t zc_launch(const ZcArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_u64, dim3(1024), dim3(256), 0, s, a.stream, (int64_t)a.stream_words, (uint64_t)0);
  // result: maxerr 0, vmin +inf, vmax -inf (as ordered bits)
  hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(1), 0, s, (uint64_t *)&a.res->maxerr_bits, (int64_t)1,
                     (uint64_t)0x8000000000000000ull);
  hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(1), 0, s, (uint64_t *)&a.res->vmin_bits, (int64_t)1,
                     (uint64_t)0xFFF0000000000000ull);
  hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(1), 0, s, (uint64_t *)&a.res->vmax_bits, (int64_t)1,
                     (uint64_t)0x000FFFFFFFFFFFFFull);
  hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(1), 0, s, (uint64_t *)&a.res->nonfinite, (int64_t)1, (uint64_t)0);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (a.dtype == SZSEL_F32) {
    switch (a.nd) {
      case 1: e = zc_typed<float, 1>(a, s); break;
      case 2: e = zc_typed<float, 2>(a, s); break;
      default: e = zc_typed<float, 3>(a, s); break;
    }
  } else {
    switch (a.nd) {
      case 1: e = zc_typed<double, 1>(a, s); break;
      case 2: e = zc_typed<double, 2>(a, s); break;
      default: e = zc_typed<double, 3>(a, s); break;
    }
  }
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

// ===========================================================================
// Step 4 for SZ: Lorenzo prediction from decompressed values, made parallel
// by quantizing first (every value to the nearest multiple of 2 eb in
// units, q; the decompressed neighbours are then q 2 eb exactly, so the
// prediction from them is the integer Lorenzo sum of their q).  The code
// q - L(q) is a symbol when it is below 32768 in magnitude and q 2 eb, in
// the field's precision, is within eb of the value; otherwise the value is
// stored raw (symbol 0, the escape).  Size: the optimal prefix code of the
// symbols (the Huffman pass), W bits per escape, and 32 bits per distinct
// symbol for the code table.
// ===========================================================================
namespace {

constexpr int kSz4Threads = 256;
constexpr int kSz4Rounds = 256;                 // rounds of 256 consecutive points
constexpr int64_t kSz4Chunk = (int64_t)kSz4Threads * kSz4Rounds;  // points per workgroup
constexpr int kSz4Win = 16384;                  // LDS window of symbols around code 0
constexpr int kSz4WinLo = 32768 - kSz4Win / 2;

__device__ inline int64_t sz4_prequant(double x, double inv) {
  const double t = fabs(x) * inv + 0.5;
  if (!(t < 1125899906842624.0)) return 0;  // 2^50
  const int64_t q = (int64_t)floor(t);
  return x < 0.0 ? -q : q;
}

template <typename T, int D>
__device__ inline int64_t sz4_q_at(const SzArgs &a, const int64_t (&p)[3], int S) {
  // q of the neighbour p - e_S (0 outside the field)
  int64_t lin = 0;
#pragma unroll
  for (int k = 0; k < D; k++) {
    const int64_t c = p[k] - ((S >> k) & 1);
    if (c < 0) return 0;
    lin = lin * a.dims[k] + c;
  }
  return sz4_prequant((double)((const T *)a.field)[lin], a.inv);
}

template <typename T, int D>
__global__ __launch_bounds__(kSz4Threads) void k_sz4(SzArgs a) {
  __shared__ uint32_t win[kSz4Win];
  __shared__ double stk[2][kSz4Threads / kWave];
  __shared__ double lstk[8];
  for (int k = threadIdx.x; k < kSz4Win; k += kSz4Threads) win[k] = 0;
  __syncthreads();
  const int t = threadIdx.x, lane = t & (kWave - 1), w = t / kWave;
  const int64_t base = (int64_t)blockIdx.x * kSz4Chunk;
  uint32_t *gh = a.hist + (size_t)(blockIdx.x % kSzCopies) * kBins;
  uint32_t esc = 0;
  double maxerr = 0.0, vmin = INFINITY, vmax = -INFINITY;
  bool bad = false;
  double acc = 0.0;  // binary counter over the rounds (thread 0)
  for (int r = 0; r < kSz4Rounds; r++) {
    const int64_t i = base + (int64_t)r * kSz4Threads + t;
    double e2 = 0.0;
    if (i < a.n) {
      int64_t p[3];
      int64_t rem = i;
#pragma unroll
      for (int k = D - 1; k >= 0; k--) {
        p[k] = rem % a.dims[k];
        rem /= a.dims[k];
      }
      const T xv = ((const T *)a.field)[i];
      const double x = (double)xv;
      const int64_t q = sz4_prequant(x, a.inv);
      int64_t pred = 0;
#pragma unroll
      for (int S = 1; S < (1 << D); S++) {
        const int card = __builtin_popcount(S);
        const int64_t v = sz4_q_at<T, D>(a, p, S);
        pred = (card & 1) ? pred + v : pred - v;
      }
      const int64_t code = q - pred;
      const T recon = (T)((double)q * a.delta);
      int sym = 0;
      T xh = xv;
      if (code > -32768 && code < 32768 && fabs(x - (double)recon) <= a.eb) {
        sym = (int)code + 32768;
        xh = recon;
      }
      if (sym == 0) {
        esc++;
      } else {
        const int wi = sym - kSz4WinLo;
        if (wi >= 0 && wi < kSz4Win)
          atomicAdd(&win[wi], 1u);
        else
          atomicAdd(&gh[sym], 1u);
      }
      const double e = x - (double)xh;
      e2 = e * e;
      maxerr = fmax(maxerr, fabs(e));
      vmin = fmin(vmin, x);
      vmax = fmax(vmax, x);
      bad = bad || !isfinite(x);
      if (a.decoded) ((T *)a.decoded)[i] = xh;
      if (a.symbols) a.symbols[i] = (uint16_t)sym;
    }
    // the round's 256 squared errors as an aligned pair tree, folded into
    // the chunk's subtree by a binary counter over the rounds
    e2 = group_tree_sum<kWave>(e2);
    if (lane == 0) stk[r & 1][w] = e2;
    __syncthreads();
    if (t == 0) {
      double v = (stk[r & 1][0] + stk[r & 1][1]) + (stk[r & 1][2] + stk[r & 1][3]);
      for (int l = 0; l < 8; l++) {
        if ((r >> l) & 1) {
          v = lstk[l] + v;
        } else {
          lstk[l] = v;
          break;
        }
      }
      if (r == kSz4Rounds - 1) acc = v;
    }
  }
  __syncthreads();
  for (int k = threadIdx.x; k < kSz4Win; k += kSz4Threads)
    if (win[k]) atomicAdd(&gh[kSz4WinLo + k], win[k]);
  esc = group_isum<kWave>(esc);
  maxerr = group_max<kWave>(maxerr);
  vmin = group_min<kWave>(vmin);
  vmax = group_max<kWave>(vmax);
  const bool any_bad = __ballot(bad) != 0;
  if (lane == 0) {
    if (any_bad) atomicOr((unsigned long long *)&a.res->nonfinite, 1ull);
    atomicAdd((unsigned long long *)&a.res->escapes, (unsigned long long)esc);
    atomicMax((unsigned long long *)&a.res->maxerr_bits, (unsigned long long)ordered_bits(maxerr));
    atomicMin((unsigned long long *)&a.res->vmin_bits, (unsigned long long)ordered_bits(vmin));
    atomicMax((unsigned long long *)&a.res->vmax_bits, (unsigned long long)ordered_bits(vmax));
  }
  if (t == 0) a.chunk_sse[blockIdx.x] = acc;
}

// Final counts: the copies summed, the escapes in bin 0.
__global__ void k_sz4_combine(SzArgs a) {
  const int b = blockIdx.x * blockDim.x + threadIdx.x;
  if (b >= kBins) return;
  uint32_t h = 0;
#pragma unroll
  for (int c = 0; c < kSzCopies; c++) h += a.hist[(size_t)c * kBins + b];
  a.hfinal[b] = b == 0 ? (uint32_t)a.res->escapes : h;
}

// Optimal code bits and sum h log2 h of the final counts (one workgroup).
// The run list holds 16,384 runs (any histogram of up to 2^27 values); a
// round's new runs go to the histogram copies, no longer needed once the
// final counts are combined (they are cleared at the start of every call).
constexpr int kSz4HuffCap = 16384;
__global__ __launch_bounds__(kHuffThreads) void k_sz4_huff(SzArgs a) {
  __shared__ HuffLdsT<kSz4HuffCap, false> S;
  __shared__ double wsum[kHuffThreads / kWave];
  __shared__ uint32_t wsym[kHuffThreads / kWave];
  // sum of h log2 h: the pair tree over the 65,536 bins (64 per thread)
  constexpr int kPer = kBins / kHuffThreads;
  const int t = threadIdx.x;
  double stkv[8];
  double v = 0.0;
  uint32_t nsym = 0;
  for (int k = 0; k < kPer; k++) {
    const uint32_t h = a.hfinal[t * kPer + k];
    nsym += h ? 1u : 0u;
    const double hd = (double)h;
    double x = h ? hd * log2(hd) : 0.0;
    for (int l = 0; l < 6; l++) {
      if ((k >> l) & 1) {
        x = stkv[l] + x;
      } else {
        stkv[l] = x;
        break;
      }
    }
    if (k == kPer - 1) v = x;
  }
  v = group_tree_sum<kWave>(v);
  nsym = group_isum<kWave>(nsym);
  if ((t & (kWave - 1)) == 0) {
    wsum[t / kWave] = v;
    wsym[t / kWave] = nsym;
  }
  __syncthreads();
  uint64_t total;
  static_assert((size_t)kSzCopies * kBins >= 2 * (size_t)kSz4HuffCap, "room for the new runs");
  const bool ok = huff_cost(a.hfinal, (uint64_t)a.n, S, a.hist, a.hist + kSz4HuffCap, total);
  if (t == 0) {
    double w16[kHuffThreads / kWave];
    for (int q = 0; q < kHuffThreads / kWave; q++) w16[q] = wsum[q];
    for (int m = kHuffThreads / kWave; m > 1; m >>= 1)
      for (int q = 0; q < m / 2; q++) w16[q] = w16[2 * q] + w16[2 * q + 1];
    a.res->hsum = w16[0];
    a.res->code_bits = ok ? total : 0;
    a.res->huff_ok = ok ? 1 : 0;
    uint64_t syms = 0;
    for (int q = 0; q < kHuffThreads / kWave; q++) syms += wsym[q];
    a.res->symbols = syms;
  }
}

template <typename T, int D>
hipError_t sz4_typed(const SzArgs &a, hipStream_t s) {
  hipLaunchKernelGGL((k_sz4<T, D>), dim3((unsigned)a.nchunks), dim3(kSz4Threads), 0, s, a);
  hipLaunchKernelGGL(k_sz4_combine, dim3(kBins / 256), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_sz4_huff, dim3(1), dim3(kHuffThreads), 0, s, a);
  const double *in = a.chunk_sse;
  int64_t n = a.nchunks;
  double *bufs[2] = {a.red, a.red + a.red_half};
  int k = 0;
  do {
    const int64_t m = (n + kRedChunk - 1) / kRedChunk;
    hipLaunchKernelGGL(k_tree_level, dim3((unsigned)m), dim3(kRedThreads), 0, s, in, n, bufs[k]);
    in = bufs[k];
    k ^= 1;
    n = m;
  } while (n > 1);
  return hipMemcpyAsync(&a.res->sse, in, sizeof(double), hipMemcpyDeviceToDevice, s);
}

}  // namespace

size_t sz4_chunks(int64_t n) { return (size_t)((n + kSz4Chunk - 1) / kSz4Chunk); }

hipError_t sz4_launch(const SzArgs &a, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_u64, dim3(1024), dim3(256), 0, s, (uint64_t *)a.hist,
                     (int64_t)((size_t)kSzCopies * kBins / 2), (uint64_t)0);
  hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(64), 0, s, (uint64_t *)a.res,
                     (int64_t)(sizeof(SzResult) / 8), (uint64_t)0);
  hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(1), 0, s, (uint64_t *)&a.res->maxerr_bits, (int64_t)1,
                     (uint64_t)0x8000000000000000ull);
  hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(1), 0, s, (uint64_t *)&a.res->vmin_bits, (int64_t)1,
                     (uint64_t)0xFFF0000000000000ull);
  hipLaunchKernelGGL(k_fill_u64, dim3(1), dim3(1), 0, s, (uint64_t *)&a.res->vmax_bits, (int64_t)1,
                     (uint64_t)0x000FFFFFFFFFFFFFull);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (a.dtype == SZSEL_F32) {
    switch (a.nd) {
      case 1: e = sz4_typed<float, 1>(a, s); break;
      case 2: e = sz4_typed<float, 2>(a, s); break;
      default: e = sz4_typed<float, 3>(a, s); break;
    }
  } else {
    switch (a.nd) {
      case 1: e = sz4_typed<double, 1>(a, s); break;
      case 2: e = sz4_typed<double, 2>(a, s); break;
      default: e = sz4_typed<double, 3>(a, s); break;
    }
  }
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

}  // namespace szsel
