// gfx950 kernels of the progressive compressor.  Wave64 throughout: in the
// bitplane codec each lane owns one 64-code word and moves between codes and
// plane words with in-register bit-matrix transposes; sign bits of newly
// significant codes are placed through per-(plane, word) cursors in LDS.
//
// Every kernel walks a table of segments (field x level x region) in
// 4096-element work blocks with a persistent block loop, so one launch serves
// any number of fields; index arithmetic uses multiply-high division.
//
// Floating point: every interpolation is evaluated in float64 with exactly
// the operation order of the stencil definitions (the library is built with
// -ffp-contract=off, so no multiply-add is fused).  Codes are exact integers.
#include <algorithm>
#include <type_traits>

#include "apc_internal.h"

namespace apc {

namespace {

constexpr int kThreads = 256;

// Global-memory pointers: the tables hand out generic pointers, and loads
// through them would compile to flat instructions (which also wait on LDS
// traffic); every kernel re-types them into the global address space.
#define GAS __attribute__((address_space(1)))

// Raw buffer access: a wave-uniform base address and byte range held in
// scalar registers plus a 32-bit per-lane byte offset.  The hardware range
// check returns 0 for loads past the range and drops stores past it, which
// stands in for per-lane bounds tests.  Dword 3 of the descriptor selects the
// 32-bit data format (raw loads and stores ignore it, a zero format would mark
// the buffer invalid).
using BufRsrc = __amdgpu_buffer_rsrc_t;
typedef uint32_t u32x2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ BufRsrc buf_rsrc(const void* p, int64_t bytes) {
  const int64_t b = bytes < 0 ? 0 : (bytes > 0x7fffffff ? 0x7fffffff : bytes);
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(p), (short)0, (int)b, 0x00020000);
}
template <typename V>
__device__ __forceinline__ V buf_load(BufRsrc r, uint32_t voff, uint32_t soff) {
  if constexpr (sizeof(V) == 4) {
    const uint32_t x = __builtin_amdgcn_raw_buffer_load_b32(r, (int)voff, (int)soff, 0);
    return __builtin_bit_cast(V, x);
  } else {
    const u32x2 x = __builtin_amdgcn_raw_buffer_load_b64(r, (int)voff, (int)soff, 0);
    return __builtin_bit_cast(V, x);
  }
}
// A wave-uniform 64-bit value (held in vector registers) moved to scalar ones.
__device__ __forceinline__ int64_t readfirst64(int64_t v) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
template <typename V>
__device__ __forceinline__ void buf_store(V v, BufRsrc r, uint32_t voff, uint32_t soff) {
  if constexpr (sizeof(V) == 4)
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(uint32_t, v), r, (int)voff, (int)soff, 0);
  else
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, (int)voff, (int)soff, 0);
}
constexpr int kPerThread = kBlockElems / kThreads;  // 16
constexpr unsigned kMaxGrid = 4096;

enum { ST_COPY = 0, ST_LINEAR = 1, ST_LQUAD = 2, ST_RQUAD = 3, ST_CUBIC = 4 };

__device__ __forceinline__ uint32_t fdiv(uint32_t n, const FastDiv& f) {
  return f.one ? n : (uint32_t)__umul64hi(f.M, (uint64_t)n);
}

__device__ __forceinline__ int node_of(int t, int kind) {
  return kind == AX_ODD ? 2 * t + 1 : (kind == AX_EVEN ? 2 * t : t);
}
__device__ __forceinline__ int lat_of(int i, int kind) {
  return kind == AX_ODD ? (i - 1) >> 1 : (kind == AX_EVEN ? i >> 1 : i);
}

// Stencil choice for odd index j on an axis of m points (Section IV: cubic
// where four neighbours exist, quadratic with three, linear with two, copy
// with one).
__device__ __forceinline__ int stencil_kind(int j, int m, int degree) {
  if (j + 1 > m - 1) return ST_COPY;
  if (degree == 1) return ST_LINEAR;
  const bool left = j - 3 >= 0;
  const bool right = j + 3 <= m - 1;
  if (left && right) return ST_CUBIC;
  if (right) return ST_LQUAD;
  if (left) return ST_RQUAD;
  return ST_LINEAR;
}

// tap(o) returns the neighbour at offset o in {-3, -1, 1, 3}; only the taps
// the stencil uses are read.
template <typename F>
__device__ __forceinline__ double stencil_eval(int kind, F tap) {
  switch (kind) {
    case ST_CUBIC: {
      const double a = tap(-3), b = tap(-1), c = tap(1), e = tap(3);
      const double t1 = b + c;
      const double t2 = a + e;
      return (9.0 * t1 - t2) * 0.0625;
    }
    case ST_LQUAD: {
      const double b = tap(-1), c = tap(1), e = tap(3);
      return ((3.0 * b + 6.0 * c) - e) * 0.125;
    }
    case ST_RQUAD: {
      const double a = tap(-3), b = tap(-1), c = tap(1);
      return ((6.0 * b + 3.0 * c) - a) * 0.125;
    }
    case ST_LINEAR: {
      const double b = tap(-1), c = tap(1);
      return (b + c) * 0.5;
    }
    default:
      return tap(-1) * 1.0;
  }
}

// The same stencils with all four taps given, every form evaluated and the
// one of `kind` selected: no branches where the kind varies across a wave
// (each form keeps its own operation order, so results are bit-equal).
__device__ __forceinline__ double stencil_select(int kind, double a, double b, double c, double e) {
  const double cub = (9.0 * (b + c) - (a + e)) * 0.0625;
  const double lq = ((3.0 * b + 6.0 * c) - e) * 0.125;
  const double rq = ((6.0 * b + 3.0 * c) - a) * 0.125;
  const double lin = (b + c) * 0.5;
  return kind == ST_CUBIC ? cub : (kind == ST_LQUAD ? lq : (kind == ST_RQUAD ? rq : (kind == ST_LINEAR ? lin : b)));
}

__device__ __forceinline__ uint64_t lanemask_lt(int lane) {
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

__device__ __forceinline__ int bitlen64(uint64_t v) { return v ? 64 - __clzll((long long)v) : 0; }

template <typename Q>
__device__ __forceinline__ uint64_t absq(Q q) {
  return q < 0 ? (uint64_t)(-(int64_t)q) : (uint64_t)q;
}

// 32-bit part p of a code's magnitude (an int32 code's magnitude fits 32 bits).
__device__ __forceinline__ uint32_t mag_part(int32_t q, int) { return q < 0 ? 0u - (uint32_t)q : (uint32_t)q; }
__device__ __forceinline__ uint32_t mag_part(int64_t q, int p) { return (uint32_t)(absq(q) >> (32 * p)); }
// Lead byte of a code for the sign pass: 0x80 | plane << 1 | negative, where
// plane = B - bit length of the magnitude is where the code becomes
// significant; 0 for a zero code.
__device__ __forceinline__ uint32_t code_lead(int32_t q, int B) {
  const uint32_t m = mag_part(q, 0);
  const uint32_t v = 0x80u | (((uint32_t)(B - 32 + __clz((int)m)) & 63u) << 1) | ((uint32_t)q >> 31);
  return m ? v : 0u;
}
__device__ __forceinline__ uint32_t code_lead(int64_t q, int B) {
  const uint64_t m = absq(q);
  const uint32_t v = 0x80u | (((uint32_t)(B - bitlen64(m)) & 63u) << 1) | (uint32_t)((uint64_t)q >> 63);
  return m ? v : 0u;
}

// Unsigned type that holds a code's magnitude, and bit lengths.
template <typename Q> struct MagOf { using type = uint64_t; };
template <> struct MagOf<int32_t> { using type = uint32_t; };
__device__ __forceinline__ int bitlen_of(uint32_t v) { return 32 - __clz((int)v); }
__device__ __forceinline__ int bitlen_of(uint64_t v) { return bitlen64(v); }

// Codes truncated to the first k of B planes (magnitude bits below plane k
// cleared, sign kept), through a mask on the magnitude computed once per
// segment: zero when k <= 0 or B <= 0 (a stream without planes is never
// decoded, so its code buffer may hold anything), all ones when k >= B.
template <typename Q> struct UOf { using type = uint64_t; };
template <> struct UOf<int32_t> { using type = uint32_t; };
template <typename Q>
__device__ __forceinline__ typename UOf<Q>::type code_mask(int B, int k) {
  using U = typename UOf<Q>::type;
  if (k <= 0 || B <= 0) return (U)0;
  if (k >= B) return ~(U)0;
  return ~(U)0 << (B - k);  // 1 <= B - k < bits of U
}
// Apply a magnitude mask to a sign-magnitude code held in two's complement
// (branch-free: s is 0 or all ones, (x ^ s) - s negates when s is set).
template <typename Q>
__device__ __forceinline__ Q apply_mask(Q q, typename UOf<Q>::type m) {
  using U = typename UOf<Q>::type;
  const U s = (U)(q >> (8 * sizeof(Q) - 1));
  const U mag = ((U)q ^ s) - s;
  return (Q)(((mag & m) ^ s) - s);
}
template <typename Q>
__device__ __forceinline__ Q mask_code(Q q, int B, int k) {
  return apply_mask<Q>(q, code_mask<Q>(B, k));
}

__device__ __forceinline__ double block_max(double v) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  __shared__ double sm[kThreads / 64];
  __syncthreads();
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = v;
  __syncthreads();
  double m = sm[0];
  for (int w = 1; w < kThreads / 64; ++w) m = fmax(m, sm[w]);
  return m;
}

__device__ __forceinline__ unsigned long long ordered_bits(double d) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(d);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

// Inclusive prefix sum over the 64 lanes of a wave with DPP moves: shifts by
// 1, 2, 4, 8 inside each row of 16 lanes (zero shifted in), then the last
// lane of row 0 is added to row 1 and of row 2 to row 3 (row_bcast:15), and
// the last lane of row 1 to rows 2 and 3 (row_bcast:31).
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v, int lane) {
  (void)lane;
  int x = (int)v;
  x += __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, true);  // row_shr:1
  x += __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, true);  // row_shr:2
  x += __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, true);  // row_shr:4
  x += __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, true);  // row_shr:8
  x += __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false); // row_bcast:15 into rows 1, 3
  x += __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false); // row_bcast:31 into rows 2, 3
  return (uint32_t)x;
}

// The same prefix sum over N independent values per lane, one DPP step at a
// time across all N, so consecutive DPP reads never wait on the VALU write
// just before them.
template <int CTRL, int ROWS, bool BC, int N>
__device__ __forceinline__ void wave_scan_step(uint32_t (&x)[N]) {
#pragma unroll
  for (int i = 0; i < N; ++i) x[i] += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x[i], CTRL, ROWS, 0xf, BC);
}
template <int N>
__device__ __forceinline__ void wave_incl_scan_n(uint32_t (&x)[N]) {
  wave_scan_step<0x111, 0xf, true>(x);
  wave_scan_step<0x112, 0xf, true>(x);
  wave_scan_step<0x114, 0xf, true>(x);
  wave_scan_step<0x118, 0xf, true>(x);
  wave_scan_step<0x142, 0xa, false>(x);
  wave_scan_step<0x143, 0xc, false>(x);
}

// Workgroups go to the device's 8 XCDs in turn (workgroup i to XCD i mod 8,
// also for the blocks a grid-stride loop takes on, the grid being a multiple
// of 8 or the whole table), and every XCD has an L2 of its own.  This
// renumbers the n blocks of one segment so that runs of g consecutive tiles
// go to one XCD, the runs dealt to the XCDs in turn: neighbouring tiles of a
// run then meet each other's halo reads in that L2 instead of fetching them
// again, while all XCDs still work on one window of the segment at a time
// (ranges far apart, a power of two bytes from each other, would meet in
// the same memory channels).  A bijection of [0, n): block lb is the i-th
// of its class x = lb mod 8; blocks past the last whole round of 8 runs keep
// their number.
__device__ __forceinline__ int64_t xcd_local(int64_t lb, int64_t n, int64_t g) {
  constexpr int64_t kXcd = 8;
  const int64_t whole = n / (kXcd * g) * (kXcd * g);
  if (lb >= whole) return lb;
  const int64_t x = lb % kXcd, i = lb / kXcd;
  return ((i / g) * kXcd + x) * g + i % g;
}

// Segment of global work block b (segments are sorted by blk_begin).
template <typename S>
__device__ __forceinline__ int find_seg(const S* segs, int nseg, int64_t b) {
  int lo = 0, hi = nseg - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (segs[mid].blk_begin <= b)
      lo = mid;
    else
      hi = mid - 1;
  }
  return __builtin_amdgcn_readfirstlane(lo);
}

__device__ __forceinline__ int64_t lat_count(const Lattice& L) { return (int64_t)L.c[0] * L.c[1] * L.c[2]; }

// Lattice element e -> node coordinates.
__device__ __forceinline__ void lattice_node(const Lattice& L, uint32_t e, int i[3]) {
  const uint32_t r = fdiv(e, L.f2);
  const int t2 = (int)(e - r * (uint32_t)L.c[2]);
  const uint32_t t0 = fdiv(r, L.f1);
  const int t1 = (int)(r - t0 * (uint32_t)L.c[1]);
  i[0] = node_of((int)t0, L.kind[0]);
  i[1] = node_of(t1, L.kind[1]);
  i[2] = node_of(t2, L.kind[2]);
}

// The region a neighbour point belongs to: the last earlier region whose
// axis coordinate is odd; -1 = a point of the next coarser level.
__device__ __forceinline__ int source_region(const RegionArgs& ra, const int i[3]) {
  int rp = -1;
  for (int r = 0; r < ra.rho; ++r)
    if (i[ra.sigma[r]] & 1) rp = r;
  return rp;
}

// Neighbour values held in the buffer of an earlier region (its lattice is
// "even" along this region's axis).
__device__ __forceinline__ double predict_from_region(const RegionArgs& ra, int rp, const int i[3], int ax, int j,
                                                      int sk) {
  // rp differs between lanes: read both regions' (uniform) descriptors and
  // select, rather than indexing the table per lane
  const Lattice& P0 = ra.prl[0];
  const Lattice& P1 = ra.prl[1];
  const bool r1 = rp == 1;
  int tt[3];
  for (int a = 0; a < 3; ++a) tt[a] = (a == ax) ? (j - 1) >> 1 : lat_of(i[a], r1 ? P1.kind[a] : P0.kind[a]);
  const int64_t c1 = r1 ? P1.c[1] : P0.c[1], c2 = r1 ? P1.c[2] : P0.c[2];
  const int64_t ls[3] = {c1 * c2, c2, 1};
  const GAS double* pp =
      (const GAS double*)(r1 ? ra.pr[1] : ra.pr[0]) + tt[0] * ls[0] + tt[1] * ls[1] + tt[2] * ls[2];
  const int64_t st = ls[ax];
  return stencil_eval(sk, [&](int o) { return pp[((o + 1) / 2) * st]; });
}

inline unsigned grid_for(int64_t nblk) { return (unsigned)std::min<int64_t>(nblk, (int64_t)kMaxGrid); }

// Running maximum / minimum / union of a value that only moves one way: the
// current value is read first and the atomic is issued only when it would
// change it, so the many blocks whose partial result is already covered do
// not queue on one contended address.  A stale read only costs an atomic
// that was not needed.
__device__ __forceinline__ void max_u64(unsigned long long* p, unsigned long long v) {
  if (v > *(volatile unsigned long long*)p) atomicMax(p, v);
}
__device__ __forceinline__ void min_u64(unsigned long long* p, unsigned long long v) {
  if (v < *(volatile unsigned long long*)p) atomicMin(p, v);
}
__device__ __forceinline__ void or_u64(unsigned long long* p, unsigned long long v) {
  if ((*(volatile unsigned long long*)p & v) != v) atomicOr(p, v);
}

// Exponent alignment of a quantization group, P - E, where E is the binary
// exponent of the group's largest |coefficient| M (M = m 2^E, 1/2 <= m < 1)
// as the max pass left it in the group's accumulator (double bits); 0 for
// an all-zero group.  P = 29 bits for float32 input, 52 for float64.  The
// host derives the same value from the same accumulator for the metadata.
template <typename T>
__device__ __forceinline__ int group_k_shift(const unsigned long long* gmax) {
  constexpr int P = sizeof(T) == 4 ? 29 : 52;
  const double M = __longlong_as_double((long long)*gmax);
  if (!(M > 0.0)) return 0;
  int E;
  (void)frexp(M, &E);
  return P - E;
}

// ------------------------------------------------------------- range pass
template <typename T>
__global__ __launch_bounds__(kThreads) void k_range(const FlatSeg* __restrict__ segs, int nseg, int64_t nblk) {
  int cur = -1;
  double lo = INFINITY, hi = -INFINITY, am = 0.0;
  bool bad = false;
  __shared__ unsigned long long sbad;
  auto flush = [&](int si) {
    const double l = -block_max(-lo), h = block_max(hi), a = block_max(am);
    if (threadIdx.x == 0) sbad = 0;
    __syncthreads();
    if (bad) atomicOr(&sbad, 1ull);
    __syncthreads();
    if (threadIdx.x == 0) {
      unsigned long long* acc = segs[si].acc;
      if (l <= h) {
        min_u64(&acc[0], ordered_bits(l));
        max_u64(&acc[1], ordered_bits(h));
      }
      max_u64(&acc[2], (unsigned long long)__double_as_longlong(a));
      if (sbad) or_u64(&acc[3], 1ull);
    }
  };
  for (int64_t b = blockIdx.x; b < nblk; b += gridDim.x) {
    const int si = find_seg(segs, nseg, b);
    if (si != cur) {
      if (cur >= 0) flush(cur);
      cur = si;
      lo = INFINITY;
      hi = -INFINITY;
      am = 0.0;
      bad = false;
    }
    const FlatSeg& S = segs[si];
    const GAS T* x = (const GAS T*)S.src;
    const int64_t e0 = (b - S.blk_begin) * kBlockElems;
    auto take = [&](double v) {
      if (!isfinite(v)) {
        bad = true;
      } else {
        lo = fmin(lo, v);
        hi = fmax(hi, v);
        am = fmax(am, fabs(v));
      }
    };
    constexpr int VW = 16 / sizeof(T);  // elements per 16-byte load
    if (e0 + kBlockElems <= S.n && (((uintptr_t)(x + e0)) & 15) == 0) {
      typedef T vec_t __attribute__((ext_vector_type(VW)));
      const GAS vec_t* xv = (const GAS vec_t*)(x + e0);
      vec_t r[kPerThread / VW];
#pragma unroll
      for (int it = 0; it < kPerThread / VW; ++it) r[it] = xv[it * kThreads + threadIdx.x];
#pragma unroll
      for (int it = 0; it < kPerThread / VW; ++it)
#pragma unroll
        for (int c = 0; c < VW; ++c) take((double)r[it][c]);
    } else {
#pragma unroll 4
      for (int it = 0; it < kPerThread; ++it) {
        const int64_t e = e0 + it * kThreads + threadIdx.x;
        if (e < S.n) take((double)x[e]);
      }
    }
  }
  if (cur >= 0) flush(cur);
}

// ------------------------------------- strided gather (compact level grids)
template <typename T>
__global__ __launch_bounds__(kThreads) void k_gather(const FlatSeg* __restrict__ segs, int nseg, int64_t nblk) {
  for (int64_t b = blockIdx.x; b < nblk; b += gridDim.x) {
    const int si = find_seg(segs, nseg, b);
    const FlatSeg& S = segs[si];
    const GAS T* src = (const GAS T*)S.src;
    GAS T* dst = (GAS T*)S.dst;
    const int64_t e0 = (b - S.blk_begin) * kBlockElems;
    for (int it = 0; it < kPerThread; ++it) {
      const int64_t e = e0 + it * kThreads + threadIdx.x;
      if (e < S.n) {
        const uint32_t r = fdiv((uint32_t)e, S.f2);
        const uint32_t i2 = (uint32_t)e - r * (uint32_t)S.dm[2];
        const uint32_t i0 = fdiv(r, S.f1);
        const uint32_t i1 = r - i0 * (uint32_t)S.dm[1];
        dst[e] = src[i0 * S.s[0] + i1 * S.s[1] + i2 * S.s[2]];
      }
    }
  }
}

// ------------------------------------------- refactor: coefficients of a region
// MODE 0: max |c| into the group maximum.  MODE 1: q = rint(c * 2^k_shift).
// Per-level: the predictions of this region are stored in pr_out for the
// regions after it; neighbours in earlier regions are their predictions.
// Per-region: every neighbour is an original value (no pre-quantization).
template <typename T, typename Q, int MODE>
__global__ __launch_bounds__(kThreads) void k_coef(const CoefSeg* __restrict__ segs, int nseg, int64_t nblk) {
  int cur = -1;
  double am = 0.0;
  int kq = 0, kseg = -1;
  for (int64_t b = blockIdx.x; b < nblk; b += gridDim.x) {
    const int si = find_seg(segs, nseg, b);
    if (MODE == 0 && si != cur) {
      if (cur >= 0) {
        const double m = block_max(am);
        if (threadIdx.x == 0) max_u64(segs[cur].gmax, (unsigned long long)__double_as_longlong(m));
      }
      cur = si;
      am = 0.0;
    }
    const CoefSeg& S = segs[si];
    if (MODE == 1 && si != kseg) {  // the group's shift, read once per segment
      kq = group_k_shift<T>(S.gmax);
      kseg = si;
    }
    const RegionArgs& ra = S.ra;
    const Lattice& L = ra.lat;
    const GAS T* G = (const GAS T*)S.G;
    const int64_t total = lat_count(L);
    const int64_t e0 = (b - S.blk_begin) * kBlockElems;
    const int ax = L.ax;
    const int64_t gs[3] = {(int64_t)L.m[1] * L.m[2], (int64_t)L.m[2], 1};
#pragma unroll 4
    for (int it = 0; it < kPerThread; ++it) {
      const int64_t e = e0 + it * kThreads + threadIdx.x;
      if (e >= total) continue;
      int i[3];
      lattice_node(L, (uint32_t)e, i);
      const int j = i[ax];
      const int sk = stencil_kind(j, L.m[ax], ra.degree);
      const int64_t gbase = i[0] * gs[0] + i[1] * gs[1] + i[2] * gs[2];
      const double xv = (double)G[gbase];
      const int rp = ra.per_level ? source_region(ra, i) : -1;
      double p;
      if (rp < 0) {
        const GAS T* g = G + gbase;
        const int64_t st = gs[ax];
        p = stencil_eval(sk, [&](int o) { return (double)g[o * st]; });
      } else {
        p = predict_from_region(ra, rp, i, ax, j, sk);
      }
      if (ra.pr_out) ((GAS double*)ra.pr_out)[e] = p;
      const double c = xv - p;
      if (MODE == 0)
        am = fmax(am, fabs(c));
      else
        ((GAS Q*)S.codes)[e] = (Q)(long long)rint(ldexp(c, kq));
    }
  }
  if (MODE == 0 && cur >= 0) {
    const double m = block_max(am);
    if (threadIdx.x == 0) max_u64(segs[cur].gmax, (unsigned long long)__double_as_longlong(m));
  }
}

// ------------------------------------------------- per-level tensor-product pass
// Per-level interpolation predicts every point of level l from the coarser
// level by one-dimensional stencils along axis 2, then axis 1, then axis 0,
// each pass reading the predictions of the previous one (tensor product).
// A block owns a kT1 x kT2 tile of (axis 1, axis 2) and walks a run of up
// to 128 planes along axis 0 (shorter runs on small levels, for
// parallelism): each coarse plane is upsampled in-plane through LDS (axis 2,
// then axis 1) into registers, a four-plane register window gives the
// axis-0 stencil, and every point of the level is visited once.  The coarse
// tile of the next plane is fetched one step ahead and the point values (or
// codes) of the current planes before the plane's LDS passes (a whole step
// ahead in the quantization and reconstruction passes of 4-byte inputs), so
// their latency overlaps the LDS passes.  Stencils are selected without
// branches, and outside the max pass the loads are issued on every lane.
// MODE 0: max |x - p| of the level.  MODE 1: codes q = rint(c * 2^k_shift)
// into the three region lattices.  MODE 2: x = p + Delta * q' on the level
// grid (coarse points are copied), written as float64 for the next level;
// MODE 3: the same for level 0, written as the output field (type T).
// Tile shapes: kT2 columns (axis 2) by kT1 = 4 * (256 / kT2) rows (axis 1);
// every thread owns one column and four consecutive rows.  Levels with a
// single plane along axis 0 come presented as m1 x m2 x 1 and take
// one-column tiles (kT2 = 1: 1024 rows, contiguous in memory); there a
// thread owns two pairs of adjacent rows half a tile apart, so that a wave's
// loads of one of its points cover adjacent addresses.
// With 4-byte per-point inputs (float32 fields; codes of float32 fields),
// the quantization and reconstruction passes fetch a step's inputs one
// whole step ahead, at four waves per SIMD (the extra registers cost the
// fifth wave, which the max pass keeps: there the early fetch does not pay).
template <typename T, typename Q, int MODE>
constexpr bool level_ahead() {
  return MODE != 0 && (MODE >= 2 ? sizeof(Q) : sizeof(T)) == 4;
}
template <typename T, typename Q, int MODE, int kT2>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(
    (level_ahead<T, Q, MODE>() || sizeof(T) == 8) ? 4 : 5))) void k_level(const LevelSeg* __restrict__ segs, int nseg, int64_t nblk) {
  constexpr bool kCol = kT2 == 1;        // one-column tiles
  constexpr int kNRG = kThreads / kT2;  // row groups
  constexpr int kT1 = 4 * kNRG;
  constexpr int kC1 = kT1 / 2 + 3, kC2 = kCol ? 1 : kT2 / 2 + 3;
  constexpr int kCPer = (kC1 * kC2 + kThreads - 1) / kThreads;  // coarse tile entries per thread
  using V = typename std::conditional<MODE >= 2, Q, T>::type;  // per-point input: code or value
  __shared__ double ctile[kC1 * kC2];
  __shared__ double u2[kC1 * kT2];
  __shared__ int sbad;
  int cur = -1;
  double am = 0.0;
  // range of the field (max pass over level 0): min, max, max |x|, non-finite
  // seen; kept in the field's own type (exact: every value is one of the
  // field's values), which for float32 fields halves their registers
  T rlo = (T)INFINITY, rhi = (T)-INFINITY, ram = (T)0;
  bool rbad = false;
  auto take = [&](T v) {
    if (!isfinite(v)) {
      rbad = true;
    } else {
      rlo = fmin(rlo, v);
      rhi = fmax(rhi, v);
      ram = fmax(ram, fabs(v));
    }
  };
  auto flush = [&](int si) {
    const double m = block_max(am);
    if (threadIdx.x == 0) max_u64(segs[si].gmax, (unsigned long long)__double_as_longlong(m));
    unsigned long long* acc = segs[si].racc;
    if (acc) {
      const double l = -block_max(-(double)rlo), h = block_max((double)rhi), a = block_max((double)ram);
      if (threadIdx.x == 0) sbad = 0;
      __syncthreads();
      if (rbad) sbad = 1;
      __syncthreads();
      if (threadIdx.x == 0) {
        if (l <= h) {
          min_u64(&acc[0], ordered_bits(l));
          max_u64(&acc[1], ordered_bits(h));
        }
        max_u64(&acc[2], (unsigned long long)__double_as_longlong(a));
        if (sbad) or_u64(&acc[3], 1ull);
      }
    }
  };
  const int tid = threadIdx.x, col = tid % kT2, rg = tid / kT2;
  for (int64_t b = blockIdx.x; b < nblk; b += gridDim.x) {
    const int si = find_seg(segs, nseg, b);
    if (MODE == 0 && si != cur) {
      if (cur >= 0) flush(cur);
      cur = si;
      am = 0.0;
      rlo = (T)INFINITY, rhi = (T)-INFINITY, ram = (T)0;
      rbad = false;
    }
    const LevelSeg& S = segs[si];
    unsigned long long* const racc = S.racc;
    const int m0 = S.m[0], m1 = S.m[1], m2 = S.m[2];
    const int mc0 = S.mc[0], mc1 = S.mc[1], mc2 = S.mc[2];
    const int deg = S.degree;
    const int nrun = (m0 + S.ch - 1) / S.ch;
    int lb = (int)xcd_local(b - S.blk_begin, (int64_t)S.nt1 * S.nt2 * nrun, S.nt2);
    const int t2 = (lb % S.nt2) * kT2;
    lb /= S.nt2;
    const int t1 = (lb % S.nt1) * kT1;
    const int f0a = (lb / S.nt1) * S.ch;
    const int f0b = min(m0, f0a + S.ch);
    const int c1s = t1 / 2 - 1, c2s = kCol ? 0 : t2 / 2 - 1;
    // segment operands, held in registers (stores through the segment's
    // pointers must not force the table to be reloaded; a lane picks the
    // operands of its region)
    Q* const qr[3] = {(Q*)S.q[0], (Q*)S.q[1], (Q*)S.q[2]};
    using UM = typename UOf<Q>::type;
    const UM Mr[3] = {code_mask<Q>(S.B[0], S.k[0]), code_mask<Q>(S.B[1], S.k[1]), code_mask<Q>(S.B[2], S.k[2])};
    auto qptr = [&](int rr) -> GAS Q* { return (GAS Q*)(rr == 0 ? qr[0] : (rr == 1 ? qr[1] : qr[2])); };
    const void* const src = S.src;
    void* const outp = S.out;
    const int64_t xs0 = S.xs[0], xs1 = S.xs[1], xs2 = S.xs[2];
    constexpr bool fin = MODE == 3;  // level 0: the T output field
    const double delta = S.delta;
    const int kshift = MODE == 1 ? group_k_shift<T>(S.gmax) : 0;

    // in-plane geometry of this thread (constant along axis 0)
    const int f2 = t2 + col;
    const bool odd2 = !kCol && (f2 & 1);
    const int sk2 = odd2 ? stencil_kind(f2, m2, deg) : 0;
    const int tc2 = odd2 ? ((f2 - 1) >> 1) - c2s : (f2 >> 1) - c2s;  // coarse tile column of f2 (or left of it)
    // The thread's four points are on rows f1b + ro(i), i = 0..3, with f1b
    // even (tiles start on even rows) and ro(i) of the parity of i, so odd i
    // means an odd row.  Everything about point i is a cheap function of i
    // and a few per-thread values, recomputed where used instead of being
    // held in registers.
    const int f1b = t1 + (kCol ? 2 : 4) * rg;
    auto ro = [](int i) { return kCol ? (i >> 1) * (kT1 / 2) + (i & 1) : i; };
    const int sk1o[2] = {stencil_kind(f1b + ro(1), m1, deg), stencil_kind(f1b + ro(3), m1, deg)};
    auto sk1 = [&](int i) { return (i & 1) ? sk1o[i >> 1] : 0; };
    auto tr1 = [&](int i) { return (f1b >> 1) + (ro(i) >> 1) - c1s; };  // coarse tile row of the row (or above it)
    // offsets of the thread's four points, split into a per-plane part and a
    // part fixed along axis 0 (all below 2^32: fields hold < 2^32 points):
    // grid offset = f0 * m1 * m2 + rg2(i); region lattice index = c * P + R
    // with c = f0 / 2 (region 2 on odd planes; region 0 or 1, or a coarse
    // point, on even planes); source offset = f0 * xs0 + rsrc(i)
    const uint32_t pl2 = (uint32_t)m1 * (uint32_t)m2;
    const uint32_t rg2b = (uint32_t)f1b * (uint32_t)m2 + (uint32_t)f2;
    const uint32_t rsrcb = (uint32_t)((int64_t)f1b * xs1 + (int64_t)f2 * xs2);
    const uint32_t pe_odd = (uint32_t)(m1 >> 1) * (uint32_t)m2;                 // region 1 plane size
    const uint32_t pe_even = (uint32_t)((m1 + 1) >> 1) * (uint32_t)(m2 >> 1);  // region 0 plane size
    const uint32_t re_odd = (uint32_t)(f1b >> 1) * (uint32_t)m2 + (uint32_t)f2;
    const uint32_t re_even = (uint32_t)(f1b >> 1) * (uint32_t)(m2 >> 1) + (uint32_t)(f2 >> 1);
    auto okp = [&](int i) { return f1b + ro(i) < m1 && f2 < m2; };
    auto rg2 = [&](int i) { return rg2b + (uint32_t)ro(i) * (uint32_t)m2; };
    auto rsrc = [&](int i) { return rsrcb + (uint32_t)ro(i) * (uint32_t)xs1; };
    auto rre = [&](int i) { return (i & 1) ? 1 : (odd2 ? 0 : -1); };  // region on even planes (-1: coarse point)
    auto pe = [&](int i) { return (i & 1) ? pe_odd : pe_even; };
    auto re = [&](int i) {
      return (i & 1) ? re_odd + (uint32_t)(ro(i) >> 1) * (uint32_t)m2
                     : re_even + (uint32_t)(ro(i) >> 1) * (uint32_t)(m2 >> 1);
    };
    // coarse tile entries of this thread: global offsets within a plane (-1 = outside the grid)
    int64_t coff[kCPer];
#pragma unroll
    for (int k = 0; k < kCPer; ++k) {
      const int e = tid + k * kThreads;
      const int r = e / kC2, kk = e - r * kC2;
      const int c1 = c1s + r, c2 = c2s + kk;
      coff[k] = -1;
      if (e < kC1 * kC2 && c1 >= 0 && c1 < mc1 && c2 >= 0 && c2 < mc2)
        coff[k] = MODE >= 2 ? (int64_t)c1 * mc2 + c2 : (int64_t)(2 * c1) * xs1 + (int64_t)(2 * c2) * xs2;
    }
    const int64_t cplane = MODE >= 2 ? (int64_t)mc1 * mc2 : 2 * xs0;  // coarse plane stride
    // The next coarse tile, held as loaded (the field's type, or float64)
    // and converted, zeroed outside the grid and (max pass over level 0)
    // taken into the range when it goes to LDS, so that the load's wait
    // falls there and not right after the load.
    using CT = typename std::conditional<MODE <= 1, T, double>::type;
    CT cpre[kCPer];
    // Loads are issued on every lane, a lane without a point reading a
    // harmless address (the segment table) and dropping the value: branches
    // around per-lane loads cost more than the loads.
    const void* const safe = (const void*)segs;
    auto fetch_tile = [&](int cc) {
#pragma unroll
      for (int k = 0; k < kCPer; ++k) {
        const bool ok = coff[k] >= 0;
        const int64_t o = (int64_t)cc * cplane + coff[k];
        if (MODE == 0) {  // as in fetch_in
          cpre[k] = (T)0;
          if (ok) cpre[k] = ((const GAS T*)src)[o];
          continue;
        }
        if (MODE >= 2)
          cpre[k] = *(ok ? (const GAS double*)src + o : (const GAS double*)safe);
        else
          cpre[k] = *(ok ? (const GAS T*)src + o : (const GAS T*)safe);
      }
    };

    // prediction of coarse plane cc (its tile is in cpre) on the thread's
    // four points; fetches the tile of cc + 1.  Block-uniform call.
    auto plane = [&](int cc, double (&u)[4]) {
      // No barrier is needed before the tile is overwritten: its readers
      // (the previous plane's axis-2 pass) all passed that plane's last
      // barrier, and the readers of u2 (its axis-1 pass) pass the next one
      // before u2 is written again.
#pragma unroll
      for (int k = 0; k < kCPer; ++k) {
        if (MODE == 0 && racc && coff[k] >= 0) take(cpre[k]);
        if (tid + k * kThreads < kC1 * kC2) ctile[tid + k * kThreads] = coff[k] >= 0 ? (double)cpre[k] : 0.0;
      }
      if (cc + 1 < mc0) fetch_tile(cc + 1);
      __syncthreads();
#pragma unroll
      for (int k = 0; k < (kC1 + kNRG - 1) / kNRG; ++k) {
        const int r = rg + kNRG * k;
        if (r < kC1) {
          const double* row = ctile + r * kC2 + tc2;  // taps row[-1..2] lie inside the tile row
          const double b0 = row[0];
          u2[r * kT2 + col] = odd2 ? stencil_select(sk2, row[-1], b0, row[1], row[2]) : b0;
        }
      }
      __syncthreads();
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const double* cp = u2 + tr1(i) * kT2 + col;  // taps cp[-1..2 rows] lie inside the tile
        u[i] = (i & 1) ? stencil_select(sk1(i), cp[-kT2], cp[0], cp[kT2], cp[2 * kT2]) : cp[0];
      }
    };

    // inputs of the two fine planes 2c and 2c + 1 (codes, or the field's
    // values); fetched a whole step ahead (kAhead) into two buffers used in
    // turn, their latency is hidden behind a plane's LDS passes and the
    // emission of the current step
    constexpr bool kAhead = level_ahead<T, Q, MODE>();
    V in[8], nx[8];
    auto fetch_points = [&](int c, V (&dst)[8]) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int f0 = 2 * c + h;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int rr = h ? 2 : rre(i);
          const bool ok = f0 < f0b && okp(i) && rr >= 0;
          V x;
          if (MODE >= 2) {
            const int rho = h ? 2 : (i & 1);  // the region of this row (rr, where there is a point)
            const uint32_t li = (uint32_t)c * (h ? pl2 : pe(i)) + (h ? rg2(i) : re(i));
            x = (V) * (ok ? (const GAS Q*)qr[rho] + li : (const GAS Q*)safe);
          } else {
            x = (V) * (ok ? (const GAS T*)src + (int64_t)f0 * xs0 + rsrc(i) : (const GAS T*)safe);
          }
          dst[h * 4 + i] = ok ? x : (V)0;
        }
      }
    };
    // the same into in[] (a separate copy: sharing the one above costs the
    // max pass registers)
    auto fetch_in = [&](int c) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int f0 = 2 * c + h;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int rr = h ? 2 : rre(i);
          const bool ok = f0 < f0b && okp(i) && rr >= 0;
          if (MODE == 0) {  // the max pass keeps branches here (its registers are tight)
            in[h * 4 + i] = (V)0;
            if (ok) in[h * 4 + i] = (V)((const GAS T*)src)[(int64_t)f0 * xs0 + rsrc(i)];
            continue;
          }
          V x;
          if (MODE >= 2) {
            const int rho = h ? 2 : (i & 1);  // the region of this row (rr, where there is a point)
            const uint32_t li = (uint32_t)c * (h ? pl2 : pe(i)) + (h ? rg2(i) : re(i));
            x = (V) * (ok ? (const GAS Q*)qr[rho] + li : (const GAS Q*)safe);
          } else {
            x = (V) * (ok ? (const GAS T*)src + (int64_t)f0 * xs0 + rsrc(i) : (const GAS T*)safe);
          }
          in[h * 4 + i] = ok ? x : (V)0;
        }
      }
    };
    auto emit = [&](int f0, int i, double p, V v) {
      const int h = f0 & 1;
      if (f0 >= f0b || !okp(i)) return;
      const int rr = h ? 2 : rre(i);
      if (MODE >= 2) {
        double x = p;  // a coarse point keeps its reconstructed value
        if (rr >= 0) {
          const UM m = rr == 0 ? Mr[0] : (rr == 1 ? Mr[1] : Mr[2]);
          x = p + (double)apply_mask<Q>((Q)v, m) * delta;
        }
        const uint32_t o = (uint32_t)f0 * pl2 + rg2(i);
        if (fin)
          ((GAS T*)outp)[o] = (T)x;
        else
          ((GAS double*)outp)[o] = x;
      } else if (rr >= 0) {
        const double c = (double)v - p;
        if (MODE == 0 && racc) take((T)v);
        if (MODE == 0) {
          am = fmax(am, fabs(c));
        } else {
          const uint32_t li = (uint32_t)(f0 >> 1) * (h ? pl2 : pe(i)) + (h ? rg2(i) : re(i));
          qptr(rr)[li] = (Q)(long long)rint(ldexp(c, kshift));
        }
      }
    };

    double w0[4] = {}, w1[4] = {}, w2[4] = {}, w3[4] = {};  // predictions of coarse planes c-1, c, c+1, c+2
    const int cb = f0a >> 1;
    fetch_tile(max(cb - 1, 0));
    if (cb - 1 >= 0) plane(cb - 1, w0);
    plane(cb, w1);
    fetch_in(cb);
    if (cb + 1 < mc0) plane(cb + 1, w2);
    if (cb + 2 < mc0) plane(cb + 2, w3);
    // one step: fine planes 2c and 2c + 1 from the inputs in cur
    auto step = [&](int c, V (&cur)[8], V (&nxt)[8]) {
      fetch_points(c + 1, nxt);  // planes at or past f0b are not read
      if (c > cb) {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          w0[i] = w1[i];
          w1[i] = w2[i];
          w2[i] = w3[i];
        }
        if (c + 2 < mc0) plane(c + 2, w3);
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) emit(2 * c, i, w1[i], cur[i]);
      if (2 * c + 1 < f0b) {
        const int sk0 = stencil_kind(2 * c + 1, m0, deg);
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const double p = stencil_select(sk0, w0[i], w1[i], w2[i], w3[i]);
          emit(2 * c + 1, i, p, cur[4 + i]);
        }
      }
    };
    if constexpr (kAhead) {
      for (int c = cb; 2 * c < f0b; c += 2) {
        step(c, in, nx);
        if (2 * (c + 1) < f0b) step(c + 1, nx, in);
      }
    } else {
      for (int c = cb; 2 * c < f0b; ++c) {
        if (c > cb) {
          fetch_in(c);
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            w0[i] = w1[i];
            w1[i] = w2[i];
            w2[i] = w3[i];
          }
          if (c + 2 < mc0) plane(c + 2, w3);
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) emit(2 * c, i, w1[i], in[i]);
        if (2 * c + 1 < f0b) {
          const int sk0 = stencil_kind(2 * c + 1, m0, deg);
#pragma unroll
          for (int i = 0; i < 4; ++i) {
            const double p = stencil_select(sk0, w0[i], w1[i], w2[i], w3[i]);
            emit(2 * c + 1, i, p, in[4 + i]);
          }
        }
      }
    }
  }
  if (MODE == 0 && cur >= 0) flush(cur);
}

// Coarsest level: the values themselves are the coefficients.
template <typename T, typename Q, int MODE>
__global__ __launch_bounds__(kThreads) void k_coarse(const FlatSeg* __restrict__ segs, int nseg, int64_t nblk) {
  int cur = -1;
  double am = 0.0;
  int kq = 0, kseg = -1;
  for (int64_t b = blockIdx.x; b < nblk; b += gridDim.x) {
    const int si = find_seg(segs, nseg, b);
    if (MODE == 0 && si != cur) {
      if (cur >= 0) {
        const double m = block_max(am);
        if (threadIdx.x == 0) max_u64(segs[cur].acc, (unsigned long long)__double_as_longlong(m));
      }
      cur = si;
      am = 0.0;
    }
    const FlatSeg& S = segs[si];
    if (MODE == 1 && si != kseg) {  // the group's shift, read once per segment
      kq = group_k_shift<T>(S.acc);
      kseg = si;
    }
    const GAS T* G = (const GAS T*)S.src;
    const int64_t e0 = (b - S.blk_begin) * kBlockElems;
#pragma unroll 4
    for (int it = 0; it < kPerThread; ++it) {
      const int64_t e = e0 + it * kThreads + threadIdx.x;
      if (e >= S.n) continue;
      const double v = (double)G[e];
      if (MODE == 0)
        am = fmax(am, fabs(v));
      else
        ((GAS Q*)S.dst)[e] = (Q)(long long)rint(ldexp(v, kq));
    }
  }
  if (MODE == 0 && cur >= 0) {
    const double m = block_max(am);
    if (threadIdx.x == 0) max_u64(segs[cur].acc, (unsigned long long)__double_as_longlong(m));
  }
}

// ---------------------------------------------- coefficient decomposition

struct Rng1 {
  int64_t c4, c2, call;
};
__device__ __forceinline__ Rng1 rng_prefix(int64_t x) { return {(x + 3) / 4, (x + 1) / 2, x}; }
__device__ __forceinline__ Rng1 rng_single(int64_t y) {
  return {(y % 4 == 0) ? 1 : 0, (y % 2 == 0) ? 1 : 0, 1};
}
__device__ __forceinline__ int64_t cls_count(int cls, Rng1 ru, Rng1 rv) {
  const int64_t h2 = ru.c4 * rv.c4, h1 = ru.c2 * rv.c2, all = ru.call * rv.call;
  return cls == 0 ? h2 : (cls == 1 ? h1 - h2 : all - h1);
}
__device__ __forceinline__ int cd_class(int u, int v) {
  if ((u & 3) == 0 && (v & 3) == 0) return 0;
  if ((u & 1) == 0 && (v & 1) == 0) return 1;
  return 2;
}

// Row walk of a region lattice: each wave takes whole lattice rows (t0, t1)
// with lanes along t2, so the stacking axis a and the (u, v) plane give
// per-row (uniform) stream offsets and every class stream is written in runs.
constexpr int kCDRowsPerBlock = kThreads / 64;

// Elements of class cls before the start of row (t0, t1) in row-major
// lattice order, i.e. the rank of (t0, t1, 0) in the class-cls stream.
template <int A>
__device__ __forceinline__ int64_t cd_row_base(int c1, int c2, int cls, int t0, int t1) {
  if (A == 0)  // (a, u, v) = (t0, t1, t2)
    return (int64_t)t0 * cls_count(cls, rng_prefix(c1), rng_prefix(c2)) + cls_count(cls, rng_prefix(t1), rng_prefix(c2));
  if (A == 1)  // (u, a, v) = (t0, t1, t2)
    return (int64_t)c1 * cls_count(cls, rng_prefix(t0), rng_prefix(c2)) +
           (int64_t)t1 * cls_count(cls, rng_single(t0), rng_prefix(c2));
  // (u, v, a) = (t0, t1, t2): whole rows belong to one class
  return (int64_t)c2 * (cls_count(cls, rng_prefix(t0), rng_prefix(c1)) + cls_count(cls, rng_single(t0), rng_prefix(t1)));
}
template <int A>
__device__ __forceinline__ int64_t cd_row_base(const CDSeg& S, int cls, int t0, int t1) {
  return cd_row_base<A>(S.c[1], S.c[2], cls, t0, t1);
}
// Elements of class cls in the row before column t2 (u is the row's plane
// coordinate when v runs along the row).
template <int A>
__device__ __forceinline__ int64_t cd_in_row(int cls, int u, int t2) {
  if (A == 2) return t2;
  const int64_t u4 = (u & 3) == 0, u2 = (u & 1) == 0;
  const int64_t c4 = (t2 + 3) >> 2, c2 = (t2 + 1) >> 1;
  return cls == 0 ? u4 * c4 : (cls == 1 ? u2 * c2 - u4 * c4 : (int64_t)t2 - u2 * c2);
}

// Lifting arithmetic width: 32-bit codes stay below 2^30 in magnitude, so
// their sums and residuals fit in int32.
template <typename Q>
using LiftT = typename std::conditional<sizeof(Q) == 4, int32_t, int64_t>::type;

template <typename W>
__device__ __forceinline__ W avgw(W x, W y) { return (x + y) >> 1; }

// Neighbour pattern of a lifting prediction: rows r0 (and r1 if hr), columns
// c0 (and c1 if hc), in (u, v) offsets; the prediction averages over columns
// and then over rows (Section V).
struct CDNb {
  int r0, r1, c0, c1;
  bool hr, hc;
};
// S2 points from stride-4 (H2) neighbours at distance 2
__device__ __forceinline__ CDNb cd_nb_s2(int u, int v, int Nu, int Nv) {
  CDNb n;
  if ((u & 3) == 0) {
    n.r0 = n.r1 = 0;
    n.hr = false;
    n.c0 = -2, n.c1 = 2, n.hc = v + 2 <= Nv - 1;
  } else {
    n.r0 = -2, n.r1 = 2, n.hr = u + 2 <= Nu - 1;
    if ((v & 3) == 0)
      n.c0 = n.c1 = 0, n.hc = false;
    else
      n.c0 = -2, n.c1 = 2, n.hc = v + 2 <= Nv - 1;
  }
  return n;
}
// S3 points from stride-2 (H1) neighbours at distance 1
__device__ __forceinline__ CDNb cd_nb_s3(int u, int v, int Nu, int Nv) {
  CDNb n;
  if ((u & 1) == 0) {
    n.r0 = n.r1 = 0;
    n.hr = false;
    n.c0 = -1, n.c1 = 1, n.hc = v + 1 <= Nv - 1;
  } else {
    n.r0 = -1, n.r1 = 1, n.hr = u + 1 <= Nu - 1;
    if ((v & 1) == 0)
      n.c0 = n.c1 = 0, n.hc = false;
    else
      n.c0 = -1, n.c1 = 1, n.hc = v + 1 <= Nv - 1;
  }
  return n;
}
template <typename W>
__device__ __forceinline__ W cd_combine(const CDNb& n, W h00, W h01, W h10, W h11) {
  const W a = n.hc ? avgw<W>(h00, h01) : h00;
  const W b = n.hc ? avgw<W>(h10, h11) : h10;
  return n.hr ? avgw<W>(a, b) : a;
}

// Row geometry.  A region lattice holds at most half of a field's points
// (< 2^31), so offsets inside it are 32-bit.
struct CDGeo {
  int t0, t1;          // row
  int Nu, Nv;
  int su, sv;          // lattice strides of u and v
  int64_t rowoff;      // lattice offset of (t0, t1, 0)
};
template <int A>
__device__ __forceinline__ CDGeo cd_geo(const CDSeg& S, uint32_t row) {
  constexpr int U = A == 0 ? 1 : 0, V = A == 2 ? 1 : 2;
  CDGeo g;
  g.t0 = (int)fdiv(row, S.f1);
  g.t1 = (int)(row - (uint32_t)g.t0 * (uint32_t)S.c[1]);
  g.Nu = S.c[U];
  g.Nv = S.c[V];
  const int st[3] = {S.c[1] * S.c[2], S.c[2], 1};
  g.su = st[U];
  g.sv = st[V];
  g.rowoff = (int64_t)row * S.c[2];
  return g;
}

constexpr int kCDBatch = 4;  // row elements per lane whose loads are issued together

// Forward lifting of each region lattice into its S1/S2/S3 streams, with
// the largest residual magnitude of each stream.
template <typename Q, int A>
__global__ __launch_bounds__(kThreads) void k_cd_forward(const CDSeg* __restrict__ segs, int nseg, int64_t nblk) {
  using W = LiftT<Q>;
  using UW = typename std::make_unsigned<W>::type;
  int cur = -1;
  UW am[3] = {0, 0, 0};
  auto flush = [&](int si) {
    for (int c = 0; c < 3; ++c) {
      const double m = block_max((double)am[c]);
      if (threadIdx.x == 0) max_u64(segs[si].smax[c], (unsigned long long)__double_as_longlong(m));
    }
  };
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int64_t b = blockIdx.x; b < nblk; b += gridDim.x) {
    const int si = find_seg(segs, nseg, b);
    if (si != cur) {
      if (cur >= 0) flush(cur);
      cur = si;
      am[0] = am[1] = am[2] = 0;
    }
    const CDSeg& S = segs[si];
    const int64_t row = (b - S.blk_begin) * kCDRowsPerBlock + wave;
    if (row >= (int64_t)S.c[0] * S.c[1]) continue;
    const CDGeo g = cd_geo<A>(S, (uint32_t)row);
    const int u = A == 0 ? g.t1 : g.t0;
    GAS Q* const so[3] = {(GAS Q*)S.S[0] + cd_row_base<A>(S, 0, g.t0, g.t1),
                          (GAS Q*)S.S[1] + cd_row_base<A>(S, 1, g.t0, g.t1),
                          (GAS Q*)S.S[2] + cd_row_base<A>(S, 2, g.t0, g.t1)};
    const GAS Q* R = (const GAS Q*)S.R + g.rowoff;
    const int c2 = S.c[2];
    for (int t2b = 0; t2b < c2; t2b += 64 * kCDBatch) {
      W x[kCDBatch], h[kCDBatch][4];
      CDNb nb[kCDBatch];
      int cls[kCDBatch];
#pragma unroll
      for (int i = 0; i < kCDBatch; ++i) {
        const int t2 = t2b + lane + 64 * i;
        const int v = A == 2 ? g.t1 : t2;
        cls[i] = cd_class(u, v);
        nb[i] = cls[i] == 1 ? cd_nb_s2(u, v, g.Nu, g.Nv) : cd_nb_s3(u, v, g.Nu, g.Nv);
        x[i] = 0;
        h[i][0] = h[i][1] = h[i][2] = h[i][3] = 0;
        if (t2 < c2) {
          const GAS Q* p = R + t2;
          x[i] = (W)p[0];
          if (cls[i] != 0) {
            const CDNb& n = nb[i];
            h[i][0] = (W)p[n.r0 * g.su + n.c0 * g.sv];
            if (n.hc) h[i][1] = (W)p[n.r0 * g.su + n.c1 * g.sv];
            if (n.hr) h[i][2] = (W)p[n.r1 * g.su + n.c0 * g.sv];
            if (n.hr && n.hc) h[i][3] = (W)p[n.r1 * g.su + n.c1 * g.sv];
          }
        }
      }
#pragma unroll
      for (int i = 0; i < kCDBatch; ++i) {
        const int t2 = t2b + lane + 64 * i;
        if (t2 >= c2) continue;
        W res = x[i];
        if (cls[i] != 0) res -= cd_combine<W>(nb[i], h[i][0], h[i][1], h[i][2], h[i][3]);
        GAS Q* dst = cls[i] == 0 ? so[0] : (cls[i] == 1 ? so[1] : so[2]);
        dst[(int)cd_in_row<A>(cls[i], u, t2)] = (Q)res;
        const UW mag = res < 0 ? (UW)(-res) : (UW)res;
        am[cls[i]] = am[cls[i]] > mag ? am[cls[i]] : mag;
      }
    }
  }
  if (cur >= 0) flush(cur);
}

// Inverse lifting.  PHASE 0 rebuilds the stride-2 points (S1 and S2 classes)
// from the truncated S1/S2 streams (stride-4 neighbours read from S1 at their
// stream offsets); PHASE 1 rebuilds the rest from S3 and the stride-2 points
// written by phase 0.
template <typename Q, int PHASE, int A>
__global__ __launch_bounds__(kThreads) void k_cd_inverse(const CDSeg* __restrict__ segs, int nseg, int64_t nblk) {
  using W = LiftT<Q>;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int64_t b = blockIdx.x; b < nblk; b += gridDim.x) {
    const int si = find_seg(segs, nseg, b);
    const CDSeg& S = segs[si];
    const int64_t row = (b - S.blk_begin) * kCDRowsPerBlock + wave;
    if (row >= (int64_t)S.c[0] * S.c[1]) continue;
    const CDGeo g = cd_geo<A>(S, (uint32_t)row);
    const int u = A == 0 ? g.t1 : g.t0;  // u of the row
    if (PHASE == 0 && (u & 1)) continue;
    if (A == 2 && PHASE == 0 && (g.t1 & 1)) continue;
    if (A == 2 && PHASE == 1 && !((u & 1) || (g.t1 & 1))) continue;
    GAS Q* out = (GAS Q*)S.Rout + g.rowoff;
    const int Bc = PHASE == 0 ? S.B[1] : S.B[2], kc = PHASE == 0 ? S.k[1] : S.k[2];
    const int B0 = S.B[0], k0 = S.k[0];
    const GAS Q* S1 = (const GAS Q*)S.S[0];
    const GAS Q* sc = (const GAS Q*)S.S[PHASE == 0 ? 1 : 2] + cd_row_base<A>(S, PHASE == 0 ? 1 : 2, g.t0, g.t1);
    // phase 0: S1 offsets of the rows at u + du (du = -2, 0, 2; v along the
    // row), or of the rows (u + du, v + dv) when whole rows share one class
    int64_t b0[3][3];
    if (PHASE == 0) {
#pragma unroll
      for (int ku = 0; ku < 3; ++ku)
#pragma unroll
        for (int kv = 0; kv < 3; ++kv) {
          const int uu = u + 2 * ku - 2, vv = g.t1 + 2 * kv - 2;
          b0[ku][kv] = 0;
          if (A != 2) {
            if (kv == 1 && uu >= 0 && uu < g.Nu)
              b0[ku][kv] = A == 0 ? cd_row_base<A>(S, 0, g.t0, uu) : cd_row_base<A>(S, 0, uu, g.t1);
          } else if (uu >= 0 && uu < g.Nu && vv >= 0 && vv < g.Nv) {
            b0[ku][kv] = cd_row_base<A>(S, 0, uu, vv);
          }
        }
    }
    // H2 value at offset (du, dv) from column t2 (phase 0), as an S1 stream index
    auto s1_at = [&](int du, int dv, int t2, int v) -> int64_t {
      const int ku = du < 0 ? 0 : (du > 0 ? 2 : 1), kv = dv < 0 ? 0 : (dv > 0 ? 2 : 1);
      return A == 2 ? b0[ku][kv] + t2 : b0[ku][1] + ((v + dv) >> 2);
    };
    for (int t2b = 0; t2b < S.c[2]; t2b += 64 * kCDBatch) {
      W xs[kCDBatch], h[kCDBatch][4];
      CDNb nb[kCDBatch];
      int cls[kCDBatch];
      bool act[kCDBatch];
#pragma unroll
      for (int i = 0; i < kCDBatch; ++i) {
        const int t2 = t2b + lane + 64 * i;
        const int v = A == 2 ? g.t1 : t2;
        cls[i] = cd_class(u, v);
        act[i] = t2 < S.c[2] && (PHASE == 0 ? cls[i] != 2 : cls[i] == 2);
        nb[i] = PHASE == 0 ? cd_nb_s2(u, v, g.Nu, g.Nv) : cd_nb_s3(u, v, g.Nu, g.Nv);
        xs[i] = 0;
        h[i][0] = h[i][1] = h[i][2] = h[i][3] = 0;
        if (!act[i]) continue;
        const CDNb& n = nb[i];
        if (PHASE == 0) {
          if (cls[i] == 0) {
            h[i][0] = (W)mask_code<Q>(S1[s1_at(0, 0, t2, v)], B0, k0);
          } else {
            xs[i] = (W)mask_code<Q>(sc[cd_in_row<A>(1, u, t2)], Bc, kc);
            h[i][0] = (W)mask_code<Q>(S1[s1_at(n.r0, n.c0, t2, v)], B0, k0);
            if (n.hc) h[i][1] = (W)mask_code<Q>(S1[s1_at(n.r0, n.c1, t2, v)], B0, k0);
            if (n.hr) h[i][2] = (W)mask_code<Q>(S1[s1_at(n.r1, n.c0, t2, v)], B0, k0);
            if (n.hr && n.hc) h[i][3] = (W)mask_code<Q>(S1[s1_at(n.r1, n.c1, t2, v)], B0, k0);
          }
        } else {
          const GAS Q* p = out + t2;
          xs[i] = (W)mask_code<Q>(sc[cd_in_row<A>(2, u, t2)], Bc, kc);
          h[i][0] = (W)p[n.r0 * g.su + n.c0 * g.sv];
          if (n.hc) h[i][1] = (W)p[n.r0 * g.su + n.c1 * g.sv];
          if (n.hr) h[i][2] = (W)p[n.r1 * g.su + n.c0 * g.sv];
          if (n.hr && n.hc) h[i][3] = (W)p[n.r1 * g.su + n.c1 * g.sv];
        }
      }
#pragma unroll
      for (int i = 0; i < kCDBatch; ++i) {
        if (!act[i]) continue;
        const int t2 = t2b + lane + 64 * i;
        const W val = (PHASE == 0 && cls[i] == 0) ? h[i][0] : xs[i] + cd_combine<W>(nb[i], h[i][0], h[i][1], h[i][2], h[i][3]);
        out[t2] = (Q)val;
      }
    }
  }
}

// Inverse lifting in one pass when v runs along lattice rows (stacking axis
// 0 or 1).  A block rebuilds a tile of 8 rows (u) x 256 columns (v) of one
// slice: the stride-2 points of the tile and a one-point halo go to LDS first
// (from the S1/S2 streams), then every row of the tile is written whole, the
// remaining points rebuilt from S3 and those LDS values.  Whole rows keep the
// stores full-width (no partial-line writes).  Slices one row deep (the
// region lattices of 2D fields) are rebuilt eight to a tile, each u = 0 row
// by one wave straight from its streams, four columns a lane.
constexpr int kCITU = 8, kCITV = 256;
constexpr int kCIHU = kCITU / 2 + 1, kCIHV = kCITV / 2 + 1;  // stride-2 rows/columns incl. halo
// staged stream runs: S1 rows (3 x 65 points), S2 of the u = 0 mod 4 rows
// (3 x 64) and of the u = 2 mod 4 rows (2 x 129)
constexpr int kCIS1 = kCITV / 4 + 1, kCIS2C = kCITV / 4;
constexpr int kCIN1 = 3 * kCIS1, kCIN2C = 3 * kCIS2C, kCIN = kCIN1 + kCIN2C + 2 * kCIHV;
constexpr int kCIL = (kCIN + kThreads - 1) / kThreads;

template <typename Q, int A>
__global__ __launch_bounds__(kThreads) void k_cd_inverse_tile(const CDSeg* __restrict__ segs, int nseg, int64_t nblk) {
  using W = LiftT<Q>;
  constexpr int U = A == 0 ? 1 : 0;
  // both padded to whole turns of the block, so every thread writes every turn
  __shared__ W h1[(kCIHU * kCIHV + kThreads - 1) / kThreads * kThreads];
  __shared__ W lt[kCIL * kThreads];
  __shared__ int64_t rb0[3], rb1[kCIHU], rb2[kCITU];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int64_t b = blockIdx.x; b < nblk; b += gridDim.x) {
    const int si = find_seg(segs, nseg, b);
    const CDSeg& S = segs[si];
    const int Nu = S.c[U], Nv = S.c[2];
    // tile coordinates by multiply-high division (tiles along v, then u)
    const uint32_t lb = (uint32_t)(b - S.blk_begin);
    const uint32_t lq = fdiv(lb, S.ftv);
    const int V0 = (int)(lb - lq * S.ftv.d) * kCITV;
    const uint32_t sq = fdiv(lq, S.ftu);
    const int U0 = (int)(lq - sq * S.ftu.d) * kCITU;
    const int sa = (int)sq;  // index along the stacking axis (slices one row deep: the group of eight)
    if (Nu == 1) {
      // a u = 0 row: S1 at v = 0 mod 4; S2 at v = 2 mod 4 plus the average
      // of the S1 points two columns away; S3 at odd v plus the average of
      // its even neighbours (an absent right neighbour repeats the left one)
      const int Ns = S.c[A];
      using UM = typename UOf<Q>::type;
      const UM M0 = code_mask<Q>(S.B[0], S.k[0]), M1 = code_mask<Q>(S.B[1], S.k[1]), M2 = code_mask<Q>(S.B[2], S.k[2]);
      const int v = V0 + 4 * lane;
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        const int sl = sa * kCITU + wave + 4 * k;
        if (sl >= Ns || v >= Nv) continue;
        const int t0 = A == 0 ? sl : 0, t1 = A == 0 ? 0 : sl;
        const GAS Q* s1 = (const GAS Q*)S.S[0] + cd_row_base<A>(S, 0, t0, t1) + (v >> 2);
        const GAS Q* s2 = (const GAS Q*)S.S[1] + cd_row_base<A>(S, 1, t0, t1) + (v >> 2);
        const GAS Q* s3 = (const GAS Q*)S.S[2] + cd_row_base<A>(S, 2, t0, t1) + (v >> 1);
        GAS Q* o = (GAS Q*)S.Rout + ((int64_t)t0 * S.c[1] + t1) * S.c[2] + v;
        const bool e1 = v + 1 <= Nv - 1, e2 = v + 2 <= Nv - 1, e3 = v + 3 <= Nv - 1, e4 = v + 4 <= Nv - 1;
        const W x0 = (W)apply_mask<Q>(s1[0], M0);
        const W x4 = e4 ? (W)apply_mask<Q>(s1[1], M0) : x0;
        const W x2 = e2 ? (W)apply_mask<Q>(s2[0], M1) + avgw<W>(x0, x4) : x0;
        o[0] = (Q)x0;
        if (e1) o[1] = (Q)((W)apply_mask<Q>(s3[0], M2) + avgw<W>(x0, x2));
        if (e2) o[2] = (Q)x2;
        if (e3) o[3] = (Q)((W)apply_mask<Q>(s3[1], M2) + avgw<W>(x2, e4 ? x4 : x2));
      }
      continue;
    }
    auto tt = [&](int u, int& t0, int& t1) {
      t0 = A == 0 ? sa : u;
      t1 = A == 0 ? u : sa;
    };
    auto rowoff = [&](int u) -> int64_t {
      int t0, t1;
      tt(u, t0, t1);
      return ((int64_t)t0 * S.c[1] + t1) * S.c[2];
    };
    __syncthreads();  // LDS of the previous tile is free
    // stream offsets of the rows this tile touches
    if (tid < 3) {  // S1 rows U0 + 4k
      const int u = U0 + 4 * tid;
      int t0, t1;
      tt(u, t0, t1);
      rb0[tid] = u < Nu ? cd_row_base<A>(S, 0, t0, t1) : 0;
    } else if (tid >= 16 && tid < 16 + kCIHU) {  // S2 rows U0 + 2k
      const int u = U0 + 2 * (tid - 16);
      int t0, t1;
      tt(u, t0, t1);
      rb1[tid - 16] = (u < Nu) ? cd_row_base<A>(S, 1, t0, t1) : 0;
    } else if (tid >= 32 && tid < 32 + kCITU) {  // S3 rows U0 + k
      const int u = U0 + tid - 32;
      int t0, t1;
      tt(u, t0, t1);
      rb2[tid - 32] = (u < Nu) ? cd_row_base<A>(S, 2, t0, t1) : 0;
    }
    __syncthreads();
    const GAS Q* S1 = (const GAS Q*)S.S[0];
    const GAS Q* S2 = (const GAS Q*)S.S[1];
    const GAS Q* S3 = (const GAS Q*)S.S[2];
    using UM = typename UOf<Q>::type;
    const UM M0 = code_mask<Q>(S.B[0], S.k[0]), M1 = code_mask<Q>(S.B[1], S.k[1]), M2 = code_mask<Q>(S.B[2], S.k[2]);
    GAS Q* const Rout = (GAS Q*)S.Rout;
    // The tile's runs of the S1 and S2 streams, one coalesced load per point
    // (in a row, each class's points of a column range are consecutive in its
    // stream): S1 of rows U0 + 4i at v = V0 + 4l, S2 of those rows at
    // v = V0 + 4l + 2, S2 of rows U0 + 2 + 4i at v = V0 + 2l.
    {
      // every lane loads (one of the three runs, by its slot), a slot
      // without a point reading a harmless address and dropping the value
      W lv[kCIL];
#pragma unroll
      for (int i = 0; i < kCIL; ++i) {
        const int e = tid + i * kThreads;
        const bool s1 = e < kCIN1, s2c = !s1 && e < kCIN1 + kCIN2C;
        const int e2 = e - kCIN1, e3 = e - kCIN1 - kCIN2C;
        const int i1 = e / kCIS1, i2 = e2 / kCIS2C, i3 = e3 / kCIHV;
        const int ii = s1 ? i1 : (s2c ? i2 : i3);
        const int l = s1 ? e - i1 * kCIS1 : (s2c ? e2 - i2 * kCIS2C : e3 - i3 * kCIHV);
        const int uu = U0 + 4 * ii + (s1 || s2c ? 0 : 2);
        const int vv = s1 ? V0 + 4 * l : (s2c ? V0 + 4 * l + 2 : V0 + 2 * l);
        const bool ok = e < kCIN && uu < Nu && vv < Nv;
        // run start: rb0[ii] (S1), rb1[2 ii] or rb1[2 ii + 1] (S2); index kept inside the tables
        const int64_t rb = s1 ? rb0[min(ii, 2)] : rb1[min(s2c ? 2 * ii : 2 * ii + 1, kCIHU - 1)];
        const int64_t o = rb + (s1 || s2c ? (V0 >> 2) : (V0 >> 1)) + l;
        const Q q = *(ok ? (s1 ? S1 : S2) + o : (const GAS Q*)segs);
        lv[i] = ok ? (W)apply_mask<Q>(q, s1 ? M0 : M1) : (W)0;
      }
#pragma unroll
      for (int i = 0; i < kCIL; ++i)
        lt[tid + i * kThreads] = lv[i];  // zero past the runs
    }
    __syncthreads();
    // stride-2 points (u, v even) of the tile and halo: S1 points as they are,
    // S2 points plus their prediction from S1 (rows u -+ 2 and columns v -+ 2;
    // an absent neighbour repeats the present one)
    {
      const W* s1t = lt;
      const W* s2c = lt + kCIN1;
      const W* s2b = lt + kCIN1 + kCIN2C;
      // branch-free: every lane reads the S1 values around it and both S2
      // candidates (indices kept inside the staged runs) and selects
      // whole turns: entries past the last (padding) take values from reads
      // that stay inside the staging and are never used
      for (int e = tid; e < (kCIHU * kCIHV + kThreads - 1) / kThreads * kThreads; e += kThreads) {
        const int r = e / kCIHV, k = e - r * kCIHV;
        const int u = U0 + 2 * r, v = V0 + 2 * k;
        const int rh = r >> 1, c0 = k >> 1;
        const int c1 = (k & 1) && v + 2 <= Nv - 1 ? c0 + 1 : c0;
        const bool r2 = r & 1;  // u = 2 mod 4 (else 0 mod 4)
        const W* ra = s1t + rh * kCIS1;
        const W* rb = r2 && u + 2 <= Nu - 1 ? ra + kCIS1 : ra;
        const W a0 = ra[c0], a1 = ra[c1], b0 = rb[c0], b1 = rb[c1];
        const W sc = s2c[rh * kCIS2C + c0];          // inside the staging for every lane
        const W sb = s2b[(r2 ? rh : 0) * kCIHV + k];  // row 0 for u = 0 mod 4 (not used)
        const W v2 = sb + avgw<W>(avgw<W>(a0, a1), avgw<W>(b0, b1));
        const W v0 = (k & 1) ? sc + avgw<W>(a0, a1) : a0;
        h1[e] = (u < Nu && v < Nv) ? (r2 ? v2 : v0) : (W)0;
      }
    }
    __syncthreads();
    // whole rows: stride-2 points from LDS, the rest from S3.  A lane takes
    // column pairs (v0 = V0 + 2p, v1 = v0 + 1), which share their stride-2
    // neighbours: on an even row, v0 is a stride-2 point and v1 averages its
    // left and right neighbours; on an odd row, v0 averages the rows above
    // and below, v1 the four diagonal neighbours (columns first, as the
    // lifting predicts).  A missing right or lower neighbour repeats the
    // present one, which leaves that average equal to it.
#pragma unroll
    for (int rr = 0; rr < kCITU / 4; ++rr) {
      const int r = wave * (kCITU / 4) + rr;
      const int u = U0 + r;
      if (u >= Nu) continue;
      const bool uodd = u & 1;
      // the row's S3 run and its output row as buffers: a column past the
      // row is out of their range, so its load reads zero and its store is
      // dropped (no per-lane branches)
      const BufRsrc s3b = buf_rsrc((const void*)(S3 + readfirst64(rb2[r])), (int64_t)(uodd ? Nv : Nv >> 1) * (int64_t)sizeof(Q));
      const BufRsrc ob = buf_rsrc((const void*)(Rout + rowoff(u)), (int64_t)Nv * (int64_t)sizeof(Q));
      W x0[kCITV / 128], x1[kCITV / 128];
#pragma unroll
      for (int c = 0; c < kCITV / 128; ++c) {
        const int v0 = V0 + 2 * (c * 64 + lane), v1 = v0 + 1;
        x0[c] = 0;
        if (uodd) x0[c] = (W)apply_mask<Q>(buf_load<Q>(s3b, (uint32_t)cd_in_row<A>(2, u, v0) * sizeof(Q), 0u), M2);
        x1[c] = (W)apply_mask<Q>(buf_load<Q>(s3b, (uint32_t)cd_in_row<A>(2, u, v1) * sizeof(Q), 0u), M2);
      }
      const W* ht = h1 + (r >> 1) * kCIHV;                         // row u (even u) or u - 1
      const W* hb = (uodd && u + 1 <= Nu - 1) ? ht + kCIHV : ht;  // row u + 1 (odd u)
#pragma unroll
      for (int c = 0; c < kCITV / 128; ++c) {
        const int p = c * 64 + lane, v0 = V0 + 2 * p, v1 = v0 + 1;  // p + 1 <= kCIHV - 1
        const bool hc = v1 + 1 <= Nv - 1;
        const W t0 = ht[p], t1 = hc ? ht[p + 1] : t0;
        const W b0 = hb[p], b1 = hc ? hb[p + 1] : b0;
        const W o0 = uodd ? x0[c] + avgw<W>(t0, b0) : t0;
        const W o1 = x1[c] + (uodd ? avgw<W>(avgw<W>(t0, t1), avgw<W>(b0, b1)) : avgw<W>(t0, t1));
        buf_store<Q>((Q)o0, ob, (uint32_t)v0 * sizeof(Q), 0u);
        buf_store<Q>((Q)o1, ob, (uint32_t)v1 * sizeof(Q), 0u);
      }
    }
  }
}

// Forward lifting in one pass when v runs along lattice rows (stacking axis
// 0 or 1).  A block lifts a tile of 8 rows (u) x 256 columns (v) of one
// slice: the tile's codes with a halo (the next row, two columns on each
// side) are staged in LDS, then wave w lifts rows w and w + 4, which have
// the same type (u = 0 mod 4, u = 2 mod 4, or odd), and writes each class of
// a row as one run of its stream.  Each prediction is the column-then-row
// average of four LDS values; an absent neighbour repeats the present one,
// and since the floor average of a value with itself is that value this is
// the same result as averaging only over the neighbours that exist.
// Slices one row deep (the region lattices of 2D fields) have only u = 0
// rows and no neighbours across rows: there the tile's eight rows are eight
// consecutive slices, each lifted as a u = 0 row by its own wave.
constexpr int kCFP = kCITV + 4;  // LDS row pitch: two halo columns each side

template <typename Q, int A>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(sizeof(Q) == 4 ? 5 : 4))) void k_cd_forward_tile(const CDSeg* __restrict__ segs, int nseg, int64_t nblk) {
  using W = LiftT<Q>;
  using UW = typename std::make_unsigned<W>::type;
  constexpr int U = A == 0 ? 1 : 0;
  __shared__ W L[(kCITU + 1) * kCFP];
  int cur = -1;
  UW am[3] = {0, 0, 0};
  auto flush = [&](int si) {
    for (int c = 0; c < 3; ++c) {
      const double m = block_max((double)am[c]);
      if (threadIdx.x == 0) max_u64(segs[si].smax[c], (unsigned long long)__double_as_longlong(m));
    }
  };
  auto upd = [&](int c, W res) {
    const UW mag = res < 0 ? (UW)(-res) : (UW)res;
    am[c] = am[c] > mag ? am[c] : mag;
  };
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // the current segment's fields, reloaded only when a tile of the next
  // segment comes up (tiles of a block only move forward)
  int64_t seg_end = -1, blk0 = 0;
  int c0 = 0, c1 = 0, c2 = 0;
  const GAS Q* R = nullptr;
  GAS Q* Sp[3] = {nullptr, nullptr, nullptr};
  for (int64_t b = blockIdx.x; b < nblk; b += gridDim.x) {
    if (b >= seg_end) {
      const int si = find_seg(segs, nseg, b);
      if (cur >= 0) flush(cur);
      cur = si;
      am[0] = am[1] = am[2] = 0;
      const CDSeg& F = segs[si];
      seg_end = si + 1 < nseg ? segs[si + 1].blk_begin : nblk;
      blk0 = F.blk_begin;
      c0 = F.c[0], c1 = F.c[1], c2 = F.c[2];
      R = (const GAS Q*)F.R;
      Sp[0] = (GAS Q*)F.S[0], Sp[1] = (GAS Q*)F.S[1], Sp[2] = (GAS Q*)F.S[2];
    }
    const int Nu = A == 0 ? c1 : c0, Nv = c2, Ns = A == 0 ? c0 : c1;
    const bool flat = Nu == 1;  // tile rows are slices
    const int nTu = (Nu + kCITU - 1) / kCITU, nTv = (Nv + kCITV - 1) / kCITV;
    int lb = (int)(b - blk0);
    const int V0 = (lb % nTv) * kCITV;
    lb /= nTv;
    const int U0 = (lb % nTu) * kCITU;
    const int sa = flat ? lb * kCITU : lb / nTu;  // index along the stacking axis (of row 0)
    // lattice row of tile row r, and whether it exists
    auto tt = [&](int r, int& t0, int& t1) {
      const int u = flat ? 0 : U0 + r, a = flat ? sa + r : sa;
      t0 = A == 0 ? a : u;
      t1 = A == 0 ? u : a;
    };
    auto row_ok = [&](int r) { return flat ? r < kCITU && sa + r < Ns : U0 + r < Nu; };
    auto rowoff = [&](int r) -> int64_t {
      int t0, t1;
      tt(r, t0, t1);
      return ((int64_t)t0 * c1 + t1) * c2;
    };
    __syncthreads();  // LDS of the previous tile is free
    // thread t loads column V0 + t of every row (row offsets are uniform),
    // threads 0..35 one halo point each; all loads precede the LDS stores
    static_assert(kCITV == kThreads && 4 * (kCITU + 1) <= kThreads, "tile shape");
    W xv[kCITU + 1], xh = 0;
#pragma unroll
    for (int r = 0; r < kCITU + 1; ++r) {
      xv[r] = 0;
      if (row_ok(r) && V0 + tid < Nv) xv[r] = (W)R[rowoff(r) + V0 + tid];
    }
    const int hr = tid >> 2, hc = (tid & 3) < 2 ? (tid & 3) : kCITV + (tid & 3);
    {
      const int v = V0 - 2 + hc;
      if (tid < 4 * (kCITU + 1) && row_ok(hr) && v >= 0 && v < Nv) xh = (W)R[rowoff(hr) + v];
    }
#pragma unroll
    for (int r = 0; r < kCITU + 1; ++r) L[r * kCFP + 2 + tid] = xv[r];
    if (tid < 4 * (kCITU + 1)) L[hr * kCFP + hc] = xh;
    __syncthreads();
    // Each wave computes the residuals of both its rows first (straight-line
    // LDS reads, rows past the lattice read zeros), then stores what exists.
    W res[2][kCITV / 64];
    const int jc = 4 * lane;  // lane's column group in a u = 0 mod 4 row
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int r = wave + 4 * k;
      const int u = U0 + r;
      const W* Lr = L + r * kCFP + 2;  // column v at Lr[v - V0]
      if (wave == 0 || flat) {  // u = 0 mod 4: S1 at v = 0 mod 4, S2 at v = 2 mod 4, S3 at odd v
        res[k][0] = Lr[jc];
        res[k][1] = Lr[jc + 2] - avgw<W>(Lr[jc], Lr[V0 + jc + 4 <= Nv - 1 ? jc + 4 : jc]);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int j = 2 * (lane + 64 * h) + 1;
          res[k][2 + h] = Lr[j] - avgw<W>(Lr[j - 1], Lr[V0 + j + 1 <= Nv - 1 ? j + 1 : j - 1]);
        }
      } else if (wave == 2) {  // u = 2 mod 4: S2 at even v (rows u -+ 2), S3 at odd v
        const W* Ld = Lr - 2 * kCFP;
        const W* Lu = u + 2 <= Nu - 1 ? Lr + 2 * kCFP : Ld;
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int j = 2 * (lane + 64 * h);
          const int j0 = (j & 2) ? j - 2 : j;
          const int j1 = (j & 2) ? (V0 + j + 2 <= Nv - 1 ? j + 2 : j - 2) : j;
          res[k][h] = Lr[j] - avgw<W>(avgw<W>(Ld[j0], Ld[j1]), avgw<W>(Lu[j0], Lu[j1]));
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int j = 2 * (lane + 64 * h) + 1;
          res[k][2 + h] = Lr[j] - avgw<W>(Lr[j - 1], Lr[V0 + j + 1 <= Nv - 1 ? j + 1 : j - 1]);
        }
      } else {  // odd u: S3 everywhere, from rows u -+ 1
        const W* Ld = Lr - kCFP;
        const W* Lu = u + 1 <= Nu - 1 ? Lr + kCFP : Ld;
#pragma unroll
        for (int h = 0; h < kCITV / 64; ++h) {
          const int j = lane + 64 * h;
          const int j0 = (j & 1) ? j - 1 : j;
          const int j1 = (j & 1) ? (V0 + j + 1 <= Nv - 1 ? j + 1 : j - 1) : j;
          res[k][h] = Lr[j] - avgw<W>(avgw<W>(Ld[j0], Ld[j1]), avgw<W>(Lu[j0], Lu[j1]));
        }
      }
    }
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const int r = wave + 4 * k;
      if (!row_ok(r)) continue;
      int t0, t1;
      tt(r, t0, t1);
      if (wave == 0 || flat) {
        GAS Q* s1 = Sp[0] + cd_row_base<A>(c1, c2, 0, t0, t1) + (V0 >> 2);
        GAS Q* s2 = Sp[1] + cd_row_base<A>(c1, c2, 1, t0, t1) + (V0 >> 2);
        GAS Q* s3 = Sp[2] + cd_row_base<A>(c1, c2, 2, t0, t1) + (V0 >> 1);
        if (V0 + jc < Nv) s1[lane] = (Q)res[k][0], upd(0, res[k][0]);
        if (V0 + jc + 2 < Nv) s2[lane] = (Q)res[k][1], upd(1, res[k][1]);
#pragma unroll
        for (int h = 0; h < 2; ++h)
          if (V0 + 2 * (lane + 64 * h) + 1 < Nv) s3[lane + 64 * h] = (Q)res[k][2 + h], upd(2, res[k][2 + h]);
      } else if (wave == 2) {
        GAS Q* s2 = Sp[1] + cd_row_base<A>(c1, c2, 1, t0, t1) + (V0 >> 1);
        GAS Q* s3 = Sp[2] + cd_row_base<A>(c1, c2, 2, t0, t1) + (V0 >> 1);
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          if (V0 + 2 * (lane + 64 * h) < Nv) s2[lane + 64 * h] = (Q)res[k][h], upd(1, res[k][h]);
          if (V0 + 2 * (lane + 64 * h) + 1 < Nv) s3[lane + 64 * h] = (Q)res[k][2 + h], upd(2, res[k][2 + h]);
        }
      } else {
        GAS Q* s3 = Sp[2] + cd_row_base<A>(c1, c2, 2, t0, t1) + V0;
#pragma unroll
        for (int h = 0; h < kCITV / 64; ++h)
          if (V0 + lane + 64 * h < Nv) s3[lane + 64 * h] = (Q)res[k][h], upd(2, res[k][h]);
      }
    }
  }
  if (cur >= 0) flush(cur);
}

// ------------------------------------------------------------ bitplane codec
__device__ __forceinline__ int find_stream(const StreamDev* sd, int ns, int64_t gch) {
  int lo = 0, hi = ns - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (sd[mid].chunk_begin <= gch)
      lo = mid;
    else
      hi = mid - 1;
  }
  return __builtin_amdgcn_readfirstlane(lo);
}

// One round of the bit-matrix transpose: swap the off-diagonal S x S bit
// blocks of every 2S x 2S block (M selects the low S bits of each 2S group).
template <int S, uint32_t M, int N = 32>
__device__ __forceinline__ void transpose_round(uint32_t (&a)[N]) {
#pragma unroll
  for (int k = 0; k < N; ++k) {
    if (k & S) continue;
    const uint32_t t = ((a[k] >> S) ^ a[k + S]) & M;
    a[k] ^= t << S;
    a[k + S] ^= t;
  }
}

// Bit-matrix transpose of 32 words: afterwards bit k of a[p] is what bit p of
// a[k] was (five rounds of block swaps, 2s x 2s blocks at round s).  Each round
// is its own instantiation so every register index is a compile-time constant.
__device__ __forceinline__ void transpose32(uint32_t (&a)[32]) {
  transpose_round<16, 0x0000FFFFu>(a);
  transpose_round<8, 0x00FF00FFu>(a);
  transpose_round<4, 0x0F0F0F0Fu>(a);
  transpose_round<2, 0x33333333u>(a);
  transpose_round<1, 0x55555555u>(a);
}

// Two 16 x 16 bit-matrix transposes at once, one in each half of 16 words:
// afterwards bit k of the low (high) half of a[p] is what bit p of the low
// (high) half of a[k] was.  The masks of the four rounds keep the halves apart.
__device__ __forceinline__ void transpose16x2(uint32_t (&a)[16]) {
  transpose_round<8, 0x00FF00FFu, 16>(a);
  transpose_round<4, 0x0F0F0F0Fu, 16>(a);
  transpose_round<2, 0x33333333u, 16>(a);
  transpose_round<1, 0x55555555u, 16>(a);
}

constexpr int kRow = 33;  // LDS row pitch (codes) of the half-word staging tile

// Stage half h of every 64-code word of a chunk in LDS: row r holds codes
// 64 r + 32 h + [0, 32) of the chunk (zero past the stream's end, which is
// where the chunk's buffer range ends).  Lane pairs of rows per load.
template <typename Q>
__device__ __forceinline__ void stage_half(BufRsrc rc, int h, Q* cst, int lane) {
  const uint32_t k = lane & 31, rr = lane >> 5;
  const uint32_t o = (32u * h + k + 64u * rr) * (uint32_t)sizeof(Q);
#pragma unroll 8
  for (uint32_t it = 0; it < 32; ++it) cst[(2 * it + rr) * kRow + k] = buf_load<Q>(rc, o, 128u * it * sizeof(Q));
}
template <typename Q>
__device__ __forceinline__ void unstage_half(BufRsrc rc, int h, const Q* cst, int lane) {
  const uint32_t k = lane & 31, rr = lane >> 5;
  const uint32_t o = (32u * h + k + 64u * rr) * (uint32_t)sizeof(Q);
#pragma unroll 8
  for (uint32_t it = 0; it < 32; ++it) buf_store<Q>(cst[(2 * it + rr) * kRow + k], rc, o, 128u * it * sizeof(Q));
}
// A chunk's codes as a buffer: base + [0, min(n - base, chunk)).
template <typename Q>
__device__ __forceinline__ BufRsrc chunk_rsrc(const void* codes, int64_t base, int64_t n) {
  return buf_rsrc((const Q*)codes + base, (n - base < kChunk ? n - base : (int64_t)kChunk) * (int64_t)sizeof(Q));
}
// Plane j's magnitude words of a chunk as a buffer (64 words, fewer at the end).
__device__ __forceinline__ BufRsrc plane_rsrc(const void* mag, int64_t j, int64_t M, int64_t chunk) {
  const int64_t w0 = chunk * 64;
  return buf_rsrc((const uint64_t*)mag + j * M + w0, (M - w0 < 64 ? M - w0 : 64) * 8);
}

// One wave per 4096-code chunk, one lane per 64-code word.  Each lane
// transposes its word into per-plane magnitude words (stored plane-major,
// coalesced across lanes), counts the codes that become significant at each
// plane, and a wave scan of those counts gives every word its offset in the
// chunk's plane-major sign staging.  The sign bits are then placed with one
// LDS fetch-and-add per nonzero code on a (plane, word) cursor, visiting the
// word's codes in order.
template <typename Q, int MAXB>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(sizeof(Q) == 4 ? 3 : 2))) void k_encode(const StreamDev* __restrict__ sd, int ns) {
  constexpr int QW = (int)sizeof(Q) / 4;
  constexpr int kStageBytes = 64 * kRow * (int)sizeof(Q);
  constexpr int kTabBytes = MAXB * 64 * 4;
  __shared__ __align__(16) unsigned char lds[kStageBytes > kTabBytes ? kStageBytes : kTabBytes];
  __shared__ unsigned long long sstage[128];  // [64, 128): per-lane sinks of empty ORs
  Q* cst = (Q*)lds;                 // half-word staging tile
  uint32_t* ptab = (uint32_t*)lds;  // then: next staging position per (plane, word)
  const int lane = threadIdx.x;
  const int64_t gch = blockIdx.x;
  const int u = find_stream(sd, ns, gch);
  const StreamDev& S = sd[u];
  const int64_t chunk = gch - S.chunk_begin;
  GAS uint64_t* mag = (GAS uint64_t*)S.mag;
  GAS uint32_t* cnt = (GAS uint32_t*)S.cnt;
  GAS uint64_t* stg = (GAS uint64_t*)S.stage;
  const int B = S.B;
  const int64_t M = S.M, n = S.n;
  const int64_t base = chunk * kChunk;
  const BufRsrc rc = chunk_rsrc<Q>(S.codes, base, n);
  sstage[lane] = 0ull;

  uint64_t P[MAXB];   // P[b]: bit b of the word's 64 magnitudes
  uint32_t lead[16];  // per code: 0x80 | plane << 1 | negative; 0 for a zero code
#pragma unroll
  for (int b = 0; b < MAXB; ++b) P[b] = 0ull;
#pragma unroll
  for (int i = 0; i < 16; ++i) lead[i] = 0u;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    stage_half<Q>(rc, h, cst, lane);
    __syncthreads();
#pragma unroll
    for (int p = 0; p < QW; ++p) {
      uint32_t r[32];
#pragma unroll
      for (int k = 0; k < 32; ++k) {
        const Q q = cst[lane * kRow + k];
        r[k] = mag_part(q, p);
        if (p == 0) {
          const int kk = 32 * h + k;
          lead[kk >> 2] |= code_lead(q, B) << (8 * (kk & 3));
        }
      }
      // Make the packed lead words opaque: otherwise the compiler sees
      // through the byte packing and keeps every code's lead byte (or what
      // it is made of) in a register of its own until the sign pass.
      if (p == 0) {
#pragma unroll
        for (int i = 0; i < 8; ++i) asm volatile("" : "+v"(lead[8 * h + i]));
      }
      transpose32(r);
#pragma unroll
      for (int bb = 0; bb < 32; ++bb)
        if (32 * p + bb < MAXB) P[32 * p + bb] |= (uint64_t)r[bb] << (32 * h);
    }
    __syncthreads();
  }

  // planes from the most significant: magnitude words, newcomer counts, cursors
  uint32_t cc[MAXB], incl[MAXB];
  uint64_t sig = 0ull;
#pragma unroll
  for (int b = MAXB - 1; b >= 0; --b) {
    const uint64_t pw = P[b];
    if (b < B) buf_store<uint64_t>(pw, plane_rsrc(S.mag, B - 1 - b, M, chunk), 8u * lane, 0u);
    cc[b] = b < B ? (uint32_t)__popcll(pw & ~sig) : 0u;
    incl[b] = cc[b];
    sig |= pw;
    // lossless stage: this chunk's nonzero words of the plane (the ballot is
    // taken by the whole wave, the count stored by lane 0)
    if (S.zcnt && b < B) {
      const uint64_t nzm = __ballot(pw != 0ull);
      if (lane == 0) ((GAS uint32_t*)S.zcnt)[chunk * B + (B - 1 - b)] = (uint32_t)__popcll(nzm);
    }
  }
  wave_incl_scan_n<MAXB>(incl);
  uint32_t toff = 0, mycnt = 0;
#pragma unroll
  for (int b = MAXB - 1; b >= 0; --b) {
    if (b >= B) continue;
    const int j = B - 1 - b;
    const uint32_t tot = (uint32_t)__builtin_amdgcn_readlane((int)incl[b], 63);
    mycnt = lane == j ? tot : mycnt;
    ptab[j * 64 + lane] = toff + incl[b] - cc[b];
    toff += tot;
  }
  if (lane < B) cnt[chunk * B + lane] = mycnt;
  // sign bits, word by word in code order (each lane owns its cursor column);
  // cursors are taken 16 codes at a time so their LDS round trips overlap.
  // Every lane issues every LDS operation: a zero code adds 0 to its own
  // plane-0 cursor and a code with no sign bit to place ORs 0 into a word of
  // its own past the staging, so no operation needs an exec-mask branch.
#pragma unroll
  for (int g = 0; g < 64; g += 16) {
    uint32_t pos[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const uint32_t v = (lead[(g + k) >> 2] >> (8 * ((g + k) & 3))) & 0xffu;
      pos[k] = atomicAdd(&ptab[((v >> 1) & 63u) * 64 + lane], v >> 7);
    }
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      const uint32_t v = (lead[(g + k) >> 2] >> (8 * ((g + k) & 3))) & 0xffu;
      if ((v & 0x81u) == 0x81u && pos[k] < (uint32_t)kChunk) atomicOr(&sstage[pos[k] >> 6], 1ull << (pos[k] & 63));
    }
  }
  __syncthreads();
  stg[chunk * 64 + lane] = sstage[lane];
}

// Exclusive scan of the per-chunk counts of one (stream, plane): the index
// section entries and the plane's total.
__global__ __launch_bounds__(kThreads) void k_scan(const StreamDev* __restrict__ sd, const int32_t* job_s,
                                                    const int32_t* job_j, int64_t* totals) {
  __shared__ uint32_t wsum[kThreads / 64];
  const int job = blockIdx.x;
  const StreamDev& S = sd[job_s[job]];
  const int j = job_j[job];
  const int64_t C = S.C, B = S.B;
  const GAS uint32_t* c = (const GAS uint32_t*)S.cnt + j;  // chunk-major: entry i at i * B
  GAS uint32_t* o = (GAS uint32_t*)S.idx + (int64_t)j * C;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  // kScanPer consecutive chunks per thread and turn: a long stream takes a
  // quarter of the barrier-separated turns
  constexpr int kScanPer = 4;
  uint64_t carry = 0;
  for (int64_t base = 0; base < C; base += kThreads * kScanPer) {
    const int64_t i0 = base + (int64_t)threadIdx.x * kScanPer;
    uint32_t v[kScanPer], t = 0;
#pragma unroll
    for (int q = 0; q < kScanPer; ++q) {
      v[q] = (i0 + q < C) ? c[(i0 + q) * B] : 0u;
      t += v[q];
    }
    const uint32_t incl = wave_incl_scan(t, lane);
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    uint32_t before = 0, all = 0;
    for (int w = 0; w < kThreads / 64; ++w) {
      if (w < wave) before += wsum[w];
      all += wsum[w];
    }
    uint32_t run = (uint32_t)carry + before + incl - t;
#pragma unroll
    for (int q = 0; q < kScanPer; ++q) {
      if (i0 + q < C) o[i0 + q] = run;
      run += v[q];
    }
    carry += all;
    __syncthreads();
  }
  if (threadIdx.x == 0) totals[job] = (int64_t)carry;
}

// Sign-section layout from the plane totals (one block of kLayoutThreads).
// Job k takes ceil(totals[k] / 64) words; prefix[] is their exclusive prefix
// sum over all jobs (prefix[njobs] = the sum).  A plane's run starts
// prefix[k] - prefix[first job of its stream] words into its stream's run,
// and a stream's run starts prefix[first] - prefix[first job of its field]
// words into its field's sign arena.  A stream whose run would end past the
// arena is not placed (its plane count is set to zero, so the sign placement
// skips it) and err is set (it is cleared first).
constexpr int kLayoutThreads = 1024;
__global__ __launch_bounds__(kLayoutThreads) void k_sign_layout(const int64_t* __restrict__ totals, int njobs,
                                                                const SignJob* __restrict__ jobs, int ns,
                                                                const SignStream* __restrict__ ss, StreamDev* sd,
                                                                int64_t* prefix, int32_t* err) {
  __shared__ int64_t part[kLayoutThreads];
  const int t = threadIdx.x;
  if (t == 0) *err = 0;  // set below, after the barriers
  // each thread sums a contiguous range of jobs, a block scan of the range
  // sums gives each range's start, and the range is written out in order
  const int per = (njobs + kLayoutThreads - 1) / kLayoutThreads;
  const int k0 = min(njobs, t * per), k1 = min(njobs, k0 + per);
  int64_t sum = 0;
  for (int k = k0; k < k1; ++k) sum += (totals[k] + 63) >> 6;
  part[t] = sum;
  __syncthreads();
  for (int off = 1; off < kLayoutThreads; off <<= 1) {
    const int64_t v = t >= off ? part[t - off] : 0;
    __syncthreads();
    part[t] += v;
    __syncthreads();
  }
  int64_t run = part[t] - sum;  // exclusive
  for (int k = k0; k < k1; ++k) {
    prefix[k] = run;
    run += (totals[k] + 63) >> 6;
  }
  if (t == kLayoutThreads - 1) prefix[njobs] = part[t];
  __syncthreads();  // prefix[] is read below by other threads of the block
  for (int k = t; k < njobs; k += kLayoutThreads) *jobs[k].pso_dst = prefix[k] - prefix[jobs[k].s_first];
  for (int i = t; i < ns; i += kLayoutThreads) {
    const SignStream& S = ss[i];
    const int64_t off = prefix[S.first] - prefix[S.f_first];
    const int64_t end = prefix[S.first + S.njob] - prefix[S.f_first];
    if (end > S.ub) {
      sd[i].B = 0;
      atomicOr(err, 1);
    } else {
      sd[i].sign += off;
    }
  }
}

// ------------------------------------------------ negabinary digit planes
// A code q is written in base -2 with B digits: w = (q + A) ^ A in the code's
// width, A the odd bit positions below B (modular arithmetic gives the digits
// exactly whenever q is in the B-digit range).  Digit plane j holds digit
// B - 1 - j of every code; with XOR chaining, stored plane j > 0 is the XOR
// of digit planes j and j - 1.  No sign bits: negabinary has none.
template <typename U>
__device__ __forceinline__ U nb_mask(int B) {
  const U odd = (U)0xAAAAAAAAAAAAAAAAull;
  return B >= (int)(8 * sizeof(U)) ? odd : (odd & (((U)1 << B) - (U)1));
}

// One wave per 4096-code chunk, lane per 64-code word: digit words through
// two half-word LDS stagings and bit-matrix transposes into plane words,
// stored plane-major (with the lossless stage's nonzero-word counts).
template <typename Q, int MAXB>
__global__ __launch_bounds__(64) void k_encode_nb(const StreamDev* __restrict__ sd, int ns) {
  using U = typename UOf<Q>::type;
  constexpr int QW = (int)sizeof(Q) / 4;
  __shared__ __align__(16) Q cst[64 * kRow];
  const int lane = threadIdx.x;
  const int64_t gch = blockIdx.x;
  const int u = find_stream(sd, ns, gch);
  const StreamDev& S = sd[u];
  const int64_t chunk = gch - S.chunk_begin;
  const int B = S.B;
  const int64_t M = S.M, n = S.n;
  const BufRsrc rc = chunk_rsrc<Q>(S.codes, chunk * kChunk, n);
  const U A = nb_mask<U>(B);
  uint64_t P[MAXB];
#pragma unroll
  for (int b = 0; b < MAXB; ++b) P[b] = 0ull;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    stage_half<Q>(rc, h, cst, lane);
    __syncthreads();
#pragma unroll
    for (int p = 0; p < QW; ++p) {
      uint32_t r[32];
#pragma unroll
      for (int k = 0; k < 32; ++k) {
        const U w = ((U)cst[lane * kRow + k] + A) ^ A;
        r[k] = (uint32_t)(w >> (32 * p));
      }
      transpose32(r);
#pragma unroll
      for (int bb = 0; bb < 32; ++bb)
        if (32 * p + bb < MAXB) P[32 * p + bb] |= (uint64_t)r[bb] << (32 * h);
    }
    __syncthreads();
  }
  uint64_t above = 0ull;
#pragma unroll
  for (int b = MAXB - 1; b >= 0; --b) {
    if (b >= B) continue;
    const uint64_t pw = P[b];
    const uint64_t sw = S.xor_chain ? (pw ^ above) : pw;
    above = pw;
    buf_store<uint64_t>(sw, plane_rsrc(S.mag, B - 1 - b, M, chunk), 8u * lane, 0u);
    if (S.zcnt) {
      const uint64_t nzm = __ballot(sw != 0ull);
      if (lane == 0) ((GAS uint32_t*)S.zcnt)[chunk * B + (B - 1 - b)] = (uint32_t)__popcll(nzm);
    }
  }
}

// One wave per chunk, lane per word: stored planes [k0, k1) loaded, the XOR
// chain undone from the digit plane above k0 (read off the resident words),
// transposed back and OR-ed into the resident digit words.
template <typename Q, int MAXB>
__global__ __launch_bounds__(64) void k_decode_nb(const StreamDev* __restrict__ sd, int ns) {
  using U = typename UOf<Q>::type;
  constexpr int QW = (int)sizeof(Q) / 4;
  __shared__ __align__(16) Q cst[64 * kRow];
  const int lane = threadIdx.x;
  const int64_t gch = blockIdx.x;
  const int u = find_stream(sd, ns, gch);
  const StreamDev& S = sd[u];
  const int64_t chunk = gch - S.chunk_begin;
  const int B = S.B, k0 = S.k0, k1 = S.k1;
  const bool fresh = S.fresh != 0;
  const int64_t M = S.M, n = S.n;
  const BufRsrc rc = chunk_rsrc<Q>(S.codes, chunk * kChunk, n);
  uint64_t above = 0ull;  // digit plane k0 - 1 of this lane's 64 codes
  if (S.xor_chain && k0 > 0 && !fresh) {
    const int d = B - k0;  // its digit position
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      stage_half<Q>(rc, h, cst, lane);
      __syncthreads();
#pragma unroll
      for (int k = 0; k < 32; ++k) above |= (uint64_t)(((U)cst[lane * kRow + k] >> d) & (U)1) << (32 * h + k);
      __syncthreads();
    }
  }
  uint64_t P[MAXB];
#pragma unroll
  for (int b = MAXB - 1; b >= 0; --b) {
    const int j = B - 1 - b;
    P[b] = 0ull;
    if (b < B && j >= k0 && j < k1) {
      const uint64_t sw = buf_load<uint64_t>(plane_rsrc(S.mag, j, M, chunk), 8u * lane, 0u);
      const uint64_t pw = S.xor_chain ? (sw ^ above) : sw;
      above = pw;
      P[b] = pw;
    }
  }
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    if (!fresh) {
      stage_half<Q>(rc, h, cst, lane);
      __syncthreads();
    }
    uint32_t nb[QW][32];
#pragma unroll
    for (int p = 0; p < QW; ++p) {
#pragma unroll
      for (int bb = 0; bb < 32; ++bb) nb[p][bb] = (32 * p + bb < MAXB) ? (uint32_t)(P[32 * p + bb] >> (32 * h)) : 0u;
      transpose32(nb[p]);
    }
#pragma unroll
    for (int k = 0; k < 32; ++k) {
      U w = fresh ? (U)0 : (U)cst[lane * kRow + k];
      w |= (U)nb[0][k];
      if constexpr (QW == 2) w |= (U)nb[QW - 1][k] << 32;
      cst[lane * kRow + k] = (Q)w;
    }
    __syncthreads();
    unstage_half<Q>(rc, h, cst, lane);
    __syncthreads();
  }
}

// Zero n 64-bit words at dst of every segment (the sign arenas of a batch,
// cleared in one launch instead of one fill per field).
__global__ __launch_bounds__(kThreads) void k_zero_words(const FlatSeg* __restrict__ segs, int nseg, int64_t nblk) {
  for (int64_t b = blockIdx.x; b < nblk; b += gridDim.x) {
    const int si = find_seg(segs, nseg, b);
    const FlatSeg& S = segs[si];
    GAS uint64_t* dst = (GAS uint64_t*)S.dst;
    const int64_t e0 = (b - S.blk_begin) * kBlockElems;
#pragma unroll 4
    for (int it = 0; it < kPerThread; ++it) {
      const int64_t e = e0 + it * kThreads + threadIdx.x;
      if (e < S.n) dst[e] = 0ull;
    }
  }
}

// The integers of resident digit words truncated to their first k of B
// digit planes: ((w & top k digits) ^ A) - A.
template <typename Q>
__global__ __launch_bounds__(kThreads) void k_nb_values(const FlatSeg* __restrict__ segs, int nseg, int64_t nblk) {
  using U = typename UOf<Q>::type;
  for (int64_t b = blockIdx.x; b < nblk; b += gridDim.x) {
    const int si = find_seg(segs, nseg, b);
    const FlatSeg& S = segs[si];
    const GAS U* src = (const GAS U*)S.src;
    GAS Q* dst = (GAS Q*)S.dst;
    constexpr int kBits = (int)(8 * sizeof(U));
    const U A = nb_mask<U>(S.B);
    const int kk = S.k < S.B ? S.k : S.B;
    const U all = S.B >= kBits ? ~(U)0 : (((U)1 << S.B) - (U)1);          // the B digits
    const U low = S.B - kk >= kBits ? ~(U)0 : (((U)1 << (S.B - kk)) - (U)1);  // the dropped ones
    const U keep = kk <= 0 ? (U)0 : (all & ~low);
    const int64_t e0 = (b - S.blk_begin) * kBlockElems;
#pragma unroll 4
    for (int it = 0; it < kPerThread; ++it) {
      const int64_t e = e0 + it * kThreads + threadIdx.x;
      if (e >= S.n) continue;
      dst[e] = (Q)(((src[e] & keep) ^ A) - A);
    }
  }
}

// ------------------------------------------------ lossless stage (zero words)
// One wave per (stream, plane, chunk) item, lane per magnitude word of the
// chunk; a ballot over the lanes gives the chunk's presence word.
// (The encoder counts each chunk's nonzero words per plane; the index scan
// gives each chunk's count before it and the plane's total.)  MODE 1: the
// stored section of every plane (suppressed: presence word and count by lane
// 0, each nonzero word at its rank; raw: every word).  MODE 2: the raw words
// back from the stored sections (and the counts into zoff, for a later
// MODE 1).  Wave-uniform branches only (on the plane's storage kind).
template <int MODE>
__global__ __launch_bounds__(256) void k_zws(const ZwsSeg* __restrict__ segs, int nseg, int64_t items) {
  const int lane = threadIdx.x & 63;
  const int64_t waves = (int64_t)gridDim.x * (blockDim.x >> 6);
  for (int64_t it = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6); it < items; it += waves) {
    const int si = find_seg(segs, nseg, it);
    const ZwsSeg& S = segs[si];
    const int64_t i = it - S.blk_begin;
    const int64_t C = S.C, M = S.M;
    const int j = (int)(i / C);
    const int64_t c = i - (int64_t)j * C;
    const int64_t w = 64 * c + lane;
    const bool inw = w < M;
    const bool sup = (S.zmask >> j) & 1ull;
    if (MODE == 1) {
      const GAS uint64_t* raw = (const GAS uint64_t*)S.raw_in + (int64_t)j * M;
      const uint64_t v = inw ? raw[w] : 0ull;
      const uint64_t nz = __ballot(v != 0ull);
      GAS uint64_t* out = (GAS uint64_t*)S.comp_out + S.pmo[j];
      if (sup) {
        const uint32_t before = ((const GAS uint32_t*)S.zoff)[(int64_t)j * C + c];
        if (lane == 0) {
          out[c] = nz;
          ((GAS uint32_t*)(out + C))[c] = before;
          if (c == C - 1 && (C & 1)) ((GAS uint32_t*)(out + C))[C] = 0u;  // padding of the counts
        }
        if (v != 0ull) out[C + (C + 1) / 2 + before + __popcll(nz & lanemask_lt(lane))] = v;
      } else if (inw) {
        out[w] = v;
      }
    } else {
      const GAS uint64_t* in = (const GAS uint64_t*)S.comp_in + S.pmo[j];
      GAS uint64_t* raw = (GAS uint64_t*)S.raw_out + (int64_t)j * M;
      if (sup) {
        const uint64_t nz = in[c];
        const uint32_t before = ((const GAS uint32_t*)(in + C))[c];
        const bool has = (nz >> lane) & 1ull;
        const uint64_t v = has ? in[C + (C + 1) / 2 + before + __popcll(nz & lanemask_lt(lane))] : 0ull;
        if (inw) raw[w] = v;
        if (lane == 0) ((GAS uint32_t*)S.zoff)[(int64_t)j * C + c] = before;
      } else if (inw) {
        raw[w] = in[w];
      }
    }
  }
}

// Bits [pos, pos + nb) of a little-endian bit string held in words w.
__device__ __forceinline__ uint64_t extract_bits(const uint64_t* w, int pos, int nb, int nwords) {
  const int w0 = pos >> 6, sh = pos & 63;
  uint64_t v = w[w0] >> sh;
  if (sh && w0 + 1 < nwords) v |= w[w0 + 1] << (64 - sh);
  if (nb < 64) v &= (1ull << nb) - 1ull;
  return v;
}

__device__ __forceinline__ int64_t readlane64(int64_t v, int lane) {
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, lane);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), lane);
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

// Move each chunk's staged sign bits to their place in the stream's sign
// section (dense, plane-major); one wave per chunk.  Lane j fetches plane j's
// count and destination at once, wave scans give each plane's offset in the
// staging and its first destination word, and the destination words of all
// planes are spread over the lanes.  Words shared with a neighbouring chunk
// are combined with atomic OR; whole words are stored.
__global__ __launch_bounds__(64) void k_sign_move(const StreamDev* __restrict__ sd, int ns) {
  __shared__ uint64_t st[64];
  __shared__ int64_t pD[64];     // plane j: first bit of its run in the sign section
  __shared__ uint32_t pc[64];    // plane j: sign bits of this chunk
  __shared__ uint32_t ps[64];    // plane j: first bit of its run in the staging
  __shared__ uint32_t pW[64];    // plane j: first of its destination words, counted over all planes
  const int64_t gch = blockIdx.x;
  const int u = find_stream(sd, ns, gch);
  const StreamDev& S = sd[u];
  const int64_t chunk = gch - S.chunk_begin;
  const int lane = threadIdx.x;
  unsigned long long* sign = (unsigned long long*)S.sign;
  st[lane] = ((const GAS uint64_t*)S.stage)[chunk * 64 + lane];
  uint32_t cj = 0;
  int64_t Dj = 0;
  if (lane < S.B) {
    cj = ((const GAS uint32_t*)S.cnt)[chunk * S.B + lane];
    Dj = ((const GAS int64_t*)S.pso)[lane] * 64 + (int64_t)((const GAS uint32_t*)S.idx)[(int64_t)lane * S.C + chunk];
  }
  const uint32_t nw = cj ? (uint32_t)(((Dj + cj - 1) >> 6) - (Dj >> 6) + 1) : 0u;
  const uint32_t wincl = wave_incl_scan(nw, lane);
  pD[lane] = Dj;
  pc[lane] = cj;
  ps[lane] = wave_incl_scan(cj, lane) - cj;
  pW[lane] = wincl - nw;
  const uint32_t T = (uint32_t)__builtin_amdgcn_readlane((int)wincl, 63);
  __syncthreads();
  // destination words of all planes, flattened, one per lane: the plane of
  // word k is the last one whose first word is <= k (planes without bits
  // share their first word with the next plane, and are passed over)
  for (uint32_t k = lane; k < T; k += 64) {
    int lo = 0, hi = 63;
#pragma unroll
    for (int it = 0; it < 6; ++it) {
      const int mid = (lo + hi + 1) >> 1;
      if (pW[mid] <= k)
        lo = mid;
      else
        hi = mid - 1;
    }
    const int64_t D = pD[lo], c = pc[lo];
    const int64_t w = (D >> 6) + (int64_t)(k - pW[lo]);
    const int64_t blo = max(w * 64, D), bhi = min(w * 64 + 64, D + c);
    const int nb = (int)(bhi - blo);
    const uint64_t bits = extract_bits(st, (int)(blo - D) + (int)ps[lo], nb, 64);
    const uint64_t val = bits << (blo - w * 64);
    if (nb == 64)
      ((GAS unsigned long long*)sign)[w] = val;
    else if (val)
      atomicOr(&sign[w], (unsigned long long)val);
  }
}

// Incremental decode of planes [k0, k1) of each listed stream into its
// resident codes; one wave per chunk, one lane per 64-code word.  The plane
// words are transposed back onto the word's codes.  A code that becomes
// significant at plane j takes the next bit of its (plane, word) cursor in
// the chunk's run of plane-j sign bits, which starts at index[j][chunk]; the
// sign words each plane needs are first copied into LDS.
// FRESH: every stream of the launch starts from zero codes (its first
// decode), so no resident code is read.
template <typename Q, int MAXB, bool FRESH>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(sizeof(Q) == 4 ? 3 : 1))) void k_decode(const StreamDev* __restrict__ sd, int ns) {
  constexpr int QW = (int)sizeof(Q) / 4;
  constexpr int kSignWords = 64 + 2 * MAXB;
  __shared__ Q cst[64 * kRow];
  __shared__ uint32_t ptab[MAXB / 2 * 64];  // cursors, two planes per word (16 bits each)
  __shared__ unsigned long long sw[kSignWords];
  __shared__ int64_t pw0[MAXB];     // first sign word of each decoded plane's run
  __shared__ uint32_t pwoff[MAXB + 1];  // its LDS offset (prefix over decoded planes)
  const int lane = threadIdx.x;
  const int64_t gch = blockIdx.x;
  const int u = find_stream(sd, ns, gch);
  const StreamDev& S = sd[u];
  const int64_t chunk = gch - S.chunk_begin;
  const GAS uint32_t* idx = (const GAS uint32_t*)S.idx;
  const GAS uint64_t* sign = (const GAS uint64_t*)S.sign;
  const GAS int64_t* pso = (const GAS int64_t*)S.pso;
  const int B = S.B, k0 = S.k0, k1 = S.k1;
  const bool fresh = FRESH || S.fresh != 0;
  const int64_t M = S.M, C = S.C, n = S.n, sign_n = S.sign_n;
  const int64_t base = chunk * kChunk;
  const BufRsrc rc = chunk_rsrc<Q>(S.codes, base, n);

  // significance before plane k0 = nonzero resident codes
  uint64_t sig = 0ull;
  if (!fresh) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      stage_half<Q>(rc, h, cst, lane);
      __syncthreads();
#pragma unroll
      for (int k = 0; k < 32; ++k)
        if (cst[lane * kRow + k] != (Q)0) sig |= 1ull << (32 * h + k);
      __syncthreads();
    }
  }
  uint64_t P[MAXB];
#pragma unroll
  for (int b = 0; b < MAXB; ++b) {
    const int j = B - 1 - b;
    P[b] = (b < B && j >= k0 && j < k1) ? buf_load<uint64_t>(plane_rsrc(S.mag, j, M, chunk), 8u * lane, 0u) : 0ull;
  }
  // lane j: first sign bit of plane j's run for this chunk (all planes at once)
  int64_t Dl = 0;
  if (lane >= k0 && lane < k1) Dl = pso[lane] * 64 + (int64_t)idx[(int64_t)lane * C + chunk];
  // newcomer counts -> cursors; runs of sign words to fetch
  uint32_t cc[MAXB], incl[MAXB];
#pragma unroll
  for (int b = MAXB - 1; b >= 0; --b) {
    const uint64_t pw = P[b];  // zero outside the decoded planes
    cc[b] = (uint32_t)__popcll(pw & ~sig);
    incl[b] = cc[b];
    sig |= pw;
  }
  wave_incl_scan_n<MAXB>(incl);
  uint32_t woff = 0;
  int np = 0;
  int64_t mypw0 = 0;
  uint32_t mypwoff = 0;
#pragma unroll
  for (int b = MAXB - 1; b >= 0; --b) {
    const int j = B - 1 - b;
    if (b >= B || j < k0 || j >= k1) continue;
    const uint32_t tot = (uint32_t)__builtin_amdgcn_readlane((int)incl[b], 63);
    const int64_t D = readlane64(Dl, j);
    const uint32_t nw = tot ? (uint32_t)(((D + tot - 1) >> 6) - (D >> 6) + 1) : 0u;
    ((uint16_t*)ptab)[((j >> 1) * 64 + lane) * 2 + (j & 1)] = (uint16_t)(woff * 64 + (uint32_t)(D & 63) + incl[b] - cc[b]);
    mypw0 = lane == np ? (D >> 6) : mypw0;
    mypwoff = lane == np ? woff : mypwoff;
    woff += nw;
    ++np;
  }
  if (lane < np) {
    pw0[lane] = mypw0;
    pwoff[lane] = mypwoff;
  }
  if (lane == 0) pwoff[np] = woff;
  __syncthreads();
  // fetch the sign words of every run (woff <= 64 + 2 * planes by construction)
  for (uint32_t i = lane; i < woff && i < (uint32_t)kSignWords; i += 64) {
    int lo = 0, hi = np - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (pwoff[mid] <= i)
        lo = mid;
      else
        hi = mid - 1;
    }
    const int64_t gw = pw0[lo] + (int64_t)(i - pwoff[lo]);
    sw[i] = (gw >= 0 && gw < sign_n) ? sign[gw] : 0ull;
  }
  __syncthreads();

#pragma unroll
  for (int h = 0; h < 2; ++h) {
    if (!fresh) {
      stage_half<Q>(rc, h, cst, lane);
      __syncthreads();
    }
    uint32_t nb[QW][32];
#pragma unroll
    for (int p = 0; p < QW; ++p) {
#pragma unroll
      for (int bb = 0; bb < 32; ++bb) nb[p][bb] = (32 * p + bb < MAXB) ? (uint32_t)(P[32 * p + bb] >> (32 * h)) : 0u;
      transpose32(nb[p]);
    }
    // Every lane issues every cursor fetch-and-add (adding 0 to its own
    // plane-0 cursor when the code takes no sign bit), 16 codes at a time.
#pragma unroll
    for (int g = 0; g < 32; g += 16) {
      typename MagOf<Q>::type mgs[16];
      uint32_t pos[16];
      bool take[16], negs[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const Q old = fresh ? (Q)0 : cst[lane * kRow + g + k];
        typename MagOf<Q>::type mg;
        if constexpr (QW == 1)
          mg = mag_part(old, 0) | nb[0][g + k];
        else
          mg = absq(old) | (uint64_t)nb[0][g + k] | (uint64_t)nb[QW - 1][g + k] << 32;
        const int j = B - bitlen_of(mg);
        take[k] = old == (Q)0 && mg != 0 && j >= 0 && j < MAXB;
        negs[k] = old < 0;
        mgs[k] = mg;
        const int jj = take[k] ? j : 0;
        pos[k] = (atomicAdd(&ptab[(jj >> 1) * 64 + lane], take[k] ? 1u << (16 * (jj & 1)) : 0u) >> (16 * (jj & 1))) & 0xffffu;
      }
      uint64_t wv[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        take[k] = take[k] & (pos[k] < (uint32_t)(kSignWords * 64));
        wv[k] = sw[(take[k] ? pos[k] : 0u) >> 6];
      }
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const bool sbit = (uint32_t)(wv[k] >> (pos[k] & 63)) & 1u;
        const bool neg = (take[k] & sbit) | (!take[k] & negs[k]);
        cst[lane * kRow + g + k] = neg ? (Q)(-(int64_t)mgs[k]) : (Q)mgs[k];
      }
    }
    __syncthreads();
    unstage_half<Q>(rc, h, cst, lane);
    __syncthreads();
  }
}

// First decode of 32-bit codes whose plans take at most kDW planes (every
// stream of the launch): the algorithm of k_decode with the decoded planes
// held in a window of kDW bit positions [lo, lo + kDW) (half the registers)
// and the codes staged through LDS a quarter word (16 codes) at a time (half
// the LDS), so that more waves fit a CU.
constexpr int kDW = 16;
constexpr int kRowQ = 17;  // LDS row pitch (codes) of the quarter-word staging tile
__device__ __forceinline__ void unstage_quarter(BufRsrc rc, int qi, const int32_t* cst, int lane) {
  const uint32_t k = lane & 15, rr = lane >> 4;  // four rows per store
  const uint32_t o = (16u * qi + k + 64u * rr) * 4u;
#pragma unroll 8
  for (uint32_t it = 0; it < 16; ++it) buf_store<int32_t>(cst[(4 * it + rr) * kRowQ + k], rc, o, 1024u * it);
}
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(4))) void k_decode_w16(const StreamDev* __restrict__ sd, int ns) {
  constexpr int kSignWords = 64 + 2 * kDW;
  __shared__ int32_t cst[64 * kRowQ];
  __shared__ uint32_t ptab[kDW / 2 * 64];  // cursors of planes j < kDW, two per word (16 bits each)
  __shared__ unsigned long long sw[128];  // kSignWords, padded to two whole turns
  __shared__ int64_t pw0[kDW];
  __shared__ uint32_t pwoff[kDW + 1];
  const int lane = threadIdx.x;
  const int64_t gch = blockIdx.x;
  const int u = find_stream(sd, ns, gch);
  const StreamDev& S = sd[u];
  const int64_t chunk = gch - S.chunk_begin;
  const GAS uint32_t* idx = (const GAS uint32_t*)S.idx;
  const GAS uint64_t* sign = (const GAS uint64_t*)S.sign;
  const GAS int64_t* pso = (const GAS int64_t*)S.pso;
  const int B = S.B, k1 = S.k1;  // planes [0, k1), k1 <= kDW
  const int64_t M = S.M, C = S.C, n = S.n, sign_n = S.sign_n;
  const BufRsrc rc = chunk_rsrc<int32_t>(S.codes, chunk * kChunk, n);
  // plane j is bit position B - 1 - j >= B - k1 >= B - kDW: window from lo
  const int lo = B > kDW ? B - kDW : 0;
  uint64_t P[kDW];
#pragma unroll
  for (int r = 0; r < kDW; ++r) {
    const int j = B - 1 - lo - r;
    P[r] = (j >= 0 && j < k1) ? buf_load<uint64_t>(plane_rsrc(S.mag, j, M, chunk), 8u * lane, 0u) : 0ull;
  }
  int64_t Dl = 0;
  if (lane < k1) Dl = pso[lane] * 64 + (int64_t)idx[(int64_t)lane * C + chunk];
  uint32_t cc[kDW], incl[kDW];
  uint64_t sig = 0ull;
#pragma unroll
  for (int r = kDW - 1; r >= 0; --r) {
    const uint64_t pw = P[r];
    cc[r] = (uint32_t)__popcll(pw & ~sig);
    incl[r] = cc[r];
    sig |= pw;
  }
  wave_incl_scan_n<kDW>(incl);
  uint32_t woff = 0;
  int np = 0;
  int64_t mypw0 = 0;
  uint32_t mypwoff = 0;
#pragma unroll
  for (int r = kDW - 1; r >= 0; --r) {
    const int j = B - 1 - lo - r;
    if (j < 0 || j >= k1) continue;
    const uint32_t tot = (uint32_t)__builtin_amdgcn_readlane((int)incl[r], 63);
    const int64_t D = readlane64(Dl, j);
    const uint32_t nw = tot ? (uint32_t)(((D + tot - 1) >> 6) - (D >> 6) + 1) : 0u;
    ((uint16_t*)ptab)[((j >> 1) * 64 + lane) * 2 + (j & 1)] = (uint16_t)(woff * 64 + (uint32_t)(D & 63) + incl[r] - cc[r]);
    mypw0 = lane == np ? (D >> 6) : mypw0;
    mypwoff = lane == np ? woff : mypwoff;
    woff += nw;
    ++np;
  }
  if (lane < np) {
    pw0[lane] = mypw0;
    pwoff[lane] = mypwoff;
  }
  if (lane == 0) pwoff[np] = woff;
  __syncthreads();
  // the sign words of every run (woff <= 64 + 2 * planes by construction),
  // two whole turns; the sign section as a buffer, so a word past it (or a
  // slot past the runs) reads zero without a branch
  const BufRsrc sb = buf_rsrc((const void*)S.sign, sign_n * 8);
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const uint32_t i = lane + 64 * t;
    int lo2 = 0;
#pragma unroll
    for (int st = kDW / 2; st >= 1; st >>= 1)
      if (lo2 + st < np && pwoff[lo2 + st] <= i) lo2 += st;
    const int64_t gw = pw0[lo2] + (int64_t)(i - pwoff[lo2]);
    const bool ok = i < woff && i < (uint32_t)kSignWords && gw >= 0 && gw < sign_n;
    sw[i] = buf_load<uint64_t>(sb, ok ? (uint32_t)gw * 8u : 0x80000000u, 0u);
  }
  __syncthreads();
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    uint32_t x[kDW];
#pragma unroll
    for (int r = 0; r < kDW; ++r) x[r] = (uint32_t)(P[r] >> (32 * h));
    transpose16x2(x);  // low half of x[k]: code 32h + k; high half: code 32h + 16 + k
#pragma unroll
    for (int g = 0; g < 2; ++g) {
      uint32_t mgs[16], pos[16];
      bool take[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const uint32_t mg = (g ? (x[k] >> 16) : (x[k] & 0xffffu)) << lo;
        const int j = B - (mg ? 32 - __clz((int)mg) : 0);
        take[k] = mg != 0u;
        mgs[k] = mg;
        const int jj = take[k] ? j : 0;
        pos[k] = (atomicAdd(&ptab[(jj >> 1) * 64 + lane], take[k] ? 1u << (16 * (jj & 1)) : 0u) >> (16 * (jj & 1))) & 0xffffu;
      }
      uint64_t wv[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        take[k] = take[k] & (pos[k] < (uint32_t)(kSignWords * 64));
        wv[k] = sw[(take[k] ? pos[k] : 0u) >> 6];
      }
#pragma unroll
      for (int k = 0; k < 16; ++k) {
        const bool neg = take[k] & ((uint32_t)(wv[k] >> (pos[k] & 63)) & 1u);
        cst[lane * kRowQ + k] = neg ? -(int32_t)mgs[k] : (int32_t)mgs[k];
      }
      __syncthreads();
      unstage_quarter(rc, 2 * h + g, cst, lane);
      __syncthreads();
    }
  }
}

// ----------------------------------------------------------- reconstruction
template <typename T, typename Q>
__global__ __launch_bounds__(kThreads) void k_coarsest(const FlatSeg* __restrict__ segs, int nseg, int64_t nblk) {
  for (int64_t b = blockIdx.x; b < nblk; b += gridDim.x) {
    const int si = find_seg(segs, nseg, b);
    const FlatSeg& S = segs[si];
    const GAS Q* q = (const GAS Q*)S.src;
    const int64_t e0 = (b - S.blk_begin) * kBlockElems;
#pragma unroll 4
    for (int it = 0; it < kPerThread; ++it) {
      const int64_t e = e0 + it * kThreads + threadIdx.x;
      if (e >= S.n) continue;
      const double x = (double)mask_code<Q>(q[e], S.B, S.k) * S.delta;
      if (S.final_out)
        ((GAS T*)S.dst)[e] = (T)x;
      else
        ((GAS double*)S.dst)[e] = x;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_inject(const FlatSeg* __restrict__ segs, int nseg, int64_t nblk) {
  for (int64_t b = blockIdx.x; b < nblk; b += gridDim.x) {
    const int si = find_seg(segs, nseg, b);
    const FlatSeg& S = segs[si];
    const GAS double* xc = (const GAS double*)S.src;
    const int64_t e0 = (b - S.blk_begin) * kBlockElems;
#pragma unroll 4
    for (int it = 0; it < kPerThread; ++it) {
      const int64_t e = e0 + it * kThreads + threadIdx.x;
      if (e >= S.n) continue;
      const uint32_t r = fdiv((uint32_t)e, S.f2);
      const uint32_t i2 = (uint32_t)e - r * (uint32_t)S.dm[2];
      const uint32_t i0 = fdiv(r, S.f1);
      const uint32_t i1 = r - i0 * (uint32_t)S.dm[1];
      const int64_t o = ((int64_t)(2 * i0) * S.dst_m1 + 2 * i1) * S.dst_m2 + 2 * i2;
      if (S.final_out)
        ((GAS T*)S.dst)[o] = (T)xc[e];
      else
        ((GAS double*)S.dst)[o] = xc[e];
    }
  }
}

// One region of one level: x' = prediction + Delta * q' (Algorithm 2).
// Neighbours on the coarser level come from xc (float64), those in earlier
// regions of this level from their buffers: predictions (per-level) or
// reconstructed values (per-region).
template <typename T, typename Q>
__global__ __launch_bounds__(kThreads) void k_recon(const ReconSeg* __restrict__ segs, int nseg, int64_t nblk) {
  for (int64_t b = blockIdx.x; b < nblk; b += gridDim.x) {
    const int si = find_seg(segs, nseg, b);
    const ReconSeg& S = segs[si];
    const RegionArgs& ra = S.ra;
    const Lattice& L = ra.lat;
    const int64_t total = lat_count(L);
    const int64_t e0 = (b - S.blk_begin) * kBlockElems;
    const int ax = L.ax;
    const GAS Q* q = (const GAS Q*)S.q;
    const int64_t cs[3] = {(int64_t)S.cm1 * S.cm2, (int64_t)S.cm2, 1};
#pragma unroll 4
    for (int it = 0; it < kPerThread; ++it) {
      const int64_t e = e0 + it * kThreads + threadIdx.x;
      if (e >= total) continue;
      int i[3];
      lattice_node(L, (uint32_t)e, i);
      const int j = i[ax];
      const int sk = stencil_kind(j, L.m[ax], ra.degree);
      const int rp = source_region(ra, i);
      double p;
      if (rp < 0) {
        int ci[3];
        for (int a = 0; a < 3; ++a) ci[a] = (a == ax) ? (j - 1) >> 1 : i[a] >> 1;
        const GAS double* pc = (const GAS double*)S.xc + ci[0] * cs[0] + ci[1] * cs[1] + ci[2] * cs[2];
        const int64_t st = cs[ax];
        p = stencil_eval(sk, [&](int o) { return pc[((o + 1) / 2) * st]; });
      } else {
        p = predict_from_region(ra, rp, i, ax, j, sk);
      }
      const double dq = (double)mask_code<Q>(q[e], S.B, S.k) * S.delta;
      const double x = p + dq;
      const int64_t o = ((int64_t)i[0] * L.m[1] + i[1]) * L.m[2] + i[2];
      if (S.final_out)
        ((GAS T*)S.out)[o] = (T)x;
      else
        ((GAS double*)S.out)[o] = x;
      if (ra.pr_out) ((GAS double*)ra.pr_out)[e] = ra.per_level ? p : x;
    }
  }
}

}  // namespace

// ------------------------------------------------------------------ launchers
#define APC_LAUNCH(kern, nblk, ...)                                                    \
  do {                                                                                 \
    if ((nblk) <= 0) return hipSuccess;                                                \
    hipLaunchKernelGGL(kern, dim3(grid_for(nblk)), dim3(kThreads), 0, s, __VA_ARGS__); \
    return hipGetLastError();                                                          \
  } while (0)
// The same with a kernel-specific cap on the grid (measured per kernel).
#define APC_LAUNCH_CAP(kern, nblk, cap, ...)                                                         \
  do {                                                                                               \
    if ((nblk) <= 0) return hipSuccess;                                                              \
    hipLaunchKernelGGL(kern, dim3((unsigned)std::min<int64_t>(nblk, (int64_t)(cap))), dim3(kThreads), \
                       0, s, __VA_ARGS__);                                                           \
    return hipGetLastError();                                                                        \
  } while (0)

template <typename T>
hipError_t launch_range(const FlatSeg* segs, int nseg, int64_t nblk, hipStream_t s) {
  APC_LAUNCH((k_range<T>), nblk, segs, nseg, nblk);
}
template <typename T>
hipError_t launch_gather(const FlatSeg* segs, int nseg, int64_t nblk, hipStream_t s) {
  APC_LAUNCH((k_gather<T>), nblk, segs, nseg, nblk);
}
template <typename T, typename Q>
hipError_t launch_coef(const CoefSeg* segs, int nseg, int64_t nblk, int mode, hipStream_t s) {
  if (mode == 0) APC_LAUNCH((k_coef<T, Q, 0>), nblk, segs, nseg, nblk);
  APC_LAUNCH((k_coef<T, Q, 1>), nblk, segs, nseg, nblk);
}
template <typename T, typename Q, int MODE>
hipError_t launch_level_mode(const LevelSeg* segs, int nseg, int64_t nblk, int t2, hipStream_t s) {
  if (t2 == 1) APC_LAUNCH((k_level<T, Q, MODE, 1>), nblk, segs, nseg, nblk);
  if (t2 == 32) APC_LAUNCH((k_level<T, Q, MODE, 32>), nblk, segs, nseg, nblk);
  if (t2 == 128) APC_LAUNCH((k_level<T, Q, MODE, 128>), nblk, segs, nseg, nblk);
  APC_LAUNCH((k_level<T, Q, MODE, 64>), nblk, segs, nseg, nblk);
}
template <typename T, typename Q>
hipError_t launch_level(const LevelSeg* segs, int nseg, int64_t nblk, int mode, int t2, hipStream_t s) {
  if (mode == 0) return launch_level_mode<T, Q, 0>(segs, nseg, nblk, t2, s);
  if (mode == 1) return launch_level_mode<T, Q, 1>(segs, nseg, nblk, t2, s);
  if (mode == 2) return launch_level_mode<T, Q, 2>(segs, nseg, nblk, t2, s);
  return launch_level_mode<T, Q, 3>(segs, nseg, nblk, t2, s);
}
template <typename T, typename Q>
hipError_t launch_coarse(const FlatSeg* segs, int nseg, int64_t nblk, int mode, hipStream_t s) {
  if (mode == 0) APC_LAUNCH((k_coarse<T, Q, 0>), nblk, segs, nseg, nblk);
  APC_LAUNCH((k_coarse<T, Q, 1>), nblk, segs, nseg, nblk);
}
template <typename Q>
hipError_t launch_cd_forward(const CDSeg* segs, int nseg, int64_t nblk, int a, int tiled, hipStream_t s) {
  if (tiled) {  // row tiles (v along rows)
    if (a == 0) APC_LAUNCH((k_cd_forward_tile<Q, 0>), nblk, segs, nseg, nblk);
    APC_LAUNCH((k_cd_forward_tile<Q, 1>), nblk, segs, nseg, nblk);
  }
  if (a == 0) APC_LAUNCH((k_cd_forward<Q, 0>), nblk, segs, nseg, nblk);
  if (a == 1) APC_LAUNCH((k_cd_forward<Q, 1>), nblk, segs, nseg, nblk);
  APC_LAUNCH((k_cd_forward<Q, 2>), nblk, segs, nseg, nblk);
}
template <typename Q>
hipError_t launch_cd_inverse(const CDSeg* segs, int nseg, int64_t nblk, int a, int phase, hipStream_t s) {
  if (phase == 2) {  // one pass over row tiles (v along rows)
    // one tile per block: measured faster than a grid-stride loop here
    if (a == 0) APC_LAUNCH_CAP((k_cd_inverse_tile<Q, 0>), nblk, 1 << 20, segs, nseg, nblk);
    APC_LAUNCH_CAP((k_cd_inverse_tile<Q, 1>), nblk, 1 << 20, segs, nseg, nblk);
  }
  if (phase == 0) {
    if (a == 0) APC_LAUNCH((k_cd_inverse<Q, 0, 0>), nblk, segs, nseg, nblk);
    if (a == 1) APC_LAUNCH((k_cd_inverse<Q, 0, 1>), nblk, segs, nseg, nblk);
    APC_LAUNCH((k_cd_inverse<Q, 0, 2>), nblk, segs, nseg, nblk);
  }
  if (a == 0) APC_LAUNCH((k_cd_inverse<Q, 1, 0>), nblk, segs, nseg, nblk);
  if (a == 1) APC_LAUNCH((k_cd_inverse<Q, 1, 1>), nblk, segs, nseg, nblk);
  APC_LAUNCH((k_cd_inverse<Q, 1, 2>), nblk, segs, nseg, nblk);
}
template <typename Q>
hipError_t launch_encode(const StreamDev* sd, int ns, int64_t chunks, hipStream_t s) {
  if (chunks <= 0) return hipSuccess;
  constexpr int MAXB = sizeof(Q) == 4 ? 32 : 64;
  hipLaunchKernelGGL((k_encode<Q, MAXB>), dim3((unsigned)chunks), dim3(64), 0, s, sd, ns);
  return hipGetLastError();
}
hipError_t launch_scan(const StreamDev* sd, const int32_t* job_s, const int32_t* job_j, int njobs, int64_t* totals,
                       hipStream_t s) {
  if (njobs <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_scan, dim3(njobs), dim3(kThreads), 0, s, sd, job_s, job_j, totals);
  return hipGetLastError();
}
hipError_t launch_sign_layout(const int64_t* totals, int njobs, const SignJob* jobs, int ns, const SignStream* ss,
                              StreamDev* sd, int64_t* prefix, int32_t* err, hipStream_t s) {
  if (njobs <= 0 || ns <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sign_layout, dim3(1), dim3(kLayoutThreads), 0, s, totals, njobs, jobs, ns, ss, sd, prefix, err);
  return hipGetLastError();
}
hipError_t launch_sign_move(const StreamDev* sd, int ns, int64_t chunks, hipStream_t s) {
  if (chunks <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_sign_move, dim3((unsigned)chunks), dim3(64), 0, s, sd, ns);
  return hipGetLastError();
}
template <typename Q>
hipError_t launch_encode_nb(const StreamDev* sd, int ns, int64_t chunks, hipStream_t s) {
  if (chunks <= 0) return hipSuccess;
  constexpr int MAXB = sizeof(Q) == 4 ? 32 : 64;
  hipLaunchKernelGGL((k_encode_nb<Q, MAXB>), dim3((unsigned)chunks), dim3(64), 0, s, sd, ns);
  return hipGetLastError();
}
template <typename Q>
hipError_t launch_decode_nb(const StreamDev* sd, int ns, int64_t chunks, hipStream_t s) {
  if (chunks <= 0) return hipSuccess;
  constexpr int MAXB = sizeof(Q) == 4 ? 32 : 64;
  hipLaunchKernelGGL((k_decode_nb<Q, MAXB>), dim3((unsigned)chunks), dim3(64), 0, s, sd, ns);
  return hipGetLastError();
}
hipError_t launch_zero_words(const FlatSeg* segs, int nseg, int64_t nblk, hipStream_t s) {
  APC_LAUNCH(k_zero_words, nblk, segs, nseg, nblk);
}
template <typename Q>
hipError_t launch_nb_values(const FlatSeg* segs, int nseg, int64_t nblk, hipStream_t s) {
  APC_LAUNCH((k_nb_values<Q>), nblk, segs, nseg, nblk);
}
template hipError_t launch_encode_nb<int32_t>(const StreamDev*, int, int64_t, hipStream_t);
template hipError_t launch_encode_nb<int64_t>(const StreamDev*, int, int64_t, hipStream_t);
template hipError_t launch_decode_nb<int32_t>(const StreamDev*, int, int64_t, hipStream_t);
template hipError_t launch_decode_nb<int64_t>(const StreamDev*, int, int64_t, hipStream_t);
template hipError_t launch_nb_values<int32_t>(const FlatSeg*, int, int64_t, hipStream_t);
template hipError_t launch_nb_values<int64_t>(const FlatSeg*, int, int64_t, hipStream_t);
hipError_t launch_zws(const ZwsSeg* segs, int nseg, int64_t items, int mode, hipStream_t s) {
  if (items <= 0) return hipSuccess;
  const unsigned grid = (unsigned)std::min<int64_t>((items + 3) / 4, (int64_t)kMaxGrid);
  if (mode == 1)
    hipLaunchKernelGGL(k_zws<1>, dim3(grid), dim3(256), 0, s, segs, nseg, items);
  else if (mode == 2)
    hipLaunchKernelGGL(k_zws<2>, dim3(grid), dim3(256), 0, s, segs, nseg, items);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}
template <typename Q>
hipError_t launch_decode(const StreamDev* sd, int ns, int64_t chunks, bool all_fresh, int max_planes, hipStream_t s) {
  if (chunks <= 0) return hipSuccess;
  constexpr int MAXB = sizeof(Q) == 4 ? 32 : 64;
  if (sizeof(Q) == 4 && all_fresh && max_planes <= kDW)
    hipLaunchKernelGGL(k_decode_w16, dim3((unsigned)chunks), dim3(64), 0, s, sd, ns);
  else if (all_fresh)
    hipLaunchKernelGGL((k_decode<Q, MAXB, true>), dim3((unsigned)chunks), dim3(64), 0, s, sd, ns);
  else
    hipLaunchKernelGGL((k_decode<Q, MAXB, false>), dim3((unsigned)chunks), dim3(64), 0, s, sd, ns);
  return hipGetLastError();
}
template <typename T, typename Q>
hipError_t launch_coarsest(const FlatSeg* segs, int nseg, int64_t nblk, hipStream_t s) {
  APC_LAUNCH((k_coarsest<T, Q>), nblk, segs, nseg, nblk);
}
template <typename T>
hipError_t launch_inject(const FlatSeg* segs, int nseg, int64_t nblk, hipStream_t s) {
  APC_LAUNCH((k_inject<T>), nblk, segs, nseg, nblk);
}
template <typename T, typename Q>
hipError_t launch_recon(const ReconSeg* segs, int nseg, int64_t nblk, hipStream_t s) {
  APC_LAUNCH((k_recon<T, Q>), nblk, segs, nseg, nblk);
}
#undef APC_LAUNCH

// explicit instantiations
template hipError_t launch_range<float>(const FlatSeg*, int, int64_t, hipStream_t);
template hipError_t launch_range<double>(const FlatSeg*, int, int64_t, hipStream_t);
template hipError_t launch_gather<float>(const FlatSeg*, int, int64_t, hipStream_t);
template hipError_t launch_gather<double>(const FlatSeg*, int, int64_t, hipStream_t);
template hipError_t launch_coef<float, int32_t>(const CoefSeg*, int, int64_t, int, hipStream_t);
template hipError_t launch_coef<double, int64_t>(const CoefSeg*, int, int64_t, int, hipStream_t);
template hipError_t launch_level<float, int32_t>(const LevelSeg*, int, int64_t, int, int, hipStream_t);
template hipError_t launch_level<double, int64_t>(const LevelSeg*, int, int64_t, int, int, hipStream_t);
template hipError_t launch_coarse<float, int32_t>(const FlatSeg*, int, int64_t, int, hipStream_t);
template hipError_t launch_coarse<double, int64_t>(const FlatSeg*, int, int64_t, int, hipStream_t);
template hipError_t launch_cd_forward<int32_t>(const CDSeg*, int, int64_t, int, int, hipStream_t);
template hipError_t launch_cd_forward<int64_t>(const CDSeg*, int, int64_t, int, int, hipStream_t);
template hipError_t launch_cd_inverse<int32_t>(const CDSeg*, int, int64_t, int, int, hipStream_t);
template hipError_t launch_cd_inverse<int64_t>(const CDSeg*, int, int64_t, int, int, hipStream_t);
template hipError_t launch_encode<int32_t>(const StreamDev*, int, int64_t, hipStream_t);
template hipError_t launch_encode<int64_t>(const StreamDev*, int, int64_t, hipStream_t);
template hipError_t launch_decode<int32_t>(const StreamDev*, int, int64_t, bool, int, hipStream_t);
template hipError_t launch_decode<int64_t>(const StreamDev*, int, int64_t, bool, int, hipStream_t);
template hipError_t launch_coarsest<float, int32_t>(const FlatSeg*, int, int64_t, hipStream_t);
template hipError_t launch_coarsest<double, int64_t>(const FlatSeg*, int, int64_t, hipStream_t);
template hipError_t launch_inject<float>(const FlatSeg*, int, int64_t, hipStream_t);
template hipError_t launch_inject<double>(const FlatSeg*, int, int64_t, hipStream_t);
template hipError_t launch_recon<float, int32_t>(const ReconSeg*, int, int64_t, hipStream_t);
template hipError_t launch_recon<double, int64_t>(const ReconSeg*, int, int64_t, hipStream_t);

}  // namespace apc
