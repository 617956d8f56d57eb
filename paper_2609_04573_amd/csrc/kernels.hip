// gfx950 kernels of the progressive compressor.  Wave64 throughout: the
// bitplane transpose uses one ballot per plane per 64-code word, and the sign
// bits of newly significant codes are ranked with popcounts of ballot masks.
//
// Floating point: every interpolation is evaluated in float64 with exactly
// the operation order of the stencil definitions (the library is built with
// -ffp-contract=off, so no multiply-add is fused).  Codes are exact integers.
#include <algorithm>

#include "apc_internal.h"

namespace apc {

namespace {

constexpr int kThreads = 256;

enum { ST_COPY = 0, ST_LINEAR = 1, ST_LQUAD = 2, ST_RQUAD = 3, ST_CUBIC = 4 };

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

__device__ __forceinline__ uint64_t lanemask_lt(int lane) {
  return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

__device__ __forceinline__ int bitlen64(uint64_t v) { return v ? 64 - __clzll((long long)v) : 0; }

template <typename Q>
__device__ __forceinline__ uint64_t absq(Q q) {
  return q < 0 ? (uint64_t)(-(int64_t)q) : (uint64_t)q;
}

// Codes truncated to the first k of B planes (low B-k bits cleared).
template <typename Q>
__device__ __forceinline__ Q mask_code(Q q, int B, int k) {
  if (k >= B) return q;
  if (k <= 0) return 0;
  const uint64_t m = absq(q) & ~((1ull << (B - k)) - 1ull);
  return q < 0 ? (Q)(-(int64_t)m) : (Q)m;
}

__device__ __forceinline__ void block_max_atomic(double v, unsigned long long* dst) {
  for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off));
  __shared__ double sm[kThreads / 64];
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m = sm[0];
    for (int w = 1; w < kThreads / 64; ++w) m = fmax(m, sm[w]);
    atomicMax(dst, (unsigned long long)__double_as_longlong(m));
  }
}

__device__ __forceinline__ unsigned long long ordered_bits(double d) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(d);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v, int lane) {
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t t = __shfl_up(v, off);
    if (lane >= off) v += t;
  }
  return v;
}

// Lattice element e -> node coordinates.
__device__ __forceinline__ void lattice_node(const Lattice& L, int64_t e, int i[3], int t[3]) {
  t[2] = (int)(e % L.c[2]);
  const int64_t r = e / L.c[2];
  t[1] = (int)(r % L.c[1]);
  t[0] = (int)(r / L.c[1]);
  for (int a = 0; a < 3; ++a) i[a] = node_of(t[a], L.kind[a]);
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
  const Lattice& PL = ra.prl[rp];
  int tt[3];
  for (int a = 0; a < 3; ++a) tt[a] = (a == ax) ? (j - 1) >> 1 : lat_of(i[a], PL.kind[a]);
  const int64_t ls[3] = {(int64_t)PL.c[1] * PL.c[2], (int64_t)PL.c[2], 1};
  const double* pp = ra.pr[rp] + tt[0] * ls[0] + tt[1] * ls[1] + tt[2] * ls[2];
  const int64_t st = ls[ax];
  return stencil_eval(sk, [&](int o) { return pp[((o + 1) / 2) * st]; });
}

// ------------------------------------------------------------- range pass
template <typename T>
__global__ __launch_bounds__(kThreads) void k_range(const T* __restrict__ x, int64_t n,
                                                     unsigned long long* acc) {
  double lo = INFINITY, hi = -INFINITY, am = 0.0;
  unsigned long long bad = 0;
  for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < n; i += (int64_t)gridDim.x * kThreads) {
    const double v = (double)x[i];
    if (!isfinite(v)) {
      bad = 1;
      continue;
    }
    lo = fmin(lo, v);
    hi = fmax(hi, v);
    am = fmax(am, fabs(v));
  }
  for (int off = 32; off > 0; off >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, off));
    hi = fmax(hi, __shfl_xor(hi, off));
    am = fmax(am, __shfl_xor(am, off));
  }
  __shared__ double s[3][kThreads / 64];
  __shared__ unsigned long long sbad;
  if (threadIdx.x == 0) sbad = 0;
  __syncthreads();
  if (bad) atomicOr(&sbad, 1ull);
  if ((threadIdx.x & 63) == 0) {
    s[0][threadIdx.x >> 6] = lo;
    s[1][threadIdx.x >> 6] = hi;
    s[2][threadIdx.x >> 6] = am;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kThreads / 64; ++w) {
      lo = fmin(s[0][0], s[0][w]);
      s[0][0] = lo;
      s[1][0] = fmax(s[1][0], s[1][w]);
      s[2][0] = fmax(s[2][0], s[2][w]);
    }
    if (s[0][0] <= s[1][0]) {
      atomicMin(&acc[0], ordered_bits(s[0][0]));
      atomicMax(&acc[1], ordered_bits(s[1][0]));
    }
    atomicMax(&acc[2], (unsigned long long)__double_as_longlong(s[2][0]));
    if (sbad) atomicOr(&acc[3], 1ull);
  }
}

// --------------------------------------------------- compact coarser level
template <typename T>
__global__ __launch_bounds__(kThreads) void k_subsample(const T* __restrict__ src, int s1, int s2,
                                                         T* __restrict__ dst, int d0, int d1, int d2) {
  const int64_t n = (int64_t)d0 * d1 * d2;
  const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (e >= n) return;
  const int i2 = (int)(e % d2);
  const int64_t r = e / d2;
  const int i1 = (int)(r % d1);
  const int i0 = (int)(r / d1);
  dst[e] = src[((int64_t)(2 * i0) * s1 + 2 * i1) * s2 + 2 * i2];
}

// ------------------------------------------- refactor: coefficients of a region
// MODE 0: max |c| into gmax.  MODE 1: q = rint(c * 2^k_shift) into codes.
// Per-level: the predictions of this region are stored in pr_out for the
// regions after it; neighbours in earlier regions are their predictions.
// Per-region: every neighbour is an original value (no pre-quantization).
template <typename T, typename Q, int MODE>
__global__ __launch_bounds__(kThreads) void k_coef(const T* __restrict__ G, RegionArgs ra,
                                                    unsigned long long* gmax, int k_shift, Q* __restrict__ codes) {
  const Lattice& L = ra.lat;
  const int64_t total = (int64_t)L.c[0] * L.c[1] * L.c[2];
  double am = 0.0;
  for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < total; e += (int64_t)gridDim.x * kThreads) {
    int i[3], t[3];
    lattice_node(L, e, i, t);
    const int ax = L.ax;
    const int j = i[ax];
    const int sk = stencil_kind(j, L.m[ax], ra.degree);
    const int64_t gs[3] = {(int64_t)L.m[1] * L.m[2], (int64_t)L.m[2], 1};
    const int64_t gbase = i[0] * gs[0] + i[1] * gs[1] + i[2] * gs[2];
    const double xv = (double)G[gbase];
    const int rp = ra.per_level ? source_region(ra, i) : -1;
    double p;
    if (rp < 0) {
      const T* g = G + gbase;
      const int64_t st = gs[ax];
      p = stencil_eval(sk, [&](int o) { return (double)g[o * st]; });
    } else {
      p = predict_from_region(ra, rp, i, ax, j, sk);
    }
    if (ra.pr_out) ra.pr_out[e] = p;
    const double c = xv - p;
    if (MODE == 0) {
      am = fmax(am, fabs(c));
    } else {
      codes[e] = (Q)(long long)rint(ldexp(c, k_shift));
    }
  }
  if (MODE == 0) block_max_atomic(am, gmax);
}

// Coarsest level: the values themselves are the coefficients.
template <typename T, typename Q, int MODE>
__global__ __launch_bounds__(kThreads) void k_coarse(const T* __restrict__ G, int64_t n, unsigned long long* gmax,
                                                      int k_shift, Q* __restrict__ codes) {
  const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  double am = 0.0;
  if (e < n) {
    const double v = (double)G[e];
    if (MODE == 0)
      am = fabs(v);
    else
      codes[e] = (Q)(long long)rint(ldexp(v, k_shift));
  }
  if (MODE == 0) block_max_atomic(am, gmax);
}

// ---------------------------------------------- coefficient decomposition
__device__ __forceinline__ int64_t avg2(int64_t x, int64_t y) { return (x + y) >> 1; }

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
// Position of lattice element t among the elements of class cls, in
// row-major order of the lattice.
template <int A, int U, int V>
__device__ __forceinline__ int64_t class_rank(int cls, const int t[3], const CDArgs& ca) {
  int64_t total = 0;
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    Rng1 r[3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
      r[a] = (a < s) ? rng_single(t[a]) : (a == s ? rng_prefix(t[a]) : rng_prefix(ca.c[a]));
    total += r[A].call * cls_count(cls, r[U], r[V]);
  }
  return total;
}
__device__ __forceinline__ int cd_class(int u, int v) {
  if ((u & 3) == 0 && (v & 3) == 0) return 0;
  if ((u & 1) == 0 && (v & 1) == 0) return 1;
  return 2;
}

template <typename Q>
__device__ __forceinline__ void block_max3_atomic(double v[3], unsigned long long* dst, const int32_t idx[3]) {
  __shared__ double sm[3][kThreads / 64];
  for (int c = 0; c < 3; ++c) {
    double x = v[c];
    for (int off = 32; off > 0; off >>= 1) x = fmax(x, __shfl_xor(x, off));
    if ((threadIdx.x & 63) == 0) sm[c][threadIdx.x >> 6] = x;
  }
  __syncthreads();
  if (threadIdx.x < 3) {
    double m = sm[threadIdx.x][0];
    for (int w = 1; w < kThreads / 64; ++w) m = fmax(m, sm[threadIdx.x][w]);
    atomicMax(&dst[idx[threadIdx.x]], (unsigned long long)__double_as_longlong(m));
  }
}

// Forward 2D integer lifting of one region lattice into S1/S2/S3.
template <typename Q, int A, int U, int V>
__global__ __launch_bounds__(kThreads) void k_cd_forward(const Q* __restrict__ R, CDArgs ca, Q* __restrict__ out,
                                                          unsigned long long* smax) {
  const int64_t total = (int64_t)ca.c[0] * ca.c[1] * ca.c[2];
  const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  double am[3] = {0.0, 0.0, 0.0};
  if (e < total) {
    int t[3];
    t[2] = (int)(e % ca.c[2]);
    const int64_t r = e / ca.c[2];
    t[1] = (int)(r % ca.c[1]);
    t[0] = (int)(r / ca.c[1]);
    const int u = t[U], v = t[V];
    const int Nu = ca.c[U], Nv = ca.c[V];
    const int64_t ls[3] = {(int64_t)ca.c[1] * ca.c[2], (int64_t)ca.c[2], 1};
    const int64_t su = ls[U], sv = ls[V];
    auto T = [&](int uu, int vv) -> int64_t { return (int64_t)R[e + (int64_t)(uu - u) * su + (int64_t)(vv - v) * sv]; };
    const int cls = cd_class(u, v);
    int64_t res;
    if (cls == 0) {
      res = T(u, v);
    } else if (cls == 1) {
      int64_t p;
      if ((u & 3) == 0) {
        p = (v + 2 <= Nv - 1) ? avg2(T(u, v - 2), T(u, v + 2)) : T(u, v - 2);
      } else {
        auto W = [&](int uu) -> int64_t {
          if ((v & 3) == 0) return T(uu, v);
          return (v + 2 <= Nv - 1) ? avg2(T(uu, v - 2), T(uu, v + 2)) : T(uu, v - 2);
        };
        p = (u + 2 <= Nu - 1) ? avg2(W(u - 2), W(u + 2)) : W(u - 2);
      }
      res = T(u, v) - p;
    } else {
      int64_t p;
      if ((u & 1) == 0) {
        p = (v + 1 <= Nv - 1) ? avg2(T(u, v - 1), T(u, v + 1)) : T(u, v - 1);
      } else {
        auto W0 = [&](int uu) -> int64_t {
          if ((v & 1) == 0) return T(uu, v);
          return (v + 1 <= Nv - 1) ? avg2(T(uu, v - 1), T(uu, v + 1)) : T(uu, v - 1);
        };
        p = (u + 1 <= Nu - 1) ? avg2(W0(u - 1), W0(u + 1)) : W0(u - 1);
      }
      res = T(u, v) - p;
    }
    out[ca.s_off[cls] + class_rank<A, U, V>(cls, t, ca)] = (Q)res;
    am[cls] = (double)(res < 0 ? -res : res);
  }
  block_max3_atomic<Q>(am, smax, ca.s_idx);
}

// Inverse lifting.  PHASE 0 rebuilds the stride-2 points (S1 and S2 classes)
// from the truncated S1/S2 streams; PHASE 1 rebuilds the rest from S3 and the
// stride-2 points written by phase 0.
template <typename Q, int PHASE, int A, int U, int V>
__global__ __launch_bounds__(kThreads) void k_cd_inverse(const Q* __restrict__ S, CDArgs ca, Q* __restrict__ out) {
  const int64_t total = (int64_t)ca.c[0] * ca.c[1] * ca.c[2];
  const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (e >= total) return;
  int t[3];
  t[2] = (int)(e % ca.c[2]);
  const int64_t r = e / ca.c[2];
  t[1] = (int)(r % ca.c[1]);
  t[0] = (int)(r / ca.c[1]);
  const int u = t[U], v = t[V];
  const int Nu = ca.c[U], Nv = ca.c[V];
  const int cls = cd_class(u, v);
  if (PHASE == 0 && cls == 2) return;
  if (PHASE == 1 && cls != 2) return;
  auto stream_val = [&](int c, int uu, int vv) -> int64_t {
    int tt[3] = {t[0], t[1], t[2]};
    tt[U] = uu;
    tt[V] = vv;
    return (int64_t)mask_code<Q>(S[ca.s_off[c] + class_rank<A, U, V>(c, tt, ca)], ca.B[c], ca.k[c]);
  };
  if (PHASE == 0) {
    int64_t val;
    if (cls == 0) {
      val = stream_val(0, u, v);
    } else {
      auto H2 = [&](int uu, int vv) -> int64_t { return stream_val(0, uu, vv); };
      int64_t p;
      if ((u & 3) == 0) {
        p = (v + 2 <= Nv - 1) ? avg2(H2(u, v - 2), H2(u, v + 2)) : H2(u, v - 2);
      } else {
        auto W = [&](int uu) -> int64_t {
          if ((v & 3) == 0) return H2(uu, v);
          return (v + 2 <= Nv - 1) ? avg2(H2(uu, v - 2), H2(uu, v + 2)) : H2(uu, v - 2);
        };
        p = (u + 2 <= Nu - 1) ? avg2(W(u - 2), W(u + 2)) : W(u - 2);
      }
      val = stream_val(1, u, v) + p;
    }
    out[e] = (Q)val;
  } else {
    const int64_t ls[3] = {(int64_t)ca.c[1] * ca.c[2], (int64_t)ca.c[2], 1};
    const int64_t su = ls[U], sv = ls[V];
    auto H1 = [&](int uu, int vv) -> int64_t { return (int64_t)out[e + (int64_t)(uu - u) * su + (int64_t)(vv - v) * sv]; };
    int64_t p;
    if ((u & 1) == 0) {
      p = (v + 1 <= Nv - 1) ? avg2(H1(u, v - 1), H1(u, v + 1)) : H1(u, v - 1);
    } else {
      auto W0 = [&](int uu) -> int64_t {
        if ((v & 1) == 0) return H1(uu, v);
        return (v + 1 <= Nv - 1) ? avg2(H1(uu, v - 1), H1(uu, v + 1)) : H1(uu, v - 1);
      };
      p = (u + 1 <= Nu - 1) ? avg2(W0(u - 1), W0(u + 1)) : W0(u - 1);
    }
    out[e] = (Q)(stream_val(2, u, v) + p);
  }
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
  return lo;
}

// One block per 4096-code chunk: magnitude words of every plane (one ballot
// per plane per word, written plane-major and coalesced from LDS), per-plane
// counts of codes whose leading bit is that plane, and the chunk's sign bits
// packed in chunk-local plane-major order.
template <typename Q, int MAXB>
__global__ __launch_bounds__(kThreads) void k_encode(const Q* __restrict__ codes, const Q* __restrict__ cd_codes,
                                                      const StreamDev* __restrict__ sd, int ns,
                                                      uint64_t* __restrict__ mag, uint32_t* __restrict__ cnt,
                                                      uint64_t* __restrict__ stage) {
  __shared__ uint64_t magbuf[MAXB][64];
  __shared__ uint16_t wpre[MAXB][64];
  __shared__ uint32_t tot[MAXB];
  __shared__ uint32_t toff[MAXB];
  __shared__ unsigned long long sstage[64];
  __shared__ int s_u;
  const int64_t gch = blockIdx.x;
  if (threadIdx.x == 0) s_u = find_stream(sd, ns, gch);
  if (threadIdx.x < 64) sstage[threadIdx.x] = 0ull;
  __syncthreads();
  const StreamDev S = sd[s_u];
  const int64_t chunk = gch - S.chunk_begin;
  const Q* src = (S.use_cd ? cd_codes : codes) + S.code_off;
  const int B = S.B;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const uint64_t lt = lanemask_lt(lane);

  int blen_r[16];
  int neg_r[16];
  int rank_r[16];
#pragma unroll
  for (int it = 0; it < 16; ++it) {
    const int wl = wave + 4 * it;
    const int64_t idx = (chunk * 64 + wl) * 64 + lane;
    const Q qv = (idx < S.n) ? src[idx] : (Q)0;
    const uint64_t mg = absq(qv);
    const int bl = bitlen64(mg);
    blen_r[it] = bl;
    neg_r[it] = qv < 0;
    int rk = 0;
    for (int j = 0; j < B; ++j) {
      const int b = B - 1 - j;
      const uint64_t mw = __ballot((mg >> b) & 1ull);
      const uint64_t nsm = __ballot(bl == b + 1);
      if (lane == 0) {
        magbuf[j][wl] = mw;
        wpre[j][wl] = (uint16_t)__popcll(nsm);
      }
      if (bl == b + 1) rk = __popcll(nsm & lt);
    }
    rank_r[it] = rk;
  }
  __syncthreads();
  for (int j = wave; j < B; j += 4) {
    const uint32_t v = wpre[j][lane];
    const uint32_t incl = wave_incl_scan(v, lane);
    wpre[j][lane] = (uint16_t)(incl - v);
    if (lane == 63) tot[j] = incl;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t off = 0;
    for (int j = 0; j < B; ++j) {
      toff[j] = off;
      off += tot[j];
      cnt[S.cnt_off + (int64_t)j * S.C + chunk] = tot[j];
    }
  }
  for (int j = wave; j < B; j += 4) {
    const int64_t w = chunk * 64 + lane;
    if (w < S.M) mag[S.mag_off + (int64_t)j * S.M + w] = magbuf[j][lane];
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < 16; ++it) {
    const int bl = blen_r[it];
    if (bl > 0 && neg_r[it]) {
      const int j = B - bl;
      const int wl = wave + 4 * it;
      const uint32_t pos = toff[j] + wpre[j][wl] + rank_r[it];
      atomicOr(&sstage[pos >> 6], 1ull << (pos & 63));
    }
  }
  __syncthreads();
  if (threadIdx.x < 64) stage[S.stage_off + chunk * 64 + threadIdx.x] = sstage[threadIdx.x];
}

// Exclusive scan of the per-chunk counts of one (stream, plane): the index
// section entries and the plane's total.
__global__ __launch_bounds__(kThreads) void k_scan(const StreamDev* __restrict__ sd, const int32_t* job_s,
                                                    const int32_t* job_j, const uint32_t* __restrict__ cnt,
                                                    uint32_t* __restrict__ idx, int64_t* totals) {
  __shared__ uint32_t wsum[kThreads / 64];
  const int job = blockIdx.x;
  const StreamDev S = sd[job_s[job]];
  const int j = job_j[job];
  const uint32_t* c = cnt + S.cnt_off + (int64_t)j * S.C;
  uint32_t* o = idx + S.idx_off + (int64_t)j * S.C;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  uint64_t carry = 0;
  for (int64_t base = 0; base < S.C; base += kThreads) {
    const int64_t i = base + threadIdx.x;
    const uint32_t v = (i < S.C) ? c[i] : 0u;
    const uint32_t incl = wave_incl_scan(v, lane);
    if (lane == 63) wsum[wave] = incl;
    __syncthreads();
    uint32_t before = 0, all = 0;
    for (int w = 0; w < kThreads / 64; ++w) {
      if (w < wave) before += wsum[w];
      all += wsum[w];
    }
    if (i < S.C) o[i] = (uint32_t)(carry + before + incl - v);
    carry += all;
    __syncthreads();
  }
  if (threadIdx.x == 0) totals[job] = (int64_t)carry;
}

__device__ __forceinline__ uint64_t extract_bits(const uint64_t* w, int pos, int nb, int nwords) {
  const int w0 = pos >> 6, sh = pos & 63;
  uint64_t v = w[w0] >> sh;
  if (sh && w0 + 1 < nwords) v |= w[w0 + 1] << (64 - sh);
  if (nb < 64) v &= (1ull << nb) - 1ull;
  return v;
}

// Move each chunk's staged sign bits to their place in the stream's sign
// section (dense, plane-major).  Words shared with a neighbouring chunk are
// combined with atomic OR; whole words are stored.
__global__ __launch_bounds__(kThreads) void k_sign_move(const StreamDev* __restrict__ sd, int ns,
                                                         const uint32_t* __restrict__ cnt,
                                                         const uint32_t* __restrict__ idx,
                                                         const int64_t* __restrict__ pso,
                                                         const uint64_t* __restrict__ stage,
                                                         unsigned long long* __restrict__ sign) {
  __shared__ int s_u;
  const int64_t gch = blockIdx.x;
  if (threadIdx.x == 0) s_u = find_stream(sd, ns, gch);
  __syncthreads();
  const StreamDev S = sd[s_u];
  const int64_t chunk = gch - S.chunk_begin;
  const uint64_t* st = stage + S.stage_off + chunk * 64;
  int64_t sbit = 0;
  for (int j = 0; j < S.B; ++j) {
    const int64_t cj = cnt[S.cnt_off + (int64_t)j * S.C + chunk];
    if (cj == 0) continue;
    const int64_t D = pso[S.psb + j] * 64 + (int64_t)idx[S.idx_off + (int64_t)j * S.C + chunk];
    const int64_t first = D >> 6, last = (D + cj - 1) >> 6;
    for (int64_t w = first + threadIdx.x; w <= last; w += kThreads) {
      const int64_t lo = max(w * 64, D), hi = min(w * 64 + 64, D + cj);
      const int nb = (int)(hi - lo);
      const uint64_t bits = extract_bits(st, (int)(lo - D + sbit), nb, 64);
      const uint64_t val = bits << (lo - w * 64);
      if (nb == 64)
        sign[S.sign_off + w] = val;
      else if (val)
        atomicOr(&sign[S.sign_off + w], (unsigned long long)val);
    }
    sbit += cj;
  }
}

// Incremental decode of planes [k0, k1) of each listed stream into its
// resident codes.  The sign of a code that becomes significant at plane j is
// found at index[j][chunk] + (rank among this chunk's plane-j newcomers).
template <typename Q, int MAXB>
__global__ __launch_bounds__(kThreads) void k_decode(const StreamDev* __restrict__ sd, int ns,
                                                      const uint64_t* __restrict__ mag,
                                                      const uint32_t* __restrict__ idx,
                                                      const uint64_t* __restrict__ sign,
                                                      const int64_t* __restrict__ pso, Q* __restrict__ codes,
                                                      Q* __restrict__ cd_codes) {
  __shared__ uint16_t wpre[MAXB][64];
  __shared__ uint64_t mws[MAXB][64];
  __shared__ int s_u;
  const int64_t gch = blockIdx.x;
  if (threadIdx.x == 0) s_u = find_stream(sd, ns, gch);
  __syncthreads();
  const StreamDev S = sd[s_u];
  const int64_t chunk = gch - S.chunk_begin;
  Q* dst = (S.use_cd ? cd_codes : codes) + S.code_off;
  const int B = S.B, k0 = S.k0, k1 = S.k1;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  for (int p = wave; p < k1 - k0; p += 4) {
    const int64_t w = chunk * 64 + lane;
    mws[p][lane] = (w < S.M) ? mag[S.mag_off + (int64_t)(k0 + p) * S.M + w] : 0ull;
  }
  __syncthreads();
  const uint64_t lt = lanemask_lt(lane);

  uint64_t nm_r[16];
  int pl_r[16];
  int rk_r[16];
  Q q_r[16];
#pragma unroll
  for (int it = 0; it < 16; ++it) {
    const int wl = wave + 4 * it;
    const int64_t word = chunk * 64 + wl;
    const int64_t e = word * 64 + lane;
    const bool valid = e < S.n;
    const Q qres = (!S.fresh && valid) ? dst[e] : (Q)0;
    bool sig = qres != 0;
    uint64_t nm = 0;
    int pl = -1, rk = 0;
    for (int j = k0; j < k1; ++j) {
      const uint64_t mw = mws[j - k0][wl];
      const bool bit = (mw >> lane) & 1ull;
      const bool nsg = bit && !sig;
      sig = sig || bit;
      if (bit) nm |= 1ull << (B - 1 - j);
      const uint64_t nsm = __ballot(nsg);
      if (lane == 0) wpre[j - k0][wl] = (uint16_t)__popcll(nsm);
      if (nsg) {
        pl = j;
        rk = __popcll(nsm & lt);
      }
    }
    nm_r[it] = nm;
    pl_r[it] = pl;
    rk_r[it] = rk;
    q_r[it] = qres;
  }
  __syncthreads();
  for (int j = wave; j < k1 - k0; j += 4) {
    const uint32_t v = wpre[j][lane];
    const uint32_t incl = wave_incl_scan(v, lane);
    wpre[j][lane] = (uint16_t)(incl - v);
  }
  __syncthreads();
#pragma unroll
  for (int it = 0; it < 16; ++it) {
    const int wl = wave + 4 * it;
    const int64_t e = (chunk * 64 + wl) * 64 + lane;
    if (e >= S.n) continue;
    const Q qres = q_r[it];
    const uint64_t m = absq(qres) | nm_r[it];
    bool neg = qres < 0;
    const int pl = pl_r[it];
    if (pl >= 0) {
      const uint64_t pos = (uint64_t)idx[S.idx_off + (int64_t)pl * S.C + chunk] + wpre[pl - k0][wl] + rk_r[it];
      const int64_t sw_i = pso[S.psb + pl] + (int64_t)(pos >> 6);
      const uint64_t sw = sw_i < S.sign_n ? sign[S.sign_off + sw_i] : 0ull;
      neg = (sw >> (pos & 63)) & 1ull;
    }
    dst[e] = neg ? (Q)(-(int64_t)m) : (Q)m;
  }
}

// ----------------------------------------------------------- reconstruction
template <typename Q>
__global__ __launch_bounds__(kThreads) void k_coarsest(const Q* __restrict__ q, int64_t n, int B, int k,
                                                        double delta, double* __restrict__ xc) {
  const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (e < n) xc[e] = (double)mask_code<Q>(q[e], B, k) * delta;
}

// One region of one level: x' = prediction + Delta * q' (Algorithm 2).
// Neighbours on the coarser level come from xc (float64), those in earlier
// regions of this level from their buffers: predictions (per-level) or
// reconstructed values (per-region).
template <typename OutT, typename Q>
__global__ __launch_bounds__(kThreads) void k_recon(const double* __restrict__ xc, int cm1, int cm2, RegionArgs ra,
                                                     const Q* __restrict__ q, int B, int k, double delta,
                                                     OutT* __restrict__ out) {
  const Lattice& L = ra.lat;
  const int64_t total = (int64_t)L.c[0] * L.c[1] * L.c[2];
  const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (e >= total) return;
  int i[3], t[3];
  lattice_node(L, e, i, t);
  const int ax = L.ax;
  const int j = i[ax];
  const int sk = stencil_kind(j, L.m[ax], ra.degree);
  const int rp = source_region(ra, i);
  double p;
  if (rp < 0) {
    const int64_t cs[3] = {(int64_t)cm1 * cm2, (int64_t)cm2, 1};
    int ci[3];
    for (int a = 0; a < 3; ++a) ci[a] = (a == ax) ? (j - 1) >> 1 : i[a] >> 1;
    const double* pc = xc + ci[0] * cs[0] + ci[1] * cs[1] + ci[2] * cs[2];
    const int64_t st = cs[ax];
    p = stencil_eval(sk, [&](int o) { return pc[((o + 1) / 2) * st]; });
  } else {
    p = predict_from_region(ra, rp, i, ax, j, sk);
  }
  const double dq = (double)mask_code<Q>(q[e], B, k) * delta;
  const double x = p + dq;
  out[((int64_t)i[0] * L.m[1] + i[1]) * L.m[2] + i[2]] = (OutT)x;
  if (ra.pr_out) ra.pr_out[e] = ra.per_level ? p : x;
}

template <typename OutT>
__global__ __launch_bounds__(kThreads) void k_inject(const double* __restrict__ xc, int c0, int c1, int c2,
                                                      OutT* __restrict__ out, int m1, int m2) {
  const int64_t n = (int64_t)c0 * c1 * c2;
  const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (e >= n) return;
  const int i2 = (int)(e % c2);
  const int64_t r = e / c2;
  const int i1 = (int)(r % c1);
  const int i0 = (int)(r / c1);
  out[((int64_t)(2 * i0) * m1 + 2 * i1) * m2 + 2 * i2] = (OutT)xc[e];
}

template <typename OutT>
__global__ __launch_bounds__(kThreads) void k_cast(const double* __restrict__ xc, int64_t n, OutT* __restrict__ out) {
  const int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x;
  if (e < n) out[e] = (OutT)xc[e];
}

inline unsigned nblocks(int64_t n) { return (unsigned)((n + kThreads - 1) / kThreads); }

}  // namespace

// ------------------------------------------------------------------ launchers
template <typename T>
hipError_t launch_range(const T* x, int64_t n, unsigned long long* acc4, hipStream_t s) {
  int64_t blocks = (n + kThreads * 8 - 1) / (kThreads * 8);
  if (blocks < 1) blocks = 1;
  if (blocks > 8192) blocks = 8192;
  hipLaunchKernelGGL((k_range<T>), dim3((unsigned)blocks), dim3(kThreads), 0, s, x, n, acc4);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_subsample(const T* src, const int32_t* msrc, T* dst, const int32_t* mdst, hipStream_t s) {
  const int64_t n = (int64_t)mdst[0] * mdst[1] * mdst[2];
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL((k_subsample<T>), dim3(nblocks(n)), dim3(kThreads), 0, s, src, msrc[1], msrc[2], dst, mdst[0],
                     mdst[1], mdst[2]);
  return hipGetLastError();
}

template <typename T, typename Q>
hipError_t launch_coef(const T* G, const RegionArgs& ra, int mode, unsigned long long* gmax, int64_t k_shift,
                       Q* codes, hipStream_t s) {
  const int64_t n = (int64_t)ra.lat.c[0] * ra.lat.c[1] * ra.lat.c[2];
  if (n == 0) return hipSuccess;
  if (mode == 0)
    hipLaunchKernelGGL((k_coef<T, Q, 0>), dim3(std::min<unsigned>(nblocks(n), 4096u)), dim3(kThreads), 0, s, G, ra, gmax,
                       (int)k_shift, codes);
  else
    hipLaunchKernelGGL((k_coef<T, Q, 1>), dim3(nblocks(n)), dim3(kThreads), 0, s, G, ra, gmax, (int)k_shift, codes);
  return hipGetLastError();
}

template <typename T, typename Q>
hipError_t launch_coarse(const T* G, int64_t n, int mode, unsigned long long* gmax, int64_t k_shift, Q* codes,
                         hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (mode == 0)
    hipLaunchKernelGGL((k_coarse<T, Q, 0>), dim3(nblocks(n)), dim3(kThreads), 0, s, G, n, gmax, (int)k_shift, codes);
  else
    hipLaunchKernelGGL((k_coarse<T, Q, 1>), dim3(nblocks(n)), dim3(kThreads), 0, s, G, n, gmax, (int)k_shift, codes);
  return hipGetLastError();
}

template <typename Q>
hipError_t launch_cd_forward(const Q* region_codes, const CDArgs& ca, Q* cd_codes, unsigned long long* smax,
                             hipStream_t s) {
  const int64_t n = (int64_t)ca.c[0] * ca.c[1] * ca.c[2];
  if (n == 0) return hipSuccess;
  if (ca.a == 0)
    hipLaunchKernelGGL((k_cd_forward<Q, 0, 1, 2>), dim3(nblocks(n)), dim3(kThreads), 0, s, region_codes, ca, cd_codes, smax);
  else if (ca.a == 1)
    hipLaunchKernelGGL((k_cd_forward<Q, 1, 0, 2>), dim3(nblocks(n)), dim3(kThreads), 0, s, region_codes, ca, cd_codes, smax);
  else
    hipLaunchKernelGGL((k_cd_forward<Q, 2, 0, 1>), dim3(nblocks(n)), dim3(kThreads), 0, s, region_codes, ca, cd_codes, smax);
  return hipGetLastError();
}

template <typename Q>
hipError_t launch_cd_inverse(const Q* cd_codes, const CDArgs& ca, Q* region_out, hipStream_t s) {
  const int64_t n = (int64_t)ca.c[0] * ca.c[1] * ca.c[2];
  if (n == 0) return hipSuccess;
#define APC_CDINV(PH, A_, U_, V_) \
  hipLaunchKernelGGL((k_cd_inverse<Q, PH, A_, U_, V_>), dim3(nblocks(n)), dim3(kThreads), 0, s, cd_codes, ca, region_out)
  for (int ph = 0; ph < 2; ++ph) {
    if (ca.a == 0) {
      if (ph == 0) APC_CDINV(0, 0, 1, 2); else APC_CDINV(1, 0, 1, 2);
    } else if (ca.a == 1) {
      if (ph == 0) APC_CDINV(0, 1, 0, 2); else APC_CDINV(1, 1, 0, 2);
    } else {
      if (ph == 0) APC_CDINV(0, 2, 0, 1); else APC_CDINV(1, 2, 0, 1);
    }
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
  }
#undef APC_CDINV
  return hipSuccess;
}

template <typename Q>
hipError_t launch_encode(const Q* codes, const Q* cd_codes, const StreamDev* sd_dev, int nstreams,
                         int64_t total_chunks, const int64_t*, int, uint64_t* mag, uint32_t* cnt, uint64_t* stage,
                         hipStream_t s) {
  if (total_chunks == 0) return hipSuccess;
  constexpr int MAXB = sizeof(Q) == 4 ? 32 : 64;
  hipLaunchKernelGGL((k_encode<Q, MAXB>), dim3((unsigned)total_chunks), dim3(kThreads), 0, s, codes, cd_codes, sd_dev,
                     nstreams, mag, cnt, stage);
  return hipGetLastError();
}

hipError_t launch_scan(const StreamDev* sd_dev, const int32_t* job_stream, const int32_t* job_plane, int njobs,
                       const uint32_t* cnt, uint32_t* idx, int64_t* totals, hipStream_t s) {
  if (njobs == 0) return hipSuccess;
  hipLaunchKernelGGL(k_scan, dim3(njobs), dim3(kThreads), 0, s, sd_dev, job_stream, job_plane, cnt, idx, totals);
  return hipGetLastError();
}

hipError_t launch_sign_move(const StreamDev* sd_dev, int nstreams, int64_t total_chunks, const uint32_t* cnt,
                            const uint32_t* idx, const int64_t* pso, const uint64_t* stage, uint64_t* sign,
                            hipStream_t s) {
  if (total_chunks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_sign_move, dim3((unsigned)total_chunks), dim3(kThreads), 0, s, sd_dev, nstreams, cnt, idx, pso,
                     stage, (unsigned long long*)sign);
  return hipGetLastError();
}

template <typename Q>
hipError_t launch_decode(const StreamDev* sd_dev, int nstreams, int64_t total_chunks, const uint64_t* mag,
                         const uint32_t* idx, const uint64_t* sign, const int64_t* pso, Q* codes, Q* cd_codes,
                         hipStream_t s) {
  if (total_chunks == 0) return hipSuccess;
  constexpr int MAXB = sizeof(Q) == 4 ? 32 : 64;
  hipLaunchKernelGGL((k_decode<Q, MAXB>), dim3((unsigned)total_chunks), dim3(kThreads), 0, s, sd_dev, nstreams, mag,
                     idx, sign, pso, codes, cd_codes);
  return hipGetLastError();
}

template <typename Q>
hipError_t launch_coarsest_q(const Q* q, int64_t n, int32_t B, int32_t k, double delta, double* xc, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL((k_coarsest<Q>), dim3(nblocks(n)), dim3(kThreads), 0, s, q, n, B, k, delta, xc);
  return hipGetLastError();
}

template <typename OutT, typename Q>
hipError_t launch_recon(const double* xc, const int32_t* cm, const RegionArgs& ra, const Q* q, int32_t B, int32_t k,
                        double delta, OutT* out, hipStream_t s) {
  const int64_t n = (int64_t)ra.lat.c[0] * ra.lat.c[1] * ra.lat.c[2];
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL((k_recon<OutT, Q>), dim3(nblocks(n)), dim3(kThreads), 0, s, xc, cm[1], cm[2], ra, q, B, k, delta,
                     out);
  return hipGetLastError();
}

template <typename OutT>
hipError_t launch_inject(const double* xc, const int32_t* cm, OutT* out, const int32_t* m, hipStream_t s) {
  const int64_t n = (int64_t)cm[0] * cm[1] * cm[2];
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL((k_inject<OutT>), dim3(nblocks(n)), dim3(kThreads), 0, s, xc, cm[0], cm[1], cm[2], out, m[1],
                     m[2]);
  return hipGetLastError();
}

template <typename OutT>
hipError_t launch_cast(const double* xc, int64_t n, OutT* out, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL((k_cast<OutT>), dim3(nblocks(n)), dim3(kThreads), 0, s, xc, n, out);
  return hipGetLastError();
}

// explicit instantiations
template hipError_t launch_cast<float>(const double*, int64_t, float*, hipStream_t);
template hipError_t launch_cast<double>(const double*, int64_t, double*, hipStream_t);
template hipError_t launch_range<float>(const float*, int64_t, unsigned long long*, hipStream_t);
template hipError_t launch_range<double>(const double*, int64_t, unsigned long long*, hipStream_t);
template hipError_t launch_subsample<float>(const float*, const int32_t*, float*, const int32_t*, hipStream_t);
template hipError_t launch_subsample<double>(const double*, const int32_t*, double*, const int32_t*, hipStream_t);
template hipError_t launch_coef<float, int32_t>(const float*, const RegionArgs&, int, unsigned long long*, int64_t,
                                                int32_t*, hipStream_t);
template hipError_t launch_coef<double, int64_t>(const double*, const RegionArgs&, int, unsigned long long*, int64_t,
                                                 int64_t*, hipStream_t);
template hipError_t launch_coarse<float, int32_t>(const float*, int64_t, int, unsigned long long*, int64_t, int32_t*,
                                                  hipStream_t);
template hipError_t launch_coarse<double, int64_t>(const double*, int64_t, int, unsigned long long*, int64_t,
                                                   int64_t*, hipStream_t);
template hipError_t launch_cd_forward<int32_t>(const int32_t*, const CDArgs&, int32_t*, unsigned long long*,
                                               hipStream_t);
template hipError_t launch_cd_forward<int64_t>(const int64_t*, const CDArgs&, int64_t*, unsigned long long*,
                                               hipStream_t);
template hipError_t launch_cd_inverse<int32_t>(const int32_t*, const CDArgs&, int32_t*, hipStream_t);
template hipError_t launch_cd_inverse<int64_t>(const int64_t*, const CDArgs&, int64_t*, hipStream_t);
template hipError_t launch_encode<int32_t>(const int32_t*, const int32_t*, const StreamDev*, int, int64_t,
                                           const int64_t*, int, uint64_t*, uint32_t*, uint64_t*, hipStream_t);
template hipError_t launch_encode<int64_t>(const int64_t*, const int64_t*, const StreamDev*, int, int64_t,
                                           const int64_t*, int, uint64_t*, uint32_t*, uint64_t*, hipStream_t);
template hipError_t launch_decode<int32_t>(const StreamDev*, int, int64_t, const uint64_t*, const uint32_t*,
                                           const uint64_t*, const int64_t*, int32_t*, int32_t*, hipStream_t);
template hipError_t launch_decode<int64_t>(const StreamDev*, int, int64_t, const uint64_t*, const uint32_t*,
                                           const uint64_t*, const int64_t*, int64_t*, int64_t*, hipStream_t);
template hipError_t launch_coarsest_q<int32_t>(const int32_t*, int64_t, int32_t, int32_t, double, double*,
                                               hipStream_t);
template hipError_t launch_coarsest_q<int64_t>(const int64_t*, int64_t, int32_t, int32_t, double, double*,
                                               hipStream_t);
template hipError_t launch_recon<float, int32_t>(const double*, const int32_t*, const RegionArgs&, const int32_t*,
                                                 int32_t, int32_t, double, float*, hipStream_t);
template hipError_t launch_recon<double, int32_t>(const double*, const int32_t*, const RegionArgs&, const int32_t*,
                                                  int32_t, int32_t, double, double*, hipStream_t);
template hipError_t launch_recon<double, int64_t>(const double*, const int32_t*, const RegionArgs&, const int64_t*,
                                                  int32_t, int32_t, double, double*, hipStream_t);
template hipError_t launch_inject<float>(const double*, const int32_t*, float*, const int32_t*, hipStream_t);
template hipError_t launch_inject<double>(const double*, const int32_t*, double*, const int32_t*, hipStream_t);

}  // namespace apc
