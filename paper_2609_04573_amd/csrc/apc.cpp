// C ABI and host orchestration of refactor (Algorithm 1) and retrieval
// (Algorithm 2) on one gfx950 device.  Metadata (group maxima, plane
// counts) is computed on the device and read back; planning is host-side.
#include <math.h>

#include <cmath>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <thread>
#include <unistd.h>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <tuple>
#include <type_traits>
#include <string>
#include <vector>

#include "../../include/apc.h"
#include "apc_internal.h"
#include "host.h"

using namespace apc;

namespace {

thread_local std::string g_last_error;

apc_status fail(apc_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_last_error = buf;
  return s;
}

#define HIP_TRY(expr)                                                                          \
  do {                                                                                         \
    hipError_t _e = (expr);                                                                    \
    if (_e != hipSuccess)                                                                      \
      return fail(_e == hipErrorOutOfMemory ? APC_E_OOM : APC_E_HIP, "%s: %s (%s:%d)", #expr, \
                  hipGetErrorString(_e), __FILE__, __LINE__);                                  \
  } while (0)

#define APC_TRY(expr)              \
  do {                             \
    apc_status _s = (expr);        \
    if (_s != APC_OK) return _s;   \
  } while (0)

// Launch profiler: when enabled, every kernel launch is bracketed by two HIP
// events on its own stream and tagged with the bytes it must move.
struct ProfRec {
  const char* name;
  hipEvent_t a, b;
  double bytes;
};
struct Profiler {
  std::atomic<bool> on{false};
  std::atomic<bool> filtered{false};  // `only` is set
  std::mutex mu;     // guards only, recs, pool (launches may come from several threads)
  std::string only;  // if set, only launches of this name are timed
  std::vector<ProfRec> recs;
  std::vector<hipEvent_t> pool;
  hipEvent_t get() {  // with mu held
    if (!pool.empty()) {
      hipEvent_t e = pool.back();
      pool.pop_back();
      return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
  }
};
Profiler g_prof;
thread_local bool g_prof_suppress = false;  // this thread's launches are not timed (graph capture)

struct ProfMark {
  hipEvent_t b = nullptr;
  hipStream_t st;
  ProfMark(const char* name, double bytes, hipStream_t s) : st(s) {
    if (!g_prof.on.load(std::memory_order_relaxed) || g_prof_suppress) return;
    std::lock_guard<std::mutex> lk(g_prof.mu);
    if (!g_prof.only.empty() && g_prof.only != name) return;
    ProfRec r{name, g_prof.get(), g_prof.get(), bytes};
    (void)hipEventRecord(r.a, st);
    g_prof.recs.push_back(r);
    b = r.b;
  }
  void stop() {
    if (b) (void)hipEventRecord(b, st);
  }
};

#define LAUNCH(name, bytes, st, expr)    \
  do {                                  \
    ProfMark _pm(name, (double)(bytes), st); \
    HIP_TRY(expr);                      \
    _pm.stop();                         \
  } while (0)

// Caching device allocator: freed blocks are kept per size and handed back to
// later requests of the same or slightly smaller size, so repeated refactors
// and retrievals do not pay hipMalloc / hipFree (both synchronize the device).
struct Pool {
  std::mutex mu;
  std::multimap<size_t, void*> free_blocks;
  size_t cached = 0;
  size_t limit = (size_t)32 << 30;

  hipError_t get(size_t n, void** p, size_t* got) {
    {
      std::lock_guard<std::mutex> lk(mu);
      auto it = free_blocks.lower_bound(n);
      if (it != free_blocks.end() && it->first <= n + n / 8 + 4096) {
        *p = it->second;
        *got = it->first;
        cached -= it->first;
        free_blocks.erase(it);
        return hipSuccess;
      }
    }
    hipError_t e = hipMalloc(p, n);
    if (e == hipErrorOutOfMemory) {
      trim(0);
      e = hipMalloc(p, n);
    }
    *got = n;
    return e;
  }
  void put(void* p, size_t n) {
    std::lock_guard<std::mutex> lk(mu);
    free_blocks.insert({n, p});
    cached += n;
    while (cached > limit && !free_blocks.empty()) {
      auto it = std::prev(free_blocks.end());
      (void)hipFree(it->second);
      cached -= it->first;
      free_blocks.erase(it);
    }
  }
  void trim(size_t keep) {
    std::lock_guard<std::mutex> lk(mu);
    while (cached > keep && !free_blocks.empty()) {
      auto it = std::prev(free_blocks.end());
      (void)hipFree(it->second);
      cached -= it->first;
      free_blocks.erase(it);
    }
  }
};
Pool& pool() {
  static Pool* p = new Pool();  // never destroyed: blocks outlive static teardown order
  return *p;
}

// Device allocation owned by a host object.
struct DevBuf;
// While set (by a DrainScope), buffers released on this thread are parked
// in this list instead of going back to the pool.
thread_local std::vector<DevBuf>* g_park = nullptr;

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  DevBuf(DevBuf&& o) noexcept : p(o.p), bytes(o.bytes) {
    o.p = nullptr;
    o.bytes = 0;
  }
  ~DevBuf() { release(); }
  void release() {
    if (p && g_park) {
      g_park->emplace_back(std::move(*this));
      return;
    }
    if (p) pool().put(p, bytes);
    p = nullptr;
    bytes = 0;
  }
  apc_status alloc(size_t nbytes) {
    if (nbytes <= bytes && p) return APC_OK;
    release();
    nbytes = (std::max<size_t>(nbytes, 8) + 255) & ~(size_t)255;
    size_t got = 0;
    hipError_t e = pool().get(nbytes, &p, &got);
    if (e != hipSuccess) {
      p = nullptr;
      return fail(e == hipErrorOutOfMemory ? APC_E_OOM : APC_E_HIP, "hipMalloc(%zu): %s", nbytes,
                  hipGetErrorString(e));
    }
    bytes = got;
    return APC_OK;
  }
  template <typename X>
  X* as() const {
    return (X*)p;
  }
};

// Device buffers that queued work may still use, kept until an event
// recorded behind that work has completed (then they go back to the pool):
// a call can return without waiting for its last kernels.
struct Retired {
  hipEvent_t ev = nullptr;
  std::vector<DevBuf> bufs;
};
std::mutex g_retired_mu;
std::deque<Retired>& retired() {
  static std::deque<Retired>* r = new std::deque<Retired>();  // never destroyed, like the pool
  return *r;
}
// Release the retired buffers whose work has finished (oldest first).
void reap_retired() {
  std::lock_guard<std::mutex> lk(g_retired_mu);
  auto& q = retired();
  while (!q.empty()) {
    const hipError_t e = hipEventQuery(q.front().ev);
    if (e == hipErrorNotReady) break;
    if (e != hipSuccess) (void)hipGetLastError();  // the stream is gone: nothing runs on it any more
    (void)hipEventDestroy(q.front().ev);
    q.pop_front();
  }
}
// Keep bufs until the work queued on st so far has finished.
apc_status retire(std::vector<DevBuf>&& bufs, hipStream_t st) {
  Retired r;
  hipError_t e = hipEventCreateWithFlags(&r.ev, hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventRecord(r.ev, st);
  if (e != hipSuccess) {  // fall back to waiting here
    if (r.ev) (void)hipEventDestroy(r.ev);
    (void)hipStreamSynchronize(st);
    return APC_OK;
  }
  r.bufs = std::move(bufs);
  std::lock_guard<std::mutex> lk(g_retired_mu);
  retired().push_back(std::move(r));
  return APC_OK;
}

// Scope of a call that queues work on stream st and may return early: every
// device buffer released on this thread while the scope lives is parked
// instead of going back to the pool.  When the scope ends, an armed scope
// (an error return) waits for the stream before the parked buffers are
// released; a disarmed one (the call completed) retires them behind an event
// on st.  Buffers released by destructors that run before the scope's own
// (locals declared after it) are therefore never handed out while queued
// kernels may still use them.
struct DrainScope {
  hipStream_t st;
  bool armed = true;
  std::vector<DevBuf> parked;
  std::vector<DevBuf>* prev;
  explicit DrainScope(hipStream_t s) : st(s), prev(g_park) { g_park = &parked; }
  DrainScope(const DrainScope&) = delete;
  DrainScope& operator=(const DrainScope&) = delete;
  ~DrainScope() {
    g_park = prev;
    if (parked.empty()) return;
    if (armed) {
      (void)hipStreamSynchronize(st);
      (void)hipGetLastError();
      parked.clear();
    } else {
      (void)retire(std::move(parked), st);
    }
  }
};

// Field geometry in the 3D embedding.
struct Geo {
  int d = 3;
  int64_t N[3] = {1, 1, 1};
  int L = 1;
  int sigma_user[3] = {2, 1, 0};
  int sigma3[3] = {2, 1, 0};
  std::vector<std::array<int32_t, 3>> m;  // compact dims per level
  int64_t n() const { return N[0] * N[1] * N[2]; }
};

int default_levels(const int64_t* N) {
  int64_t nmax = std::max(N[0], std::max(N[1], N[2]));
  if (nmax <= 2) return 1;
  int64_t v = nmax - 2;
  int bl = 0;
  while (v) {
    ++bl;
    v >>= 1;
  }
  return 1 + bl;
}

Lattice lattice(const Geo& g, int l, int rho) {
  Lattice L{};
  for (int a = 0; a < 3; ++a) {
    L.m[a] = g.m[l][a];
    L.kind[a] = AX_EVEN;
  }
  for (int j = 0; j < g.d; ++j) {
    const int ax = g.sigma3[j];
    L.kind[ax] = j < rho ? AX_ALL : (j == rho ? AX_ODD : AX_EVEN);
  }
  for (int a = 0; a < 3; ++a) {
    const int m = L.m[a];
    L.c[a] = L.kind[a] == AX_ALL ? m : (L.kind[a] == AX_ODD ? m / 2 : (m + 1) / 2);
  }
  L.ax = g.sigma3[rho];
  L.f2 = make_fastdiv((uint32_t)std::max(1, L.c[2]));
  L.f1 = make_fastdiv((uint32_t)std::max(1, L.c[1]));
  return L;
}

int64_t lat_count(const Lattice& L) { return (int64_t)L.c[0] * L.c[1] * L.c[2]; }

struct Rng1h {
  int64_t c4, c2, call;
};
int64_t cls_count_h(int cls, Rng1h ru, Rng1h rv) {
  const int64_t h2 = ru.c4 * rv.c4, h1 = ru.c2 * rv.c2, all = ru.call * rv.call;
  return cls == 0 ? h2 : (cls == 1 ? h1 - h2 : all - h1);
}
Rng1h prefix_h(int64_t x) { return {(x + 3) / 4, (x + 1) / 2, x}; }

int bitlen(int64_t v) {
  int b = 0;
  uint64_t u = (uint64_t)v;
  while (u) {
    ++b;
    u >>= 1;
  }
  return b;
}

unsigned long long double_bits(double d) {
  unsigned long long b;
  memcpy(&b, &d, 8);
  return b;
}
double bits_double(unsigned long long b) {
  double d;
  memcpy(&d, &b, 8);
  return d;
}
double unordered(unsigned long long ob) {
  return bits_double((ob >> 63) ? (ob & 0x7fffffffffffffffull) : ~ob);
}

}  // namespace

// One level-0 region under coefficient decomposition.
struct CDInfo {
  int32_t c[3];      // region lattice dims
  int32_t a;         // stacking axis (3D)
  int s_idx[3];      // streams S1..S3
  int64_t s_off[3];  // their offsets in the decomposition code buffer
  int64_t reg_off;   // offset of the region in the recomposition buffer
};

// Pinned host blocks for table uploads.  Pinning is slow (it dominates a
// small retrieval), so blocks are pooled for the life of the process; each
// carries an event recorded after the last copy queued out of it, and a
// block is handed out again only once that event has completed.
struct PinnedBlock {
  void* p = nullptr;
  size_t cap = 0;
  hipEvent_t ev = nullptr;
};
struct PinnedPool {
  std::mutex mu;
  std::vector<PinnedBlock> free_;
  // a block of at least `bytes`; pooled blocks are idle (their copies done)
  bool get(size_t bytes, PinnedBlock& out) {
    {
      std::lock_guard<std::mutex> lk(mu);
      int best = -1;
      for (int i = 0; i < (int)free_.size(); ++i)
        if (free_[i].cap >= bytes && (best < 0 || free_[i].cap < free_[best].cap)) best = i;
      if (best >= 0) {
        out = free_[best];
        free_.erase(free_.begin() + best);
        return true;
      }
    }
    size_t cap = (size_t)1 << 16;
    while (cap < bytes) cap <<= 1;
    if (hipHostMalloc(&out.p, cap) != hipSuccess) {
      out = PinnedBlock();
      return false;
    }
    out.cap = cap;
    if (hipEventCreateWithFlags(&out.ev, hipEventDisableTiming) != hipSuccess) {
      (void)hipHostFree(out.p);
      out = PinnedBlock();
      return false;
    }
    return true;
  }
  // Return a block once the copies queued out of it are done (`pending`:
  // the last one was queued on stream st and not yet marked by its event).
  // Waiting here keeps pooled blocks free of events on streams that may be
  // destroyed later.
  void put(PinnedBlock& b, hipStream_t st, bool pending) {
    if (!b.p) return;
    if (pending) (void)hipEventRecord(b.ev, st);
    if (hipEventSynchronize(b.ev) != hipSuccess) {
      // the event is unusable (its stream is gone): replace it, and clear
      // the error so it is not reported by an unrelated later call
      (void)hipGetLastError();
      (void)hipEventDestroy(b.ev);
      b.ev = nullptr;
      if (hipEventCreateWithFlags(&b.ev, hipEventDisableTiming) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipHostFree(b.p);
        b = PinnedBlock();
        return;
      }
    }
    std::lock_guard<std::mutex> lk(mu);
    free_.push_back(b);
    b = PinnedBlock();
  }
};
PinnedPool g_pinned;

struct apc_handle {
  Meta meta;
  Geo geo;
  apc_scheme scheme{};
  int dtype = APC_F32;
  std::vector<int64_t> region_off;  // (l * 3 + rho) -> offset in the region code buffer
  int64_t code_n = 0;               // codes in the region code buffer
  int64_t cd_n = 0;                 // codes in the decomposition buffer
  int64_t cdreg_n = 0;              // codes in the recomposition buffer
  std::vector<CDInfo> cd;           // per level-0 region
  std::vector<int> psb;             // per stream: first entry in pso
  // stored representation
  DevBuf mag, idx, sign, pso;
  DevBuf zoff;  // lossless stage: per-(plane, chunk) nonzero words before the chunk (layout of idx)
  // retrieval state: decoded codes and planes decoded so far per stream
  DevBuf codes, cd_codes;
  DevBuf pcodes, pcd_codes;  // digit-plane handles: truncated integers of the last retrieval
  std::vector<int> k_res;
  DevBuf xc, xb[2], pr[2], cdreg, tables;
  bool work_ready = false;
  PinnedBlock pinned;  // staging of table uploads (its event follows the last upload)
  hipEvent_t ready = nullptr;  // follows the refactor's last kernel (work on other streams waits for it)
  std::shared_ptr<void> ready_owner;  // the handles of one batch share `ready`: destroyed with the last
  hipEvent_t tab_ev = nullptr;  // follows the last retrieval that read `tables`
  int interp = INTERP_GREEDY;    // retrieval interpreter
  bool host_only = false;        // rebuilt from bytes without device data: planning only
  ~apc_handle() {
    g_pinned.put(pinned, nullptr, false);
    if (tab_ev) {
      (void)hipEventSynchronize(tab_ev);
      (void)hipEventDestroy(tab_ev);
    }
    if (ready) {  // the buffers go back to the shared pool only after the refactor's last kernels
      (void)hipEventSynchronize(ready);
      if (!ready_owner) (void)hipEventDestroy(ready);
    }
  }
};

namespace {

size_t qsize(int dtype) { return dtype == APC_F32 ? 4 : 8; }

// ------------------------------------------------------------ segment tables
// Byte buffers of segment tables, kept per thread from call to call: a
// table then lands in memory whose pages exist and whose capacity fits (a
// fresh buffer of megabytes pays page faults and regrowth copies on every
// call).  At most 8 buffers of at most 64 MiB each are kept.
thread_local std::vector<std::vector<char>> g_table_bufs;
struct TableBuilder {
  std::vector<char> bytes;
  TableBuilder() {
    if (!g_table_bufs.empty()) {
      bytes.swap(g_table_bufs.back());
      g_table_bufs.pop_back();
      bytes.clear();
    }
  }
  ~TableBuilder() {
    if (bytes.capacity() >= ((size_t)64 << 10) && bytes.capacity() <= ((size_t)64 << 20) && g_table_bufs.size() < 8) {
      bytes.clear();
      g_table_bufs.push_back(std::move(bytes));
    }
  }
  TableBuilder(TableBuilder&&) = default;
  TableBuilder& operator=(TableBuilder&&) = default;
  TableBuilder(const TableBuilder&) = delete;
  TableBuilder& operator=(const TableBuilder&) = delete;
  template <typename S>
  size_t add(const std::vector<S>& v) {
    return add_raw(v.data(), sizeof(S) * v.size());
  }
  size_t add_raw(const void* p, size_t n) {
    size_t off = (bytes.size() + 255) & ~(size_t)255;
    bytes.resize(off + n);
    if (n) memcpy(bytes.data() + off, p, n);
    return off;
  }
};

enum LaunchKind {
  K_RANGE, K_GATHER, K_COEF0, K_COEF1, K_COARSE0, K_COARSE1, K_CDF, K_CDI0, K_CDI1,
  K_ENCODE, K_SIGN, K_DECODE, K_COARSEST, K_INJECT, K_RECON, K_LEVEL0, K_LEVEL1, K_LEVEL2, K_LEVEL3, K_CDIT, K_CDFT,
  // two-stream retrieval: the helper stream starts after what the main one
  // queued so far (FORK), marks its end (JOIN_REC), and the main one waits
  // for that mark (JOIN_WAIT); without a helper stream these do nothing
  K_FORK, K_JOIN_REC, K_JOIN_WAIT,
  K_DECODE_NB, K_NB_VALUES,  // digit planes: decode, truncated integers
  K_ZERO                     // clear 64-bit words (sign arenas)
};

struct Launch {
  int kind;
  size_t off;
  int nseg;
  int64_t nblk;   // work blocks, or chunks for the codec kernels
  int a;          // stacking axis (decomposition kernels)
  double bytes;   // bytes the launch must move (profiling)
  const char* name;
  int side = 0;   // 1: runs on the helper stream, when there is one
  int stage = 0;  // retrieval: dependency order (launches of one stage are independent)
};

// Dependency stage of a retrieval launch: decodes, the inverse
// decomposition, the coarsest level, then levels from coarse to fine
// (per-region levels: injection, then regions in order).  Launches of
// several retrievals with the same stage, kind and argument can be merged
// into one launch over all their segments.
int level_stage(int l, int sub) { return 100 + 10 * (64 - l) + sub; }

template <typename S>
int64_t assign_blocks(std::vector<S>& segs, std::function<int64_t(const S&)> count) {
  int64_t b = 0;
  for (S& s : segs) {
    s.blk_begin = b;
    b += (count(s) + kBlockElems - 1) / kBlockElems;
  }
  return b;
}

// ------------------------------------------------ per-level sweep tile shapes
// A tile is t2 columns (axis 2) by 1024 / t2 rows (axis 1).  The autotuner
// records the fastest width per (dtype, log2 of the level's axis-1 and axis-2
// extents); unseen shapes use a default.
std::mutex g_tile_mu;
std::map<std::tuple<int, int, int>, int> g_tiles;
int g_tile_override = 0;

int ceil_log2(int64_t v) {
  int b = 0;
  while (((int64_t)1 << b) < v) ++b;
  return b;
}
int default_tile(int m2) { return m2 <= 32 ? 32 : 64; }
int tile_for(int dtype, int m1, int m2) {
  std::lock_guard<std::mutex> lk(g_tile_mu);
  if (g_tile_override) return g_tile_override;
  auto it = g_tiles.find(std::make_tuple(dtype, ceil_log2(m1), ceil_log2(m2)));
  return it != g_tiles.end() ? it->second : default_tile(m2);
}

// Per-level pass geometry of level l (the coarser level is l + 1) for tiles
// t2 wide; the caller fills in the operands and then calls shape_level_seg.
LevelSeg level_seg(const apc_handle* h, int l) {
  const Geo& g = h->geo;
  LevelSeg s{};
  for (int a = 0; a < 3; ++a) {
    s.m[a] = g.m[l][a];
    s.mc[a] = g.m[l + 1][a];
  }
  s.degree = h->scheme.degree;
  return s;
}
// Tile counts and runs of a level segment whose operands (xs, q, B, k) are
// set for the field's own axes and regions; returns the tile width it takes.
// A level with one plane along axis 0 (every level of a 2D or 1D field, the
// coarse levels of a thin 3D one) is presented as m1 x m2 x 1 and swept with
// one-column tiles of 1024 points of a row, a block walking a run of rows as
// it walks planes of a 3D level.  The flat index of every point, the region
// lattices and the stencil order (axis 2, then 1, then 0) are unchanged:
// region 0 (odd along axis 2) is then empty and regions 0 and 1 become 1
// and 2.
int shape_level_seg(LevelSeg& s, int t2, int64_t min_blocks = 1024) {
  if (s.m[0] == 1) {
    for (int a = 0; a < 2; ++a) {
      s.m[a] = s.m[a + 1];
      s.mc[a] = s.mc[a + 1];
      s.xs[a] = s.xs[a + 1];
    }
    s.m[2] = s.mc[2] = 1;
    s.xs[2] = 0;
    for (int r = 2; r > 0; --r) {
      s.q[r] = s.q[r - 1];
      s.B[r] = s.B[r - 1];
      s.k[r] = s.k[r - 1];
    }
    s.q[0] = nullptr;  // never addressed: no point is odd along axis 2
    t2 = 1;
  }
  const int t1 = 1024 / t2;
  s.nt1 = (s.m[1] + t1 - 1) / t1;
  s.nt2 = (s.m[2] + t2 - 1) / t2;
  // runs along axis 0: as long as possible while the level still spreads
  // over min_blocks blocks
  s.ch = kLvlCH;
  while (s.ch > 2 && (int64_t)s.nt1 * s.nt2 * ((s.m[0] + s.ch - 1) / s.ch) < min_blocks) s.ch /= 2;
  return t2;
}
int64_t assign_level_blocks(std::vector<LevelSeg>& segs) {
  int64_t b = 0;
  for (LevelSeg& s : segs) {
    s.blk_begin = b;
    b += (int64_t)s.nt1 * s.nt2 * ((s.m[0] + s.ch - 1) / s.ch);
  }
  return b;
}

// Decomposition passes: one wave per lattice row, four rows a block.
int64_t assign_cd_blocks(std::vector<CDSeg>& segs) {
  int64_t b = 0;
  for (CDSeg& s : segs) {
    s.blk_begin = b;
    b += ((int64_t)s.c[0] * s.c[1] + 3) / 4;
  }
  return b;
}

// One-pass decomposition passes: tiles of 8 rows x 256 columns per slice,
// or of eight slices one row deep (tiles along v first).
int64_t assign_cd_tile_blocks(std::vector<CDSeg>& segs, int a) {
  int64_t b = 0;
  for (CDSeg& s : segs) {
    s.blk_begin = b;
    const int64_t nu = s.c[a == 0 ? 1 : 0], ns = s.c[a];
    s.ftu = make_fastdiv((uint32_t)std::max<int64_t>(1, (nu + 7) / 8));
    s.ftv = make_fastdiv((uint32_t)std::max<int64_t>(1, (s.c[2] + 255) / 256));
    b += (nu == 1 ? (ns + 7) / 8 : ns * ((nu + 7) / 8)) * ((s.c[2] + 255) / 256);
  }
  return b;
}

template <typename T, typename Q>
apc_status issue(const std::vector<Launch>& ls, const char* base, hipStream_t st0, hipStream_t aux = nullptr,
                 hipEvent_t ev_fork = nullptr, hipEvent_t ev_join = nullptr) {
  for (const Launch& l : ls) {
    const void* p = base + l.off;
    const hipStream_t st = aux && l.side ? aux : st0;
    switch (l.kind) {
      case K_FORK:
        if (aux) {
          HIP_TRY(hipEventRecord(ev_fork, st0));
          HIP_TRY(hipStreamWaitEvent(aux, ev_fork, 0));
        }
        break;
      case K_JOIN_REC:
        if (aux) HIP_TRY(hipEventRecord(ev_join, aux));
        break;
      case K_JOIN_WAIT:
        if (aux) HIP_TRY(hipStreamWaitEvent(st0, ev_join, 0));
        break;
      case K_RANGE: LAUNCH(l.name, l.bytes, st, launch_range<T>((const FlatSeg*)p, l.nseg, l.nblk, st)); break;
      case K_GATHER: LAUNCH(l.name, l.bytes, st, launch_gather<T>((const FlatSeg*)p, l.nseg, l.nblk, st)); break;
      case K_COEF0: LAUNCH(l.name, l.bytes, st, (launch_coef<T, Q>((const CoefSeg*)p, l.nseg, l.nblk, 0, st))); break;
      case K_COEF1: LAUNCH(l.name, l.bytes, st, (launch_coef<T, Q>((const CoefSeg*)p, l.nseg, l.nblk, 1, st))); break;
      case K_COARSE0:
        LAUNCH(l.name, l.bytes, st, (launch_coarse<T, Q>((const FlatSeg*)p, l.nseg, l.nblk, 0, st)));
        break;
      case K_COARSE1:
        LAUNCH(l.name, l.bytes, st, (launch_coarse<T, Q>((const FlatSeg*)p, l.nseg, l.nblk, 1, st)));
        break;
      case K_CDF: LAUNCH(l.name, l.bytes, st, launch_cd_forward<Q>((const CDSeg*)p, l.nseg, l.nblk, l.a, 0, st)); break;
      case K_CDFT: LAUNCH(l.name, l.bytes, st, launch_cd_forward<Q>((const CDSeg*)p, l.nseg, l.nblk, l.a, 1, st)); break;
      case K_CDI0:
        LAUNCH(l.name, l.bytes, st, launch_cd_inverse<Q>((const CDSeg*)p, l.nseg, l.nblk, l.a, 0, st));
        break;
      case K_CDI1:
        LAUNCH(l.name, l.bytes, st, launch_cd_inverse<Q>((const CDSeg*)p, l.nseg, l.nblk, l.a, 1, st));
        break;
      case K_CDIT:
        LAUNCH(l.name, l.bytes, st, launch_cd_inverse<Q>((const CDSeg*)p, l.nseg, l.nblk, l.a, 2, st));
        break;
      case K_ENCODE: LAUNCH(l.name, l.bytes, st, launch_encode<Q>((const StreamDev*)p, l.nseg, l.nblk, st)); break;
      case K_SIGN: LAUNCH(l.name, l.bytes, st, launch_sign_move((const StreamDev*)p, l.nseg, l.nblk, st)); break;
      case K_DECODE:  // a: bit 0 marks the level-0 decode, bit 1 a launch of first decodes only,
                      // bit 2 one whose streams add at most 16 planes each
        LAUNCH(l.name, l.bytes, st,
               launch_decode<Q>((const StreamDev*)p, l.nseg, l.nblk, (l.a & 2) != 0, (l.a & 4) ? 16 : 64, st));
        break;
      case K_COARSEST:
        LAUNCH(l.name, l.bytes, st, (launch_coarsest<T, Q>((const FlatSeg*)p, l.nseg, l.nblk, st)));
        break;
      case K_DECODE_NB:
        LAUNCH(l.name, l.bytes, st, launch_decode_nb<Q>((const StreamDev*)p, l.nseg, l.nblk, st));
        break;
      case K_NB_VALUES:
        LAUNCH(l.name, l.bytes, st, launch_nb_values<Q>((const FlatSeg*)p, l.nseg, l.nblk, st));
        break;
      case K_ZERO: LAUNCH(l.name, l.bytes, st, launch_zero_words((const FlatSeg*)p, l.nseg, l.nblk, st)); break;
      case K_INJECT: LAUNCH(l.name, l.bytes, st, launch_inject<T>((const FlatSeg*)p, l.nseg, l.nblk, st)); break;
      case K_RECON: LAUNCH(l.name, l.bytes, st, (launch_recon<T, Q>((const ReconSeg*)p, l.nseg, l.nblk, st))); break;
      case K_LEVEL0:
      case K_LEVEL1:
      case K_LEVEL2:
      case K_LEVEL3:
        LAUNCH(l.name, l.bytes, st,
               (launch_level<T, Q>((const LevelSeg*)p, l.nseg, l.nblk, l.kind - K_LEVEL0, l.a, st)));
        break;
      default: return fail(APC_E_INVALID, "unknown launch kind");
    }
  }
  return APC_OK;
}

// Device -> host copy on stream st through a pinned block, then wait for it:
// a copy straight into pageable memory is staged by the runtime and costs
// tens of microseconds of idle device time at every such read-back.
// Waits by polling the block's event: a blocking wait puts the thread to
// sleep and its wake-up alone costs tens of microseconds, during which the
// device would idle.
apc_status read_back(void* host, const void* dev, size_t bytes, hipStream_t st) {
  if (bytes == 0) return APC_OK;
  PinnedBlock b;
  if (!g_pinned.get(bytes, b)) return fail(APC_E_OOM, "pinned read-back of %zu bytes", bytes);
  hipError_t e = hipMemcpyAsync(b.p, dev, bytes, hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipEventRecord(b.ev, st);
  if (e == hipSuccess) {
    while ((e = hipEventQuery(b.ev)) == hipErrorNotReady) {
    }
  }
  if (e == hipSuccess) memcpy(host, b.p, bytes);
  g_pinned.put(b, st, e != hipSuccess);
  if (e != hipSuccess) return fail(APC_E_HIP, "read-back: %s", hipGetErrorString(e));
  return APC_OK;
}

// A read-back in two halves: start() queues the copy, finish() waits for it
// (polling, as read_back does) and copies the result out, so the host can
// queue more work in between.
struct PendingRead {
  PinnedBlock b;
  void* host = nullptr;
  size_t bytes = 0;
  hipStream_t st = nullptr;
  bool queued = false;
  ~PendingRead() { g_pinned.put(b, st, queued); }
  apc_status start(void* h, const void* dev, size_t n, hipStream_t s) {
    host = h;
    bytes = n;
    st = s;
    if (n == 0) return APC_OK;
    if (!g_pinned.get(n, b)) return fail(APC_E_OOM, "pinned read-back of %zu bytes", n);
    HIP_TRY(hipMemcpyAsync(b.p, dev, n, hipMemcpyDeviceToHost, s));
    queued = true;
    HIP_TRY(hipEventRecord(b.ev, s));
    return APC_OK;
  }
  apc_status finish() {
    if (bytes == 0) return APC_OK;
    hipError_t e;
    while ((e = hipEventQuery(b.ev)) == hipErrorNotReady) {
    }
    if (e != hipSuccess) return fail(APC_E_HIP, "read-back: %s", hipGetErrorString(e));
    queued = false;
    memcpy(host, b.p, bytes);
    return APC_OK;
  }
};

// Wait for the work queued on st by polling an event (see read_back).
apc_status spin_sync(hipStream_t st) {
  hipEvent_t ev = nullptr;
  HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
  hipError_t e = hipEventRecord(ev, st);
  if (e == hipSuccess) {
    while ((e = hipEventQuery(ev)) == hipErrorNotReady) {
    }
  }
  (void)hipEventDestroy(ev);
  if (e != hipSuccess) return fail(APC_E_HIP, "stream wait: %s", hipGetErrorString(e));
  return APC_OK;
}

// Pinned staging that stays valid until the process ends; append-only
// within one refactor call.
struct Staging {
  PinnedBlock b;
  size_t used = 0;
  hipStream_t last = nullptr;
  ~Staging() { g_pinned.put(b, nullptr, false); }  // its event follows its last copy
  apc_status put(const std::vector<char>& bytes, void* dev, hipStream_t st) {
    if (bytes.empty()) return APC_OK;
    if (used + bytes.size() > b.cap) {
      // the old block may still feed queued copies: its event guards reuse
      g_pinned.put(b, nullptr, false);
      if (!g_pinned.get(std::max<size_t>(bytes.size() * 2, (size_t)1 << 20), b))
        return fail(APC_E_OOM, "pinned staging of %zu bytes", bytes.size());
      used = 0;
    }
    char* dst = (char*)b.p + used;
    memcpy(dst, bytes.data(), bytes.size());
    used += (bytes.size() + 255) & ~(size_t)255;
    HIP_TRY(hipMemcpyAsync(dev, dst, bytes.size(), hipMemcpyHostToDevice, st));
    HIP_TRY(hipEventRecord(b.ev, st));
    last = st;
    return APC_OK;
  }
};

apc_status setup_geometry(apc_handle* h, const int64_t* dims, int32_t ndim, const apc_scheme* sc) {
  if (ndim < 1 || ndim > 3) return fail(APC_E_INVALID, "ndim must be 1..3 (got %d)", ndim);
  Geo& g = h->geo;
  g.d = ndim;
  for (int a = 0; a < 3; ++a) g.N[a] = 1;
  for (int a = 0; a < ndim; ++a) {
    if (dims[a] < 1 || dims[a] > (1ll << 30))
      return fail(APC_E_INVALID, "dims[%d]=%lld out of range", a, (long long)dims[a]);
    g.N[3 - ndim + a] = dims[a];
  }
  if (g.n() > (1ll << 32) - 1) return fail(APC_E_INVALID, "field too large (more than 2^32-1 points)");
  if (sc->kind != APC_PER_LEVEL && sc->kind != APC_PER_REGION) return fail(APC_E_INVALID, "scheme.kind");
  if (sc->degree != 1 && sc->degree != 3) return fail(APC_E_INVALID, "scheme.degree must be 1 or 3");
  if (sc->cd_axis < -1 || sc->cd_axis >= ndim) return fail(APC_E_INVALID, "scheme.cd_axis out of range");
  if (sc->cd_axis >= 0 && ndim < 2) return fail(APC_E_INVALID, "coefficient decomposition needs 2D or 3D data");
  if (sc->levels < 0 || sc->levels > 40) return fail(APC_E_INVALID, "scheme.levels out of range");
  if (sc->lossless != 0 && sc->lossless != 1) return fail(APC_E_INVALID, "scheme.lossless must be 0 or 1");
  if (sc->encoding < 0 || sc->encoding > 2) return fail(APC_E_INVALID, "scheme.encoding must be 0, 1 or 2");
  if (sc->kind == APC_PER_LEVEL) {
    for (int j = 0; j < ndim; ++j) g.sigma_user[j] = ndim - 1 - j;
  } else {
    bool seen[3] = {false, false, false};
    for (int j = 0; j < ndim; ++j) {
      const int a = sc->order[j];
      if (a < 0 || a >= ndim || seen[a]) return fail(APC_E_INVALID, "scheme.order is not a permutation");
      seen[a] = true;
      g.sigma_user[j] = a;
    }
  }
  for (int j = 0; j < ndim; ++j) g.sigma3[j] = g.sigma_user[j] + (3 - ndim);
  g.L = sc->levels > 0 ? sc->levels : default_levels(g.N);
  g.m.resize(g.L);
  for (int l = 0; l < g.L; ++l)
    for (int a = 0; a < 3; ++a) g.m[l][a] = (int32_t)((g.N[a] - 1) / ((int64_t)1 << l) + 1);
  h->scheme = *sc;
  return APC_OK;
}

// Offsets of every (level, region) lattice in the region code buffer (the
// coarsest level first, then levels L-2 .. 0, regions in pass order) and
// the buffer's length in codes.
int64_t region_layout(const Geo& g, std::vector<int64_t>& region_off) {
  const int d = g.d, L = g.L;
  region_off.assign((size_t)std::max(1, L) * 3, 0);
  int64_t off = (int64_t)g.m[L - 1][0] * g.m[L - 1][1] * g.m[L - 1][2];
  for (int l = L - 2; l >= 0; --l)
    for (int rho = 0; rho < d; ++rho) {
      region_off[l * 3 + rho] = off;
      off += lat_count(lattice(g, l, rho));
    }
  return off;
}

// Groups, streams, units and buffer offsets, in unit order.
void build_layout(apc_handle* h, int P) {
  Geo& g = h->geo;
  Meta& m = h->meta;
  const int d = g.d, L = g.L;
  const bool per_level = h->scheme.kind == APC_PER_LEVEL;
  const int cd_axis = h->scheme.cd_axis;
  m = Meta();
  m.d = d;
  m.L = L;
  m.P = P;
  m.n = g.n();
  m.lossless = h->scheme.lossless != 0;
  m.enc = h->scheme.encoding;
  h->code_n = region_layout(g, h->region_off);
  const int64_t ncoarse = (int64_t)g.m[L - 1][0] * g.m[L - 1][1] * g.m[L - 1][2];

  Group gc;
  gc.kind = G_COARSE;
  gc.level = L - 1;
  gc.n = ncoarse;
  m.groups.push_back(gc);
  Stream sc;
  sc.kind = S_COARSE;
  sc.level = L - 1;
  sc.group = 0;
  sc.n = ncoarse;
  sc.code_off = 0;
  m.streams.push_back(sc);
  Unit uc;
  uc.group = 0;
  uc.stream = 0;
  m.units.push_back(uc);

  h->cd.clear();
  h->cd_n = 0;
  h->cdreg_n = 0;
  for (int l = L - 2; l >= 0; --l) {
    const bool use_cd = cd_axis >= 0 && l == 0;
    auto add_cd = [&](int rho, int group) {
      const Lattice lat = lattice(g, 0, rho);
      CDInfo ci{};
      for (int a = 0; a < 3; ++a) ci.c[a] = lat.c[a];
      ci.a = cd_axis + (3 - d);
      int rest[2], nr = 0;
      for (int a = 0; a < 3; ++a)
        if (a != ci.a) rest[nr++] = a;
      std::vector<int> trip;
      for (int t = 0; t < 3; ++t) {
        Stream s;
        s.kind = S_CD;
        s.level = 0;
        s.rho = rho;
        s.t = t + 1;
        s.group = group;
        s.n = (int64_t)ci.c[ci.a] * cls_count_h(t, prefix_h(ci.c[rest[0]]), prefix_h(ci.c[rest[1]]));
        s.use_cd = true;
        s.code_off = h->cd_n;
        ci.s_off[t] = h->cd_n;
        ci.s_idx[t] = (int)m.streams.size();
        h->cd_n += s.n;
        trip.push_back((int)m.streams.size());
        m.streams.push_back(s);
      }
      ci.reg_off = h->cdreg_n;
      h->cdreg_n += lat_count(lat);
      h->cd.push_back(ci);
      return trip;
    };
    if (per_level) {
      Group gr;
      gr.kind = G_LEVEL;
      gr.level = l;
      for (int rho = 0; rho < d; ++rho) gr.n += lat_count(lattice(g, l, rho));
      gr.cd = use_cd ? CD_STAIR : CD_NONE;
      const int gi = (int)m.groups.size();
      m.groups.push_back(gr);
      if (!use_cd) {
        Stream s;
        s.kind = S_LEVEL;
        s.level = l;
        s.group = gi;
        s.n = gr.n;
        s.code_off = h->region_off[l * 3 + 0];
        Unit u;
        u.group = gi;
        u.stream = (int)m.streams.size();
        m.streams.push_back(s);
        m.units.push_back(u);
      } else {
        for (int rho = 0; rho < d; ++rho) add_cd(rho, gi);
        Unit u;  // the staircase is built once plane counts are known
        u.group = gi;
        u.stair = true;
        m.units.push_back(u);
      }
    } else {
      for (int rho = 0; rho < d; ++rho) {
        Group gr;
        gr.kind = G_REGION;
        gr.level = l;
        gr.rho = rho;
        gr.n = lat_count(lattice(g, l, rho));
        gr.cd = use_cd ? CD_SUM : CD_NONE;
        const int gi = (int)m.groups.size();
        m.groups.push_back(gr);
        if (!use_cd) {
          Stream s;
          s.kind = S_REGION;
          s.level = l;
          s.rho = rho;
          s.group = gi;
          s.n = gr.n;
          s.code_off = h->region_off[l * 3 + rho];
          Unit u;
          u.group = gi;
          u.stream = (int)m.streams.size();
          m.streams.push_back(s);
          m.units.push_back(u);
        } else {
          for (int s : add_cd(rho, gi)) {
            Unit u;
            u.group = gi;
            u.stream = s;
            m.units.push_back(u);
          }
        }
      }
    }
  }
  for (Stream& S : m.streams) {
    S.lossless = m.lossless;
    S.enc = m.enc;
  }
}

// Weights of every group (exact chain norms of the user axes).
// Host worker threads kept for the life of the process (starting threads
// for every call costs tens of microseconds each): up to 15 workers plus
// the calling thread.  One call uses them at a time.  A worker runs every
// job once; the caller waits until all have.
struct HostPool {
  std::mutex busy;  // held by the call using the workers
  std::mutex mu;
  std::condition_variable wake, done;
  const std::function<void()>* job = nullptr;
  uint64_t gen = 0;
  size_t pending = 0;
  size_t nworkers = 0;
  pid_t pid;
  HostPool() : pid(getpid()) {
    const size_t hw = std::max(1u, std::thread::hardware_concurrency());
    const size_t want = std::min<size_t>(16, hw) - 1;
    for (size_t t = 0; t < want; ++t) {
      try {
        std::thread([this] { loop(); }).detach();
      } catch (...) {  // no more threads to be had
        break;
      }
      ++nworkers;
    }
  }
  void loop() {
    uint64_t seen = 0;
    for (;;) {
      const std::function<void()>* j;
      {
        std::unique_lock<std::mutex> lk(mu);
        wake.wait(lk, [&] { return gen != seen; });
        seen = gen;
        j = job;
      }
      (*j)();
      std::lock_guard<std::mutex> lk(mu);
      if (--pending == 0) done.notify_one();
    }
  }
  void run(const std::function<void()>& f) {
    {
      std::lock_guard<std::mutex> lk(mu);
      job = &f;
      pending = nworkers;
      ++gen;
    }
    wake.notify_all();
    f();
    std::unique_lock<std::mutex> lk(mu);
    done.wait(lk, [&] { return pending == 0; });
  }
};
HostPool& host_pool() {
  static HostPool* p = new HostPool();  // never destroyed: its threads wait until the process ends
  return *p;
}

// f(i) for i in [0, n) on the host pool (the caller among the threads); for
// independent per-handle host work of a batch.  f must not throw.  A call
// made from inside f, or while another call holds the pool, or in a process
// forked from the one that started the pool, runs on its own thread.
thread_local bool g_in_parallel = false;
template <typename F>
void parallel_for(size_t n, F&& f) {
  if (n <= 1 || g_in_parallel) {
    for (size_t i = 0; i < n; ++i) f(i);
    return;
  }
  HostPool& pool = host_pool();
  if (pool.nworkers == 0 || pool.pid != getpid() || !pool.busy.try_lock()) {
    for (size_t i = 0; i < n; ++i) f(i);
    return;
  }
  std::atomic<size_t> next{0};
  const std::function<void()> work = [&] {
    const bool was = g_in_parallel;
    g_in_parallel = true;
    for (size_t i; (i = next.fetch_add(1)) < n;) f(i);
    g_in_parallel = was;
  };
  pool.run(work);
  pool.busy.unlock();
}

void assign_weights(apc_handle* h) {
  Geo& g = h->geo;
  Meta& m = h->meta;
  const int d = g.d;
  std::vector<std::vector<double>> ninf(d), none(d);
  for (int a = 0; a < d; ++a) axis_norms(g.N[3 - d + a], g.L, h->scheme.degree, ninf[a], none[a]);
  for (Group& gr : m.groups) {
    int levs[3];
    for (int a = 0; a < d; ++a) levs[a] = gr.kind == G_COARSE ? g.L - 1 : gr.level;
    if (gr.kind == G_REGION)
      for (int j = 0; j < d; ++j) levs[g.sigma_user[j]] = j <= gr.rho ? gr.level : gr.level + 1;
    double w = 1.0;
    double r = sqrt((double)gr.n / (double)m.n);
    for (int a = 0; a < d; ++a) {
      const double li = ninf[a][levs[a]], l1 = none[a][levs[a]];
      w = w * li;
      r = r * sqrt(li * l1);
    }
    gr.w = w;
    gr.rho_w = r;
  }
}

void finalize_units(apc_handle* h) {
  Meta& m = h->meta;
  for (Unit& u : m.units) {
    if (!u.stair) continue;
    std::vector<std::vector<int>> rs;
    for (int s = 0; s < (int)m.streams.size(); ++s) {
      const Stream& st = m.streams[s];
      if (st.kind == S_CD && st.group == u.group) {
        if (st.t == 1) rs.push_back({});
        rs.back().push_back(s);
      }
    }
    const int g = u.group;
    u = build_staircase(g, rs, m.streams);
  }
  for (Group& gr : m.groups) {
    gr.wd_inf = gr.w * gr.delta;
    gr.wd_2 = gr.rho_w * gr.delta;
  }
  finalize_meta(m);
}

RegionArgs region_args(const apc_handle* h, int l, int rho, bool per_level, double* const pr[2], bool with_pr,
                       bool write_pr) {
  const Geo& g = h->geo;
  RegionArgs ra{};
  ra.lat = lattice(g, l, rho);
  ra.rho = rho;
  for (int j = 0; j < 3; ++j) ra.sigma[j] = g.sigma3[j];
  ra.degree = h->scheme.degree;
  ra.per_level = per_level ? 1 : 0;
  for (int r = 0; r < 2; ++r) {
    if (r < rho && with_pr) {
      ra.prl[r] = lattice(g, l, r);
      ra.pr[r] = pr[r];
    }
  }
  ra.pr_out = (write_pr && rho < g.d - 1) ? pr[rho] : nullptr;
  return ra;
}

int group_of(const Meta& m, int l, int rho) {
  for (int gi = 0; gi < (int)m.groups.size(); ++gi) {
    const Group& gr = m.groups[gi];
    if (gr.kind == G_LEVEL && gr.level == l) return gi;
    if (gr.kind == G_REGION && gr.level == l && gr.rho == rho) return gi;
  }
  return 0;
}

int stream_of(const Meta& m, int l, int rho) {
  for (int s = 0; s < (int)m.streams.size(); ++s) {
    const Stream& S = m.streams[s];
    if (S.kind == S_LEVEL && S.level == l) return s;
    if (S.kind == S_REGION && S.level == l && S.rho == rho) return s;
  }
  return -1;
}

// ------------------------------------------------------------- refactoring
// Refactor a batch of fields (one dtype): every pass is one launch over the
// segments of all fields; the host syncs three times for the whole batch.
template <typename T, typename Q>
apc_status refactor_batch(std::vector<apc_handle*>& H, const std::vector<const T*>& X, hipStream_t st) {
  const int nf = (int)H.size();
  reap_retired();
  // on an early (error) return, queued work is waited for before any
  // buffer is released; a completed call retires its temporaries instead
  DrainScope drain(st);
  const int P = sizeof(T) == 4 ? 29 : 52;
  struct Tmp {
    DevBuf grids, codes, cdc;
    std::vector<int64_t> goff;   // level -> offset in grids
    int64_t acc = 0;             // offset in the accumulator buffer
  };
  std::vector<Tmp> tmp(nf);
  int64_t nacc = 0;
  // each field's layout (groups, streams, units, offsets) is its own host work
  parallel_for((size_t)nf, [&](size_t f) { build_layout(H[f], P); });
  for (int f = 0; f < nf; ++f) {
    apc_handle* h = H[f];
    const Geo& g = h->geo;
    Tmp& t = tmp[f];
    t.goff.assign(g.L, 0);
    int64_t gtot = 0;
    // compact level grids: per-level fields read the field at strides and
    // only need the coarsest level here
    const bool per_level = h->scheme.kind == APC_PER_LEVEL;
    for (int l = per_level ? g.L - 1 : 1; l < g.L; ++l) {
      if (l == 0) continue;
      t.goff[l] = gtot;
      gtot += (int64_t)g.m[l][0] * g.m[l][1] * g.m[l][2];
    }
    APC_TRY(t.grids.alloc(sizeof(T) * (size_t)std::max<int64_t>(1, gtot)));
    APC_TRY(t.codes.alloc(sizeof(Q) * (size_t)h->code_n));
    if (h->cd_n) APC_TRY(t.cdc.alloc(sizeof(Q) * (size_t)h->cd_n));
    t.acc = nacc;
    nacc += 4 + (int64_t)h->meta.groups.size() + (int64_t)h->meta.streams.size();
  }
  DevBuf accb, tab;
  APC_TRY(accb.alloc(8 * (size_t)nacc));
  std::vector<unsigned long long> init((size_t)nacc, 0ull);
  for (int f = 0; f < nf; ++f) init[(size_t)tmp[f].acc] = ~0ull;
  Staging stage;
  {
    std::vector<char> b(init.size() * 8);
    memcpy(b.data(), init.data(), b.size());
    APC_TRY(stage.put(b, accb.p, st));
  }
  unsigned long long* acc = accb.as<unsigned long long>();
  auto grid_ptr = [&](int f, int l) -> const T* { return l == 0 ? X[f] : tmp[f].grids.template as<T>() + tmp[f].goff[l]; };
  // per-level fields: one tensor-product pass per level (all levels in one launch)
  // every segment of a launch shares one tile width: the one chosen for the
  // largest level in the batch
  int lvl_t2 = 64;
  {
    int64_t big = -1;
    for (int f = 0; f < nf; ++f) {
      const apc_handle* h = H[f];
      if (h->scheme.kind != APC_PER_LEVEL || h->geo.L < 2 || h->geo.m[0][0] == 1) continue;
      const Geo& g = h->geo;
      const int64_t n = g.n();
      if (n > big) {
        big = n;
        lvl_t2 = tile_for(h->dtype, (int)g.m[0][1], (int)g.m[0][2]);
      }
    }
  }
  // runs along axis 0: a field alone spreads each level over 1024 blocks or
  // more; in a batch the fields share the launch, and each level is cut
  // into fewer, longer runs (the coarse planes a run needs before its first
  // step are fewer per point)
  int64_t lvl_min_blocks = 1024;
  {
    int nlev = 0;
    for (int f = 0; f < nf; ++f) nlev += H[f]->scheme.kind == APC_PER_LEVEL;
    lvl_min_blocks = std::max<int64_t>(64, 1024 / std::max(1, nlev));
  }
  // segments of levels with several planes (tiles lvl_t2 wide) and of
  // single-plane levels (one-column tiles): one launch each
  auto level_segs = [&](int mode, double& by, bool flat) {
    std::vector<LevelSeg> ls2;
    for (int f = 0; f < nf; ++f) {
      const apc_handle* h = H[f];
      if (h->scheme.kind != APC_PER_LEVEL) continue;
      for (int l = 0; l < h->geo.L - 1; ++l) {
        if ((h->geo.m[l][0] == 1) != flat) continue;
        LevelSeg c = level_seg(h, l);
        const Geo& g = h->geo;
        c.src = X[f];
        const int64_t sl = (int64_t)1 << l;
        c.xs[0] = sl * g.N[1] * g.N[2];
        c.xs[1] = sl * g.N[2];
        c.xs[2] = sl;
        if (mode == 0 && l == 0) c.racc = acc + tmp[f].acc;  // the field's range, in the same pass
        const int gi = group_of(h->meta, l, 0);
        c.gmax = acc + tmp[f].acc + 4 + gi;
        for (int rho = 0; rho < h->geo.d; ++rho) c.q[rho] = tmp[f].codes.template as<Q>() + h->region_off[l * 3 + rho];
        shape_level_seg(c, lvl_t2, lvl_min_blocks);
        // bytes the method moves: each fine point of the level read once (and
        // its code written in the quantization pass); coarse points are
        // counted at their own, coarser level, the coarsest by its own pass
        const int64_t nfine = (int64_t)c.m[0] * c.m[1] * c.m[2] - (int64_t)c.mc[0] * c.mc[1] * c.mc[2];
        by += (double)nfine * (sizeof(T) + (mode == 1 ? sizeof(Q) : 0));
        ls2.push_back(c);
      }
    }
    return ls2;
  };

  // ---- tables of the first pass
  TableBuilder tb;
  std::vector<Launch> ls;
  {
    std::vector<FlatSeg> rs, gs;
    for (int f = 0; f < nf; ++f) {
      FlatSeg s{};
      s.src = X[f];
      s.n = H[f]->geo.n();
      s.acc = acc + tmp[f].acc;
      const Geo& g = H[f]->geo;
      const bool per_level = H[f]->scheme.kind == APC_PER_LEVEL;
      if (!per_level || g.L < 2) rs.push_back(s);  // per-level: the level-0 max pass finds the range
      for (int l = per_level ? g.L - 1 : 1; l < g.L; ++l) {
        if (l == 0) continue;
        FlatSeg q{};
        q.src = X[f];
        q.dst = tmp[f].grids.template as<T>() + tmp[f].goff[l];
        q.n = (int64_t)g.m[l][0] * g.m[l][1] * g.m[l][2];
        const int64_t sl = (int64_t)1 << l;
        q.s[0] = sl * g.N[1] * g.N[2];
        q.s[1] = sl * g.N[2];
        q.s[2] = sl;
        for (int a = 0; a < 3; ++a) q.dm[a] = g.m[l][a];
        q.f2 = make_fastdiv((uint32_t)q.dm[2]);
        q.f1 = make_fastdiv((uint32_t)q.dm[1]);
        gs.push_back(q);
      }
    }
    double nb = 0, gb = 0;
    for (auto& s : rs) nb += (double)sizeof(T) * s.n;
    for (auto& s : gs) gb += 2.0 * sizeof(T) * s.n;
    const int64_t b1 = assign_blocks<FlatSeg>(rs, [](const FlatSeg& s) { return s.n; });
    const int64_t b2 = assign_blocks<FlatSeg>(gs, [](const FlatSeg& s) { return s.n; });
    if (!rs.empty()) ls.push_back({K_RANGE, tb.add(rs), (int)rs.size(), b1, 0, nb, "range"});
    if (!gs.empty()) ls.push_back({K_GATHER, tb.add(gs), (int)gs.size(), b2, 0, gb, "subsample"});
    for (int flat = 0; flat < 2; ++flat) {
      double by = 0;
      std::vector<LevelSeg> lv = level_segs(0, by, flat);
      const int64_t nbk = assign_level_blocks(lv);
      if (!lv.empty()) ls.push_back({K_LEVEL0, tb.add(lv), (int)lv.size(), nbk, flat ? 1 : lvl_t2, by, "coef_max"});
    }
    for (int rho = 0; rho < 3; ++rho) {  // per-region fields: one pass per region
      std::vector<CoefSeg> cs;
      double by = 0;
      for (int f = 0; f < nf; ++f) {
        const apc_handle* h = H[f];
        if (rho >= h->geo.d || h->scheme.kind == APC_PER_LEVEL) continue;
        for (int l = 0; l < h->geo.L - 1; ++l) {
          CoefSeg c{};
          double* pr[2] = {nullptr, nullptr};
          c.ra = region_args(h, l, rho, false, pr, false, false);
          if (lat_count(c.ra.lat) == 0) continue;
          c.G = grid_ptr(f, l);
          c.gmax = acc + tmp[f].acc + 4 + group_of(h->meta, l, rho);
          by += (double)lat_count(c.ra.lat) * sizeof(T);
          cs.push_back(c);
        }
      }
      const int64_t nbk = assign_blocks<CoefSeg>(cs, [](const CoefSeg& c) { return lat_count(c.ra.lat); });
      if (!cs.empty()) ls.push_back({K_COEF0, tb.add(cs), (int)cs.size(), nbk, 0, by, "coef_max"});
    }
    std::vector<FlatSeg> cs;
    double by = 0;
    for (int f = 0; f < nf; ++f) {
      FlatSeg s{};
      s.src = grid_ptr(f, H[f]->geo.L - 1);
      s.n = H[f]->meta.streams[0].n;
      s.acc = acc + tmp[f].acc + 4;
      by += (double)sizeof(T) * s.n;
      cs.push_back(s);
    }
    const int64_t nbk = assign_blocks<FlatSeg>(cs, [](const FlatSeg& s) { return s.n; });
    ls.push_back({K_COARSE0, tb.add(cs), (int)cs.size(), nbk, 0, by, "coarse"});
  }
  APC_TRY(tab.alloc(tb.bytes.size()));
  APC_TRY(stage.put(tb.bytes, tab.p, st));
  APC_TRY((issue<T, Q>(ls, (const char*)tab.p, st)));

  // ---- second pass: codes, then coefficient decomposition.  It is queued
  // right behind the first: the quantization kernels derive each group's
  // shift P - E from the group maximum the first pass left on the device, and
  // the host reads the maxima (with the range and the decomposition maxima)
  // once, after the decomposition.
  TableBuilder tb2;
  ls.clear();
  for (int flat = 0; flat < 2; ++flat) {
    double by = 0;
    std::vector<LevelSeg> lv = level_segs(1, by, flat);
    const int64_t nbk = assign_level_blocks(lv);
    if (!lv.empty()) ls.push_back({K_LEVEL1, tb2.add(lv), (int)lv.size(), nbk, flat ? 1 : lvl_t2, by, "coef_quant"});
  }
  for (int rho = 0; rho < 3; ++rho) {
    std::vector<CoefSeg> cs;
    double by = 0;
    for (int f = 0; f < nf; ++f) {
      const apc_handle* h = H[f];
      if (rho >= h->geo.d || h->scheme.kind == APC_PER_LEVEL) continue;
      for (int l = 0; l < h->geo.L - 1; ++l) {
        CoefSeg c{};
        double* pr[2] = {nullptr, nullptr};
        c.ra = region_args(h, l, rho, false, pr, false, false);
        if (lat_count(c.ra.lat) == 0) continue;
        c.G = grid_ptr(f, l);
        c.codes = tmp[f].codes.template as<Q>() + h->region_off[l * 3 + rho];
        c.gmax = acc + tmp[f].acc + 4 + group_of(h->meta, l, rho);
        by += (double)lat_count(c.ra.lat) * (sizeof(T) + sizeof(Q));
        cs.push_back(c);
      }
    }
    const int64_t nbk = assign_blocks<CoefSeg>(cs, [](const CoefSeg& c) { return lat_count(c.ra.lat); });
    if (!cs.empty()) ls.push_back({K_COEF1, tb2.add(cs), (int)cs.size(), nbk, 0, by, "coef_quant"});
  }
  {
    std::vector<FlatSeg> cs;
    double by = 0;
    for (int f = 0; f < nf; ++f) {
      FlatSeg s{};
      s.src = grid_ptr(f, H[f]->geo.L - 1);
      s.dst = tmp[f].codes.p;
      s.n = H[f]->meta.streams[0].n;
      s.acc = acc + tmp[f].acc + 4;  // the coarsest level's group (group 0)
      by += (double)(sizeof(T) + sizeof(Q)) * s.n;
      cs.push_back(s);
    }
    const int64_t nbk = assign_blocks<FlatSeg>(cs, [](const FlatSeg& s) { return s.n; });
    ls.push_back({K_COARSE1, tb2.add(cs), (int)cs.size(), nbk, 0, by, "coarse"});
  }
  for (int a3 = 0; a3 < 3; ++a3) {
    std::vector<CDSeg> cs;
    double by = 0;
    for (int f = 0; f < nf; ++f) {
      apc_handle* h = H[f];
      for (int rho = 0; rho < (int)h->cd.size(); ++rho) {
        const CDInfo& ci = h->cd[rho];
        if (ci.a != a3) continue;
        CDSeg c{};
        for (int a = 0; a < 3; ++a) c.c[a] = ci.c[a];
        c.f2 = make_fastdiv((uint32_t)std::max(1, c.c[2]));
        c.f1 = make_fastdiv((uint32_t)std::max(1, c.c[1]));
        c.R = tmp[f].codes.template as<Q>() + h->region_off[0 * 3 + rho];
        for (int t = 0; t < 3; ++t) {
          c.S[t] = tmp[f].cdc.template as<Q>() + ci.s_off[t];
          c.smax[t] = acc + tmp[f].acc + 4 + h->meta.groups.size() + ci.s_idx[t];
        }
        const int64_t cnt = (int64_t)c.c[0] * c.c[1] * c.c[2];
        if (cnt == 0) continue;
        by += 2.0 * sizeof(Q) * cnt;
        cs.push_back(c);
      }
    }
    if (cs.empty()) continue;
    if (a3 < 2) {  // v runs along lattice rows: one pass over row tiles
      const int64_t nbk = assign_cd_tile_blocks(cs, a3);
      ls.push_back({K_CDFT, tb2.add(cs), (int)cs.size(), nbk, a3, by, "cd_forward"});
    } else {
      const int64_t nbk = assign_cd_blocks(cs);
      ls.push_back({K_CDF, tb2.add(cs), (int)cs.size(), nbk, a3, by, "cd_forward"});
    }
  }
  // Sign arenas, sized by a bound known before any count (each code takes at
  // most one sign bit and each plane's run is rounded up to whole words) and
  // cleared (one launch for the batch) behind the passes above, instead of
  // between the count read-back and the sign placement.
  std::vector<int64_t> sign_ub(nf, 0);
  {
    std::vector<FlatSeg> zs;
    for (int f = 0; f < nf; ++f) {
      apc_handle* h = H[f];
      for (const Stream& S : h->meta.streams) sign_ub[f] += (S.n + 63) / 64 + 8 * (int64_t)sizeof(Q);
      sign_ub[f] = std::max<int64_t>(1, sign_ub[f]);
      APC_TRY(h->sign.alloc(8 * (size_t)sign_ub[f]));
      FlatSeg z{};
      z.dst = h->sign.p;
      z.n = sign_ub[f];
      zs.push_back(z);
    }
    const int64_t nbk = assign_blocks<FlatSeg>(zs, [](const FlatSeg& z) { return z.n; });
    double by = 0;
    for (const FlatSeg& z : zs) by += 8.0 * (double)z.n;
    ls.push_back({K_ZERO, tb2.add(zs), (int)zs.size(), nbk, 0, by, "sign_clear"});
  }
  DevBuf tab2;
  APC_TRY(tab2.alloc(tb2.bytes.size()));
  APC_TRY(stage.put(tb2.bytes, tab2.p, st));
  APC_TRY((issue<T, Q>(ls, (const char*)tab2.p, st)));
  std::vector<unsigned long long> hv((size_t)nacc);
  APC_TRY(read_back(hv.data(), acc, 8 * hv.size(), st));
  for (int f = 0; f < nf; ++f) {
    const unsigned long long* v = hv.data() + tmp[f].acc;
    if (v[3]) return fail(APC_E_NONFINITE, "field %d holds NaN or Inf", f);
    Meta& m = H[f]->meta;
    m.xmin = unordered(v[0]);
    m.xmax = unordered(v[1]);
    m.A = bits_double(v[2]);
    for (size_t gi = 0; gi < m.groups.size(); ++gi) {
      Group& gr = m.groups[gi];
      gr.M = bits_double(v[4 + gi]);
      if (gr.M > 0.0) {  // the shift the quantization kernels used (group_k_shift)
        int E;
        frexp(gr.M, &E);
        gr.E = E;
        gr.k_shift = P - E;
        gr.delta = ldexp(1.0, E - P);
      } else {
        gr.E = 0;
        gr.k_shift = 0;
        gr.delta = 0.0;
      }
    }
  }
  for (int f = 0; f < nf; ++f) {
    apc_handle* h = H[f];
    Meta& m = h->meta;
    const unsigned long long* v = hv.data() + tmp[f].acc + 4 + m.groups.size();
    for (int s = 0; s < (int)m.streams.size(); ++s) {
      Stream& S = m.streams[s];
      if (S.use_cd) {
        S.maxabs = (int64_t)bits_double(v[s]);
      } else {
        const Group& gr = m.groups[S.group];
        S.maxabs = gr.M > 0.0 ? (int64_t)rint(ldexp(gr.M, gr.k_shift)) : 0;
      }
      if (S.n == 0) S.maxabs = 0;
      S.B = S.enc ? nb_digits(S.maxabs) : bitlen(S.maxabs);
    }
  }

  // ---- bitplane encoding of every stream of every field
  std::vector<StreamDev> sds, nsd;             // generic streams, negabinary streams
  std::vector<std::pair<int, int>> sd_of, nsd_of;  // (field, stream)
  int64_t chunks = 0, cnt_n = 0, stage_w = 0, nchunks = 0;
  for (int f = 0; f < nf; ++f) {
    apc_handle* h = H[f];
    Meta& m = h->meta;
    int64_t mag_w = 0, idx_n = 0;
    for (Stream& S : m.streams) {
      S.mag_off = mag_w;
      S.idx_off = idx_n;
      if (S.B == 0 || S.n == 0) continue;
      mag_w += (int64_t)S.B * S.words();
      idx_n += (int64_t)S.B * S.chunks();
    }
    APC_TRY(h->mag.alloc(8 * (size_t)std::max<int64_t>(1, mag_w)));
    APC_TRY(h->idx.alloc(4 * (size_t)std::max<int64_t>(1, idx_n)));
    for (int s = 0; s < (int)m.streams.size(); ++s) {
      Stream& S = m.streams[s];
      if (S.B == 0 || S.n == 0) continue;
      if (S.enc) {  // digit planes: no index, no signs
        StreamDev nd{};
        nd.codes = (S.use_cd ? tmp[f].cdc.template as<Q>() : tmp[f].codes.template as<Q>()) + S.code_off;
        nd.mag = h->mag.as<uint64_t>() + S.mag_off;
        nd.n = S.n;
        nd.M = S.words();
        nd.C = S.chunks();
        nd.chunk_begin = nchunks;
        nd.B = S.B;
        nd.xor_chain = S.enc == 2 ? 1 : 0;
        nchunks += nd.C;
        nsd.push_back(nd);
        nsd_of.push_back({f, s});
        continue;
      }
      StreamDev sd{};
      sd.codes = (S.use_cd ? tmp[f].cdc.template as<Q>() : tmp[f].codes.template as<Q>()) + S.code_off;
      sd.mag = h->mag.as<uint64_t>() + S.mag_off;
      sd.idx = h->idx.as<uint32_t>() + S.idx_off;
      sd.cnt = (uint32_t*)(intptr_t)cnt_n;      // offsets, rebased below
      sd.stage = (uint64_t*)(intptr_t)stage_w;
      sd.n = S.n;
      sd.M = S.words();
      sd.C = S.chunks();
      sd.chunk_begin = chunks;
      sd.B = S.B;
      cnt_n += (int64_t)S.B * sd.C;
      stage_w += 64 * sd.C;
      chunks += sd.C;
      sds.push_back(sd);
      sd_of.push_back({f, s});
    }
  }
  DevBuf cntb, stageb, sdb, jobs, totals;
  APC_TRY(cntb.alloc(4 * (size_t)std::max<int64_t>(1, cnt_n)));
  APC_TRY(stageb.alloc(8 * (size_t)std::max<int64_t>(1, stage_w)));
  double eb = 0;
  for (StreamDev& sd : sds) {
    sd.cnt = cntb.as<uint32_t>() + (intptr_t)sd.cnt;
    sd.stage = stageb.as<uint64_t>() + (intptr_t)sd.stage;
    eb += (double)sizeof(Q) * sd.n + 8.0 * sd.B * sd.M + 512.0 * sd.C + 4.0 * sd.B * sd.C;
  }
  std::vector<int32_t> job;
  int njobs = 0;
  for (size_t i = 0; i < sds.size(); ++i) njobs += sds[i].B;
  job.resize(2 * (size_t)njobs);
  {
    int k = 0;
    for (size_t i = 0; i < sds.size(); ++i)
      for (int j = 0; j < sds[i].B; ++j, ++k) {
        job[k] = (int32_t)i;
        job[njobs + k] = j;
      }
  }
  std::vector<int64_t> tot((size_t)njobs);
  PendingRead rd_tot;
  DevBuf prefix, errb;
  DevBuf zcnt, ztot;  // lossless stage: per-chunk nonzero words, per-plane totals
  // ---- sign sections: laid out on the device from the plane totals
  // (k_sign_layout), then placed; the totals come back to the host meanwhile
  // and the host repeats the layout for the metadata.  The layout tables
  // (each plane's offset slot, each stream's jobs) travel with the encode
  // table, and the layout kernel adds each stream's offset to its sign
  // pointer in that table, which the sign placement then reads.
  {
    size_t i = 0;
    std::vector<int> nplanes(nf, 0);
    for (int f = 0; f < nf; ++f) H[f]->psb.assign(H[f]->meta.streams.size(), 0);
    std::vector<SignJob> sj((size_t)njobs);
    std::vector<SignStream> ss(sds.size());
    std::vector<int32_t> f_first(nf, 0);
    {
      int k = 0, prev_f = -1;
      for (i = 0; i < sds.size(); ++i) {
        const int f = sd_of[i].first, s = sd_of[i].second;
        if (f != prev_f) {
          f_first[f] = k;
          prev_f = f;
        }
        H[f]->psb[s] = nplanes[f];
        ss[i].first = k;
        ss[i].njob = sds[i].B;
        ss[i].f_first = f_first[f];
        ss[i].ub = sign_ub[f];
        for (int j = 0; j < sds[i].B; ++j, ++k) {
          sj[k].pso_dst = (int64_t*)(intptr_t)(nplanes[f] + j);  // rebased below
          sj[k].s_first = ss[i].first;
        }
        nplanes[f] += sds[i].B;
      }
    }
    for (int f = 0; f < nf; ++f) APC_TRY(H[f]->pso.alloc(8 * std::max<size_t>(1, (size_t)nplanes[f])));
    for (int k = 0; k < njobs; ++k) {
      const int f = sd_of[job[k]].first;
      sj[k].pso_dst = H[f]->pso.as<int64_t>() + (intptr_t)sj[k].pso_dst;
    }
    double sb = 0;
    for (i = 0; i < sds.size(); ++i) {
      const int f = sd_of[i].first, s = sd_of[i].second;
      sds[i].sign = H[f]->sign.as<uint64_t>();  // the stream's offset is added on the device
      sds[i].pso = H[f]->pso.as<int64_t>() + H[f]->psb[s];
      sds[i].sign_n = 0;
      sb += 512.0 * sds[i].C + 8.0 * (sds[i].n / 64 + sds[i].B);
    }
    // lossless stage: the encoder counts each chunk's nonzero words per plane
    // (zcnt); a scan gives per plane the counts before each chunk (kept on
    // the handle for packing stored sections) and the totals, read back with
    // the sign totals
    std::vector<StreamDev> zsd;
    std::vector<int32_t> zjs, zjj;
    std::vector<size_t> zof;  // encode-table entry of each lossless stream
    std::vector<StreamDev*> all;  // generic then negabinary encode-table entries
    std::vector<std::pair<int, int>> all_of;
    for (i = 0; i < sds.size(); ++i) {
      all.push_back(&sds[i]);
      all_of.push_back(sd_of[i]);
    }
    for (i = 0; i < nsd.size(); ++i) {
      all.push_back(&nsd[i]);
      all_of.push_back(nsd_of[i]);
    }
    int64_t zcnt_n = 0;
    for (i = 0; i < all.size(); ++i)
      if (H[all_of[i].first]->meta.lossless) zcnt_n += (int64_t)all[i]->B * all[i]->C;
    if (zcnt_n) APC_TRY(zcnt.alloc(4 * (size_t)zcnt_n));
    zcnt_n = 0;
    for (i = 0; i < all.size(); ++i) {
      const int f = all_of[i].first, s = all_of[i].second;
      apc_handle* h = H[f];
      if (!h->meta.lossless) continue;
      if (!h->zoff.p) {
        int64_t nz = 0;
        for (const Stream& S : h->meta.streams)
          if (S.B && S.n) nz += (int64_t)S.B * S.chunks();
        APC_TRY(h->zoff.alloc(4 * (size_t)std::max<int64_t>(1, nz)));
      }
      all[i]->zcnt = zcnt.as<uint32_t>() + zcnt_n;
      zcnt_n += (int64_t)all[i]->B * all[i]->C;
      StreamDev d = *all[i];
      d.cnt = all[i]->zcnt;
      d.idx = h->zoff.as<uint32_t>() + h->meta.streams[s].idx_off;
      for (int j = 0; j < d.B; ++j) {
        zjs.push_back((int32_t)zsd.size());
        zjj.push_back(j);
      }
      zsd.push_back(d);
      zof.push_back(i);
    }
    std::vector<int64_t> ztv(zjs.size(), 0);
    PendingRead rd_z;
    if (!sds.empty() || !nsd.empty()) {
      TableBuilder tb3;
      const size_t o_sd = tb3.add(sds);
      const size_t o_job = tb3.add(job);
      const size_t o_sj = tb3.add(sj);
      const size_t o_ss = tb3.add(ss);
      const size_t o_nd = tb3.add(nsd);
      const size_t o_zd = tb3.add(zsd), o_zs = tb3.add(zjs), o_zj = tb3.add(zjj);
      APC_TRY(sdb.alloc(tb3.bytes.size()));
      APC_TRY(totals.alloc(8 * (size_t)std::max(1, njobs)));
      APC_TRY(prefix.alloc(8 * ((size_t)njobs + 1)));
      APC_TRY(errb.alloc(4));
      APC_TRY(stage.put(tb3.bytes, sdb.p, st));
      StreamDev* sdd = (StreamDev*)((char*)sdb.p + o_sd);
      const int32_t* jd = (const int32_t*)((const char*)sdb.p + o_job);
      if (!sds.empty()) {
        LAUNCH("encode", eb, st, launch_encode<Q>(sdd, (int)sds.size(), chunks, st));
        LAUNCH("scan", 8.0 * cnt_n, st, launch_scan(sdd, jd, jd + njobs, njobs, totals.as<int64_t>(), st));
        APC_TRY(rd_tot.start(tot.data(), totals.p, 8 * (size_t)njobs, st));
      }
      if (!nsd.empty()) {
        double nbb = 0;
        for (const StreamDev& d : nsd) nbb += (double)sizeof(Q) * d.n + 8.0 * d.B * d.M;
        LAUNCH("encode_nb", nbb, st,
               launch_encode_nb<Q>((const StreamDev*)((char*)sdb.p + o_nd), (int)nsd.size(), nchunks, st));
      }
      if (!zsd.empty()) {
        APC_TRY(ztot.alloc(8 * ztv.size()));
        const char* zb = (const char*)sdb.p;
        LAUNCH("zws_scan", 8.0 * zcnt_n, st,
               launch_scan((const StreamDev*)(zb + o_zd), (const int32_t*)(zb + o_zs), (const int32_t*)(zb + o_zj),
                           (int)zjs.size(), ztot.as<int64_t>(), st));
        APC_TRY(rd_z.start(ztv.data(), ztot.p, 8 * ztv.size(), st));
      }
      if (!sds.empty()) LAUNCH("sign_layout", 16.0 * njobs, st,
             launch_sign_layout(totals.as<int64_t>(), njobs, (const SignJob*)((const char*)sdb.p + o_sj),
                                (int)sds.size(), (const SignStream*)((const char*)sdb.p + o_ss), sdd,
                                prefix.as<int64_t>(), errb.as<int32_t>(), st));
      if (!sds.empty()) LAUNCH("sign_move", sb, st, launch_sign_move(sdd, (int)sds.size(), chunks, st));
    }
    // the same layout on the host, for the metadata
    APC_TRY(rd_tot.finish());
    APC_TRY(rd_z.finish());
    {
      size_t k = 0;
      for (size_t z = 0; z < zof.size(); ++z) {
        Stream& S = H[all_of[zof[z]].first]->meta.streams[all_of[zof[z]].second];
        S.nnz.assign(S.B, 0);
        for (int j = 0; j < S.B; ++j) S.nnz[j] = ztv[k++];
      }
    }
    std::vector<int64_t> sign_words(nf, 0);
    for (int f = 0; f < nf; ++f)
      for (Stream& S : H[f]->meta.streams) {
        S.nsig.clear();
        S.pso.clear();
      }
    size_t jb = 0;
    for (i = 0; i < sds.size(); ++i) {
      const int f = sd_of[i].first, s = sd_of[i].second;
      Stream& S = H[f]->meta.streams[s];
      S.nsig.assign(S.B, 0);
      S.pso.assign(S.B, 0);
      S.sign_off = sign_words[f];
      int64_t w = 0;
      for (int j = 0; j < S.B; ++j, ++jb) {
        S.nsig[j] = tot[jb];
        S.pso[j] = w;
        w += (tot[jb] + 63) / 64;
      }
      sign_words[f] += w;
    }
    for (const auto& fs : nsd_of) {  // digit planes carry no signs
      Stream& S = H[fs.first]->meta.streams[fs.second];
      S.nsig.assign(S.B, 0);
      S.pso.assign(S.B, 0);
      S.sign_off = sign_words[fs.first];
    }
    for (int f = 0; f < nf; ++f)
      if (sign_words[f] > sign_ub[f]) return fail(APC_E_INVALID, "internal: sign section exceeds its bound");
  }
  // The rest of the metadata is host work on counts already read back; it
  // runs while the sign placement is on the device, and so does the
  // interpreter's greedy sequence for error-bound targets (kept in the
  // handle for its first retrieval).
  // (independent per field: spread over host threads for large batches)
  parallel_for((size_t)nf, [&](size_t f) {
    assign_weights(H[f]);
    finalize_units(H[f]);
    H[f]->k_res.assign(H[f]->meta.streams.size(), 0);
    ensure_sequence(H[f]->meta, 0);
  });
  // The call returns while the sign placement may still run: each handle
  // gets an event behind it (work on other streams waits for that), and the
  // temporaries stay allocated until it has finished.  (The layout kernel's
  // bound check repeats the host's, above, which has already passed.)
  {  // one event for the whole batch, shared by its handles
    hipEvent_t ev = nullptr;
    HIP_TRY(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
    std::shared_ptr<void> owner((void*)ev, [](void* e) { (void)hipEventDestroy((hipEvent_t)e); });
    HIP_TRY(hipEventRecord(ev, st));
    for (int f = 0; f < nf; ++f) {
      apc_handle* h = H[f];
      if (h->ready && !h->ready_owner) (void)hipEventDestroy(h->ready);
      h->ready = ev;
      h->ready_owner = owner;
    }
  }
  std::vector<DevBuf> keep;
  for (Tmp& t : tmp) {
    keep.push_back(std::move(t.grids));
    keep.push_back(std::move(t.codes));
    keep.push_back(std::move(t.cdc));
  }
  for (DevBuf* b : {&accb, &tab, &tab2, &cntb, &stageb, &sdb, &jobs, &totals, &prefix, &errb, &zcnt, &ztot})
    keep.push_back(std::move(*b));
  APC_TRY(retire(std::move(keep), st));
  drain.armed = false;
  return APC_OK;
}

// ---------------------------------------------------------------- retrieval
// Work buffers of one retrieval (the handle's own, or a server slot's).
struct WorkPtrs {
  double* xc = nullptr;
  double* xb[2] = {nullptr, nullptr};
  double* pr[2] = {nullptr, nullptr};
  void* cdreg = nullptr;
  // decoded codes (region codes, decomposition codes); null = the handle's
  // resident buffers
  void* codes = nullptr;
  void* cd_codes = nullptr;
  // digit-plane handles: the truncated integers of this retrieval (layout of
  // the decoded codes), which the recomposition and reconstruction read
  void* pcodes = nullptr;
  void* pcd_codes = nullptr;
};

// Bytes of work buffers a retrieval of this handle needs (layout of carve_work).
size_t work_bytes(const apc_handle* h) {
  const Geo& g = h->geo;
  const int L = g.L;
  size_t b = 8 * (size_t)((int64_t)g.m[L - 1][0] * g.m[L - 1][1] * g.m[L - 1][2]) + 256;
  if (L >= 2) {
    b += 2 * (8 * (size_t)((int64_t)g.m[1][0] * g.m[1][1] * g.m[1][2]) + 256);
    if (h->scheme.kind != APC_PER_LEVEL) {  // earlier regions' values (per-region reconstruction)
      if (g.d >= 2) b += 8 * (size_t)lat_count(lattice(g, 0, 0)) + 256;
      if (g.d >= 3) b += 8 * (size_t)lat_count(lattice(g, 0, 1)) + 256;
    }
    b += qsize(h->dtype) * (size_t)h->cdreg_n + 256;
  }
  if (h->meta.enc)  // truncated integers of the digit words
    b += qsize(h->dtype) * (size_t)(std::max<int64_t>(1, h->code_n) + std::max<int64_t>(1, h->cd_n)) + 512;
  return b;
}

WorkPtrs carve_work(const apc_handle* h, void* base) {
  const Geo& g = h->geo;
  const int L = g.L;
  WorkPtrs w;
  char* p = (char*)base;
  auto take = [&](size_t n) {
    char* r = p;
    p += (n + 255) & ~(size_t)255;
    return r;
  };
  w.xc = (double*)take(8 * (size_t)((int64_t)g.m[L - 1][0] * g.m[L - 1][1] * g.m[L - 1][2]));
  if (L >= 2) {
    const size_t n1 = (size_t)((int64_t)g.m[1][0] * g.m[1][1] * g.m[1][2]);
    w.xb[0] = (double*)take(8 * n1);
    w.xb[1] = (double*)take(8 * n1);
    if (h->scheme.kind != APC_PER_LEVEL) {
      if (g.d >= 2) w.pr[0] = (double*)take(8 * (size_t)lat_count(lattice(g, 0, 0)));
      if (g.d >= 3) w.pr[1] = (double*)take(8 * (size_t)lat_count(lattice(g, 0, 1)));
    }
    w.cdreg = take(qsize(h->dtype) * (size_t)h->cdreg_n);
  }
  if (h->meta.enc) {
    w.pcodes = take(qsize(h->dtype) * (size_t)std::max<int64_t>(1, h->code_n));
    w.pcd_codes = take(qsize(h->dtype) * (size_t)std::max<int64_t>(1, h->cd_n));
  }
  return w;
}

apc_status ensure_codes(apc_handle* h) {
  const size_t qs = qsize(h->dtype);
  if (!h->codes.p) APC_TRY(h->codes.alloc(qs * (size_t)std::max<int64_t>(1, h->code_n)));
  if (!h->cd_codes.p) APC_TRY(h->cd_codes.alloc(qs * (size_t)std::max<int64_t>(1, h->cd_n)));
  return APC_OK;
}

apc_status ensure_work(apc_handle* h) {
  if (h->work_ready) return APC_OK;
  const Geo& g = h->geo;
  const size_t qs = qsize(h->dtype);
  APC_TRY(ensure_codes(h));
  const int L = g.L;
  const int64_t nc = (int64_t)g.m[L - 1][0] * g.m[L - 1][1] * g.m[L - 1][2];
  APC_TRY(h->xc.alloc(8 * (size_t)nc));
  if (L >= 2) {
    const int64_t n1 = (int64_t)g.m[1][0] * g.m[1][1] * g.m[1][2];
    APC_TRY(h->xb[0].alloc(8 * (size_t)n1));
    APC_TRY(h->xb[1].alloc(8 * (size_t)n1));
    if (h->scheme.kind != APC_PER_LEVEL) {  // earlier regions' values (per-region reconstruction)
      if (g.d >= 2) APC_TRY(h->pr[0].alloc(8 * (size_t)std::max<int64_t>(1, lat_count(lattice(g, 0, 0)))));
      if (g.d >= 3) APC_TRY(h->pr[1].alloc(8 * (size_t)std::max<int64_t>(1, lat_count(lattice(g, 0, 1)))));
    }
    if (h->cdreg_n) APC_TRY(h->cdreg.alloc(qs * (size_t)h->cdreg_n));
  }
  if (h->meta.enc) {
    APC_TRY(h->pcodes.alloc(qs * (size_t)std::max<int64_t>(1, h->code_n)));
    APC_TRY(h->pcd_codes.alloc(qs * (size_t)std::max<int64_t>(1, h->cd_n)));
  }
  h->work_ready = true;
  return APC_OK;
}

WorkPtrs handle_work(apc_handle* h) {
  WorkPtrs w;
  w.xc = h->xc.as<double>();
  w.xb[0] = h->xb[0].as<double>();
  w.xb[1] = h->xb[1].as<double>();
  w.pr[0] = h->pr[0].as<double>();
  w.pr[1] = h->pr[1].as<double>();
  w.cdreg = h->cdreg.p;
  w.pcodes = h->pcodes.p;
  w.pcd_codes = h->pcd_codes.p;
  return w;
}

// Tables and launches of one retrieval; kres tracks the planes resident
// after it (incremental decode).  The decode part and the reconstruction
// part can be built separately (a server runs them on different streams).
// `split`: queue the levels coarser than level 0 (their decode, the coarsest
// level and their reconstruction) so that they can run on a helper stream
// beside the level-0 decode and recomposition (per-level fields with a
// decomposition and at least three levels; the launches carry fork and join
// marks, which do nothing when issued on one stream).
template <typename T, typename Q>
void build_retrieve(apc_handle* h, const std::vector<int>& planes, T* out, std::vector<int>& kres,
                    TableBuilder& tb, std::vector<Launch>& ls, int64_t* fetched, const WorkPtrs& w,
                    bool with_decode = true, bool with_recon = true, bool split = false,
                    int64_t lvl_min_blocks = 1024) {
  Meta& m = h->meta;
  const Geo& g = h->geo;
  const int d = g.d, L = g.L;
  const bool per_level = h->scheme.kind == APC_PER_LEVEL;
  const bool nb = m.enc != 0;  // digit planes: decoded words are not codes yet
  const bool split_on = split && with_decode && with_recon && per_level && !h->cd.empty() && L >= 3 && !nb;
  const size_t base = ls.size();
  Q* const codes = w.codes ? (Q*)w.codes : h->codes.as<Q>();
  Q* const cd_codes = w.cd_codes ? (Q*)w.cd_codes : h->cd_codes.as<Q>();
  // what the recomposition and reconstruction read: the decoded codes
  // truncated to the plan by each consumer (generic planes), or the
  // truncated integers this retrieval makes from the digit words
  Q* const rcodes = nb ? (Q*)w.pcodes : codes;
  Q* const rcd_codes = nb ? (Q*)w.pcd_codes : cd_codes;
  auto cB = [&](int s) { return nb ? 64 : m.streams[s].B; };
  auto ck = [&](int s) { return nb ? 64 : planes[s]; };
  std::vector<StreamDev> nbv;  // digit-plane decodes
  int64_t nbch = 0;
  double nbb = 0;
  // decode launches by (level 0 or not) x (first decode adding at most 16
  // planes, which the windowed kernel takes, or any other)
  std::vector<StreamDev> sdv[4];
  int64_t chv[4] = {0, 0, 0, 0}, fb = 0;
  double dbv[4] = {0, 0, 0, 0};
  bool frv[4] = {true, true, true, true};  // every stream of the launch decodes from zero
  for (int s = 0; s < (int)m.streams.size() && with_decode; ++s) {
    const Stream& S = m.streams[s];
    if (S.B == 0 || S.n == 0 || planes[s] <= kres[s]) continue;
    if (S.enc) {
      StreamDev sd{};
      sd.codes = (S.use_cd ? cd_codes : codes) + S.code_off;
      sd.mag = h->mag.as<uint64_t>() + S.mag_off;
      sd.n = S.n;
      sd.M = S.words();
      sd.C = S.chunks();
      sd.chunk_begin = nbch;
      sd.B = S.B;
      sd.k0 = kres[s];
      sd.k1 = planes[s];
      sd.fresh = kres[s] == 0 ? 1 : 0;
      sd.xor_chain = S.enc == 2 ? 1 : 0;
      for (int j = sd.k0; j < sd.k1; ++j) fb += S.plane_bytes(j);
      nbb += (double)(sd.k1 - sd.k0) * 8.0 * sd.M + (double)sizeof(Q) * S.n * (sd.fresh ? 1 : 2);
      nbch += sd.C;
      nbv.push_back(sd);
      kres[s] = planes[s];
      continue;
    }
    const bool fine = split_on && S.level == 0 && S.kind != S_COARSE;
    const bool win = kres[s] == 0 && planes[s] <= 16;
    const int cat = (fine ? 2 : 0) + (win ? 1 : 0);
    StreamDev sd{};
    sd.codes = (S.use_cd ? cd_codes : codes) + S.code_off;
    sd.mag = h->mag.as<uint64_t>() + S.mag_off;
    sd.idx = h->idx.as<uint32_t>() + S.idx_off;
    sd.sign = h->sign.as<uint64_t>() + S.sign_off;
    sd.pso = h->pso.as<int64_t>() + h->psb[s];
    sd.sign_n = S.sign_words();
    sd.n = S.n;
    sd.M = S.words();
    sd.C = S.chunks();
    sd.chunk_begin = chv[cat];
    sd.B = S.B;
    sd.k0 = kres[s];
    sd.k1 = planes[s];
    sd.fresh = kres[s] == 0 ? 1 : 0;
    double b = 0.0;
    for (int j = sd.k0; j < sd.k1; ++j) {
      fb += S.plane_bytes(j);
      b += 8.0 * ((S.nsig[j] + 63) / 64);
    }
    b += (double)(sd.k1 - sd.k0) * (8.0 * sd.M + 4.0 * sd.C) + (double)sizeof(Q) * S.n * (sd.fresh ? 1 : 2);
    chv[cat] += sd.C;
    dbv[cat] += b;
    sdv[cat].push_back(sd);
    frv[cat] = frv[cat] && sd.fresh != 0;
    kres[s] = planes[s];
  }
  if (fetched) *fetched = fb;
  // `a`: bit 0 marks a level-0 decode (for the reordering below), bit 1 a
  // launch of first decodes only, bit 2 one whose streams add at most 16 planes
  for (int cat = 0; cat < 4; ++cat)
    if (!sdv[cat].empty())
      ls.push_back({K_DECODE, tb.add(sdv[cat]), (int)sdv[cat].size(), chv[cat],
                    ((cat & 2) ? 1 : 0) | (frv[cat] ? 2 : 0) | ((cat & 1) ? 4 : 0), dbv[cat], "decode"});
  if (!nbv.empty()) ls.push_back({K_DECODE_NB, tb.add(nbv), (int)nbv.size(), nbch, 0, nbb, "decode"});
  if (!with_recon) return;
  if (nb) {  // the plan's truncated integers of every stream
    std::vector<FlatSeg> vs;
    double by = 0;
    for (int s = 0; s < (int)m.streams.size(); ++s) {
      const Stream& S = m.streams[s];
      if (S.n == 0) continue;
      FlatSeg v{};
      v.src = (S.use_cd ? cd_codes : codes) + S.code_off;
      v.dst = (S.use_cd ? rcd_codes : rcodes) + S.code_off;
      v.n = S.n;
      v.B = S.B;
      v.k = planes[s];
      by += 2.0 * sizeof(Q) * S.n;
      vs.push_back(v);
    }
    const int64_t nbk = assign_blocks<FlatSeg>(vs, [](const FlatSeg& v) { return v.n; });
    if (!vs.empty()) {
      ls.push_back({K_NB_VALUES, tb.add(vs), (int)vs.size(), nbk, 0, by, "nb_values"});
      ls.back().stage = 1;
    }
  }
  // inverse decomposition of every level-0 region
  if (!h->cd.empty() && L >= 2) {
    std::vector<CDSeg> cs;
    double by = 0;
    for (int rho = 0; rho < (int)h->cd.size(); ++rho) {
      const CDInfo& ci = h->cd[rho];
      CDSeg c{};
      for (int a = 0; a < 3; ++a) c.c[a] = ci.c[a];
      c.f2 = make_fastdiv((uint32_t)std::max(1, c.c[2]));
      c.f1 = make_fastdiv((uint32_t)std::max(1, c.c[1]));
      c.Rout = (Q*)w.cdreg + ci.reg_off;
      for (int t = 0; t < 3; ++t) {
        c.S[t] = rcd_codes + ci.s_off[t];
        c.B[t] = cB(ci.s_idx[t]);
        c.k[t] = ck(ci.s_idx[t]);
      }
      const int64_t cnt = (int64_t)c.c[0] * c.c[1] * c.c[2];
      if (cnt == 0) continue;
      by += 2.0 * sizeof(Q) * cnt;
      cs.push_back(c);
    }
    if (!cs.empty()) {
      const int a3 = h->cd[0].a;
      if (a3 < 2) {  // v runs along lattice rows: one pass over row tiles
        const int64_t nbk = assign_cd_tile_blocks(cs, a3);
        ls.push_back({K_CDIT, tb.add(cs), (int)cs.size(), nbk, a3, by, "cd_inverse"});
        ls.back().stage = 2;
      } else {
        const int64_t nbk = assign_cd_blocks(cs);
        const size_t off = tb.add(cs);
        ls.push_back({K_CDI0, off, (int)cs.size(), nbk, a3, by * 0.5, "cd_inverse"});
        ls.back().stage = 2;
        ls.push_back({K_CDI1, off, (int)cs.size(), nbk, a3, by * 0.5, "cd_inverse"});
        ls.back().stage = 3;
      }
    }
  }
  // coarsest level
  {
    const Stream& s0 = m.streams[0];
    FlatSeg c{};
    c.src = rcodes;
    c.dst = L == 1 ? (void*)out : (void*)w.xc;
    c.n = s0.n;
    c.B = cB(0);
    c.k = ck(0);
    c.delta = m.groups[s0.group].delta;
    c.final_out = L == 1 ? 1 : 0;
    std::vector<FlatSeg> cs{c};
    const int64_t nbk = assign_blocks<FlatSeg>(cs, [](const FlatSeg& s) { return s.n; });
    ls.push_back({K_COARSEST, tb.add(cs), 1, nbk, 0, (8.0 + sizeof(Q)) * s0.n, "coarsest"});
    ls.back().stage = 4;
  }
  const double* xin = w.xc;
  for (int l = L - 2; l >= 0; --l) {
    double* xout = l > 0 ? w.xb[l % 2] : nullptr;
    void* dst = l > 0 ? (void*)xout : (void*)out;
    if (per_level) {  // one tensor-product pass writes the whole level grid
      LevelSeg c = level_seg(h, l);
      c.src = xin;
      c.out = dst;
      c.final_out = l == 0 ? 1 : 0;
      c.delta = m.groups[group_of(m, l, 0)].delta;
      const bool cd0 = l == 0 && !h->cd.empty();
      const int s = cd0 ? -1 : stream_of(m, l, 0);
      for (int rho = 0; rho < d; ++rho) {
        if (cd0) {
          c.q[rho] = (Q*)w.cdreg + h->cd[rho].reg_off;
          c.B[rho] = 64;
          c.k[rho] = 64;
        } else {
          c.q[rho] = rcodes + h->region_off[l * 3 + rho];
          c.B[rho] = cB(s);
          c.k[rho] = ck(s);
        }
      }
      const int t2 = shape_level_seg(c, tile_for(h->dtype, g.m[l][1], g.m[l][2]), lvl_min_blocks);
      std::vector<LevelSeg> cs{c};
      const int64_t nbk = assign_level_blocks(cs);
      // codes of the level's fine points and the coarser grid read, every
      // point of the level written
      const int64_t n = (int64_t)c.m[0] * c.m[1] * c.m[2], nc = (int64_t)c.mc[0] * c.mc[1] * c.mc[2];
      const double by = (double)(n - nc) * sizeof(Q) + (double)n * (l ? 8 : sizeof(T)) + 8.0 * nc;
      // level 0 writes the output field: its own kernel and profile name
      ls.push_back({l == 0 ? K_LEVEL3 : K_LEVEL2, tb.add(cs), 1, nbk, t2, by, l == 0 ? "recon" : "recon_coarse"});
      ls.back().stage = level_stage(l, 0);
      xin = xout;
      continue;
    }
    {
      FlatSeg c{};
      c.src = xin;
      c.dst = dst;
      for (int a = 0; a < 3; ++a) c.dm[a] = g.m[l + 1][a];
      c.n = (int64_t)c.dm[0] * c.dm[1] * c.dm[2];
      c.f2 = make_fastdiv((uint32_t)c.dm[2]);
      c.f1 = make_fastdiv((uint32_t)c.dm[1]);
      c.dst_m1 = g.m[l][1];
      c.dst_m2 = g.m[l][2];
      c.final_out = l == 0 ? 1 : 0;
      std::vector<FlatSeg> cs{c};
      const int64_t nbk = assign_blocks<FlatSeg>(cs, [](const FlatSeg& s) { return s.n; });
      ls.push_back({K_INJECT, tb.add(cs), 1, nbk, 0, (8.0 + (l ? 8 : sizeof(T))) * c.n, "inject"});
      ls.back().stage = level_stage(l, 0);
    }
    for (int rho = 0; rho < d; ++rho) {
      ReconSeg r{};
      double* pr[2] = {w.pr[0], w.pr[1]};
      r.ra = region_args(h, l, rho, per_level, pr, true, true);
      const int64_t cnt = lat_count(r.ra.lat);
      if (cnt == 0) continue;
      r.xc = xin;
      r.cm1 = g.m[l + 1][1];
      r.cm2 = g.m[l + 1][2];
      if (l == 0 && !h->cd.empty()) {
        const CDInfo& ci = h->cd[rho];
        r.q = (const Q*)w.cdreg + ci.reg_off;
        r.B = 64;
        r.k = 64;
        r.delta = m.groups[m.streams[ci.s_idx[0]].group].delta;
      } else {
        const int s = stream_of(m, l, rho);
        const Stream& S = m.streams[s];
        r.q = rcodes + h->region_off[l * 3 + rho];
        r.B = cB(s);
        r.k = ck(s);
        r.delta = m.groups[S.group].delta;
      }
      r.out = dst;
      r.final_out = l == 0 ? 1 : 0;
      std::vector<ReconSeg> cs{r};
      const int64_t nbk = assign_blocks<ReconSeg>(cs, [](const ReconSeg& s) { return lat_count(s.ra.lat); });
      const double by = (double)cnt * (sizeof(Q) + (l ? 8 : sizeof(T)) + (r.ra.pr_out ? 8 : 0));
      ls.push_back({K_RECON, tb.add(cs), 1, nbk, 0, by, "recon"});
      ls.back().stage = level_stage(l, 1 + rho);
    }
    xin = xout;
  }
  if (split_on) {
    // queued as: fork | level-0 decode, recomposition | coarse decode,
    // coarsest, levels L-2..2 (helper) | join mark | join wait | level 1,
    // level 0.  The critical path is queued first, so the device starts on
    // it while the host is still queueing the helper's many small launches;
    // level 1, the largest of the coarse levels, runs on the main stream,
    // where it has the device to itself instead of sharing it with the
    // recomposition.
    std::vector<Launch> dec_c, dec_f, cdi, chain, lev0;
    for (size_t i = base; i < ls.size(); ++i) {
      Launch x = ls[i];
      if (x.kind == K_DECODE)
        ((x.a & 1) ? dec_f : dec_c).push_back(x);
      else if (x.kind == K_CDIT || x.kind == K_CDI0 || x.kind == K_CDI1)
        cdi.push_back(x);
      else if (x.kind == K_LEVEL3)
        lev0.push_back(x);
      else {
        x.side = 1;
        chain.push_back(x);
      }
    }
    std::vector<Launch> lev1;
    if (!chain.empty() && chain.back().kind == K_LEVEL2) {  // levels run coarse to fine: the last is level 1
      lev1.push_back(chain.back());
      lev1.back().side = 0;
      chain.pop_back();
    }
    ls.resize(base);
    auto mark = [&](int kind) { ls.push_back({kind, 0, 0, 0, 0, 0.0, "mark"}); };
    mark(K_FORK);
    for (const Launch& x : dec_f) ls.push_back(x);
    for (const Launch& x : cdi) ls.push_back(x);
    for (Launch x : dec_c) {
      x.side = 1;
      ls.push_back(x);
    }
    for (const Launch& x : chain) ls.push_back(x);
    mark(K_JOIN_REC);
    mark(K_JOIN_WAIT);
    for (const Launch& x : lev1) ls.push_back(x);
    for (const Launch& x : lev0) ls.push_back(x);
  }
}

// Segment size of each retrieval launch kind, and the shift of a segment's
// first work block (first chunk for decodes).
size_t seg_size_of(int kind) {
  switch (kind) {
    case K_DECODE:
    case K_DECODE_NB: return sizeof(StreamDev);
    case K_NB_VALUES: return sizeof(FlatSeg);
    case K_CDIT:
    case K_CDI0:
    case K_CDI1: return sizeof(CDSeg);
    case K_COARSEST:
    case K_INJECT: return sizeof(FlatSeg);
    case K_RECON: return sizeof(ReconSeg);
    case K_LEVEL2:
    case K_LEVEL3: return sizeof(LevelSeg);
    default: return 0;
  }
}
void rebase_seg(int kind, char* seg, int64_t add) {
  switch (kind) {
    case K_DECODE:
    case K_DECODE_NB: ((StreamDev*)seg)->chunk_begin += add; break;
    case K_NB_VALUES: ((FlatSeg*)seg)->blk_begin += add; break;
    case K_CDIT:
    case K_CDI0:
    case K_CDI1: ((CDSeg*)seg)->blk_begin += add; break;
    case K_COARSEST:
    case K_INJECT: ((FlatSeg*)seg)->blk_begin += add; break;
    case K_RECON: ((ReconSeg*)seg)->blk_begin += add; break;
    case K_LEVEL2:
    case K_LEVEL3: ((LevelSeg*)seg)->blk_begin += add; break;
    default: break;
  }
}

// The launches of several retrievals (each list with its own table) merged:
// launches with equal (stage, kind, argument) become one launch over the
// concatenated segments, work blocks (chunks for decodes) numbered on from
// the previous list's, in stage order.  Launches of one stage never depend
// on each other, and every retrieval's own order is kept.
struct LaunchPart {
  const TableBuilder* tb;
  const std::vector<Launch>* ls;
};
void merge_launches(const std::vector<LaunchPart>& parts, TableBuilder& tb, std::vector<Launch>& out) {
  struct Acc {
    Launch l{};
    std::vector<char> segs;
  };
  std::map<std::tuple<int, int, int>, Acc> acc;
  for (const LaunchPart& p : parts)
    for (const Launch& l : *p.ls) {
      const size_t sz = seg_size_of(l.kind);
      auto key = std::make_tuple(l.stage, l.kind, l.a);
      auto it = acc.find(key);
      if (it == acc.end()) {
        Acc a;
        a.l = l;
        a.l.nseg = 0;
        a.l.nblk = 0;
        a.l.bytes = 0.0;
        it = acc.emplace(key, std::move(a)).first;
      }
      Acc& a = it->second;
      const size_t at = a.segs.size();
      a.segs.resize(at + sz * (size_t)l.nseg);
      memcpy(a.segs.data() + at, p.tb->bytes.data() + l.off, sz * (size_t)l.nseg);
      for (int i = 0; i < l.nseg; ++i) rebase_seg(l.kind, a.segs.data() + at + sz * (size_t)i, a.l.nblk);
      a.l.nseg += l.nseg;
      a.l.nblk += l.nblk;
      a.l.bytes += l.bytes;
    }
  for (auto& kv : acc) {
    Launch l = kv.second.l;
    l.off = tb.add_raw(kv.second.segs.data(), kv.second.segs.size());
    out.push_back(l);
  }
}

// Plane bytes of planes [kcur[s], planes[s]) of every stream; kcur advances.
int64_t fetch_bytes(const Meta& m, std::vector<int>& kcur, const std::vector<int>& planes) {
  int64_t b = 0;
  for (size_t s = 0; s < planes.size(); ++s) {
    for (int j = kcur[s]; j < planes[s]; ++j) b += m.streams[s].plane_bytes(j);
    kcur[s] = std::max(kcur[s], planes[s]);
  }
  return b;
}

apc_status upload_tables(apc_handle* h, const std::vector<char>& bytes, hipStream_t st) {
  if (bytes.empty()) return APC_OK;
  if (h->pinned.cap < bytes.size()) {
    g_pinned.put(h->pinned, nullptr, false);  // its event already follows its last upload
    if (!g_pinned.get(bytes.size() * 2, h->pinned)) return fail(APC_E_OOM, "pinned staging of %zu bytes", bytes.size());
  } else {
    HIP_TRY(hipEventSynchronize(h->pinned.ev));  // the previous copy has left the staging
  }
  memcpy(h->pinned.p, bytes.data(), bytes.size());
  if (h->tables.bytes < bytes.size() && h->tab_ev) {
    // a larger table: the previous retrieval (on any stream) may still read
    // the old one, which goes back to the shared pool only after it
    HIP_TRY(hipEventSynchronize(h->tab_ev));
  }
  APC_TRY(h->tables.alloc(bytes.size()));
  HIP_TRY(hipMemcpyAsync(h->tables.p, h->pinned.p, bytes.size(), hipMemcpyHostToDevice, st));
  HIP_TRY(hipEventRecord(h->pinned.ev, st));
  return APC_OK;
}

// Helper streams (with a fork and a join event) for two-stream retrievals,
// checked out per call and returned as soon as the work is queued: later
// users queue behind it, and the events are read when a wait is queued, so
// re-recording them afterwards is safe.  Created on first use on a device
// (default priority, non-blocking) and kept until the process ends.
struct AuxStream {
  int dev = -1;
  hipStream_t s = nullptr;
  hipEvent_t fork = nullptr, join = nullptr;
};
struct AuxPool {
  std::mutex mu;
  std::vector<AuxStream> free_;
  bool get(AuxStream& out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return false;
    {
      std::lock_guard<std::mutex> lk(mu);
      for (size_t i = 0; i < free_.size(); ++i)
        if (free_[i].dev == dev) {
          out = free_[i];
          free_.erase(free_.begin() + (long)i);
          return true;
        }
    }
    out = AuxStream();
    out.dev = dev;
    if (hipStreamCreateWithFlags(&out.s, hipStreamNonBlocking) != hipSuccess) return false;
    if (hipEventCreateWithFlags(&out.fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&out.join, hipEventDisableTiming) != hipSuccess) {
      (void)hipGetLastError();
      return false;  // the stream is kept (never destroyed)
    }
    return true;
  }
  void put(const AuxStream& a) {
    std::lock_guard<std::mutex> lk(mu);
    free_.push_back(a);
  }
};
AuxPool g_aux;

template <typename T, typename Q>
apc_status retrieve_impl(apc_handle* h, const std::vector<int>& planes, T* out, hipStream_t st, int64_t* fetched) {
  if (h->ready) HIP_TRY(hipStreamWaitEvent(st, h->ready, 0));  // the refactor's last kernels
  APC_TRY(ensure_work(h));
  TableBuilder tb;
  std::vector<Launch> ls;
  std::vector<int> kres = h->k_res;
  build_retrieve<T, Q>(h, planes, out, kres, tb, ls, fetched, handle_work(h), true, true, true);
  APC_TRY(upload_tables(h, tb.bytes, st));
  // two streams, except while every launch is timed (the per-kernel
  // breakdown is taken on one stream so that no kernel's time includes
  // another's running beside it)
  bool split = !(g_prof.on && !g_prof.filtered);
  bool marks = false;
  for (const Launch& l : ls) marks = marks || l.kind == K_FORK;
  split = split && marks;
  AuxStream aux;
  if (split && g_aux.get(aux)) {
    const apc_status r = issue<T, Q>(ls, (const char*)h->tables.p, st, aux.s, aux.fork, aux.join);
    g_aux.put(aux);
    APC_TRY(r);
  } else {
    APC_TRY((issue<T, Q>(ls, (const char*)h->tables.p, st)));
  }
  if (!h->tab_ev) HIP_TRY(hipEventCreateWithFlags(&h->tab_ev, hipEventDisableTiming));
  HIP_TRY(hipEventRecord(h->tab_ev, st));  // the helper stream, if any, has joined st
  h->k_res = kres;
  return APC_OK;
}

apc_status target_tau(const apc_handle* h, const apc_target* t, double& tau, int& mode) {
  const double rng = h->meta.range();
  switch (t->kind) {
    case APC_EB_ABS:
      tau = t->value;
      mode = 0;
      return APC_OK;
    case APC_EB_REL:
      tau = t->value * rng;
      mode = 0;
      return APC_OK;
    case APC_RMSE_ABS:
      tau = t->value;
      mode = 1;
      return APC_OK;
    case APC_PSNR:
      tau = rng * pow(10.0, -t->value / 20.0);
      mode = 1;
      return APC_OK;
    default:
      return fail(APC_E_INVALID, "unknown target kind %d", t->kind);
  }
}

// The plan for a target with the handle's interpreter.  resident: planes
// already fetched (free for the dynamic program and best-first search;
// ignored by the greedy, whose plans are nested anyway), or null.
apc_status plan_for(apc_handle* h, const apc_target* target, std::vector<int>& planes, apc_retrieve_info* info,
                    const std::vector<int>* resident) {
  double tau;
  int mode;
  APC_TRY(target_tau(h, target, tau, mode));
  double b;
  int nsteps;
  if (make_plan_with(h->meta, h->interp, h->scheme.kind == APC_PER_REGION, tau, mode, resident, planes, b, nsteps) != 0)
    return fail(APC_E_BELOW_FLOOR, "tolerance %.17g is below the floor of this representation", tau);
  if (info) {
    info->bytes_total = plan_bytes(h->meta, planes);
    info->bytes_fetched = 0;
    info->bound = b;
    info->tau = tau;
    info->bitrate = 8.0 * (double)info->bytes_total / (double)h->meta.n;
    info->n_streams = (int32_t)planes.size();
    info->nsteps = nsteps;
  }
  return APC_OK;
}

apc_status need_device(const apc_handle* h) {
  if (h->host_only) return fail(APC_E_INVALID, "handle holds no device data (rebuilt for planning only)");
  return APC_OK;
}

// Many retrievals in shared launches (Algorithm 2 for each request): every
// handle decodes once, up to the largest plan among its requests, and the
// recomposition and reconstruction of every request run merged, each reading
// the resident codes truncated to its own plan into its own work buffers
// (the handle's for its first request, temporaries for further ones).
template <typename T, typename Q>
apc_status retrieve_batch_impl(apc_handle* const* hs, int32_t n, const apc_target* targets, void* const* outs,
                               apc_retrieve_info* infos, hipStream_t st) {
  DrainScope drain(st);
  std::vector<std::vector<int>> planes((size_t)n);
  std::vector<apc_retrieve_info> inf((size_t)n);
  std::vector<apc_handle*> uniq;
  std::map<apc_handle*, size_t> idx;
  for (int32_t i = 0; i < n; ++i) {
    apc_handle* h = hs[i];
    APC_TRY(plan_for(h, &targets[i], planes[i], &inf[i], &h->k_res));
    if (!idx.count(h)) {
      idx[h] = uniq.size();
      uniq.push_back(h);
    }
  }
  for (apc_handle* h : uniq) {
    if (h->ready) HIP_TRY(hipStreamWaitEvent(st, h->ready, 0));  // the refactor's last kernels
    APC_TRY(ensure_work(h));
  }
  // decodes: each request is credited with the planes it adds, in order
  std::vector<std::vector<int>> want(uniq.size()), kres(uniq.size());
  for (size_t u = 0; u < uniq.size(); ++u) want[u] = kres[u] = uniq[u]->k_res;
  for (int32_t i = 0; i < n; ++i) inf[i].bytes_fetched = fetch_bytes(hs[i]->meta, want[idx[hs[i]]], planes[i]);
  std::vector<TableBuilder> tbs(uniq.size() + (size_t)n);
  std::vector<std::vector<Launch>> lss(uniq.size() + (size_t)n);
  std::vector<LaunchPart> parts;
  for (size_t u = 0; u < uniq.size(); ++u) {
    build_retrieve<T, Q>(uniq[u], want[u], nullptr, kres[u], tbs[u], lss[u], nullptr, WorkPtrs(), true, false);
    if (!lss[u].empty()) parts.push_back({&tbs[u], &lss[u]});
  }
  std::vector<DevBuf> tmp;
  tmp.reserve((size_t)n);
  std::vector<bool> own_used(uniq.size(), false);
  for (int32_t i = 0; i < n; ++i) {
    apc_handle* h = hs[i];
    const size_t u = idx[h];
    WorkPtrs w;
    if (!own_used[u]) {
      w = handle_work(h);
      own_used[u] = true;
    } else {
      tmp.emplace_back();
      APC_TRY(tmp.back().alloc(work_bytes(h)));
      w = carve_work(h, tmp.back().p);
    }
    std::vector<int> kdone = kres[u];  // decoded above
    const size_t j = uniq.size() + (size_t)i;
    // the requests share each launch: longer level runs, as in a batched refactor
    build_retrieve<T, Q>(h, planes[i], (T*)outs[i], kdone, tbs[j], lss[j], nullptr, w, false, true, false,
                         std::max<int64_t>(64, 1024 / std::max(1, n)));
    parts.push_back({&tbs[j], &lss[j]});
  }
  TableBuilder tb;
  std::vector<Launch> ls;
  merge_launches(parts, tb, ls);
  // the merged table travels in the first handle's table buffer, as a
  // retrieval of that handle's own would
  apc_handle* h0 = uniq[0];
  APC_TRY(upload_tables(h0, tb.bytes, st));
  APC_TRY((issue<T, Q>(ls, (const char*)h0->tables.p, st)));
  if (!h0->tab_ev) HIP_TRY(hipEventCreateWithFlags(&h0->tab_ev, hipEventDisableTiming));
  HIP_TRY(hipEventRecord(h0->tab_ev, st));
  for (size_t u = 0; u < uniq.size(); ++u) uniq[u]->k_res = kres[u];
  if (infos)
    for (int32_t i = 0; i < n; ++i) infos[i] = inf[i];
  // the temporary work buffers stay allocated until the queued work has finished
  APC_TRY(retire(std::move(tmp), st));
  drain.armed = false;
  return APC_OK;
}

apc_status do_retrieve(apc_handle* h, const std::vector<int>& planes, void* out_dev, void* hip_stream,
                       int64_t* fetched) {
  hipStream_t st = (hipStream_t)hip_stream;
  if (h->dtype == APC_F32) return retrieve_impl<float, int32_t>(h, planes, (float*)out_dev, st, fetched);
  return retrieve_impl<double, int64_t>(h, planes, (double*)out_dev, st, fetched);
}

apc_status make_handles(int nf, const int32_t dtype, const int64_t* dims, const int32_t* ndims,
                        const apc_scheme* schemes, std::vector<std::unique_ptr<apc_handle>>& own) {
  own.clear();
  int64_t doff = 0;
  for (int f = 0; f < nf; ++f) {
    std::unique_ptr<apc_handle> h(new apc_handle());
    h->dtype = dtype;
    APC_TRY(setup_geometry(h.get(), dims + doff, ndims[f], &schemes[f]));
    doff += ndims[f];
    own.push_back(std::move(h));
  }
  return APC_OK;
}

apc_status refactor_many(const void* const* fields, int32_t dtype, const int64_t* dims, const int32_t* ndims,
                         const apc_scheme* schemes, int32_t nf, hipStream_t st,
                         std::vector<std::unique_ptr<apc_handle>>& own) {
  if (dtype != APC_F32 && dtype != APC_F64) return fail(APC_E_DTYPE, "dtype must be APC_F32 or APC_F64");
  // target-driven selection first for the fields that ask for it
  std::vector<apc_scheme> sc(schemes, schemes + nf);
  int64_t doff = 0;
  for (int f = 0; f < nf; ++f) {
    if (sc[f].kind == APC_AUTO || sc[f].kind == APC_AUTO_PSNR) {
      apc_scheme chosen{};
      APC_TRY(apc_select_pipeline(fields[f], dtype, dims + doff, ndims[f],
                                  sc[f].kind == APC_AUTO ? APC_MODE_EB : APC_MODE_PSNR, &chosen, st));
      chosen.levels = sc[f].levels;
      chosen.lossless = sc[f].lossless;
      chosen.encoding = sc[f].encoding;
      sc[f] = chosen;
    }
    doff += ndims[f];
  }
  APC_TRY(make_handles(nf, dtype, dims, ndims, sc.data(), own));
  std::vector<apc_handle*> hs;
  for (auto& h : own) hs.push_back(h.get());
  if (dtype == APC_F32) {
    std::vector<const float*> xs;
    for (int f = 0; f < nf; ++f) xs.push_back((const float*)fields[f]);
    return refactor_batch<float, int32_t>(hs, xs, st);
  }
  std::vector<const double*> xs;
  for (int f = 0; f < nf; ++f) xs.push_back((const double*)fields[f]);
  return refactor_batch<double, int64_t>(hs, xs, st);
}

// ------------------------------------------------ retrieval without allocation
// Every device buffer of apc_retrieve_static (decoded codes, the float64
// coarse grids, the recomposition buffer, the launch tables) is carved from
// this array, which each device holds from module load until the process
// ends.  Host code never passes the array's name to the device: its address
// on the current device is looked up once per device (static_scratch) and
// kept.
constexpr size_t kStaticScratchBytes = (size_t)256 << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
std::mutex g_scratch_mu;
char* g_scratch_ptr[kMaxDevices] = {};

apc_status static_scratch(char** base) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(APC_E_INVALID, "device %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(APC_E_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
    g_scratch_ptr[dev] = (char*)p;
  }
  *base = g_scratch_ptr[dev];
  return APC_OK;
}

// One retrieval from no resident planes with every buffer in the static
// scratch: [region codes | decomposition codes | work grids | tables].
template <typename T, typename Q>
apc_status retrieve_static_impl(apc_handle* h, const std::vector<int>& planes, T* out, hipStream_t st,
                                int64_t* fetched) {
  char* base = nullptr;
  APC_TRY(static_scratch(&base));
  auto up = [](size_t n) { return (n + 255) & ~(size_t)255; };
  size_t off = 0;
  const size_t o_codes = off;
  off += up(sizeof(Q) * (size_t)std::max<int64_t>(1, h->code_n));
  const size_t o_cd = off;
  off += up(sizeof(Q) * (size_t)std::max<int64_t>(1, h->cd_n));
  const size_t o_work = off;
  off += up(work_bytes(h));
  if (off > kStaticScratchBytes)
    return fail(APC_E_INVALID, "field needs %zu bytes of retrieval buffers; the static scratch holds %zu", off,
                kStaticScratchBytes);
  WorkPtrs w = carve_work(h, base + o_work);
  w.codes = base + o_codes;
  w.cd_codes = base + o_cd;
  TableBuilder tb;
  std::vector<Launch> ls;
  std::vector<int> kres(h->meta.streams.size(), 0);  // every plane of the plan is decoded from zero
  build_retrieve<T, Q>(h, planes, out, kres, tb, ls, fetched, w, true, true, false);
  const size_t o_tab = off;
  off += up(tb.bytes.size());
  if (off > kStaticScratchBytes)
    return fail(APC_E_INVALID, "field needs %zu bytes of retrieval buffers; the static scratch holds %zu", off,
                kStaticScratchBytes);
  if (h->ready) HIP_TRY(hipStreamWaitEvent(st, h->ready, 0));  // the refactor's last kernels
  // from pageable memory: the runtime has consumed the source when the call returns
  if (!tb.bytes.empty())
    HIP_TRY(hipMemcpyAsync(base + o_tab, tb.bytes.data(), tb.bytes.size(), hipMemcpyHostToDevice, st));
  APC_TRY((issue<T, Q>(ls, base + o_tab, st)));
  return APC_OK;
}

}  // namespace

// ------------------------------------------------------------ serialization
// The stored representation as one byte string (all integers little endian):
//   [0, 8)    magic "APCREP01"
//   [8, 16)   total length in bytes
//   [16, 24)  length of the metadata section
//   [24, 32)  checksum of the metadata section
//   metadata  dtype, ndim (int32); dims[3] (int64, unused ones 0); scheme:
//             kind, degree, order[3] (the pass order; unused entries 0),
//             cd_axis, levels (= L) (int32); L, P, 0 (int32); xmin, xmax, A
//             (float64); group and stream counts (uint32); M per group
//             (float64); per stream: n, max |code| (int64), B, 0 (int32),
//             new-significant counts of its B planes (int64)
//   streams   per stream in stream order: blob length, blob checksum
//             (uint64), then the blob in the layout of apc_stream_blob
// Every section is a multiple of 8 bytes long.
namespace {

constexpr char kRepMagic[8] = {'A', 'P', 'C', 'R', 'E', 'P', '0', '1'};

// 64-bit checksum of a byte range: the length, then every little-endian
// 64-bit word (the last one zero padded), each folded in by xor, a multiply
// by an odd constant and an xor-shift.  It catches truncation and stray
// changes; it is not a cryptographic hash.
uint64_t rep_hash(const unsigned char* p, size_t n) {
  uint64_t h = 0x6a09e667f3bcc909ull ^ (uint64_t)n;
  auto mix = [&](uint64_t w) {
    h ^= w;
    h *= 0x9e3779b97f4a7c15ull;
    h ^= h >> 32;
  };
  size_t i = 0;
  for (; i + 8 <= n; i += 8) {
    uint64_t w;
    memcpy(&w, p + i, 8);
    mix(w);
  }
  if (i < n) {
    uint64_t w = 0;
    memcpy(&w, p + i, n - i);
    mix(w);
  }
  return h;
}

template <typename V>
void put(std::vector<unsigned char>& b, V v) {
  const size_t at = b.size();
  b.resize(at + sizeof(V));
  memcpy(b.data() + at, &v, sizeof(V));
}

void rep_meta(const apc_handle* h, std::vector<unsigned char>& b) {
  const Geo& g = h->geo;
  const Meta& m = h->meta;
  put<int32_t>(b, h->dtype);
  put<int32_t>(b, g.d);
  for (int a = 0; a < 3; ++a) put<int64_t>(b, a < g.d ? g.N[3 - g.d + a] : 0);
  put<int32_t>(b, h->scheme.kind);
  put<int32_t>(b, h->scheme.degree);
  for (int j = 0; j < 3; ++j) put<int32_t>(b, j < g.d ? g.sigma_user[j] : 0);
  put<int32_t>(b, h->scheme.cd_axis);
  put<int32_t>(b, g.L);
  put<int32_t>(b, g.L);
  put<int32_t>(b, m.P);
  put<int32_t>(b, m.lossless ? 1 : 0);
  put<int32_t>(b, m.enc);
  put<int32_t>(b, 0);
  put<double>(b, m.xmin);
  put<double>(b, m.xmax);
  put<double>(b, m.A);
  put<uint32_t>(b, (uint32_t)m.groups.size());
  put<uint32_t>(b, (uint32_t)m.streams.size());
  for (const Group& gr : m.groups) put<double>(b, gr.M);
  for (const Stream& S : m.streams) {
    put<int64_t>(b, S.n);
    put<int64_t>(b, S.maxabs);
    put<int32_t>(b, S.B);
    put<int32_t>(b, 0);
    for (int j = 0; j < S.B; ++j) put<int64_t>(b, S.nsig[j]);
    if (m.lossless)
      for (int j = 0; j < S.B; ++j) put<int64_t>(b, S.nnz[j]);
  }
}

struct RepReader {
  const unsigned char* p;
  size_t n, at = 0;
  bool ok = true;
  template <typename V>
  V get() {
    V v{};
    if (!ok || n - at < sizeof(V)) {
      ok = false;
      return v;
    }
    memcpy(&v, p + at, sizeof(V));
    at += sizeof(V);
    return v;
  }
};

#define REP_CHECK(cond, ...)                         \
  do {                                               \
    if (!(cond)) return fail(APC_E_CORRUPT, __VA_ARGS__); \
  } while (0)

// Check a serialized representation and rebuild the host side of its handle
// (geometry, layout, metadata, the interpreter's sequence); blobs[s] points
// at stream s's blob inside src.  No device work.
apc_status rep_parse(const unsigned char* src, int64_t len, std::unique_ptr<apc_handle>& out,
                     std::vector<const unsigned char*>& blobs, bool verify_streams = true) {
  REP_CHECK(len >= 32, "%lld bytes: shorter than the header", (long long)len);
  REP_CHECK(memcmp(src, kRepMagic, 8) == 0, "bad magic");
  uint64_t tl, ml, mh;
  memcpy(&tl, src + 8, 8);
  memcpy(&ml, src + 16, 8);
  memcpy(&mh, src + 24, 8);
  REP_CHECK(tl == (uint64_t)len, "length field %llu, %lld bytes given (truncated or padded)",
            (unsigned long long)tl, (long long)len);
  REP_CHECK(ml <= (uint64_t)len - 32 && ml % 8 == 0, "metadata length %llu out of range", (unsigned long long)ml);
  REP_CHECK(rep_hash(src + 32, (size_t)ml) == mh, "metadata checksum mismatch");
  RepReader r{src + 32, (size_t)ml};
  const int32_t dtype = r.get<int32_t>(), ndim = r.get<int32_t>();
  int64_t dims[3];
  for (int a = 0; a < 3; ++a) dims[a] = r.get<int64_t>();
  apc_scheme sc{};
  sc.kind = r.get<int32_t>();
  sc.degree = r.get<int32_t>();
  for (int j = 0; j < 3; ++j) sc.order[j] = r.get<int32_t>();
  sc.cd_axis = r.get<int32_t>();
  sc.levels = r.get<int32_t>();
  const int32_t L = r.get<int32_t>(), P = r.get<int32_t>();
  sc.lossless = r.get<int32_t>();
  sc.encoding = r.get<int32_t>();
  (void)r.get<int32_t>();
  const double xmin = r.get<double>(), xmax = r.get<double>(), A = r.get<double>();
  const uint32_t ng = r.get<uint32_t>(), ns = r.get<uint32_t>();
  REP_CHECK(r.ok, "metadata truncated");
  REP_CHECK(dtype == APC_F32 || dtype == APC_F64, "dtype %d", dtype);
  REP_CHECK(P == (dtype == APC_F32 ? 29 : 52), "precision %d does not match the dtype", P);
  std::unique_ptr<apc_handle> h(new apc_handle());
  h->dtype = dtype;
  if (setup_geometry(h.get(), dims, ndim, &sc) != APC_OK)
    return fail(APC_E_CORRUPT, "geometry or scheme: %s", g_last_error.c_str());
  REP_CHECK(h->geo.L == L, "level count %d, the geometry gives %d", L, h->geo.L);
  build_layout(h.get(), P);
  Meta& m = h->meta;
  REP_CHECK(ng == m.groups.size() && ns == m.streams.size(), "%u groups / %u streams, the layout has %zu / %zu", ng,
            ns, m.groups.size(), m.streams.size());
  REP_CHECK(std::isfinite(xmin) && std::isfinite(xmax) && xmin <= xmax && A == std::max(fabs(xmin), fabs(xmax)),
            "range fields inconsistent");
  m.xmin = xmin;
  m.xmax = xmax;
  m.A = A;
  for (Group& gr : m.groups) {
    gr.M = r.get<double>();
    REP_CHECK(r.ok && std::isfinite(gr.M) && gr.M >= 0.0, "group maximum out of range");
    if (gr.M > 0.0) {
      int E;
      frexp(gr.M, &E);
      gr.E = E;
      gr.k_shift = P - E;
      gr.delta = ldexp(1.0, E - P);
    }
  }
  const int maxB = dtype == APC_F32 ? (sc.encoding ? 32 : 31) : 62;
  for (Stream& S : m.streams) {
    const int64_t n = r.get<int64_t>(), mx = r.get<int64_t>();
    const int32_t B = r.get<int32_t>();
    (void)r.get<int32_t>();
    REP_CHECK(r.ok, "metadata truncated");
    REP_CHECK(n == S.n, "stream length %lld, the layout gives %lld", (long long)n, (long long)S.n);
    REP_CHECK(mx >= 0 && B == (S.enc ? nb_digits(mx) : bitlen(mx)) && B <= maxB,
              "stream maximum / plane count inconsistent");
    const Group& gr = m.groups[S.group];
    if (!S.use_cd) {
      const int64_t want = gr.M > 0.0 ? (int64_t)rint(ldexp(gr.M, gr.k_shift)) : 0;
      REP_CHECK(S.n == 0 || mx == want, "stream maximum does not follow its group maximum");
    } else {
      REP_CHECK(gr.M > 0.0 || mx == 0, "decomposition stream of an all-zero group");
    }
    S.maxabs = mx;
    S.B = B;
    S.nsig.assign(B, 0);
    int64_t tot = 0;
    for (int j = 0; j < B; ++j) {
      S.nsig[j] = r.get<int64_t>();
      REP_CHECK(r.ok && S.nsig[j] >= 0 && S.nsig[j] <= S.n, "plane counts out of range");
      tot += S.nsig[j];
    }
    REP_CHECK(tot <= S.n, "more new-significant codes than codes");
    if (S.enc)
      REP_CHECK(tot == 0, "digit planes carry no signs");
    else
      REP_CHECK(B == 0 || S.nsig[0] > 0, "the top plane holds no new-significant code");
    if (S.lossless) {
      S.nnz.assign(B, 0);
      for (int j = 0; j < B; ++j) {
        S.nnz[j] = r.get<int64_t>();
        REP_CHECK(r.ok && S.nnz[j] >= 0 && S.nnz[j] <= S.words(), "nonzero word counts out of range");
      }
    }
  }
  REP_CHECK(r.at == r.n, "metadata section has %zu trailing bytes", r.n - r.at);
  // stream blobs
  size_t at = 32 + (size_t)ml;
  blobs.assign(m.streams.size(), nullptr);
  int64_t mag_w = 0, idx_n = 0, sign_w = 0, nplanes = 0;
  h->psb.assign(m.streams.size(), 0);
  for (int s = 0; s < (int)m.streams.size(); ++s) {
    Stream& S = m.streams[s];
    REP_CHECK((uint64_t)len - at >= 16, "stream %d header truncated", s);
    uint64_t bl, bh;
    memcpy(&bl, src + at, 8);
    memcpy(&bh, src + at + 8, 8);
    REP_CHECK(bl == (uint64_t)S.blob_bytes(), "stream %d: %llu blob bytes, its metadata gives %lld", s,
              (unsigned long long)bl, (long long)S.blob_bytes());
    REP_CHECK((uint64_t)len - at - 16 >= bl, "stream %d blob truncated", s);
    const unsigned char* b = src + at + 16;
    REP_CHECK(!verify_streams || rep_hash(b, (size_t)bl) == bh, "stream %d checksum mismatch", s);
    blobs[s] = b;
    at += 16 + (size_t)bl;
    S.mag_off = mag_w;
    S.idx_off = idx_n;
    S.sign_off = sign_w;
    S.pso.assign(S.B, 0);
    if (S.B == 0 || S.n == 0) continue;
    // index entries: per plane, counts before each chunk, starting at zero,
    // non-decreasing by at most a chunk, and within the plane's total
    const int64_t C = S.chunks();
    if (S.lossless) {
      // stored magnitude sections: a suppressed plane's presence words stop
      // at its last word, its counts follow them, its kept words are nonzero
      // and number nnz; a raw plane holds nnz nonzero words
      const unsigned char* ms = b + S.index_bytes();
      const int64_t M = S.words();
      for (int j = 0; j < S.B; ++j) {
        if (S.suppressed(j)) {
          int64_t run = 0;
          for (int64_t c = 0; c < C; ++c) {
            uint64_t pw;
            uint32_t cv;
            memcpy(&pw, ms + 8 * c, 8);
            memcpy(&cv, ms + 8 * C + 4 * c, 4);
            const int64_t valid = std::min<int64_t>(64, M - 64 * c);
            REP_CHECK(valid == 64 || (pw >> valid) == 0, "stream %d plane %d: presence past the last word", s, j);
            REP_CHECK((int64_t)cv == run, "stream %d plane %d: chunk counts out of order", s, j);
            run += __builtin_popcountll(pw);
          }
          REP_CHECK(run == S.nnz[j], "stream %d plane %d: %lld kept words, metadata says %lld", s, j, (long long)run,
                    (long long)S.nnz[j]);
          const unsigned char* kept = ms + 8 * S.zws_head_words();
          for (int64_t k = 0; k < run; ++k) {
            uint64_t v;
            memcpy(&v, kept + 8 * k, 8);
            REP_CHECK(v != 0, "stream %d plane %d: a kept word is zero", s, j);
          }
        } else {
          int64_t nz = 0;
          for (int64_t w = 0; w < M; ++w) {
            uint64_t v;
            memcpy(&v, ms + 8 * w, 8);
            nz += v != 0;
          }
          REP_CHECK(nz == S.nnz[j], "stream %d plane %d: %lld nonzero words, metadata says %lld", s, j,
                    (long long)nz, (long long)S.nnz[j]);
        }
        ms += 8 * S.mag_words(j);
      }
    }
    for (int j = 0; j < S.B && !S.enc; ++j) {
      uint32_t prev = 0;
      for (int64_t c = 0; c < C; ++c) {
        uint32_t v;
        memcpy(&v, b + 4 * ((int64_t)j * C + c), 4);
        REP_CHECK((c == 0 ? v == 0 : (v >= prev && v - prev <= 4096)) && v <= (uint64_t)S.nsig[j],
                  "stream %d plane %d: index entry %lld out of order", s, j, (long long)c);
        prev = v;
      }
    }
    int64_t w = 0;
    for (int j = 0; j < S.B; ++j) {
      S.pso[j] = w;
      w += (S.nsig[j] + 63) / 64;
    }
    h->psb[s] = (int)nplanes;
    mag_w += (int64_t)S.B * S.words();
    idx_n += (int64_t)S.B * C;
    sign_w += w;
    nplanes += S.B;
  }
  REP_CHECK(at == (size_t)len, "%lld trailing bytes", (long long)(len - (int64_t)at));
  assign_weights(h.get());
  finalize_units(h.get());
  h->k_res.assign(m.streams.size(), 0);
  ensure_sequence(m, 0);
  out = std::move(h);
  return APC_OK;
}

// Device arenas of a handle rebuilt from bytes, and its planes uploaded:
// every plane, or per stream only the first kmax[s] (index entries, stored
// magnitude sections and sign words of those planes are prefixes of their
// sections, so a partial upload is three prefix copies per stream).
// Copies from pageable memory: the runtime has consumed each source when a
// copy call returns, and the stream is synchronized before returning.
apc_status upload_planes(apc_handle* h, const std::vector<const unsigned char*>& blobs, const std::vector<int>* kmax,
                         hipStream_t st) {
  Meta& m = h->meta;
  int64_t mag_w = 0, idx_n = 0, sign_w = 0, nplanes = 0;
  for (const Stream& S : m.streams) {
    if (S.B == 0 || S.n == 0) continue;
    mag_w += (int64_t)S.B * S.words();
    idx_n += (int64_t)S.B * S.chunks();
    sign_w += S.sign_words();
    nplanes += S.B;
  }
  APC_TRY(h->mag.alloc(8 * (size_t)std::max<int64_t>(1, mag_w)));
  APC_TRY(h->idx.alloc(4 * (size_t)std::max<int64_t>(1, idx_n)));
  APC_TRY(h->sign.alloc(8 * (size_t)std::max<int64_t>(1, sign_w)));
  APC_TRY(h->pso.alloc(8 * (size_t)std::max<int64_t>(1, nplanes)));
  if (m.lossless) APC_TRY(h->zoff.alloc(4 * (size_t)std::max<int64_t>(1, idx_n)));
  std::vector<int64_t> pso((size_t)std::max<int64_t>(1, nplanes), 0);
  // copies from pageable memory: the runtime has consumed each source when
  // the call returns, and the stream is synchronized before returning
  for (int s = 0; s < (int)m.streams.size(); ++s) {
    const Stream& S = m.streams[s];
    if (S.B == 0 || S.n == 0) continue;
    const unsigned char* b = blobs[s];
    const int K = kmax ? std::min(S.B, std::max(0, (*kmax)[s])) : S.B;  // planes uploaded
    for (int j = 0; j < S.B; ++j) pso[(size_t)h->psb[s] + j] = S.pso[j];
    if (K == 0) continue;
    const int64_t ibp = S.index_bytes();
    const int64_t mb = 8 * (int64_t)K * S.words();
    const int64_t sb = 8 * (K < S.B ? S.pso[K] : S.sign_words());
    int64_t stored_k = 0;  // stored magnitude words of the first K planes
    for (int j = 0; j < K; ++j) stored_k += S.mag_words(j);
    if (ibp)
      HIP_TRY(hipMemcpyAsync(h->idx.as<uint32_t>() + S.idx_off, b, 4 * (size_t)K * S.chunks(), hipMemcpyHostToDevice,
                             st));
    if (!S.lossless) {
      HIP_TRY(hipMemcpyAsync(h->mag.as<uint64_t>() + S.mag_off, b + ibp, (size_t)mb, hipMemcpyHostToDevice, st));
    } else {
      // stored sections uploaded as they are, expanded to raw planes on the device
      const int64_t smb = 8 * stored_k;
      std::vector<int64_t> pmo((size_t)K + 1, 0);
      uint64_t zmask = 0;
      for (int j = 0; j < K; ++j) {
        pmo[j + 1] = pmo[j] + S.mag_words(j);
        if (S.suppressed(j)) zmask |= 1ull << j;
      }
      DevBuf in, tab;
      APC_TRY(in.alloc((size_t)smb));
      HIP_TRY(hipMemcpyAsync(in.p, b + ibp, (size_t)smb, hipMemcpyHostToDevice, st));
      ZwsSeg z{};
      z.raw_out = h->mag.as<uint64_t>() + S.mag_off;
      z.zoff = h->zoff.as<uint32_t>() + S.idx_off;
      z.comp_in = in.as<uint64_t>();
      z.zmask = zmask;
      z.M = S.words();
      z.C = S.chunks();
      z.B = K;
      TableBuilder tb;
      const size_t o_p = tb.add(pmo);
      APC_TRY(tab.alloc(tb.bytes.size() + 256 + sizeof(ZwsSeg)));
      z.pmo = (const int64_t*)((char*)tab.p + o_p);
      const size_t o_z = tb.add(std::vector<ZwsSeg>{z});
      HIP_TRY(hipMemcpyAsync(tab.p, tb.bytes.data(), tb.bytes.size(), hipMemcpyHostToDevice, st));
      HIP_TRY(launch_zws((const ZwsSeg*)((char*)tab.p + o_z), 1, (int64_t)K * S.chunks(), 2, st));
      HIP_TRY(hipStreamSynchronize(st));  // before the temporaries go back to the pool
    }
    const int64_t mbs = 8 * S.stored_mag_words();
    if (sb)
      HIP_TRY(hipMemcpyAsync(h->sign.as<uint64_t>() + S.sign_off, b + ibp + mbs, (size_t)sb, hipMemcpyHostToDevice, st));
  }
  HIP_TRY(hipMemcpyAsync(h->pso.p, pso.data(), 8 * pso.size(), hipMemcpyHostToDevice, st));
  HIP_TRY(hipStreamSynchronize(st));
  return APC_OK;
}

#undef REP_CHECK

}  // namespace

// Retrieval ladder captured as one HIP graph (a sequence of targets, each
// written to its own output).
struct apc_ladder {
  apc_handle* h = nullptr;
  DevBuf tables;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<int> k_after;
  ~apc_ladder() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
  }
};

extern "C" {

const char* apc_strerror(apc_status s) {
  switch (s) {
    case APC_OK: return "ok";
    case APC_E_INVALID: return "invalid argument";
    case APC_E_DTYPE: return "unsupported dtype";
    case APC_E_NONFINITE: return "non-finite input";
    case APC_E_BELOW_FLOOR: return "target below the representation floor";
    case APC_E_OOM: return "out of device memory";
    case APC_E_HIP: return "HIP runtime error";
    case APC_E_BUSY: return "busy";
    case APC_E_CORRUPT: return "corrupt data";
    case APC_E_NODEVICE: return "no HIP device";
    default: return "unknown status";
  }
}

const char* apc_last_error(void) { return g_last_error.c_str(); }

apc_status apc_refactor(const void* field_dev, int32_t dtype, const int64_t* dims, int32_t ndim,
                        const apc_scheme* scheme, void* hip_stream, apc_handle** out) {
  if (!field_dev || !dims || !scheme || !out) return fail(APC_E_INVALID, "null argument");
  std::vector<std::unique_ptr<apc_handle>> own;
  const void* f[1] = {field_dev};
  APC_TRY(refactor_many(f, dtype, dims, &ndim, scheme, 1, (hipStream_t)hip_stream, own));
  *out = own[0].release();
  return APC_OK;
}

apc_status apc_refactor_batch(const void* const* fields_dev, int32_t dtype, const int64_t* dims,
                              const int32_t* ndims, const apc_scheme* schemes, int32_t nfields, void* hip_stream,
                              apc_handle** out) {
  if (!fields_dev || !dims || !ndims || !schemes || !out || nfields < 1) return fail(APC_E_INVALID, "bad argument");
  for (int f = 0; f < nfields; ++f)
    if (!fields_dev[f]) return fail(APC_E_INVALID, "null field %d", f);
  std::vector<std::unique_ptr<apc_handle>> own;
  APC_TRY(refactor_many(fields_dev, dtype, dims, ndims, schemes, nfields, (hipStream_t)hip_stream, own));
  for (int f = 0; f < nfields; ++f) out[f] = own[f].release();
  return APC_OK;
}

apc_status apc_plan(apc_handle* h, const apc_target* target, int32_t* planes_out, apc_retrieve_info* info) {
  if (!h || !target) return fail(APC_E_INVALID, "null argument");
  std::vector<int> planes;
  APC_TRY(plan_for(h, target, planes, info, &h->k_res));
  if (planes_out)
    for (size_t s = 0; s < planes.size(); ++s) planes_out[s] = planes[s];
  return APC_OK;
}

apc_status apc_retrieve(apc_handle* h, const apc_target* target, void* out_dev, apc_retrieve_info* info,
                        void* hip_stream) {
  if (!h || !target || !out_dev) return fail(APC_E_INVALID, "null argument");
  APC_TRY(need_device(h));
  std::vector<int> planes;
  apc_retrieve_info inf{};
  APC_TRY(plan_for(h, target, planes, &inf, &h->k_res));
  int64_t fetched = 0;
  APC_TRY(do_retrieve(h, planes, out_dev, hip_stream, &fetched));
  inf.bytes_fetched = fetched;
  if (info) *info = inf;
  return APC_OK;
}

apc_status apc_retrieve_batch(apc_handle* const* hs, int32_t n, const apc_target* targets, void* const* outs_dev,
                              apc_retrieve_info* infos, void* hip_stream) {
  if (!hs || !targets || !outs_dev || n < 1) return fail(APC_E_INVALID, "bad argument");
  for (int32_t i = 0; i < n; ++i) {
    if (!hs[i] || !outs_dev[i]) return fail(APC_E_INVALID, "null handle or output at %d", i);
    if (hs[i]->dtype != hs[0]->dtype) return fail(APC_E_INVALID, "a batch holds handles of one dtype");
    APC_TRY(need_device(hs[i]));
  }
  hipStream_t st = (hipStream_t)hip_stream;
  if (hs[0]->dtype == APC_F32) return retrieve_batch_impl<float, int32_t>(hs, n, targets, outs_dev, infos, st);
  return retrieve_batch_impl<double, int64_t>(hs, n, targets, outs_dev, infos, st);
}

apc_status apc_retrieve_planes(apc_handle* h, const int32_t* planes, void* out_dev, void* hip_stream) {
  if (!h || !planes || !out_dev) return fail(APC_E_INVALID, "null argument");
  APC_TRY(need_device(h));
  std::vector<int> p(h->meta.streams.size());
  for (size_t s = 0; s < p.size(); ++s) p[s] = std::max(0, std::min<int>(planes[s], h->meta.streams[s].B));
  return do_retrieve(h, p, out_dev, hip_stream, nullptr);
}

apc_status apc_retrieve_static(apc_handle* h, const apc_target* target, void* out_dev, apc_retrieve_info* info,
                               void* hip_stream) {
  if (!h || !target || !out_dev) return fail(APC_E_INVALID, "null argument");
  APC_TRY(need_device(h));
  std::vector<int> planes;
  apc_retrieve_info inf{};
  APC_TRY(plan_for(h, target, planes, &inf, &h->k_res));
  int64_t fetched = 0;
  hipStream_t st = (hipStream_t)hip_stream;
  if (h->dtype == APC_F32)
    APC_TRY((retrieve_static_impl<float, int32_t>(h, planes, (float*)out_dev, st, &fetched)));
  else
    APC_TRY((retrieve_static_impl<double, int64_t>(h, planes, (double*)out_dev, st, &fetched)));
  inf.bytes_fetched = fetched;
  if (info) *info = inf;
  return APC_OK;
}

apc_status apc_ladder_create(apc_handle* h, const apc_target* targets, int32_t n, void* const* outs_dev,
                             void* hip_stream, apc_ladder** out) {
  if (!h || !targets || !outs_dev || !out || n < 1) return fail(APC_E_INVALID, "bad argument");
  APC_TRY(need_device(h));
  APC_TRY(ensure_work(h));
  hipStream_t st = (hipStream_t)hip_stream;
  if (h->ready) HIP_TRY(hipStreamWaitEvent(st, h->ready, 0));  // the refactor's last kernels
  std::unique_ptr<apc_ladder> ld(new apc_ladder());
  ld->h = h;
  TableBuilder tb;
  std::vector<Launch> ls;
  std::vector<int> kres(h->meta.streams.size(), 0);  // a replay starts from nothing resident
  for (int i = 0; i < n; ++i) {
    std::vector<int> planes;
    APC_TRY(plan_for(h, &targets[i], planes, nullptr, &kres));
    if (h->dtype == APC_F32)
      build_retrieve<float, int32_t>(h, planes, (float*)outs_dev[i], kres, tb, ls, nullptr, handle_work(h));
    else
      build_retrieve<double, int64_t>(h, planes, (double*)outs_dev[i], kres, tb, ls, nullptr, handle_work(h));
  }
  ld->k_after = kres;
  APC_TRY(ld->tables.alloc(tb.bytes.size()));
  HIP_TRY(hipStreamSynchronize(st));
  HIP_TRY(hipMemcpy(ld->tables.p, tb.bytes.data(), tb.bytes.size(), hipMemcpyHostToDevice));
  // Capture on a private stream (the legacy null stream cannot be captured);
  // the graph is later launched on the caller's stream.
  hipStream_t cs = nullptr;
  HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  hipError_t e0 = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
  if (e0 != hipSuccess) {
    (void)hipStreamDestroy(cs);
    return fail(APC_E_HIP, "hipStreamBeginCapture: %s", hipGetErrorString(e0));
  }
  g_prof_suppress = true;  // no timing events inside a capture
  apc_status s = h->dtype == APC_F32 ? issue<float, int32_t>(ls, (const char*)ld->tables.p, cs)
                                     : issue<double, int64_t>(ls, (const char*)ld->tables.p, cs);
  g_prof_suppress = false;
  hipGraph_t graph = nullptr;
  hipError_t e = hipStreamEndCapture(cs, &graph);
  (void)hipStreamDestroy(cs);
  if (s != APC_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return s;
  }
  if (e != hipSuccess) return fail(APC_E_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
  ld->graph = graph;
  HIP_TRY(hipGraphInstantiate(&ld->exec, graph, nullptr, nullptr, 0));
  *out = ld.release();
  return APC_OK;
}

apc_status apc_ladder_launch(apc_ladder* ld, void* hip_stream) {
  if (!ld) return fail(APC_E_INVALID, "null ladder");
  HIP_TRY(hipGraphLaunch(ld->exec, (hipStream_t)hip_stream));
  ld->h->k_res = ld->k_after;
  return APC_OK;
}

void apc_ladder_free(apc_ladder* ld) {
  if (!ld) return;
  (void)hipDeviceSynchronize();
  delete ld;
}

void apc_free(apc_handle* h) {
  if (!h) return;
  if (h->host_only) {  // no device data, nothing queued
    delete h;
    return;
  }
  // Work queued on any stream may still read this handle's buffers; they go
  // back to the shared pool only once the device is idle.
  (void)hipDeviceSynchronize();
  delete h;
  reap_retired();  // the device is idle: every retired buffer goes back to the pool
}

int32_t apc_num_streams(const apc_handle* h) { return h ? (int32_t)h->meta.streams.size() : 0; }
int32_t apc_num_groups(const apc_handle* h) { return h ? (int32_t)h->meta.groups.size() : 0; }
int64_t apc_num_points(const apc_handle* h) { return h ? h->meta.n : 0; }

apc_status apc_stream_info(const apc_handle* h, int32_t s, int64_t* n, int32_t* B, int64_t* maxabs,
                           int64_t* blob_bytes) {
  if (!h || s < 0 || s >= (int32_t)h->meta.streams.size()) return fail(APC_E_INVALID, "bad stream index");
  const Stream& S = h->meta.streams[s];
  if (n) *n = S.n;
  if (B) *B = S.B;
  if (maxabs) *maxabs = S.maxabs;
  if (blob_bytes) *blob_bytes = S.blob_bytes();
  return APC_OK;
}

apc_status apc_stream_blob(const apc_handle* h, int32_t s, void* host_dst, int64_t cap) {
  if (!h || s < 0 || s >= (int32_t)h->meta.streams.size() || !host_dst) return fail(APC_E_INVALID, "bad argument");
  APC_TRY(need_device(h));
  const Stream& S = h->meta.streams[s];
  if (cap < S.blob_bytes()) return fail(APC_E_INVALID, "buffer too small");
  char* dst = (char*)host_dst;
  memset(dst, 0, (size_t)S.blob_bytes());
  if (S.B == 0 || S.n == 0) return APC_OK;
  if (h->ready) HIP_TRY(hipEventSynchronize(h->ready));  // the refactor's last kernels
  const int64_t ibp = S.index_bytes();
  if (ibp)
    HIP_TRY(hipMemcpy(dst, h->idx.as<uint32_t>() + S.idx_off, 4 * (size_t)S.B * S.chunks(), hipMemcpyDeviceToHost));
  const int64_t mb = 8 * S.stored_mag_words();
  if (!S.lossless) {
    HIP_TRY(hipMemcpy(dst + ibp, h->mag.as<uint64_t>() + S.mag_off, (size_t)mb, hipMemcpyDeviceToHost));
  } else {
    // the stored sections, packed on the device from the raw planes
    std::vector<int64_t> pmo((size_t)S.B + 1, 0);
    uint64_t zmask = 0;
    for (int j = 0; j < S.B; ++j) {
      pmo[j + 1] = pmo[j] + S.mag_words(j);
      if (S.suppressed(j)) zmask |= 1ull << j;
    }
    DevBuf out, tab;
    APC_TRY(out.alloc((size_t)mb));
    ZwsSeg z{};
    z.raw_in = h->mag.as<uint64_t>() + S.mag_off;
    z.zoff = h->zoff.as<uint32_t>() + S.idx_off;
    z.comp_out = out.as<uint64_t>();
    z.zmask = zmask;
    z.M = S.words();
    z.C = S.chunks();
    z.B = S.B;
    TableBuilder tb;
    const size_t o_p = tb.add(pmo);
    APC_TRY(tab.alloc(tb.bytes.size() + 256 + sizeof(ZwsSeg)));
    z.pmo = (const int64_t*)((char*)tab.p + o_p);
    const size_t o_z = tb.add(std::vector<ZwsSeg>{z});
    HIP_TRY(hipMemcpy(tab.p, tb.bytes.data(), tb.bytes.size(), hipMemcpyHostToDevice));
    HIP_TRY(launch_zws((const ZwsSeg*)((char*)tab.p + o_z), 1, (int64_t)S.B * S.chunks(), 1, nullptr));
    HIP_TRY(hipMemcpy(dst + ibp, out.p, (size_t)mb, hipMemcpyDeviceToHost));
    HIP_TRY(hipDeviceSynchronize());  // the temporaries go back to the pool after this
  }
  const int64_t sb = 8 * S.sign_words();
  if (sb) HIP_TRY(hipMemcpy(dst + ibp + mb, h->sign.as<uint64_t>() + S.sign_off, (size_t)sb, hipMemcpyDeviceToHost));
  return APC_OK;
}

apc_status apc_metadata_json(const apc_handle* h, char* buf, int64_t cap, int64_t* len) {
  if (!h) return fail(APC_E_INVALID, "null handle");
  std::string js = meta_json(h->meta);
  {  // the scheme the handle was refactored with (levels: the number used)
    const apc_scheme& c = h->scheme;
    char tmp[320];
    snprintf(tmp, sizeof(tmp),
             ",\"scheme\":{\"kind\":%d,\"degree\":%d,\"order\":[%d,%d,%d],\"cd_axis\":%d,\"levels\":%d,"
             "\"lossless\":%d,\"encoding\":%d}}",
             c.kind, c.degree, h->geo.sigma_user[0], h->geo.sigma_user[1], h->geo.sigma_user[2], c.cd_axis, h->geo.L,
             c.lossless, c.encoding);
    js.pop_back();  // the closing brace
    js += tmp;
  }
  if (len) *len = (int64_t)js.size();
  if (buf) {
    if (cap < (int64_t)js.size() + 1) return fail(APC_E_INVALID, "buffer too small");
    memcpy(buf, js.c_str(), js.size() + 1);
  }
  return APC_OK;
}

apc_status apc_field_info(const apc_handle* h, int64_t* dims, int32_t* ndim, int32_t* dtype) {
  if (!h) return fail(APC_E_INVALID, "null handle");
  const Geo& g = h->geo;
  if (ndim) *ndim = g.d;
  if (dtype) *dtype = h->dtype;
  if (dims)
    for (int a = 0; a < g.d; ++a) dims[a] = g.N[3 - g.d + a];
  return APC_OK;
}

apc_status apc_serialize(const apc_handle* h, void* host_dst, int64_t cap, int64_t* len) {
  if (!h || !len) return fail(APC_E_INVALID, "null argument");
  APC_TRY(need_device(h));
  std::vector<unsigned char> meta;
  rep_meta(h, meta);
  int64_t total = 32 + (int64_t)meta.size();
  for (const Stream& S : h->meta.streams) total += 16 + S.blob_bytes();
  *len = total;
  if (!host_dst) return APC_OK;
  if (cap < total) return fail(APC_E_INVALID, "buffer of %lld bytes, the representation needs %lld", (long long)cap,
                               (long long)total);
  if (h->ready) HIP_TRY(hipEventSynchronize(h->ready));  // the refactor's last kernels
  unsigned char* d = (unsigned char*)host_dst;
  memcpy(d, kRepMagic, 8);
  const uint64_t tl = (uint64_t)total, ml = (uint64_t)meta.size(), mh = rep_hash(meta.data(), meta.size());
  memcpy(d + 8, &tl, 8);
  memcpy(d + 16, &ml, 8);
  memcpy(d + 24, &mh, 8);
  memcpy(d + 32, meta.data(), meta.size());
  // the stream blobs copied out in turn, then their checksums on the host
  // threads (each over its own blob)
  const int ns = (int)h->meta.streams.size();
  std::vector<int64_t> at_s((size_t)ns);
  int64_t at = 32 + (int64_t)meta.size();
  for (int s = 0; s < ns; ++s) {
    const Stream& S = h->meta.streams[s];
    const uint64_t bl = (uint64_t)S.blob_bytes();
    at_s[(size_t)s] = at;
    if (bl) APC_TRY(apc_stream_blob(h, s, d + at + 16, (int64_t)bl));
    memcpy(d + at, &bl, 8);
    at += 16 + (int64_t)bl;
  }
  parallel_for((size_t)ns, [&](size_t s) {
    const int64_t a = at_s[s];
    uint64_t bl;
    memcpy(&bl, d + a, 8);
    const uint64_t bh = rep_hash(d + a + 16, (size_t)bl);
    memcpy(d + a + 8, &bh, 8);
  });
  return APC_OK;
}

apc_status apc_deserialize_host(const void* src, int64_t len, apc_handle** out) {
  if (!src || len < 0 || !out) return fail(APC_E_INVALID, "null argument");
  std::unique_ptr<apc_handle> h;
  std::vector<const unsigned char*> blobs;
  APC_TRY(rep_parse((const unsigned char*)src, len, h, blobs));
  h->host_only = true;
  *out = h.release();
  return APC_OK;
}

apc_status apc_set_interpreter(apc_handle* h, int32_t interp) {
  if (!h) return fail(APC_E_INVALID, "null handle");
  if (interp < APC_INTERP_GREEDY || interp > APC_INTERP_PAPER) return fail(APC_E_INVALID, "interpreter %d", interp);
  h->interp = interp;
  return APC_OK;
}

apc_status apc_deserialize(const void* src, int64_t len, void* hip_stream, apc_handle** out) {
  if (!src || len < 0) return fail(APC_E_INVALID, "null argument");
  std::unique_ptr<apc_handle> h;
  std::vector<const unsigned char*> blobs;
  APC_TRY(rep_parse((const unsigned char*)src, len, h, blobs));
  if (!out) return APC_OK;  // checked only
  APC_TRY(upload_planes(h.get(), blobs, nullptr, (hipStream_t)hip_stream));
  *out = h.release();
  return APC_OK;
}

}  // extern "C"

// ------------------------------------------------------ out-of-core blocks
// A field held in host memory, split into independent blocks (the paper
// refactors fixed-size blocks independently, one per core, and stores them).
// Each block is refactored on the device and kept serialized in host memory;
// a retrieval plans every block on its host-side metadata, uploads only the
// planes the plan needs (prefixes of the stored sections), reconstructs the
// block on the device and copies it into the host output.  The device holds
// one group of blocks at a time, so the field can exceed device memory.
struct apc_blockset {
  int dtype = APC_F32;
  int ndim = 3;
  int64_t N[3] = {1, 1, 1}, bs[3] = {1, 1, 1}, nb[3] = {1, 1, 1};
  apc_scheme scheme{};
  int interp = INTERP_GREEDY;
  double xmin = 0, xmax = 0;
  std::vector<std::vector<unsigned char>> blobs;
  std::vector<std::unique_ptr<apc_handle>> plan_h;  // planning-only handles, one per block
  int64_t nblocks() const { return nb[0] * nb[1] * nb[2]; }
  void block(int64_t b, int64_t lo[3], int64_t ext[3]) const {
    const int64_t i[3] = {b / (nb[1] * nb[2]), (b / nb[2]) % nb[1], b % nb[2]};
    for (int a = 0; a < 3; ++a) {
      lo[a] = i[a] * bs[a];
      ext[a] = std::min(N[a], lo[a] + bs[a]) - lo[a];
    }
  }
};

namespace {

// Rows of a block between a row-major host field and a dense block buffer.
void block_copy(const apc_blockset* B, int64_t b, size_t es, const char* field, char* dense, bool to_dense,
                char* field_out) {
  int64_t lo[3], ext[3];
  B->block(b, lo, ext);
  const size_t row = (size_t)ext[2] * es;
  auto plane = [&](size_t z) {
    for (int64_t y = 0; y < ext[1]; ++y) {
      const size_t fo = (size_t)(((lo[0] + (int64_t)z) * B->N[1] + (lo[1] + y)) * B->N[2] + lo[2]) * es;
      const size_t bo = (size_t)(((int64_t)z * ext[1] + y) * ext[2]) * es;
      if (to_dense)
        memcpy(dense + bo, field + fo, row);
      else
        memcpy(field_out + fo, dense + bo, row);
    }
  };
  // large blocks copy their planes on the host threads (one thread's memcpy
  // moves about 9 GB/s, far below what the host memory takes)
  if ((size_t)ext[1] * row * (size_t)ext[0] >= ((size_t)8 << 20))
    parallel_for((size_t)ext[0], plane);
  else
    for (int64_t z = 0; z < ext[0]; ++z) plane((size_t)z);
}

}  // namespace

extern "C" {

apc_status apc_blocks_refactor(const void* field_host, int32_t dtype, const int64_t* dims, int32_t ndim,
                               const int64_t* block, const apc_scheme* scheme, int64_t group_bytes, void* hip_stream,
                               apc_blockset** out) {
  if (!field_host || !dims || !block || !scheme || !out || ndim < 1 || ndim > 3 || group_bytes <= 0)
    return fail(APC_E_INVALID, "bad argument");
  if (dtype != APC_F32 && dtype != APC_F64) return fail(APC_E_DTYPE, "dtype must be APC_F32 or APC_F64");
  hipStream_t st = (hipStream_t)hip_stream;
  std::unique_ptr<apc_blockset> B(new apc_blockset());
  B->dtype = dtype;
  B->ndim = ndim;
  B->scheme = *scheme;
  for (int a = 0; a < ndim; ++a) {
    if (dims[a] < 1 || block[a] < 1) return fail(APC_E_INVALID, "dims and block extents must be positive");
    B->N[3 - ndim + a] = dims[a];
    B->bs[3 - ndim + a] = std::min(dims[a], block[a]);
  }
  for (int a = 0; a < 3; ++a) B->nb[a] = (B->N[a] + B->bs[a] - 1) / B->bs[a];
  const size_t es = qsize(dtype);
  const int64_t nbk = B->nblocks();
  B->blobs.resize((size_t)nbk);
  B->plan_h.resize((size_t)nbk);
  // groups of blocks that fit the device budget, refactored in one batch
  int64_t b0 = 0;
  while (b0 < nbk) {
    std::vector<int64_t> bl;
    size_t bytes = 0;
    for (int64_t b = b0; b < nbk; ++b) {
      int64_t lo[3], ext[3];
      B->block(b, lo, ext);
      const size_t nbyte = (size_t)(ext[0] * ext[1] * ext[2]) * es;
      if (!bl.empty() && bytes + nbyte > (size_t)group_bytes) break;
      bl.push_back(b);
      bytes += nbyte;
    }
    PinnedBlock pin;
    if (!g_pinned.get(bytes, pin)) return fail(APC_E_OOM, "pinned staging of %zu bytes", bytes);
    DevBuf dev;
    apc_status r = dev.alloc(bytes);
    std::vector<const void*> ptrs;
    std::vector<int64_t> bd;
    std::vector<int32_t> nds;
    std::vector<size_t> offs;
    size_t off = 0;
    for (int64_t b : bl) {
      int64_t lo[3], ext[3];
      B->block(b, lo, ext);
      offs.push_back(off);
      ptrs.push_back((const char*)dev.p + off);
      for (int a = 3 - ndim; a < 3; ++a) bd.push_back(ext[a]);
      nds.push_back(ndim);
      off += (size_t)(ext[0] * ext[1] * ext[2]) * es;
    }
    // the blocks' gathers into the staging block (each on the host threads)
    for (size_t i = 0; i < bl.size(); ++i)
      block_copy(B.get(), bl[i], es, (const char*)field_host, (char*)pin.p + offs[i], true, nullptr);
    if (r == APC_OK && hipMemcpyAsync(dev.p, pin.p, bytes, hipMemcpyHostToDevice, st) != hipSuccess)
      r = fail(APC_E_HIP, "block upload failed");
    std::vector<std::unique_ptr<apc_handle>> own;
    if (r == APC_OK) {
      std::vector<apc_scheme> sc(bl.size(), *scheme);
      r = refactor_many(ptrs.data(), dtype, bd.data(), nds.data(), sc.data(), (int32_t)bl.size(), st, own);
    }
    g_pinned.put(pin, st, true);
    // serialization of each block (device reads, checksums) and its host
    // planning handle, on the host threads; a failure is reported with the
    // message of the thread that met it
    if (r == APC_OK) {
      int dev_id = 0;
      HIP_TRY(hipGetDevice(&dev_id));
      std::vector<apc_status> rs(bl.size(), APC_OK);
      std::vector<std::string> msg(bl.size());
      parallel_for(bl.size(), [&](size_t i) {
        apc_status q = hipSetDevice(dev_id) == hipSuccess ? APC_OK : fail(APC_E_HIP, "hipSetDevice failed");
        int64_t len = 0;
        if (q == APC_OK) q = apc_serialize(own[i].get(), nullptr, 0, &len);
        std::vector<unsigned char>& blob = B->blobs[(size_t)bl[i]];
        if (q == APC_OK) {
          blob.resize((size_t)len);
          q = apc_serialize(own[i].get(), blob.data(), len, &len);
        }
        if (q == APC_OK) {
          std::vector<const unsigned char*> bp;
          // the blob was just written here: its stream checksums are not re-verified
          q = rep_parse(blob.data(), len, B->plan_h[(size_t)bl[i]], bp, false);
          if (q == APC_OK) B->plan_h[(size_t)bl[i]]->host_only = true;
        }
        if (q != APC_OK) {
          rs[i] = q;
          msg[i] = g_last_error;
        }
      });
      for (size_t i = 0; i < bl.size() && r == APC_OK; ++i)
        if (rs[i] != APC_OK) r = fail(rs[i], "block %lld: %s", (long long)bl[i], msg[i].c_str());
    }
    (void)hipStreamSynchronize(st);
    for (auto& h : own) apc_free(h.release());
    APC_TRY(r);
    b0 += (int64_t)bl.size();
  }
  B->xmin = B->plan_h[0]->meta.xmin;
  B->xmax = B->plan_h[0]->meta.xmax;
  for (auto& h : B->plan_h) {
    B->xmin = std::min(B->xmin, h->meta.xmin);
    B->xmax = std::max(B->xmax, h->meta.xmax);
  }
  *out = B.release();
  return APC_OK;
}

apc_status apc_blocks_info(const apc_blockset* B, int64_t* nblocks, int64_t* stored_bytes, double* xmin,
                           double* xmax) {
  if (!B) return fail(APC_E_INVALID, "null block set");
  if (nblocks) *nblocks = B->nblocks();
  if (stored_bytes) {
    int64_t t = 0;
    for (const auto& b : B->blobs) t += (int64_t)b.size();
    *stored_bytes = t;
  }
  if (xmin) *xmin = B->xmin;
  if (xmax) *xmax = B->xmax;
  return APC_OK;
}

apc_status apc_blocks_blob(const apc_blockset* B, int64_t b, const void** bytes, int64_t* len) {
  if (!B || b < 0 || b >= B->nblocks() || !bytes || !len) return fail(APC_E_INVALID, "bad argument");
  *bytes = B->blobs[(size_t)b].data();
  *len = (int64_t)B->blobs[(size_t)b].size();
  return APC_OK;
}

apc_status apc_blocks_set_interpreter(apc_blockset* B, int32_t interp) {
  if (!B) return fail(APC_E_INVALID, "null block set");
  if (interp < APC_INTERP_GREEDY || interp > APC_INTERP_PAPER) return fail(APC_E_INVALID, "interpreter %d", interp);
  B->interp = interp;
  for (auto& h : B->plan_h) h->interp = interp;
  return APC_OK;
}

apc_status apc_blocks_retrieve(apc_blockset* B, const apc_target* target, void* out_host, apc_retrieve_info* info,
                               void* hip_stream) {
  if (!B || !target || !out_host) return fail(APC_E_INVALID, "null argument");
  hipStream_t st = (hipStream_t)hip_stream;
  // the target as an absolute bound every block must meet: a max error
  // within tau in every block is one within tau overall, and an RMSE within
  // r in every block is one within r overall
  const double rng = B->xmax - B->xmin;
  apc_target t = *target;
  switch (target->kind) {
    case APC_EB_REL:
      t.kind = APC_EB_ABS;
      t.value = target->value * rng;
      break;
    case APC_PSNR:
      t.kind = APC_RMSE_ABS;
      t.value = rng * pow(10.0, -target->value / 20.0);
      break;
    case APC_EB_ABS:
    case APC_RMSE_ABS: break;
    default: return fail(APC_E_INVALID, "unknown target kind %d", target->kind);
  }
  const size_t es = qsize(B->dtype);
  size_t maxb = 0;
  for (int64_t b = 0; b < B->nblocks(); ++b) {
    int64_t lo[3], ext[3];
    B->block(b, lo, ext);
    maxb = std::max(maxb, (size_t)(ext[0] * ext[1] * ext[2]) * es);
  }
  DevBuf dout;
  APC_TRY(dout.alloc(maxb));
  PinnedBlock pin;
  if (!g_pinned.get(maxb, pin)) return fail(APC_E_OOM, "pinned staging of %zu bytes", maxb);
  struct PinBack {
    PinnedBlock* p;
    hipStream_t st;
    ~PinBack() { g_pinned.put(*p, st, true); }
  } pb{&pin, st};
  apc_retrieve_info tot{};
  double sq = 0.0, worst = 0.0;
  const bool l2 = t.kind == APC_RMSE_ABS;
  for (int64_t b = 0; b < B->nblocks(); ++b) {
    apc_handle* ph = B->plan_h[(size_t)b].get();
    std::vector<int> planes;
    apc_retrieve_info bi{};
    APC_TRY(plan_for(ph, &t, planes, &bi, nullptr));
    std::unique_ptr<apc_handle> h;
    std::vector<const unsigned char*> bp;
    const std::vector<unsigned char>& blob = B->blobs[(size_t)b];
    // blobs this blockset wrote and holds: their stream checksums are not
    // re-verified at every retrieval (deserializing outside input does)
    APC_TRY(rep_parse(blob.data(), (int64_t)blob.size(), h, bp, false));
    APC_TRY(upload_planes(h.get(), bp, &planes, st));
    APC_TRY(do_retrieve(h.get(), planes, dout.p, st, nullptr));
    HIP_TRY(hipMemcpyAsync(pin.p, dout.p, (size_t)ph->meta.n * es, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    block_copy(B, b, es, nullptr, (char*)pin.p, false, (char*)out_host);
    tot.bytes_total += bi.bytes_total;
    tot.bytes_fetched += bi.bytes_total;
    tot.nsteps += bi.nsteps;
    tot.n_streams += bi.n_streams;
    worst = std::max(worst, bi.bound);
    sq += (double)ph->meta.n * bi.bound * bi.bound;
  }
  const double n = (double)(B->N[0] * B->N[1] * B->N[2]);
  tot.tau = t.value;
  tot.bound = l2 ? sqrt(sq / n) : worst;
  tot.bitrate = 8.0 * (double)tot.bytes_total / n;
  if (info) *info = tot;
  return APC_OK;
}

void apc_blocks_free(apc_blockset* B) { delete B; }

apc_status apc_axis_norms(int64_t n, int32_t L, int32_t degree, double* inf_out, double* one_out) {
  if (n < 1 || L < 1 || (degree != 1 && degree != 3) || !inf_out || !one_out)
    return fail(APC_E_INVALID, "bad argument");
  std::vector<double> a, b;
  axis_norms(n, L, degree, a, b);
  for (int l = 0; l < L; ++l) {
    inf_out[l] = a[l];
    one_out[l] = b[l];
  }
  return APC_OK;
}

apc_status apc_profile_enable(int32_t on) {
  g_prof.on = on != 0;
  return APC_OK;
}

apc_status apc_profile_only(const char* name) {
  std::lock_guard<std::mutex> lk(g_prof.mu);
  g_prof.only = name ? name : "";
  g_prof.filtered = !g_prof.only.empty();
  return APC_OK;
}

static std::string g_prof_last = "{}";

apc_status apc_profile_report(char* buf, int64_t cap, int64_t* len) {
  // Per kernel name: launches, total milliseconds, total bytes moved.  The
  // records are consumed once; the text stays available for a second call
  // (callers ask for the length first).
  std::lock_guard<std::mutex> lk(g_prof.mu);
  if (!g_prof.recs.empty()) {
    std::vector<std::string> names;
    std::vector<double> ms, bytes;
    std::vector<int64_t> count;
    for (ProfRec& r : g_prof.recs) {
      (void)hipEventSynchronize(r.b);
      float t = 0.f;
      (void)hipEventElapsedTime(&t, r.a, r.b);
      size_t k = 0;
      while (k < names.size() && names[k] != r.name) ++k;
      if (k == names.size()) {
        names.push_back(r.name);
        ms.push_back(0);
        bytes.push_back(0);
        count.push_back(0);
      }
      ms[k] += t;
      bytes[k] += r.bytes;
      count[k] += 1;
      g_prof.pool.push_back(r.a);
      g_prof.pool.push_back(r.b);
    }
    g_prof.recs.clear();
    std::string js = "{";
    char tmp[256];
    for (size_t k = 0; k < names.size(); ++k) {
      snprintf(tmp, sizeof(tmp), "%s\"%s\":{\"count\":%lld,\"ms\":%.6f,\"bytes\":%.0f}", k ? "," : "",
               names[k].c_str(), (long long)count[k], ms[k], bytes[k]);
      js += tmp;
    }
    js += "}";
    g_prof_last = js;
  }
  if (len) *len = (int64_t)g_prof_last.size();
  if (buf) {
    if (cap < (int64_t)g_prof_last.size() + 1) return fail(APC_E_INVALID, "buffer too small");
    memcpy(buf, g_prof_last.c_str(), g_prof_last.size() + 1);
  }
  return APC_OK;
}

}  // extern "C"

// ------------------------------------------------------ pipeline selection
namespace {

// Regular sample blocks of the field (about 1%): side b at every e-th block
// position per axis; at least one block per axis.
void sample_blocks(const Geo& g, std::vector<std::array<int64_t, 6>>& blocks) {
  const int d = g.d;
  const int64_t side = d == 3 ? 32 : (d == 2 ? 128 : 4096);
  const int64_t every = d == 3 ? 5 : (d == 2 ? 10 : 100);
  std::vector<int64_t> pos[3];
  for (int a = 0; a < 3; ++a) {
    const int64_t n = g.N[a];
    if (a < 3 - d) {
      pos[a].push_back(-1);  // embedded axis: whole (length 1)
      continue;
    }
    const int64_t nb = std::max<int64_t>(1, n / side);
    for (int64_t p = 0; p < nb; p += every) pos[a].push_back(p);
  }
  for (int64_t p0 : pos[0])
    for (int64_t p1 : pos[1])
      for (int64_t p2 : pos[2]) {
        std::array<int64_t, 6> b{};
        const int64_t ps[3] = {p0, p1, p2};
        for (int a = 0; a < 3; ++a) {
          if (ps[a] < 0) {
            b[a] = 0;
            b[3 + a] = 1;
          } else {
            b[a] = ps[a] * side;
            b[3 + a] = std::min(g.N[a], (ps[a] + 1) * side) - b[a];
          }
        }
        blocks.push_back(b);
      }
}

const double kTuneTol[9] = {1e-3, 5e-4, 1e-4, 5e-5, 1e-5, 5e-6, 1e-6, 5e-7, 1e-7};

template <typename T>
apc_status select_impl(const T* field, int32_t dtype, const Geo& g, int mode, apc_scheme* out, hipStream_t st) {
  std::vector<std::array<int64_t, 6>> blocks;
  sample_blocks(g, blocks);
  const int nb = (int)blocks.size();
  int64_t tot = 0;
  std::vector<int64_t> boff(nb);
  for (int b = 0; b < nb; ++b) {
    boff[b] = tot;
    tot += blocks[b][3] * blocks[b][4] * blocks[b][5];
  }
  DevBuf samp, tab, accb;
  APC_TRY(samp.alloc(sizeof(T) * (size_t)tot));
  APC_TRY(accb.alloc(32));
  std::vector<FlatSeg> gs, rs;
  for (int b = 0; b < nb; ++b) {
    FlatSeg q{};
    q.src = field + (blocks[b][0] * g.N[1] + blocks[b][1]) * g.N[2] + blocks[b][2];
    q.dst = samp.as<T>() + boff[b];
    for (int a = 0; a < 3; ++a) q.dm[a] = (int32_t)blocks[b][3 + a];
    q.n = (int64_t)q.dm[0] * q.dm[1] * q.dm[2];
    q.s[0] = g.N[1] * g.N[2];
    q.s[1] = g.N[2];
    q.s[2] = 1;
    q.f2 = make_fastdiv((uint32_t)q.dm[2]);
    q.f1 = make_fastdiv((uint32_t)q.dm[1]);
    gs.push_back(q);
  }
  FlatSeg r{};
  r.src = field;
  r.n = g.n();
  r.acc = accb.as<unsigned long long>();
  rs.push_back(r);
  TableBuilder tb;
  const int64_t b1 = assign_blocks<FlatSeg>(gs, [](const FlatSeg& s) { return s.n; });
  const int64_t b2 = assign_blocks<FlatSeg>(rs, [](const FlatSeg& s) { return s.n; });
  std::vector<Launch> ls{{K_GATHER, tb.add(gs), (int)gs.size(), b1, 0, 2.0 * sizeof(T) * tot, "subsample"},
                         {K_RANGE, tb.add(rs), 1, b2, 0, (double)sizeof(T) * g.n(), "range"}};
  unsigned long long init[4] = {~0ull, 0ull, 0ull, 0ull};
  HIP_TRY(hipMemcpyAsync(accb.p, init, 32, hipMemcpyHostToDevice, st));
  APC_TRY(tab.alloc(tb.bytes.size()));
  HIP_TRY(hipMemcpyAsync(tab.p, tb.bytes.data(), tb.bytes.size(), hipMemcpyHostToDevice, st));
  typedef typename std::conditional<sizeof(T) == 4, int32_t, int64_t>::type Q;
  APC_TRY((issue<T, Q>(ls, (const char*)tab.p, st)));
  unsigned long long hv[4];
  HIP_TRY(hipMemcpyAsync(hv, accb.p, 32, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (hv[3]) return fail(APC_E_NONFINITE, "field holds NaN or Inf");
  const double rng = unordered(hv[1]) - unordered(hv[0]);

  std::vector<const void*> fptr(nb);
  std::vector<int64_t> dims;
  std::vector<int32_t> nds(nb, g.d);
  for (int b = 0; b < nb; ++b) {
    fptr[b] = samp.as<T>() + boff[b];
    for (int a = 3 - g.d; a < 3; ++a) dims.push_back(blocks[b][3 + a]);
  }
  auto vote = [&](const std::vector<apc_scheme>& cands, int& winner) -> apc_status {
    std::vector<std::array<int64_t, 9>> sizes(cands.size());
    for (size_t c = 0; c < cands.size(); ++c) {
      std::vector<apc_scheme> sc(nb, cands[c]);
      std::vector<std::unique_ptr<apc_handle>> own;
      APC_TRY(refactor_many(fptr.data(), dtype, dims.data(), nds.data(), sc.data(), nb, st, own));
      // the blocks' plans are independent host work: spread over threads
      std::vector<std::array<int64_t, 9>> per(own.size());
      parallel_for(own.size(), [&](size_t i) {
        Meta& m = own[i]->meta;
        for (int t = 0; t < 9; ++t) {
          std::vector<int> planes;
          double b;
          int ns;
          if (make_plan(m, kTuneTol[t] * rng, mode, planes, b, ns) != 0) {
            planes.assign(m.streams.size(), 0);
            for (size_t s = 0; s < planes.size(); ++s) planes[s] = m.streams[s].B;
          }
          per[i][t] = plan_bytes(m, planes);
        }
      });
      for (int t = 0; t < 9; ++t) {
        int64_t total = 0;
        for (const auto& p : per) total += p[t];
        sizes[c][t] = total;
      }
    }
    std::vector<int> votes(cands.size(), 0);
    for (int t = 0; t < 9; ++t) {
      size_t best = 0;
      for (size_t c = 1; c < cands.size(); ++c)
        if (sizes[c][t] < sizes[best][t]) best = c;
      ++votes[best];
    }
    winner = 0;
    for (size_t c = 1; c < cands.size(); ++c)
      if (votes[c] > votes[winner]) winner = (int)c;
    return APC_OK;
  };
  std::vector<apc_scheme> cands;
  apc_scheme base{};
  base.degree = 3;
  base.cd_axis = -1;
  if (mode == 0) {
    apc_scheme s = base;
    s.kind = APC_PER_LEVEL;
    for (int j = 0; j < g.d; ++j) s.order[j] = g.d - 1 - j;
    cands.push_back(s);
  }
  int perm[3] = {0, 1, 2};
  do {
    apc_scheme s = base;
    s.kind = APC_PER_REGION;
    for (int j = 0; j < g.d; ++j) s.order[j] = perm[j];
    cands.push_back(s);
  } while (std::next_permutation(perm, perm + g.d));
  int w = 0;
  APC_TRY(vote(cands, w));
  apc_scheme best = cands[w];
  if (g.d >= 2) {
    std::vector<apc_scheme> cc{best};
    for (int a = 0; a < g.d; ++a) {
      apc_scheme s = best;
      s.cd_axis = a;
      cc.push_back(s);
    }
    APC_TRY(vote(cc, w));
    best = cc[w];
  }
  *out = best;
  return APC_OK;
}

}  // namespace

// ------------------------------------------------------------- tile autotuner
// Times the per-level max and quantization passes of every level of at
// least 2^18 points with each tile width on the given field (the codes go
// to a scratch buffer laid out as a handle's) and records the fastest width
// in the table.  The two passes prefer different widths on some shapes, so
// their sum decides.
template <typename T>
apc_status tune_impl(const T* field, int32_t dtype, const Geo& g, int degree, hipStream_t st, int32_t* tile0,
                     double* us0) {
  typedef typename std::conditional<sizeof(T) == 4, int32_t, int64_t>::type Q;
  static const int kWidths[3] = {32, 64, 128};
  std::vector<int64_t> region_off;
  const int64_t code_n = region_layout(g, region_off);
  DevBuf acc, tab, codes;
  APC_TRY(acc.alloc(64));
  HIP_TRY(hipMemsetAsync(acc.p, 0, 64, st));
  APC_TRY(codes.alloc(sizeof(Q) * (size_t)std::max<int64_t>(1, code_n)));
  apc_handle probe;
  probe.geo = g;
  probe.scheme.degree = degree;
  probe.dtype = dtype;
  if (tile0) *tile0 = 0;
  for (int l = 0; l + 1 < g.L; ++l) {
    const int64_t n = (int64_t)g.m[l][0] * g.m[l][1] * g.m[l][2];
    if (n < ((int64_t)1 << 18) || g.m[l][0] == 1) break;  // single-plane levels take one-column tiles
    double best = 1e300;
    int bw = 64;
    for (int k = 0; k < 3; ++k) {
      LevelSeg c = level_seg(&probe, l);
      c.src = field;
      const int64_t sl = (int64_t)1 << l;
      c.xs[0] = sl * g.N[1] * g.N[2];
      c.xs[1] = sl * g.N[2];
      c.xs[2] = sl;
      c.gmax = acc.as<unsigned long long>();
      for (int rho = 0; rho < g.d; ++rho) c.q[rho] = codes.as<Q>() + region_off[l * 3 + rho];
      shape_level_seg(c, kWidths[k]);
      std::vector<LevelSeg> cs{c};
      const int64_t nbk = assign_level_blocks(cs);
      APC_TRY(tab.alloc(sizeof(LevelSeg)));
      HIP_TRY(hipMemcpyAsync(tab.p, cs.data(), sizeof(LevelSeg), hipMemcpyHostToDevice, st));
      hipEvent_t e0, e1;
      HIP_TRY(hipEventCreate(&e0));
      HIP_TRY(hipEventCreate(&e1));
      // warm; the max pass also sets the group maximum the quantization shift is taken from
      HIP_TRY((launch_level<T, Q>((const LevelSeg*)tab.p, 1, nbk, 0, kWidths[k], st)));
      HIP_TRY((launch_level<T, Q>((const LevelSeg*)tab.p, 1, nbk, 1, kWidths[k], st)));
      HIP_TRY(hipEventRecord(e0, st));
      for (int r = 0; r < 3; ++r) {
        HIP_TRY((launch_level<T, Q>((const LevelSeg*)tab.p, 1, nbk, 0, kWidths[k], st)));
        HIP_TRY((launch_level<T, Q>((const LevelSeg*)tab.p, 1, nbk, 1, kWidths[k], st)));
      }
      HIP_TRY(hipEventRecord(e1, st));
      HIP_TRY(hipEventSynchronize(e1));
      float ms = 0.f;
      HIP_TRY(hipEventElapsedTime(&ms, e0, e1));
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      const double us = ms * 1e3 / 3.0;
      if (l == 0 && us0) us0[k] = us;
      // widths come in increasing order and a wider one within 3% of the
      // fastest so far is taken: in a batch, where many fields' tiles share
      // the caches, narrow tiles re-fetch more halo than a single field's
      // timing shows
      if (k == 0 || us < best * 1.03) bw = kWidths[k];
      best = std::min(best, us);
    }
    {
      std::lock_guard<std::mutex> lk(g_tile_mu);
      g_tiles[std::make_tuple((int)dtype, ceil_log2(g.m[l][1]), ceil_log2(g.m[l][2]))] = bw;
    }
    if (l == 0 && tile0) *tile0 = bw;
  }
  return APC_OK;
}

extern "C" apc_status apc_tune_tiles(const void* field_dev, int32_t dtype, const int64_t* dims, int32_t ndim,
                                     int32_t degree, void* hip_stream, int32_t* tile0, double* us0) {
  if (!field_dev || !dims) return fail(APC_E_INVALID, "null argument");
  apc_handle probe;
  apc_scheme def{};
  def.kind = APC_PER_LEVEL;
  def.degree = degree;
  def.cd_axis = -1;
  APC_TRY(setup_geometry(&probe, dims, ndim, &def));
  hipStream_t st = (hipStream_t)hip_stream;
  if (dtype == APC_F32) return tune_impl<float>((const float*)field_dev, dtype, probe.geo, degree, st, tile0, us0);
  if (dtype == APC_F64) return tune_impl<double>((const double*)field_dev, dtype, probe.geo, degree, st, tile0, us0);
  return fail(APC_E_DTYPE, "dtype must be APC_F32 or APC_F64");
}

extern "C" apc_status apc_tile_override(int32_t t2) {
  if (t2 != 0 && t2 != 32 && t2 != 64 && t2 != 128) return fail(APC_E_INVALID, "tile width must be 0, 32, 64 or 128");
  std::lock_guard<std::mutex> lk(g_tile_mu);
  g_tile_override = t2;
  return APC_OK;
}

extern "C" apc_status apc_tile_width(int32_t dtype, int64_t m1, int64_t m2, int32_t* t2) {
  if (!t2) return fail(APC_E_INVALID, "null argument");
  *t2 = tile_for(dtype, (int)m1, (int)m2);
  return APC_OK;
}

extern "C" apc_status apc_select_pipeline(const void* field_dev, int32_t dtype, const int64_t* dims, int32_t ndim,
                                          int32_t mode, apc_scheme* out, void* hip_stream) {
  if (!field_dev || !dims || !out) return fail(APC_E_INVALID, "null argument");
  if (mode != APC_MODE_EB && mode != APC_MODE_PSNR) return fail(APC_E_INVALID, "mode");
  apc_handle probe;
  apc_scheme def{};
  def.kind = APC_PER_LEVEL;
  def.degree = 3;
  def.cd_axis = -1;
  APC_TRY(setup_geometry(&probe, dims, ndim, &def));
  hipStream_t st = (hipStream_t)hip_stream;
  if (dtype == APC_F32) return select_impl<float>((const float*)field_dev, dtype, probe.geo, mode, out, st);
  if (dtype == APC_F64) return select_impl<double>((const double*)field_dev, dtype, probe.geo, mode, out, st);
  return fail(APC_E_DTYPE, "dtype must be APC_F32 or APC_F64");
}

// ------------------------------------------------------------------ serving
// A request loop over resident refactored fields with continuous batching.
// Requests queue in arrival order; whenever one of max_slots slot streams is
// free, the worker thread takes the queued requests (up to max_batch, in
// order, as long as their work buffers fit the HBM budget) as one batch:
//  - the planes the batch needs that no earlier batch decoded are decoded
//    for each field up to the largest plan of the batch on that field, every
//    field in the same launches, on the server's decode stream (decodes are
//    serialized there: each one only adds planes to the resident codes);
//  - on the slot stream, after that decode, the recomposition and
//    reconstruction of every request of the batch run as one set of merged
//    launches, each request reading the resident codes truncated to its own
//    plan into its own work buffers and output.
// Batches on different slots overlap on the device; requests that arrive
// while batches run are admitted into the next one.  A request's output
// therefore depends only on its own plan.  Plans are made at submission, on
// the caller's thread; the worker builds tables without holding the server
// lock and watches its batches' completion events without sleeping.
namespace {

struct SrvRequest {
  int64_t ticket = 0;
  int field = 0;
  void* out = nullptr;
  std::vector<int> planes;
  apc_retrieve_info info{};
  size_t footprint = 0;
  int state = 0;  // 0 pending, 1 running, 2 done, 3 failed
  apc_status status = APC_OK;
  double t_submit = 0, t_start = 0, t_done = 0;
  DevBuf work;
};

struct SrvStaging {  // device table buffer fed from pinned memory
  DevBuf dev;
  PinnedBlock pinned;  // its event follows the last copy out of it
  ~SrvStaging() { g_pinned.put(pinned, nullptr, false); }
  apc_status put(const std::vector<char>& b, hipStream_t st) {
    if (b.empty()) return APC_OK;
    if (pinned.cap < b.size()) {
      g_pinned.put(pinned, nullptr, false);
      if (!g_pinned.get(2 * b.size(), pinned)) return fail(APC_E_OOM, "pinned staging of %zu bytes", b.size());
    } else {
      HIP_TRY(hipEventSynchronize(pinned.ev));
    }
    memcpy(pinned.p, b.data(), b.size());
    if (dev.bytes < b.size()) {
      // the old table may still be read by queued work on this stream: the
      // pool hands it out again only after the device has moved past it
      HIP_TRY(hipStreamSynchronize(st));
      APC_TRY(dev.alloc(2 * b.size()));
    }
    HIP_TRY(hipMemcpyAsync(dev.p, pinned.p, b.size(), hipMemcpyHostToDevice, st));
    HIP_TRY(hipEventRecord(pinned.ev, st));
    return APC_OK;
  }
};

struct SrvSlot {
  hipStream_t st = nullptr;
  hipEvent_t done = nullptr;
  SrvStaging tab;
  std::vector<int64_t> batch;  // tickets of the batch in flight (empty: free)
};

struct SrvField {
  apc_handle* h = nullptr;
  std::vector<int> k_issued;  // planes decoded (or queued for decoding) per stream
};

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

}  // namespace

struct apc_server {
  int device = 0;
  std::vector<std::unique_ptr<SrvField>> fields;
  std::vector<std::unique_ptr<SrvSlot>> slots;
  hipStream_t dec_st = nullptr;
  hipEvent_t dec_ev = nullptr;
  bool has_dec = false;
  SrvStaging dec_tab;
  std::map<int64_t, std::unique_ptr<SrvRequest>> reqs;
  std::deque<int64_t> pending;
  std::vector<double> lat_ms;
  int64_t next_ticket = 1;
  size_t budget = 0, in_use = 0;
  int max_batch = 1;
  int max_queue = 1 << 16;
  int64_t completed = 0, failed = 0, max_running = 0, running = 0;
  std::mutex mu;
  std::condition_variable cv, done_cv;
  std::thread worker;
  bool stop = false;

  // Queue the work of one batch (called without the lock; only the worker
  // touches the fields' decode state and the slots).
  template <typename T, typename Q>
  apc_status start(const std::vector<SrvRequest*>& batch, SrvSlot& sl) {
    // decodes: per field, up to the largest plan of the batch; each request
    // is credited with the planes it adds in arrival order
    std::map<int, std::vector<int>> want;
    for (SrvRequest* r : batch) {
      SrvField& f = *fields[r->field];
      auto it = want.find(r->field);
      if (it == want.end()) it = want.emplace(r->field, f.k_issued).first;
      std::vector<int>& u = it->second;
      r->info.bytes_fetched = fetch_bytes(f.h->meta, u, r->planes);
    }
    std::vector<TableBuilder> dtb(want.size());
    std::vector<std::vector<Launch>> dls(want.size());
    std::vector<LaunchPart> parts;
    size_t i = 0;
    for (auto& kv : want) {
      SrvField& f = *fields[kv.first];
      build_retrieve<T, Q>(f.h, kv.second, nullptr, f.k_issued, dtb[i], dls[i], nullptr, WorkPtrs(), true, false);
      if (!dls[i].empty()) parts.push_back({&dtb[i], &dls[i]});
      ++i;
    }
    if (!parts.empty()) {
      TableBuilder tb;
      std::vector<Launch> ls;
      merge_launches(parts, tb, ls);
      APC_TRY(dec_tab.put(tb.bytes, dec_st));
      APC_TRY((issue<T, Q>(ls, (const char*)dec_tab.dev.p, dec_st)));
      HIP_TRY(hipEventRecord(dec_ev, dec_st));
      has_dec = true;
    }
    // recomposition and reconstruction of every request, merged, on the
    // slot stream after the decode that covers the batch
    if (has_dec) HIP_TRY(hipStreamWaitEvent(sl.st, dec_ev, 0));
    std::vector<TableBuilder> rtb(batch.size());
    std::vector<std::vector<Launch>> rls(batch.size());
    parts.clear();
    for (size_t j = 0; j < batch.size(); ++j) {
      SrvRequest* r = batch[j];
      apc_handle* h = fields[r->field]->h;
      APC_TRY(r->work.alloc(r->footprint));
      const WorkPtrs w = carve_work(h, r->work.p);
      std::vector<int> kdone = fields[r->field]->k_issued;  // no decode in this part
      build_retrieve<T, Q>(h, r->planes, (T*)r->out, kdone, rtb[j], rls[j], nullptr, w, false, true, false,
                           std::max<int64_t>(64, 1024 / (int64_t)batch.size()));
      parts.push_back({&rtb[j], &rls[j]});
    }
    TableBuilder tb;
    std::vector<Launch> ls;
    merge_launches(parts, tb, ls);
    APC_TRY(sl.tab.put(tb.bytes, sl.st));
    APC_TRY((issue<T, Q>(ls, (const char*)sl.tab.dev.p, sl.st)));
    HIP_TRY(hipEventRecord(sl.done, sl.st));
    return APC_OK;
  }

  void finish(SrvRequest& r, double t, bool ok, apc_status s) {
    r.t_done = t;
    r.state = ok ? 2 : 3;
    if (!ok) {
      r.status = s;
      ++failed;
    }
    lat_ms.push_back((r.t_done - r.t_submit) * 1e3);
    ++completed;
    r.work.release();
    in_use -= r.footprint;
    --running;
  }

  void loop() {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    while (!stop) {
      bool busy = false;
      for (auto& slp : slots) {
        SrvSlot& sl = *slp;
        if (sl.batch.empty()) continue;
        const hipError_t q = hipEventQuery(sl.done);
        if (q == hipErrorNotReady) {
          busy = true;
          continue;
        }
        const double t = now_s();
        for (int64_t tk : sl.batch) finish(*reqs[tk], t, q == hipSuccess, APC_E_HIP);
        sl.batch.clear();
        done_cv.notify_all();
      }
      while (!pending.empty()) {
        SrvSlot* free_slot = nullptr;
        for (auto& slp : slots)
          if (slp->batch.empty()) {
            free_slot = slp.get();
            break;
          }
        if (!free_slot) break;
        // the queued requests in arrival order, as many as fit
        std::vector<SrvRequest*> batch;
        size_t fp = 0;
        while (!pending.empty() && (int)batch.size() < max_batch) {
          SrvRequest& r = *reqs[pending.front()];
          if (in_use + fp + r.footprint > budget) break;
          fp += r.footprint;
          batch.push_back(&r);
          pending.pop_front();
        }
        if (batch.empty()) break;  // the head waits for running batches to free memory
        const double t = now_s();
        for (SrvRequest* r : batch) {
          r->state = 1;
          r->t_start = t;
          free_slot->batch.push_back(r->ticket);
        }
        in_use += fp;
        running += (int64_t)batch.size();
        max_running = std::max(max_running, running);
        lk.unlock();
        const bool f32 = fields[batch[0]->field]->h->dtype == APC_F32;
        apc_status st = APC_OK;
        // a batch holds one dtype: split off the requests of the other one
        std::vector<SrvRequest*> same, other;
        for (SrvRequest* r : batch) ((fields[r->field]->h->dtype == APC_F32) == f32 ? same : other).push_back(r);
        st = f32 ? start<float, int32_t>(same, *free_slot) : start<double, int64_t>(same, *free_slot);
        if (st == APC_OK && !other.empty())
          st = f32 ? start<double, int64_t>(other, *free_slot) : start<float, int32_t>(other, *free_slot);
        lk.lock();
        if (st != APC_OK) {
          // nothing of a failed batch is trusted: wait for what was queued, fail every request
          (void)hipStreamSynchronize(free_slot->st);
          (void)hipStreamSynchronize(dec_st);
          const double t2 = now_s();
          for (int64_t tk : free_slot->batch) finish(*reqs[tk], t2, false, st);
          free_slot->batch.clear();
          done_cv.notify_all();
          continue;
        }
        busy = true;
      }
      if (busy) {
        // batches in flight: watch their events without sleeping (a sleep
        // or a blocking wait costs tens of microseconds of latency)
        lk.unlock();
        std::this_thread::yield();
        lk.lock();
      } else {
        cv.wait(lk, [&] { return stop || !pending.empty(); });
      }
    }
  }
};

extern "C" {

apc_status apc_server_create(apc_handle* const* fields, int32_t nfields, int64_t hbm_budget_bytes, int32_t max_slots,
                             int32_t max_batch, apc_server** out) {
  if (!fields || nfields < 1 || max_slots < 1 || max_slots > 64 || max_batch < 1 || max_batch > 1024 ||
      hbm_budget_bytes <= 0 || !out)
    return fail(APC_E_INVALID, "bad argument");
  std::unique_ptr<apc_server> sv(new apc_server());
  HIP_TRY(hipGetDevice(&sv->device));
  sv->budget = (size_t)hbm_budget_bytes;
  sv->max_batch = max_batch;
  for (int f = 0; f < nfields; ++f) {
    if (!fields[f]) return fail(APC_E_INVALID, "null field handle %d", f);
    APC_TRY(need_device(fields[f]));
    sv->fields.emplace_back(new SrvField());
    SrvField& F = *sv->fields.back();
    F.h = fields[f];
    if (F.h->ready) HIP_TRY(hipEventSynchronize(F.h->ready));  // the refactor's last kernels
    APC_TRY(ensure_codes(F.h));
    // both greedy sequences now: later plans only read the metadata, so
    // submissions plan without any lock
    ensure_sequence(F.h->meta, 0);
    ensure_sequence(F.h->meta, 1);
    F.k_issued = F.h->k_res;
  }
  HIP_TRY(hipStreamCreateWithFlags(&sv->dec_st, hipStreamNonBlocking));
  HIP_TRY(hipEventCreateWithFlags(&sv->dec_ev, hipEventDisableTiming));
  for (int i = 0; i < max_slots; ++i) {
    sv->slots.emplace_back(new SrvSlot());
    HIP_TRY(hipStreamCreateWithFlags(&sv->slots.back()->st, hipStreamNonBlocking));
    HIP_TRY(hipEventCreateWithFlags(&sv->slots.back()->done, hipEventDisableTiming));
  }
  HIP_TRY(hipDeviceSynchronize());
  apc_server* raw = sv.get();
  sv->worker = std::thread([raw] { raw->loop(); });
  *out = sv.release();
  return APC_OK;
}

apc_status apc_server_submit(apc_server* sv, int32_t field, const apc_target* target, void* out_dev,
                             int64_t* ticket) {
  if (!sv || !target || !out_dev || !ticket) return fail(APC_E_INVALID, "null argument");
  if (field < 0 || field >= (int32_t)sv->fields.size()) return fail(APC_E_INVALID, "bad field %d", field);
  std::unique_ptr<SrvRequest> r(new SrvRequest());
  r->field = field;
  r->out = out_dev;
  r->t_submit = now_s();
  apc_handle* h = sv->fields[field]->h;
  // read-only on the handle (the greedy sequences exist); other interpreters
  // plan as for a fresh handle (the worker owns the resident planes)
  APC_TRY(plan_for(h, target, r->planes, &r->info, nullptr));
  r->footprint = work_bytes(h);
  if (r->footprint > sv->budget)
    return fail(APC_E_BUSY, "request needs %zu bytes of work buffers, budget is %zu", r->footprint, sv->budget);
  std::lock_guard<std::mutex> lk(sv->mu);
  if ((int)sv->pending.size() >= sv->max_queue) return fail(APC_E_BUSY, "request queue full");
  r->ticket = sv->next_ticket++;
  *ticket = r->ticket;
  sv->pending.push_back(r->ticket);
  sv->reqs[r->ticket] = std::move(r);
  sv->cv.notify_all();
  return APC_OK;
}

apc_status apc_server_wait(apc_server* sv, int64_t ticket, apc_retrieve_info* info) {
  if (!sv) return fail(APC_E_INVALID, "null server");
  std::unique_lock<std::mutex> lk(sv->mu);
  auto it = sv->reqs.find(ticket);
  if (it == sv->reqs.end()) return fail(APC_E_INVALID, "unknown ticket");
  SrvRequest* r = it->second.get();
  sv->done_cv.wait(lk, [&] { return r->state >= 2; });
  const apc_status s = r->status;
  if (info) *info = r->info;
  sv->reqs.erase(it);
  if (s != APC_OK) return fail(s, "request %lld failed", (long long)ticket);
  return APC_OK;
}

apc_status apc_server_poll(apc_server* sv, int64_t ticket, int32_t* done) {
  if (!sv || !done) return fail(APC_E_INVALID, "null argument");
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->reqs.find(ticket);
  if (it == sv->reqs.end()) return fail(APC_E_INVALID, "unknown ticket");
  *done = it->second->state >= 2 ? 1 : 0;
  return APC_OK;
}

apc_status apc_server_stats(apc_server* sv, double* p50_ms, double* p99_ms, double* mean_ms, int64_t* completed,
                            int64_t* max_running) {
  if (!sv) return fail(APC_E_INVALID, "null server");
  std::lock_guard<std::mutex> lk(sv->mu);
  std::vector<double> v = sv->lat_ms;
  std::sort(v.begin(), v.end());
  auto pct = [&](double q) {
    if (v.empty()) return 0.0;
    size_t i = (size_t)std::ceil(q / 100.0 * (double)v.size());
    i = std::min(v.size() - 1, i ? i - 1 : 0);
    return v[i];
  };
  double sum = 0;
  for (double x : v) sum += x;
  if (p50_ms) *p50_ms = pct(50);
  if (p99_ms) *p99_ms = pct(99);
  if (mean_ms) *mean_ms = v.empty() ? 0.0 : sum / (double)v.size();
  if (completed) *completed = sv->completed;
  if (max_running) *max_running = sv->max_running;
  return APC_OK;
}

apc_status apc_server_reset_stats(apc_server* sv) {
  if (!sv) return fail(APC_E_INVALID, "null server");
  std::lock_guard<std::mutex> lk(sv->mu);
  sv->lat_ms.clear();
  sv->completed = 0;
  sv->max_running = sv->running;
  return APC_OK;
}

void apc_server_destroy(apc_server* sv) {
  if (!sv) return;
  {
    std::unique_lock<std::mutex> lk(sv->mu);
    // let queued and running requests finish
    sv->done_cv.wait(lk, [&] {
      if (!sv->pending.empty()) return false;
      for (const auto& s : sv->slots)
        if (!s->batch.empty()) return false;
      return true;
    });
    sv->stop = true;
    sv->cv.notify_all();
  }
  sv->worker.join();
  (void)hipDeviceSynchronize();
  // staging goes back to the pool while the streams its events name exist
  for (auto& s : sv->slots) g_pinned.put(s->tab.pinned, nullptr, false);
  g_pinned.put(sv->dec_tab.pinned, nullptr, false);
  for (auto& s : sv->slots) {
    if (s->done) (void)hipEventDestroy(s->done);
    if (s->st) (void)hipStreamDestroy(s->st);
  }
  if (sv->dec_ev) (void)hipEventDestroy(sv->dec_ev);
  if (sv->dec_st) (void)hipStreamDestroy(sv->dec_st);
  for (auto& f : sv->fields) f->h->k_res = f->k_issued;
  delete sv;
}

}  // extern "C"
