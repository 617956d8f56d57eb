// C ABI and host orchestration of refactor (Algorithm 1) and retrieval
// (Algorithm 2) on one gfx950 device.  Metadata (group maxima, plane
// counts) is computed on the device and read back; planning is host-side.
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <memory>
#include <mutex>
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
  bool on = false;
  std::vector<ProfRec> recs;
  std::vector<hipEvent_t> pool;
  hipEvent_t get() {
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

struct ProfMark {
  int rec = -1;
  hipStream_t st;
  ProfMark(const char* name, double bytes, hipStream_t s) : st(s) {
    if (!g_prof.on) return;
    ProfRec r{name, g_prof.get(), g_prof.get(), bytes};
    (void)hipEventRecord(r.a, st);
    g_prof.recs.push_back(r);
    rec = (int)g_prof.recs.size() - 1;
  }
  void stop() {
    if (rec >= 0) (void)hipEventRecord(g_prof.recs[rec].b, st);
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
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
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

struct apc_handle {
  Meta meta;
  Geo geo;
  apc_scheme scheme{};
  int dtype = APC_F32;
  std::vector<int64_t> region_off;  // (l * 3 + rho) -> offset in the region code buffer
  int64_t code_n = 0;               // codes in the region code buffer
  int64_t cd_n = 0;                 // codes in the decomposition buffer
  std::vector<CDArgs> cd;           // per level-0 region
  // stored representation
  DevBuf mag, idx, sign, pso;
  // retrieval state
  DevBuf codes, cd_codes;
  std::vector<int> k_res;
  DevBuf xc, xb[2], pr[2], cdreg, sd, tmp;
  std::vector<StreamDev> sd_host;   // source of the last decode-table upload
  bool work_ready = false;
};

namespace {

size_t qsize(int dtype) { return dtype == APC_F32 ? 4 : 8; }

apc_status setup_geometry(apc_handle* h, const int64_t* dims, int32_t ndim, const apc_scheme* sc) {
  if (ndim < 1 || ndim > 3) return fail(APC_E_INVALID, "ndim must be 1..3 (got %d)", ndim);
  Geo& g = h->geo;
  g.d = ndim;
  for (int a = 0; a < 3; ++a) g.N[a] = 1;
  for (int a = 0; a < ndim; ++a) {
    if (dims[a] < 1 || dims[a] > (1ll << 30)) return fail(APC_E_INVALID, "dims[%d]=%lld out of range", a, (long long)dims[a]);
    g.N[3 - ndim + a] = dims[a];
  }
  if (g.n() > (1ll << 34)) return fail(APC_E_INVALID, "field too large");
  if (sc->kind != APC_PER_LEVEL && sc->kind != APC_PER_REGION) return fail(APC_E_INVALID, "scheme.kind");
  if (sc->degree != 1 && sc->degree != 3) return fail(APC_E_INVALID, "scheme.degree must be 1 or 3");
  if (sc->cd_axis < -1 || sc->cd_axis >= ndim) return fail(APC_E_INVALID, "scheme.cd_axis out of range");
  if (sc->cd_axis >= 0 && ndim < 2) return fail(APC_E_INVALID, "coefficient decomposition needs 2D or 3D data");
  if (sc->levels < 0 || sc->levels > 40) return fail(APC_E_INVALID, "scheme.levels out of range");
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

// Groups, streams, units and buffer offsets, in unit order.
void build_layout(apc_handle* h, int P, double xmin, double xmax, double A) {
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
  m.xmin = xmin;
  m.xmax = xmax;
  m.A = A;
  h->region_off.assign((size_t)std::max(1, L) * 3, 0);
  int64_t off = 0;
  const int64_t ncoarse = (int64_t)g.m[L - 1][0] * g.m[L - 1][1] * g.m[L - 1][2];
  off += ncoarse;
  for (int l = L - 2; l >= 0; --l)
    for (int rho = 0; rho < d; ++rho) {
      h->region_off[l * 3 + rho] = off;
      off += lat_count(lattice(g, l, rho));
    }
  h->code_n = off;

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
  for (int l = L - 2; l >= 0; --l) {
    const bool use_cd = cd_axis >= 0 && l == 0;
    auto add_cd = [&](int rho, int group) {
      const Lattice lat = lattice(g, 0, rho);
      CDArgs ca{};
      for (int a = 0; a < 3; ++a) ca.c[a] = lat.c[a];
      ca.a = cd_axis + (3 - d);
      int rest[2], nr = 0;
      for (int a = 0; a < 3; ++a)
        if (a != ca.a) rest[nr++] = a;
      ca.u = rest[0];
      ca.v = rest[1];
      std::vector<int> trip;
      for (int t = 0; t < 3; ++t) {
        Stream s;
        s.kind = S_CD;
        s.level = 0;
        s.rho = rho;
        s.t = t + 1;
        s.group = group;
        s.n = (int64_t)ca.c[ca.a] * cls_count_h(t, prefix_h(ca.c[ca.u]), prefix_h(ca.c[ca.v]));
        s.use_cd = true;
        s.code_off = h->cd_n;
        ca.s_off[t] = h->cd_n;
        ca.s_idx[t] = (int)m.streams.size();
        h->cd_n += s.n;
        trip.push_back((int)m.streams.size());
        m.streams.push_back(s);
      }
      h->cd.push_back(ca);
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
        std::vector<std::vector<int>> rs;
        for (int rho = 0; rho < d; ++rho) rs.push_back(add_cd(rho, gi));
        Unit u;  // staircase filled once plane counts are known
        u.group = gi;
        u.stair = true;
        u.seg_steps.clear();
        u.levels.clear();
        // remember the triples in seg_steps[0] temporarily is not needed: rebuilt in finalize
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
}

// Weights of every group (exact chain norms of the user axes).
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

template <typename Q>
RegionArgs region_args(apc_handle* h, int l, int rho, bool per_level, bool with_pr, bool write_pr) {
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
      ra.pr[r] = h->pr[r].as<double>();
    }
  }
  ra.pr_out = (write_pr && rho < g.d - 1) ? h->pr[rho].as<double>() : nullptr;
  return ra;
}

template <typename T, typename Q>
apc_status refactor_impl(apc_handle* h, const T* x, hipStream_t st) {
  Geo& g = h->geo;
  const int d = g.d, L = g.L;
  const int P = sizeof(T) == 4 ? 29 : 52;
  const bool per_level = h->scheme.kind == APC_PER_LEVEL;
  const int64_t n = g.n();

  // grids of levels 1..L-1 (compact copies of the original values)
  std::vector<int64_t> goff(L, 0);
  int64_t gtot = 0;
  for (int l = 1; l < L; ++l) {
    goff[l] = gtot;
    gtot += (int64_t)g.m[l][0] * g.m[l][1] * g.m[l][2];
  }
  DevBuf grids, small, codes, cdc;
  APC_TRY(grids.alloc(sizeof(T) * (size_t)gtot));
  auto grid_ptr = [&](int l) -> const T* { return l == 0 ? x : grids.as<T>() + goff[l]; };
  for (int l = 1; l < L; ++l)
    LAUNCH("subsample", 2.0 * sizeof(T) * g.m[l][0] * g.m[l][1] * g.m[l][2], st,
           launch_subsample<T>(grid_ptr(l - 1), g.m[l - 1].data(), grids.as<T>() + goff[l], g.m[l].data(), st));

  build_layout(h, P, 0, 0, 0);
  Meta& m = h->meta;
  const int ng = (int)m.groups.size(), ns = (int)m.streams.size();
  APC_TRY(small.alloc(8 * (size_t)(4 + ng + ns)));
  unsigned long long* acc = small.as<unsigned long long>();
  unsigned long long* gmax = acc + 4;
  unsigned long long* smax = gmax + ng;
  std::vector<unsigned long long> init(4 + ng + ns, 0ull);
  init[0] = ~0ull;
  HIP_TRY(hipMemcpyAsync(acc, init.data(), 8 * init.size(), hipMemcpyHostToDevice, st));
  LAUNCH("range", (double)sizeof(T) * n, st, launch_range<T>(x, n, acc, st));

  if (per_level && d >= 2) {
    APC_TRY(h->pr[0].alloc(8 * (size_t)lat_count(lattice(g, 0, 0))));
    if (d >= 3) APC_TRY(h->pr[1].alloc(8 * (size_t)lat_count(lattice(g, 0, 1))));
  }
  // group index of (level, region)
  auto group_of = [&](int l, int rho) {
    for (int gi = 0; gi < ng; ++gi) {
      const Group& gr = m.groups[gi];
      if (gr.kind == G_LEVEL && gr.level == l) return gi;
      if (gr.kind == G_REGION && gr.level == l && gr.rho == rho) return gi;
    }
    return 0;
  };
  // pass 1: coefficient maxima
  for (int l = 0; l < L - 1; ++l)
    for (int rho = 0; rho < d; ++rho) {
      RegionArgs ra = region_args<Q>(h, l, rho, per_level, per_level, per_level);
      const double nr = (double)lat_count(ra.lat);
      LAUNCH("coef_max", nr * sizeof(T) + (ra.pr_out ? 8.0 * nr : 0.0), st,
             (launch_coef<T, Q>(grid_ptr(l), ra, 0, gmax + group_of(l, rho), 0, (Q*)nullptr, st)));
    }
  const int64_t ncoarse = m.streams[0].n;
  LAUNCH("coarse", (double)sizeof(T) * ncoarse, st,
         (launch_coarse<T, Q>(grid_ptr(L - 1), ncoarse, 0, gmax + 0, 0, (Q*)nullptr, st)));
  std::vector<unsigned long long> hv(4 + ng);
  HIP_TRY(hipMemcpyAsync(hv.data(), acc, 8 * hv.size(), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (hv[3]) return fail(APC_E_NONFINITE, "field holds NaN or Inf");
  m.xmin = unordered(hv[0]);
  m.xmax = unordered(hv[1]);
  m.A = bits_double(hv[2]);
  for (int gi = 0; gi < ng; ++gi) {
    Group& gr = m.groups[gi];
    gr.M = bits_double(hv[4 + gi]);
    if (gr.M > 0.0) {
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

  // pass 2: quantized codes
  APC_TRY(codes.alloc(sizeof(Q) * (size_t)h->code_n));
  for (int l = 0; l < L - 1; ++l)
    for (int rho = 0; rho < d; ++rho) {
      RegionArgs ra = region_args<Q>(h, l, rho, per_level, per_level, per_level);
      const Group& gr = m.groups[group_of(l, rho)];
      const double nr = (double)lat_count(ra.lat);
      LAUNCH("coef_quant", nr * (sizeof(T) + sizeof(Q)) + (ra.pr_out ? 8.0 * nr : 0.0), st,
             (launch_coef<T, Q>(grid_ptr(l), ra, 1, nullptr, gr.k_shift, codes.as<Q>() + h->region_off[l * 3 + rho], st)));
    }
  LAUNCH("coarse", (double)(sizeof(T) + sizeof(Q)) * ncoarse, st,
         (launch_coarse<T, Q>(grid_ptr(L - 1), ncoarse, 1, nullptr, m.groups[0].k_shift, codes.as<Q>(), st)));
  grids.release();

  // coefficient decomposition of level 0
  if (h->scheme.cd_axis >= 0 && L >= 2) {
    APC_TRY(cdc.alloc(sizeof(Q) * (size_t)std::max<int64_t>(1, h->cd_n)));
    for (int rho = 0; rho < d; ++rho)
      LAUNCH("cd_forward", 2.0 * sizeof(Q) * h->cd[rho].c[0] * h->cd[rho].c[1] * h->cd[rho].c[2], st,
             (launch_cd_forward<Q>(codes.as<Q>() + h->region_off[rho], h->cd[rho], cdc.as<Q>(), smax, st)));
    std::vector<unsigned long long> sv(ns);
    HIP_TRY(hipMemcpyAsync(sv.data(), smax, 8 * ns, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    for (int s = 0; s < ns; ++s)
      if (m.streams[s].use_cd) m.streams[s].maxabs = (int64_t)bits_double(sv[s]);
  }
  for (Stream& s : m.streams) {
    if (!s.use_cd) {
      const Group& gr = m.groups[s.group];
      s.maxabs = gr.M > 0.0 ? (int64_t)rint(ldexp(gr.M, gr.k_shift)) : 0;
    }
    if (s.n == 0) s.maxabs = 0;
    s.B = bitlen(s.maxabs);
  }

  // bitplane encoding: magnitude words, per-chunk counts, staged signs
  int64_t mag_words = 0, idx_n = 0, stage_words = 0, chunks = 0;
  std::vector<StreamDev> sds;
  std::vector<int> sd_stream;
  for (int s = 0; s < ns; ++s) {
    Stream& S = m.streams[s];
    if (S.B == 0 || S.n == 0) continue;
    S.mag_off = mag_words;
    S.idx_off = idx_n;
    StreamDev sd{};
    sd.n = S.n;
    sd.code_off = S.code_off;
    sd.M = S.words();
    sd.C = S.chunks();
    sd.mag_off = mag_words;
    sd.idx_off = idx_n;
    sd.cnt_off = idx_n;
    sd.stage_off = stage_words;
    sd.chunk_begin = chunks;
    sd.B = S.B;
    sd.use_cd = S.use_cd ? 1 : 0;
    mag_words += (int64_t)S.B * sd.M;
    idx_n += (int64_t)S.B * sd.C;
    stage_words += 64 * sd.C;
    chunks += sd.C;
    sds.push_back(sd);
    sd_stream.push_back(s);
  }
  APC_TRY(h->mag.alloc(8 * (size_t)mag_words));
  APC_TRY(h->idx.alloc(4 * (size_t)idx_n));
  DevBuf cnt, stage, sdd, jobs, totals;
  APC_TRY(cnt.alloc(4 * (size_t)idx_n));
  APC_TRY(stage.alloc(8 * (size_t)stage_words));
  APC_TRY(sdd.alloc(sizeof(StreamDev) * std::max<size_t>(1, sds.size())));
  if (!sds.empty()) {
    HIP_TRY(hipMemcpyAsync(sdd.p, sds.data(), sizeof(StreamDev) * sds.size(), hipMemcpyHostToDevice, st));
    double eb = 8.0 * mag_words + 8.0 * stage_words + 4.0 * idx_n;
    for (const StreamDev& sd : sds) eb += (double)sizeof(Q) * sd.n;
    LAUNCH("encode", eb, st,
           (launch_encode<Q>(codes.as<Q>(), cdc.as<Q>(), sdd.as<StreamDev>(), (int)sds.size(), chunks, nullptr, 0,
                             h->mag.as<uint64_t>(), cnt.as<uint32_t>(), stage.as<uint64_t>(), st)));
  }
  std::vector<int32_t> job_s, job_j;
  for (size_t i = 0; i < sds.size(); ++i)
    for (int j = 0; j < sds[i].B; ++j) {
      job_s.push_back((int32_t)i);
      job_j.push_back(j);
    }
  const int njobs = (int)job_s.size();
  APC_TRY(jobs.alloc(8 * (size_t)std::max(1, njobs)));
  APC_TRY(totals.alloc(8 * (size_t)std::max(1, njobs)));
  std::vector<int64_t> tot(njobs);
  if (njobs) {
    HIP_TRY(hipMemcpyAsync(jobs.p, job_s.data(), 4 * njobs, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(jobs.as<int32_t>() + njobs, job_j.data(), 4 * njobs, hipMemcpyHostToDevice, st));
    LAUNCH("scan", 8.0 * idx_n, st, launch_scan(sdd.as<StreamDev>(), jobs.as<int32_t>(), jobs.as<int32_t>() + njobs, njobs,
                        cnt.as<uint32_t>(), h->idx.as<uint32_t>(), totals.as<int64_t>(), st));
    HIP_TRY(hipMemcpyAsync(tot.data(), totals.p, 8 * njobs, hipMemcpyDeviceToHost, st));
  }
  HIP_TRY(hipStreamSynchronize(st));
  // sign sections
  int64_t sign_words = 0;
  std::vector<int64_t> pso_all;
  for (size_t i = 0, jb = 0; i < sds.size(); ++i) {
    Stream& S = m.streams[sd_stream[i]];
    S.nsig.assign(S.B, 0);
    S.pso.assign(S.B, 0);
    S.sign_off = sign_words;
    sds[i].sign_off = sign_words;
    sds[i].psb = (int32_t)pso_all.size();
    int64_t w = 0;
    for (int j = 0; j < S.B; ++j, ++jb) {
      S.nsig[j] = tot[jb];
      S.pso[j] = w;
      pso_all.push_back(w);
      w += (tot[jb] + 63) / 64;
    }
    sign_words += w;
  }
  APC_TRY(h->sign.alloc(8 * (size_t)std::max<int64_t>(1, sign_words)));
  APC_TRY(h->pso.alloc(8 * std::max<size_t>(1, pso_all.size())));
  HIP_TRY(hipMemsetAsync(h->sign.p, 0, 8 * (size_t)std::max<int64_t>(1, sign_words), st));
  if (!pso_all.empty())
    HIP_TRY(hipMemcpyAsync(h->pso.p, pso_all.data(), 8 * pso_all.size(), hipMemcpyHostToDevice, st));
  if (!sds.empty()) {
    HIP_TRY(hipMemcpyAsync(sdd.p, sds.data(), sizeof(StreamDev) * sds.size(), hipMemcpyHostToDevice, st));
    LAUNCH("sign_move", 8.0 * (stage_words + sign_words), st, launch_sign_move(sdd.as<StreamDev>(), (int)sds.size(), chunks, cnt.as<uint32_t>(), h->idx.as<uint32_t>(),
                             h->pso.as<int64_t>(), stage.as<uint64_t>(), h->sign.as<uint64_t>(), st));
  }
  HIP_TRY(hipStreamSynchronize(st));
  assign_weights(h);
  finalize_units(h);
  h->k_res.assign(ns, 0);
  return APC_OK;
}

apc_status ensure_work(apc_handle* h) {
  if (h->work_ready) return APC_OK;
  const Geo& g = h->geo;
  const size_t qs = qsize(h->dtype);
  APC_TRY(h->codes.alloc(qs * (size_t)std::max<int64_t>(1, h->code_n)));
  APC_TRY(h->cd_codes.alloc(qs * (size_t)std::max<int64_t>(1, h->cd_n)));
  const int L = g.L;
  const int64_t nc = (int64_t)g.m[L - 1][0] * g.m[L - 1][1] * g.m[L - 1][2];
  APC_TRY(h->xc.alloc(8 * (size_t)nc));
  if (L >= 2) {
    const int64_t n1 = (int64_t)g.m[std::min(1, L - 1)][0] * g.m[std::min(1, L - 1)][1] * g.m[std::min(1, L - 1)][2];
    APC_TRY(h->xb[0].alloc(8 * (size_t)n1));
    APC_TRY(h->xb[1].alloc(8 * (size_t)n1));
    if (g.d >= 2) APC_TRY(h->pr[0].alloc(8 * (size_t)lat_count(lattice(g, 0, 0))));
    if (g.d >= 3) APC_TRY(h->pr[1].alloc(8 * (size_t)lat_count(lattice(g, 0, 1))));
    if (h->scheme.cd_axis >= 0) {
      int64_t mx = 0;
      for (int rho = 0; rho < g.d; ++rho) mx = std::max(mx, lat_count(lattice(g, 0, rho)));
      APC_TRY(h->cdreg.alloc(qs * (size_t)std::max<int64_t>(1, mx)));
    }
  }
  APC_TRY(h->sd.alloc(sizeof(StreamDev) * std::max<size_t>(1, h->meta.streams.size())));
  h->work_ready = true;
  return APC_OK;
}

template <typename T, typename Q>
apc_status retrieve_impl(apc_handle* h, const std::vector<int>& planes, T* out, hipStream_t st, int64_t* fetched) {
  APC_TRY(ensure_work(h));
  Meta& m = h->meta;
  const Geo& g = h->geo;
  const int d = g.d, L = g.L;
  const bool per_level = h->scheme.kind == APC_PER_LEVEL;
  // incremental decode of the planes not resident yet
  std::vector<StreamDev>& sds = h->sd_host;
  sds.clear();
  int64_t chunks = 0, fb = 0;
  double db = 0.0;
  for (int s = 0; s < (int)m.streams.size(); ++s) {
    const Stream& S = m.streams[s];
    if (S.B == 0 || S.n == 0 || planes[s] <= h->k_res[s]) continue;
    StreamDev sd{};
    sd.n = S.n;
    sd.code_off = S.code_off;
    sd.M = S.words();
    sd.C = S.chunks();
    sd.mag_off = S.mag_off;
    sd.idx_off = S.idx_off;
    sd.sign_off = S.sign_off;
    sd.sign_n = S.sign_words();
    sd.chunk_begin = chunks;
    sd.B = S.B;
    sd.use_cd = S.use_cd ? 1 : 0;
    sd.k0 = h->k_res[s];
    sd.k1 = planes[s];
    sd.fresh = h->k_res[s] == 0 ? 1 : 0;
    int psb = 0;
    for (int s2 = 0; s2 < s; ++s2) psb += m.streams[s2].n > 0 ? m.streams[s2].B : 0;
    sd.psb = psb;
    for (int j = sd.k0; j < sd.k1; ++j) {
      fb += S.plane_bytes(j);
      db += 8.0 * ((S.nsig[j] + 63) / 64);
    }
    db += (double)(sd.k1 - sd.k0) * (8.0 * sd.M + 4.0 * sd.C) + (double)sizeof(Q) * S.n * (sd.fresh ? 1 : 2);
    chunks += sd.C;
    sds.push_back(sd);
    h->k_res[s] = planes[s];
  }
  if (fetched) *fetched = fb;
  if (!sds.empty()) {
    HIP_TRY(hipMemcpyAsync(h->sd.p, sds.data(), sizeof(StreamDev) * sds.size(), hipMemcpyHostToDevice, st));
    LAUNCH("decode", db, st, (launch_decode<Q>(h->sd.as<StreamDev>(), (int)sds.size(), chunks, h->mag.as<uint64_t>(),
                              h->idx.as<uint32_t>(), h->sign.as<uint64_t>(), h->pso.as<int64_t>(), h->codes.as<Q>(),
                              h->cd_codes.as<Q>(), st)));
  }
  // coarsest level
  const Stream& s0 = m.streams[0];
  const Group& g0 = m.groups[s0.group];
  double* xc = h->xc.as<double>();
  LAUNCH("coarsest", (8.0 + sizeof(Q)) * s0.n, st, (launch_coarsest_q<Q>(h->codes.as<Q>(), s0.n, s0.B, planes[0], g0.delta, xc, st)));
  if (L == 1) {
    LAUNCH("cast", (8.0 + sizeof(T)) * s0.n, st, launch_cast<T>(xc, s0.n, out, st));
    return APC_OK;
  }
  // stream of each (level, region)
  auto stream_of = [&](int l, int rho) {
    for (int s = 0; s < (int)m.streams.size(); ++s) {
      const Stream& S = m.streams[s];
      if (S.kind == S_LEVEL && S.level == l) return s;
      if (S.kind == S_REGION && S.level == l && S.rho == rho) return s;
    }
    return -1;
  };
  const double* xin = xc;
  for (int l = L - 2; l >= 0; --l) {
    double* xout = l > 0 ? h->xb[l % 2].as<double>() : nullptr;
    const int32_t* cm = g.m[l + 1].data();
    if (l > 0)
      LAUNCH("inject", 16.0 * cm[0] * cm[1] * cm[2], st, launch_inject<double>(xin, cm, xout, g.m[l].data(), st));
    else
      LAUNCH("inject", (8.0 + sizeof(T)) * cm[0] * cm[1] * cm[2], st, launch_inject<T>(xin, cm, out, g.m[0].data(), st));
    for (int rho = 0; rho < d; ++rho) {
      RegionArgs ra = region_args<Q>(h, l, rho, per_level, true, true);
      const Q* q;
      int B, k;
      double delta;
      if (l == 0 && h->scheme.cd_axis >= 0) {
        CDArgs ca = h->cd[rho];
        for (int t = 0; t < 3; ++t) {
          const Stream& S = m.streams[ca.s_idx[t]];
          ca.B[t] = S.B;
          ca.k[t] = planes[ca.s_idx[t]];
        }
        LAUNCH("cd_inverse", 2.0 * sizeof(Q) * ca.c[0] * ca.c[1] * ca.c[2], st,
               (launch_cd_inverse<Q>(h->cd_codes.as<Q>(), ca, h->cdreg.as<Q>(), st)));
        q = h->cdreg.as<Q>();
        B = 64;
        k = 64;
        delta = m.groups[m.streams[ca.s_idx[0]].group].delta;
      } else {
        const int s = stream_of(l, rho);
        const Stream& S = m.streams[s];
        q = h->codes.as<Q>() + h->region_off[l * 3 + rho];
        B = S.B;
        k = planes[s];
        delta = m.groups[S.group].delta;
      }
      if (l > 0)
        LAUNCH("recon", (double)lat_count(ra.lat) * (sizeof(Q) + 8 + (ra.pr_out ? 8 : 0)), st,
               (launch_recon<double, Q>(xin, cm, ra, q, B, k, delta, xout, st)));
      else
        LAUNCH("recon", (double)lat_count(ra.lat) * (sizeof(Q) + sizeof(T) + (ra.pr_out ? 8 : 0)), st,
               (launch_recon<T, Q>(xin, cm, ra, q, B, k, delta, out, st)));
    }
    xin = xout;
  }
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

}  // namespace

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
  if (dtype != APC_F32 && dtype != APC_F64) return fail(APC_E_DTYPE, "dtype must be APC_F32 or APC_F64");
  std::unique_ptr<apc_handle> h(new apc_handle());
  h->dtype = dtype;
  APC_TRY(setup_geometry(h.get(), dims, ndim, scheme));
  hipStream_t st = (hipStream_t)hip_stream;
  apc_status s = dtype == APC_F32 ? refactor_impl<float, int32_t>(h.get(), (const float*)field_dev, st)
                                  : refactor_impl<double, int64_t>(h.get(), (const double*)field_dev, st);
  if (s != APC_OK) return s;
  *out = h.release();
  return APC_OK;
}

apc_status apc_plan(apc_handle* h, const apc_target* target, int32_t* planes_out, apc_retrieve_info* info) {
  if (!h || !target) return fail(APC_E_INVALID, "null argument");
  double tau;
  int mode;
  APC_TRY(target_tau(h, target, tau, mode));
  std::vector<int> planes;
  double b;
  int nsteps;
  if (make_plan(h->meta, tau, mode, planes, b, nsteps) != 0)
    return fail(APC_E_BELOW_FLOOR, "tolerance %.17g is below the floor of this representation", tau);
  if (planes_out)
    for (size_t s = 0; s < planes.size(); ++s) planes_out[s] = planes[s];
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

static apc_status do_retrieve(apc_handle* h, const std::vector<int>& planes, void* out_dev, void* hip_stream,
                              int64_t* fetched) {
  hipStream_t st = (hipStream_t)hip_stream;
  if (h->dtype == APC_F32) return retrieve_impl<float, int32_t>(h, planes, (float*)out_dev, st, fetched);
  return retrieve_impl<double, int64_t>(h, planes, (double*)out_dev, st, fetched);
}

apc_status apc_retrieve(apc_handle* h, const apc_target* target, void* out_dev, apc_retrieve_info* info,
                        void* hip_stream) {
  if (!h || !target || !out_dev) return fail(APC_E_INVALID, "null argument");
  std::vector<int32_t> planes(h->meta.streams.size());
  apc_retrieve_info inf{};
  APC_TRY(apc_plan(h, target, planes.data(), &inf));
  std::vector<int> p(planes.begin(), planes.end());
  int64_t fetched = 0;
  APC_TRY(do_retrieve(h, p, out_dev, hip_stream, &fetched));
  inf.bytes_fetched = fetched;
  if (info) *info = inf;
  return APC_OK;
}

apc_status apc_retrieve_planes(apc_handle* h, const int32_t* planes, void* out_dev, void* hip_stream) {
  if (!h || !planes || !out_dev) return fail(APC_E_INVALID, "null argument");
  std::vector<int> p(h->meta.streams.size());
  for (size_t s = 0; s < p.size(); ++s) p[s] = std::max(0, std::min<int>(planes[s], h->meta.streams[s].B));
  return do_retrieve(h, p, out_dev, hip_stream, nullptr);
}

void apc_free(apc_handle* h) {
  if (!h) return;
  // Work queued on any stream may still read this handle's buffers; they go
  // back to the shared pool only once the device is idle.
  (void)hipDeviceSynchronize();
  delete h;
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
  const Stream& S = h->meta.streams[s];
  if (cap < S.blob_bytes()) return fail(APC_E_INVALID, "buffer too small");
  char* dst = (char*)host_dst;
  memset(dst, 0, (size_t)S.blob_bytes());
  if (S.B == 0 || S.n == 0) return APC_OK;
  const int64_t ib = 4 * (int64_t)S.B * S.chunks();
  HIP_TRY(hipMemcpy(dst, h->idx.as<uint32_t>() + S.idx_off, (size_t)ib, hipMemcpyDeviceToHost));
  const int64_t ibp = ib + (8 - ib % 8) % 8;
  const int64_t mb = 8 * (int64_t)S.B * S.words();
  HIP_TRY(hipMemcpy(dst + ibp, h->mag.as<uint64_t>() + S.mag_off, (size_t)mb, hipMemcpyDeviceToHost));
  const int64_t sb = 8 * S.sign_words();
  if (sb) HIP_TRY(hipMemcpy(dst + ibp + mb, h->sign.as<uint64_t>() + S.sign_off, (size_t)sb, hipMemcpyDeviceToHost));
  return APC_OK;
}

apc_status apc_metadata_json(const apc_handle* h, char* buf, int64_t cap, int64_t* len) {
  if (!h) return fail(APC_E_INVALID, "null handle");
  const std::string js = meta_json(h->meta);
  if (len) *len = (int64_t)js.size();
  if (buf) {
    if (cap < (int64_t)js.size() + 1) return fail(APC_E_INVALID, "buffer too small");
    memcpy(buf, js.c_str(), js.size() + 1);
  }
  return APC_OK;
}

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

apc_status apc_profile_report(char* buf, int64_t cap, int64_t* len) {
  // Per kernel name: launches, total milliseconds, total bytes moved.
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
    snprintf(tmp, sizeof(tmp), "%s\"%s\":{\"count\":%lld,\"ms\":%.6f,\"bytes\":%.0f}", k ? "," : "", names[k].c_str(),
             (long long)count[k], ms[k], bytes[k]);
    js += tmp;
  }
  js += "}";
  if (len) *len = (int64_t)js.size();
  if (buf) {
    if (cap < (int64_t)js.size() + 1) return fail(APC_E_INVALID, "buffer too small");
    memcpy(buf, js.c_str(), js.size() + 1);
  }
  return APC_OK;
}

apc_status apc_select_pipeline(const void*, int32_t, const int64_t*, int32_t, int32_t, apc_scheme*, void*) {
  return fail(APC_E_INVALID, "select_pipeline is not available yet");
}

}  // extern "C"
