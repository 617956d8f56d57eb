// Error weights, max ordering and the greedy retrieval interpreter
// (Section V-C; Algorithm 2 "RetrievalInterpreter"), host side.  Float
// expressions are written in the same order as their definitions so that
// plans are reproducible bit for bit.
#include <math.h>
#include <stdio.h>

#include <algorithm>
#include <array>
#include <map>
#include <mutex>

#include "host.h"

namespace apc {

namespace {

int stencil_kind(int j, int m, int degree) {
  if (j + 1 > m - 1) return 0;           // copy
  if (degree == 1) return 1;             // linear
  const bool left = j - 3 >= 0, right = j + 3 <= m - 1;
  if (left && right) return 4;           // cubic
  if (right) return 2;                   // quadratic, missing left neighbour
  if (left) return 3;                    // quadratic, missing right neighbour
  return 1;
}

int64_t compact_len(int64_t n, int l) { return (n - 1) / ((int64_t)1 << l) + 1; }

double to_double_scaled(__int128 num, int shift4) {
  // num / 16^shift4, rounded once: the integer conversion rounds to nearest
  // even and the power-of-two scaling is exact.
  return ldexp((double)num, -4 * shift4);
}

}  // namespace

// Exact norms of the 1D interpolation chain from level l to level 0 on an
// axis of n points.  Every weight is a multiple of 1/16, so each coarse unit
// vector is prolonged level by level in integers scaled by 16 per level; its
// support only grows by a few points per level.
static void axis_norms_exact(int64_t n, int L, int degree, std::vector<double>& inf, std::vector<double>& one) {
  inf.assign(L, 1.0);
  one.assign(L, 1.0);
  std::vector<__int128> rows(n), cur, nxt;
  for (int l = 1; l < L; ++l) {
    std::fill(rows.begin(), rows.end(), (__int128)0);
    __int128 colmax = 0;
    const int64_t m_l = compact_len(n, l);
    for (int64_t k = 0; k < m_l; ++k) {
      // cur holds values on level j for indices [lo, hi]
      int64_t lo = k, hi = k;
      cur.assign(1, 1);
      for (int j = l - 1; j >= 0; --j) {
        const int64_t mf = compact_len(n, j);
        const int64_t nlo = std::max<int64_t>(0, 2 * lo - 3), nhi = std::min<int64_t>(mf - 1, 2 * hi + 3);
        nxt.assign((size_t)(nhi - nlo + 1), 0);
        auto cv = [&](int64_t c) -> __int128 { return (c >= lo && c <= hi) ? cur[(size_t)(c - lo)] : 0; };
        for (int64_t i = nlo; i <= nhi; ++i) {
          __int128 v;
          if ((i & 1) == 0) {
            v = 16 * cv(i / 2);
          } else {
            switch (stencil_kind((int)i, (int)mf, degree)) {
              case 4: v = -cv((i - 3) / 2) + 9 * cv((i - 1) / 2) + 9 * cv((i + 1) / 2) - cv((i + 3) / 2); break;
              case 2: v = 6 * cv((i - 1) / 2) + 12 * cv((i + 1) / 2) - 2 * cv((i + 3) / 2); break;
              case 3: v = -2 * cv((i - 3) / 2) + 12 * cv((i - 1) / 2) + 6 * cv((i + 1) / 2); break;
              case 1: v = 8 * cv((i - 1) / 2) + 8 * cv((i + 1) / 2); break;
              default: v = 16 * cv((i - 1) / 2); break;
            }
          }
          nxt[(size_t)(i - nlo)] = v;
        }
        cur.swap(nxt);
        lo = nlo;
        hi = nhi;
      }
      __int128 cs = 0;
      for (int64_t r = lo; r <= hi; ++r) {
        const __int128 v = cur[(size_t)(r - lo)] < 0 ? -cur[(size_t)(r - lo)] : cur[(size_t)(r - lo)];
        cs += v;
        rows[r] += v;
      }
      colmax = std::max(colmax, cs);
    }
    __int128 rowmax = 0;
    for (int64_t r = 0; r < n; ++r) rowmax = std::max(rowmax, rows[r]);
    inf[l] = to_double_scaled(rowmax, l);
    one[l] = to_double_scaled(colmax, l);
  }
}

// The norms depend only on (n, L, degree) and every refactor of a field
// needs them for each axis: they are computed once per shape and kept.
void axis_norms(int64_t n, int L, int degree, std::vector<double>& inf, std::vector<double>& one) {
  static std::mutex mu;
  static std::map<std::array<int64_t, 3>, std::pair<std::vector<double>, std::vector<double>>> memo;
  const std::array<int64_t, 3> key = {n, (int64_t)L, (int64_t)degree};
  {
    std::lock_guard<std::mutex> lk(mu);
    auto it = memo.find(key);
    if (it != memo.end()) {
      inf = it->second.first;
      one = it->second.second;
      return;
    }
  }
  axis_norms_exact(n, L, degree, inf, one);
  std::lock_guard<std::mutex> lk(mu);
  if (memo.size() < 4096) memo[key] = {inf, one};
}

// The first step count after k whose error is below err(k) (n at most):
// steps that do not lower the error (the first digit planes of a negabinary
// stream) are taken together with the step that does.
template <typename F>
static int next_lower(F err, int k, int n) {
  int k2 = k + 1;
  while (k2 < n && err(k2) >= err(k)) ++k2;
  return k2;
}

Unit build_staircase(int group, const std::vector<std::vector<int>>& rs, const std::vector<Stream>& st) {
  const int R = (int)rs.size();
  std::vector<std::vector<std::pair<int, int>>> orders(R);  // (stream t, planes taken together)
  for (int r = 0; r < R; ++r) {
    int k[3] = {0, 0, 0};
    for (;;) {
      int best = -1, best_n = 0;
      double best_r = -1.0;
      for (int t = 0; t < 3; ++t) {
        const Stream& s = st[rs[r][t]];
        if (k[t] < s.B) {
          const int k2 = next_lower([&](int kk) { return s.delta(kk); }, k[t], s.B);
          const int64_t gain = s.delta(k[t]) - s.delta(k2);
          int64_t nb = 0;
          for (int j = k[t]; j < k2; ++j) nb += s.plane_bytes(j);
          const double q = (double)gain / (double)nb;
          if (q > best_r) {
            best = t;
            best_r = q;
            best_n = k2 - k[t];
          }
        }
      }
      if (best < 0) break;
      orders[r].push_back({best, best_n});
      k[best] += best_n;
    }
  }
  std::vector<int> pos(R, 0);
  std::vector<std::array<int, 3>> kk(R, {0, 0, 0});
  auto err = [&](int r) {
    int64_t s = 0;
    for (int t = 0; t < 3; ++t) s += st[rs[r][t]].delta(kk[r][t]);
    return s;
  };
  std::vector<int64_t> e(R);
  int64_t top = 0;
  for (int r = 0; r < R; ++r) {
    e[r] = err(r);
    top = std::max(top, e[r]);
  }
  Unit u;
  u.group = group;
  u.stair = true;
  u.levels.push_back(top);
  while (u.levels.back() > 0) {
    const int64_t cur = u.levels.back();
    int64_t nb = 0;
    std::vector<std::pair<int, int>> steps;
    for (int r = 0; r < R; ++r) {
      if (e[r] == cur) {
        const int t = orders[r][pos[r]].first, cnt = orders[r][pos[r]].second;
        ++pos[r];
        const int s = rs[r][t];
        for (int c = 0; c < cnt; ++c) {
          nb += st[s].plane_bytes(kk[r][t]);
          steps.push_back({s, kk[r][t]});
          ++kk[r][t];
        }
        e[r] = err(r);
      }
    }
    int64_t nt = 0;
    for (int r = 0; r < R; ++r) nt = std::max(nt, e[r]);
    u.levels.push_back(nt);
    u.seg_bytes.push_back(nb);
    u.seg_steps.push_back(steps);
  }
  return u;
}

int unit_nsteps(const Meta& m, const Unit& u) {
  return u.stair ? (int)u.seg_bytes.size() : m.streams[u.stream].B;
}

int64_t unit_err(const Meta& m, const Unit& u, int k) {
  return u.stair ? u.levels[k] : m.streams[u.stream].delta(k);
}

static int64_t unit_step_bytes(const Meta& m, const Unit& u, int k) {
  return u.stair ? u.seg_bytes[k] : m.streams[u.stream].plane_bytes(k);
}

static int64_t group_error(const Meta& m, int g, const std::vector<int>& state) {
  const std::vector<int>& us = m.group_units[g];
  if (us.size() == 1) return unit_err(m, m.units[us[0]], state[us[0]]);
  int64_t s = 0;
  for (int u : us) s += unit_err(m, m.units[u], state[u]);
  return s;
}

double bound(const Meta& m, const std::vector<int>& state, int mode) {
  double E = 0.0;
  for (int g : m.group_order) {
    const Group& gr = m.groups[g];
    const double wd = mode == 0 ? gr.wd_inf : gr.wd_2;
    E = E + wd * (0.5 + (double)group_error(m, g, state));
  }
  return E + m.eps_fp;
}

void finalize_meta(Meta& m) {
  m.group_units.assign(m.groups.size(), {});
  m.group_order.clear();
  for (int u = 0; u < (int)m.units.size(); ++u) {
    const int g = m.units[u].group;
    if (m.group_units[g].empty()) m.group_order.push_back(g);
    m.group_units[g].push_back(u);
  }
  std::vector<int> zero(m.units.size(), 0);
  double e0 = 0.0, W = 0.0;
  for (int g : m.group_order) {
    const Group& gr = m.groups[g];
    e0 = e0 + gr.wd_inf * (0.5 + (double)group_error(m, g, zero));
    W = W + gr.w;
  }
  const double Ap = m.A + e0;
  const double u_out = m.P == 29 ? ldexp(1.0, -24) : ldexp(1.0, -53);
  m.eps_fp = u_out * Ap + (ldexp(1.0, -40) * W) * Ap;
  int64_t nseg = 0, sumB = 0;
  for (const Unit& u : m.units)
    if (u.stair) nseg += (int64_t)u.seg_bytes.size();
  for (const Stream& s : m.streams) sumB += s.B;
  // with the lossless stage every plane also records its nonzero word count
  m.meta_bytes = 64 + 16 * (int64_t)m.groups.size() + 16 * (int64_t)m.streams.size() + (m.lossless ? 8 : 4) * sumB +
                 8 * nseg;
  m.seq_ready[0] = m.seq_ready[1] = false;
}

void ensure_sequence(Meta& m, int mode) {
  if (m.seq_ready[mode]) return;
  const int nu = (int)m.units.size();
  std::vector<int> state(nu, 0);
  m.seq[mode].clear();
  m.seq_E0[mode] = bound(m, state, mode);
  // a unit's score and next step depend only on its own state: kept per
  // unit and recomputed for the unit that advances (the same choices, in
  // the same order, as recomputing every unit at every step)
  std::vector<double> score(nu, -1.0);
  std::vector<int> next_k(nu, 0);
  auto rescore = [&](int u) {
    const Unit& un = m.units[u];
    const int n = unit_nsteps(m, un);
    if (state[u] >= n) {
      score[u] = -1.0;
      return;
    }
    const Group& gr = m.groups[un.group];
    const double wd = mode == 0 ? gr.wd_inf : gr.wd_2;
    const int k = state[u];
    const int k2 = next_lower([&](int kk) { return unit_err(m, un, kk); }, k, n);
    const int64_t de = unit_err(m, un, k) - unit_err(m, un, k2);
    int64_t c = 0;
    for (int j = k; j < k2; ++j) c += unit_step_bytes(m, un, j);
    score[u] = (wd * (double)de) / (double)c;
    next_k[u] = k2;
  };
  std::vector<bool> live(nu, false);
  for (int u = 0; u < nu; ++u) {
    live[u] = state[u] < unit_nsteps(m, m.units[u]);
    if (live[u]) rescore(u);
  }
  for (;;) {
    int best = -1;
    double best_s = -1.0;
    for (int u = 0; u < nu; ++u)
      if (live[u] && score[u] > best_s) {
        best = u;
        best_s = score[u];
      }
    if (best < 0) break;
    state[best] = next_k[best];
    m.seq[mode].push_back({best, next_k[best], bound(m, state, mode)});
    live[best] = state[best] < unit_nsteps(m, m.units[best]);
    if (live[best]) rescore(best);
  }
  m.seq_ready[mode] = true;
}

int make_plan(Meta& m, double tau, int mode, std::vector<int>& planes, double& bound_out, int& nsteps) {
  if (!(tau > 0.0)) return -1;
  ensure_sequence(m, mode);
  std::vector<int> state(m.units.size(), 0);
  double E = m.seq_E0[mode];
  int n = 0;
  while (E > tau) {
    if (n == (int)m.seq[mode].size()) return -1;
    const Meta::SeqStep& st = m.seq[mode][n];
    state[st.unit] = st.k;
    E = st.E;
    ++n;
  }
  planes.assign(m.streams.size(), 0);
  for (int u = 0; u < (int)m.units.size(); ++u) {
    const Unit& un = m.units[u];
    if (!un.stair) {
      planes[un.stream] = state[u];
    } else {
      for (int j = 0; j < state[u]; ++j)
        for (const auto& sp : un.seg_steps[j]) planes[sp.first] = std::max(planes[sp.first], sp.second + 1);
    }
  }
  bound_out = E;
  nsteps = n;
  return 0;
}

int64_t plan_bytes(const Meta& m, const std::vector<int>& planes) {
  int64_t total = m.meta_bytes;
  for (size_t s = 0; s < m.streams.size(); ++s)
    for (int j = 0; j < planes[s]; ++j) total += m.streams[s].plane_bytes(j);
  return total;
}

// ------------------------------------------------------------------
// The paper's interpreters (Section V-C; Algorithm 2): dynamic programming
// for per-region interpolation, best-first search for per-level
// interpolation with decomposition.  Both minimise the bytes a retrieval
// fetches beyond the resident planes (incremental invocation) subject to the
// model bound <= tau, and fall back to the greedy plan when it fetches no
// more.  The arithmetic follows the definitions step by step in a fixed
// order, so plans are reproducible bit for bit.
namespace {

constexpr int kDPParts = 2048;
constexpr int kDPRetries = 8;
constexpr int64_t kInf = INT64_MAX / 4;

double wd_of(const Group& g, int mode) { return mode == 0 ? g.wd_inf : g.wd_2; }

std::vector<int> resident_steps(const Meta& m, const std::vector<int>* res) {
  std::vector<int> out(m.units.size(), 0);
  if (!res) return out;
  for (size_t u = 0; u < m.units.size(); ++u) {
    const Unit& un = m.units[u];
    if (!un.stair) {
      out[u] = std::min(m.streams[un.stream].B, (*res)[un.stream]);
    } else {
      int s = 0;
      while (s < (int)un.seg_steps.size()) {
        bool all = true;
        for (const auto& sp : un.seg_steps[s]) all = all && sp.second < (*res)[sp.first];
        if (!all) break;
        ++s;
      }
      out[u] = s;
    }
  }
  return out;
}

int64_t step_cost(const Meta& m, int u, int k, const std::vector<int>* res) {
  const Unit& un = m.units[u];
  if (!un.stair) {
    if (res && k < (*res)[un.stream]) return 0;
    return m.streams[un.stream].plane_bytes(k);
  }
  int64_t total = 0;
  for (const auto& sp : un.seg_steps[k])
    if (!res || sp.second >= (*res)[sp.first]) total += m.streams[sp.first].plane_bytes(sp.second);
  return total;
}

int64_t extra_bytes(const Meta& m, const std::vector<int>& planes, const std::vector<int>* res) {
  int64_t total = 0;
  for (size_t s = 0; s < m.streams.size(); ++s)
    for (int j = res ? (*res)[s] : 0; j < planes[s]; ++j) total += m.streams[s].plane_bytes(j);
  return total;
}

std::vector<int> stream_planes(const Meta& m, const std::vector<int>& state) {
  std::vector<int> planes(m.streams.size(), 0);
  for (size_t u = 0; u < m.units.size(); ++u) {
    const Unit& un = m.units[u];
    if (!un.stair) {
      planes[un.stream] = state[u];
    } else {
      for (int j = 0; j < state[u]; ++j)
        for (const auto& sp : un.seg_steps[j]) planes[sp.first] = std::max(planes[sp.first], sp.second + 1);
    }
  }
  return planes;
}

// The model's bound for any per-stream plane vector: a staircase group takes
// the largest summed stream error of its regions.
double bound_for_planes(const Meta& m, const std::vector<int>& k, int mode) {
  double E = 0.0;
  for (int g : m.group_order) {
    const Group& gr = m.groups[g];
    const std::vector<int>& us = m.group_units[g];
    int64_t e = 0;
    if (us.size() == 1 && m.units[us[0]].stair) {
      std::map<int, int64_t> per;
      for (size_t s = 0; s < m.streams.size(); ++s)
        if (m.streams[s].group == g) per[m.streams[s].rho] += m.streams[s].delta(k[s]);
      for (const auto& kv : per) e = std::max(e, kv.second);
    } else {
      for (int u : us) e += m.streams[m.units[u].stream].delta(k[m.units[u].stream]);
    }
    E = E + wd_of(gr, mode) * (0.5 + (double)e);
  }
  return E + m.eps_fp;
}

struct PlanOut {
  std::vector<int> planes;
  double bound = 0.0;
  int nsteps = 0;
};

PlanOut as_plan(const Meta& m, std::vector<int> planes, int nsteps, int mode, const std::vector<int>* res) {
  if (res)
    for (size_t s = 0; s < planes.size(); ++s) planes[s] = std::max(planes[s], (*res)[s]);
  PlanOut p;
  p.bound = bound_for_planes(m, planes, mode);
  p.planes = std::move(planes);
  p.nsteps = nsteps;
  return p;
}

double budget(const Meta& m, double tau, int mode) {
  double c = m.eps_fp;
  for (int g : m.group_order) c = c + wd_of(m.groups[g], mode) * 0.5;
  return tau - c;
}

// Fewest bytes over `units`, their error terms rounded up to parts of
// R / kDPParts, summing to at most R; false when no choice fits.
bool dp_solve(const Meta& m, int mode, const std::vector<int>& units, double R, const std::vector<int>& k0,
              const std::vector<int>* res, int64_t& bytes, std::vector<int>& state) {
  if (!(R > 0.0)) return false;
  const int P = kDPParts;
  const double q = R / P;
  std::vector<int64_t> dp(P + 1, 0), nd(P + 1);
  std::vector<std::vector<int>> ch(units.size(), std::vector<int>(P + 1, -1));
  std::vector<std::vector<int64_t>> parts_of(units.size());
  for (size_t i = 0; i < units.size(); ++i) {
    const int u = units[i];
    const Unit& un = m.units[u];
    const double wd = wd_of(m.groups[un.group], mode);
    const int n = unit_nsteps(m, un);
    std::fill(nd.begin(), nd.end(), kInf);
    parts_of[i].assign(n + 1, 0);
    int64_t c = 0;
    for (int k = k0[u]; k <= n; ++k) {
      if (k > k0[u]) c += step_cost(m, u, k - 1, res);
      const double a = wd * (double)unit_err(m, un, k);
      int64_t A = 0;
      if (a > 0.0) {
        const double v = a / q;
        A = v > (double)P ? (int64_t)P + 1 : (int64_t)ceil(v);
      }
      parts_of[i][k] = A;
      if (A > P) continue;
      for (int b = (int)A; b <= P; ++b) {
        const int64_t prev = dp[b - A];
        if (prev >= kInf) continue;
        const int64_t v = c + prev;
        if (v < nd[b]) {  // ties keep the smaller step count
          nd[b] = v;
          ch[i][b] = k;
        }
      }
    }
    dp.swap(nd);
  }
  if (dp[P] >= kInf) return false;
  bytes = dp[P];
  int b = P;
  for (int i = (int)units.size() - 1; i >= 0; --i) {
    const int k = ch[i][b];
    state[units[i]] = k;
    b -= (int)parts_of[i][k];
  }
  return true;
}

PlanOut greedy_plan(Meta& m, double tau, int mode, const std::vector<int>* res, bool& ok) {
  std::vector<int> planes;
  double E;
  int n;
  ok = make_plan(m, tau, mode, planes, E, n) == 0;
  if (!ok) return PlanOut();
  return as_plan(m, planes, n, mode, res);
}

PlanOut better(const Meta& m, const PlanOut* best, const PlanOut& greedy, const std::vector<int>* res) {
  if (!best || extra_bytes(m, best->planes, res) > extra_bytes(m, greedy.planes, res)) return greedy;
  return *best;
}

int sum_of(const std::vector<int>& v) {
  int s = 0;
  for (int x : v) s += x;
  return s;
}

PlanOut dp_plan(Meta& m, double tau, int mode, const std::vector<int>* res, bool& ok) {
  const PlanOut greedy = greedy_plan(m, tau, mode, res, ok);
  if (!ok) return greedy;
  const std::vector<int> k0 = resident_steps(m, res);
  std::vector<int> all(m.units.size());
  for (size_t u = 0; u < all.size(); ++u) all[u] = (int)u;
  double R = budget(m, tau, mode);
  for (int it = 0; it < kDPRetries; ++it) {
    std::vector<int> state(m.units.size(), 0);
    int64_t bytes;
    if (!dp_solve(m, mode, all, R, k0, res, bytes, state)) break;
    if (bound(m, state, mode) <= tau) {
      const PlanOut p = as_plan(m, stream_planes(m, state), sum_of(state), mode, res);
      return better(m, &p, greedy, res);
    }
    R = R * (1.0 - ldexp(1.0, -20));
  }
  return greedy;
}

PlanOut best_first_plan(Meta& m, double tau, int mode, const std::vector<int>* res, bool& ok) {
  int su = -1;
  for (size_t u = 0; u < m.units.size(); ++u)
    if (m.units[u].stair) {
      su = (int)u;
      break;
    }
  if (su < 0) return dp_plan(m, tau, mode, res, ok);
  const PlanOut greedy = greedy_plan(m, tau, mode, res, ok);
  if (!ok) return greedy;
  const Unit& stair = m.units[su];
  std::vector<int> others;
  for (size_t u = 0; u < m.units.size(); ++u)
    if ((int)u != su) others.push_back((int)u);
  const std::vector<int> k0 = resident_steps(m, res);
  const double wd0 = wd_of(m.groups[stair.group], mode);
  double R0 = budget(m, tau, mode);
  std::vector<std::pair<int64_t, int>> pos;  // (own cost, steps), cheapest first
  int64_t c = 0;
  for (int s = k0[su]; s <= unit_nsteps(m, stair); ++s) {
    if (s > k0[su]) c += step_cost(m, su, s - 1, res);
    pos.push_back({c, s});
  }
  std::sort(pos.begin(), pos.end());
  for (int it = 0; it < kDPRetries; ++it) {
    bool found = false;
    int64_t best_total = 0;
    std::vector<int> best_state;
    for (const auto& ps : pos) {
      if (found && ps.first >= best_total) break;
      const double a = wd0 * (double)unit_err(m, stair, ps.second);
      if (a > R0) continue;
      std::vector<int> state(m.units.size(), 0);
      int64_t bytes;
      if (!dp_solve(m, mode, others, R0 - a, k0, res, bytes, state)) continue;
      if (!found || ps.first + bytes < best_total) {
        found = true;
        best_total = ps.first + bytes;
        state[su] = ps.second;
        best_state = state;
      }
    }
    if (!found) break;
    if (bound(m, best_state, mode) <= tau) {
      const PlanOut p = as_plan(m, stream_planes(m, best_state), sum_of(best_state), mode, res);
      return better(m, &p, greedy, res);
    }
    R0 = R0 * (1.0 - ldexp(1.0, -20));
  }
  return greedy;
}

}  // namespace

int make_plan_with(Meta& m, int interp, bool per_region, double tau, int mode, const std::vector<int>* resident,
                   std::vector<int>& planes, double& bound_out, int& nsteps) {
  if (interp == INTERP_GREEDY) return make_plan(m, tau, mode, planes, bound_out, nsteps);
  if (!(tau > 0.0)) return -1;
  bool ok = true;
  PlanOut p;
  if (interp == INTERP_DP || (interp == INTERP_PAPER && per_region))
    p = dp_plan(m, tau, mode, resident, ok);
  else
    p = best_first_plan(m, tau, mode, resident, ok);
  if (!ok) return -1;
  planes = p.planes;
  bound_out = p.bound;
  nsteps = p.nsteps;
  return 0;
}

std::string meta_json(const Meta& m) {
  std::string o;
  char buf[512];
  auto add = [&](const char* fmt, auto... args) {
    snprintf(buf, sizeof(buf), fmt, args...);
    o += buf;
  };
  add("{\"d\":%d,\"L\":%d,\"P\":%d,\"n\":%lld,\"xmin\":%.17g,\"xmax\":%.17g,\"A\":%.17g,\"eps_fp\":%.17g,"
      "\"meta_bytes\":%lld,\"encoding\":%d,\"lossless\":%d,\"groups\":[",
      m.d, m.L, m.P, (long long)m.n, m.xmin, m.xmax, m.A, m.eps_fp, (long long)m.meta_bytes, m.enc, m.lossless ? 1 : 0);
  for (size_t g = 0; g < m.groups.size(); ++g) {
    const Group& gr = m.groups[g];
    add("%s{\"kind\":%d,\"level\":%d,\"rho\":%d,\"n\":%lld,\"M\":%.17g,\"E\":%d,\"delta\":%.17g,\"w\":%.17g,"
        "\"rho_w\":%.17g,\"cd\":%d}",
        g ? "," : "", gr.kind, gr.level, gr.rho, (long long)gr.n, gr.M, gr.E, gr.delta, gr.w, gr.rho_w, gr.cd);
  }
  o += "],\"streams\":[";
  for (size_t s = 0; s < m.streams.size(); ++s) {
    const Stream& st = m.streams[s];
    add("%s{\"kind\":%d,\"level\":%d,\"rho\":%d,\"t\":%d,\"group\":%d,\"n\":%lld,\"B\":%d,\"maxabs\":%lld,\"nsig\":[",
        s ? "," : "", st.kind, st.level, st.rho, st.t, st.group, (long long)st.n, st.B, (long long)st.maxabs);
    for (size_t j = 0; j < st.nsig.size(); ++j) add("%s%lld", j ? "," : "", (long long)st.nsig[j]);
    o += "]";
    if (st.lossless) {
      o += ",\"nnz\":[";
      for (size_t j = 0; j < st.nnz.size(); ++j) add("%s%lld", j ? "," : "", (long long)st.nnz[j]);
      o += "]";
    }
    o += "}";
  }
  o += "],\"units\":[";
  for (size_t u = 0; u < m.units.size(); ++u) {
    const Unit& un = m.units[u];
    add("%s{\"group\":%d,\"stair\":%d,\"stream\":%d,\"levels\":[", u ? "," : "", un.group, un.stair ? 1 : 0,
        un.stream);
    for (size_t j = 0; j < un.levels.size(); ++j) add("%s%lld", j ? "," : "", (long long)un.levels[j]);
    o += "]}";
  }
  o += "]}";
  return o;
}

}  // namespace apc
