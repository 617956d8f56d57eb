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

Unit build_staircase(int group, const std::vector<std::vector<int>>& rs, const std::vector<Stream>& st) {
  const int R = (int)rs.size();
  std::vector<std::vector<int>> orders(R);
  for (int r = 0; r < R; ++r) {
    int k[3] = {0, 0, 0};
    for (;;) {
      int best = -1;
      double best_r = -1.0;
      for (int t = 0; t < 3; ++t) {
        const Stream& s = st[rs[r][t]];
        if (k[t] < s.B) {
          const int64_t gain = s.delta(k[t]) - s.delta(k[t] + 1);
          const double q = (double)gain / (double)s.plane_bytes(k[t]);
          if (q > best_r) {
            best = t;
            best_r = q;
          }
        }
      }
      if (best < 0) break;
      orders[r].push_back(best);
      ++k[best];
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
        const int t = orders[r][pos[r]++];
        const int s = rs[r][t];
        nb += st[s].plane_bytes(kk[r][t]);
        steps.push_back({s, kk[r][t]});
        ++kk[r][t];
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
  m.meta_bytes = 64 + 16 * (int64_t)m.groups.size() + 16 * (int64_t)m.streams.size() + 4 * sumB + 8 * nseg;
  m.seq_ready[0] = m.seq_ready[1] = false;
}

void ensure_sequence(Meta& m, int mode) {
  if (m.seq_ready[mode]) return;
  std::vector<int> state(m.units.size(), 0);
  m.seq[mode].clear();
  m.seq_E0[mode] = bound(m, state, mode);
  for (;;) {
    int best = -1;
    double best_s = -1.0;
    for (int u = 0; u < (int)m.units.size(); ++u) {
      const Unit& un = m.units[u];
      if (state[u] < unit_nsteps(m, un)) {
        const Group& gr = m.groups[un.group];
        const double wd = mode == 0 ? gr.wd_inf : gr.wd_2;
        const int64_t de = unit_err(m, un, state[u]) - unit_err(m, un, state[u] + 1);
        const double s = (wd * (double)de) / (double)unit_step_bytes(m, un, state[u]);
        if (s > best_s) {
          best = u;
          best_s = s;
        }
      }
    }
    if (best < 0) break;
    ++state[best];
    m.seq[mode].push_back({best, bound(m, state, mode)});
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
    const auto& st = m.seq[mode][n];
    ++state[st.first];
    E = st.second;
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

std::string meta_json(const Meta& m) {
  std::string o;
  char buf[512];
  auto add = [&](const char* fmt, auto... args) {
    snprintf(buf, sizeof(buf), fmt, args...);
    o += buf;
  };
  add("{\"d\":%d,\"L\":%d,\"P\":%d,\"n\":%lld,\"xmin\":%.17g,\"xmax\":%.17g,\"A\":%.17g,\"eps_fp\":%.17g,"
      "\"meta_bytes\":%lld,\"groups\":[",
      m.d, m.L, m.P, (long long)m.n, m.xmin, m.xmax, m.A, m.eps_fp, (long long)m.meta_bytes);
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
    o += "]}";
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
