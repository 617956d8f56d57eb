// Host-side metadata of a refactored field and the retrieval interpreter.
#pragma once

#include <stdint.h>

#include <string>
#include <utility>
#include <vector>

namespace apc {

enum GroupKind { G_COARSE = 0, G_LEVEL = 1, G_REGION = 2 };
enum StreamKind { S_COARSE = 0, S_LEVEL = 1, S_REGION = 2, S_CD = 3 };
enum CdKind { CD_NONE = 0, CD_SUM = 1, CD_STAIR = 2 };

struct Group {
  int kind = 0, level = 0, rho = 0;
  int64_t n = 0;
  double M = 0.0;     // max |coefficient|
  int E = 0;          // frexp exponent of M
  double delta = 0.0; // quantization step 2^(E-P) (0 for an all-zero group)
  int k_shift = 0;    // P - E
  double w = 1.0, rho_w = 0.0;   // max-error and RMSE weights
  double wd_inf = 0.0, wd_2 = 0.0;
  int cd = CD_NONE;
};

struct Stream {
  int kind = 0, level = 0, rho = 0, t = 0;
  int group = 0;
  int64_t n = 0;
  int B = 0;
  int64_t maxabs = 0;
  int64_t code_off = 0;  // in the region code buffer, or the decomposition buffer
  bool use_cd = false;
  std::vector<int64_t> nsig;  // per plane (most significant first)
  std::vector<int64_t> pso;   // per plane: sign words before it in this stream
  int64_t mag_off = 0, idx_off = 0, sign_off = 0;
  // lossless stage: nonzero magnitude words per plane; a plane is stored
  // zero-word suppressed (presence words, per-chunk counts, nonzero words)
  // where that is smaller than its raw words
  bool lossless = false;
  std::vector<int64_t> nnz;
  // encoding: 0 generic bitplanes (sign-magnitude); 1 negabinary digit
  // planes; 2 negabinary digit planes, XOR-chained
  int enc = 0;

  int64_t words() const { return (n + 63) / 64; }
  int64_t chunks() const { return (n + 4095) / 4096; }
  int64_t sign_words() const {
    int64_t s = 0;
    for (int64_t v : nsig) s += (v + 63) / 64;
    return s;
  }
  int64_t zws_head_words() const { return chunks() + (chunks() + 1) / 2; }
  bool suppressed(int j) const { return lossless && 8 * (zws_head_words() + nnz[j]) < 8 * words(); }
  int64_t mag_words(int j) const { return suppressed(j) ? zws_head_words() + nnz[j] : words(); }
  int64_t plane_bytes(int j) const {
    if (enc) return 8 * mag_words(j);  // digit planes only: no index, no signs
    return 4 * chunks() + 8 * mag_words(j) + 8 * ((nsig[j] + 63) / 64);
  }
  // Largest error of a code truncated to k of B planes: sign-magnitude
  // truncation leaves less than one unit of the first dropped plane; dropped
  // negabinary digits are worth at most floor((2^(B-k+1) - 1) / 3).
  int64_t delta(int k) const {
    if (k <= 0) return maxabs;
    if (enc) return (int64_t)(((1ull << (B - k + 1)) - 1ull) / 3ull);
    return (int64_t)((1ull << (B - k)) - 1ull);
  }
  int64_t stored_mag_words() const {
    int64_t w = 0;
    for (int j = 0; j < B; ++j) w += mag_words(j);
    return w;
  }
  int64_t index_bytes() const {  // the index section, padded to 8 bytes (none for digit planes)
    if (enc) return 0;
    const int64_t ib = 4 * (int64_t)B * chunks();
    return ib + (8 - ib % 8) % 8;
  }
  int64_t blob_bytes() const { return index_bytes() + 8 * stored_mag_words() + 8 * sign_words(); }
};

struct Unit {
  int group = 0;
  bool stair = false;
  int stream = -1;
  std::vector<int64_t> levels, seg_bytes;
  std::vector<std::vector<std::pair<int, int>>> seg_steps;  // (stream, plane) per segment
};

// Fewest negabinary digits whose range holds [-V, V]: B digits hold
// [-2 (4^floor(B/2) - 1) / 3, (4^ceil(B/2) - 1) / 3].
inline int nb_digits(int64_t V) {
  int B = 0;
  for (;;) {
    const unsigned __int128 p = (((unsigned __int128)1 << (2 * ((B + 1) / 2))) - 1) / 3;
    const unsigned __int128 q = 2 * ((((unsigned __int128)1 << (2 * (B / 2))) - 1) / 3);
    if (p >= (unsigned __int128)V && q >= (unsigned __int128)V) return B;
    ++B;
  }
}

struct Meta {
  int d = 3, L = 1, P = 29;
  bool lossless = false;  // planes stored through the lossless stage
  int enc = 0;            // encoding of every stream (Stream::enc)
  int64_t n = 0;
  double xmin = 0, xmax = 0, A = 0;
  double eps_fp = 0;
  int64_t meta_bytes = 0;
  std::vector<Group> groups;
  std::vector<Stream> streams;
  std::vector<Unit> units;
  std::vector<std::vector<int>> group_units;
  std::vector<int> group_order;
  // greedy sequences, per mode (0 = max error, 1 = RMSE): unit advanced, its
  // step count after the step, bound after the step
  struct SeqStep {
    int unit, k;
    double E;
  };
  bool seq_ready[2] = {false, false};
  double seq_E0[2] = {0, 0};
  std::vector<SeqStep> seq[2];

  double range() const { return xmax - xmin; }
};

// Planner (plan.cpp)
void axis_norms(int64_t n, int L, int degree, std::vector<double>& inf, std::vector<double>& one);
Unit build_staircase(int group, const std::vector<std::vector<int>>& region_streams,
                     const std::vector<Stream>& streams);
void finalize_meta(Meta& m);
int64_t unit_err(const Meta& m, const Unit& u, int k);
int unit_nsteps(const Meta& m, const Unit& u);
double bound(const Meta& m, const std::vector<int>& state, int mode);
void ensure_sequence(Meta& m, int mode);
// Returns 0 on success, -1 if tau is below the floor.
int make_plan(Meta& m, double tau, int mode, std::vector<int>& planes, double& bound_out, int& nsteps);
int64_t plan_bytes(const Meta& m, const std::vector<int>& planes);
// Interpreters: the greedy above, the dynamic program, the best-first search
// (the dynamic program without a staircase), or the paper's choice (dynamic
// program for per-region interpolation, best-first search otherwise).
// resident: planes already fetched per stream (they cost nothing), or null.
enum { INTERP_GREEDY = 0, INTERP_DP = 1, INTERP_BEST_FIRST = 2, INTERP_PAPER = 3 };
int make_plan_with(Meta& m, int interp, bool per_region, double tau, int mode, const std::vector<int>* resident,
                   std::vector<int>& planes, double& bound_out, int& nsteps);
std::string meta_json(const Meta& m);

}  // namespace apc
