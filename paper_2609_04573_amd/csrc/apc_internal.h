// Internal declarations shared by the host orchestration and the gfx950
// kernels.  Fields are handled in a 3D embedding (leading axes of length 1).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace apc {

constexpr int kChunk = 4096;        // codes per chunk (sign index granularity)
constexpr int kWordsPerChunk = 64;  // 64-bit magnitude words per chunk

enum AxisKind : int32_t { AX_ALL = 0, AX_ODD = 1, AX_EVEN = 2 };

// One region of one level, as a lattice on that level's compact grid:
// node coordinate i = t (all), 2t+1 (odd) or 2t (even) on each axis.
struct Lattice {
  int32_t m[3];     // compact grid dims of the level
  int32_t c[3];     // lattice dims
  int32_t kind[3];  // AxisKind per axis
  int32_t ax;       // interpolation axis of the region (the odd one)
};

// Where the interpolation of one region reads its neighbours.
struct RegionArgs {
  Lattice lat;            // this region
  int32_t rho;            // region index in pass order
  int32_t sigma[3];       // pass order (3D axes); only [0, rho) are consulted
  int32_t degree;         // 1 or 3
  int32_t per_level;      // 1 = per-level, 0 = per-region
  Lattice prl[2];         // lattices of regions 0 and 1 of this level
  const double* pr[2];    // their buffers (predictions or reconstructed values)
  double* pr_out;         // this region's buffer to fill (null if not needed)
};

// Device-side description of one bitplane stream for the codec kernels.
struct StreamDev {
  int64_t n;          // codes
  int64_t code_off;   // offset of the stream's codes in its code buffer
  int64_t M;          // magnitude words per plane
  int64_t C;          // chunks
  int64_t mag_off;    // words, in the magnitude arena
  int64_t idx_off;    // uint32 entries, in the index arena
  int64_t cnt_off;    // uint32 entries, in the per-chunk count scratch (B*C)
  int64_t stage_off;  // words, in the sign staging scratch (64 per chunk)
  int64_t sign_off;   // words, in the sign arena
  int64_t sign_n;     // sign words of the stream (decode bound)
  int64_t chunk_begin;// first global chunk id of this stream (combined launches)
  int32_t B;          // planes
  int32_t use_cd;     // codes live in the decomposition code buffer
  int32_t k0, k1;     // decode: planes [k0, k1) to add
  int32_t fresh;      // decode: resident codes are all zero (skip reading them)
  int32_t psb;        // first entry of this stream's per-plane sign offsets (pso array)
};

// Coefficient-decomposition view of one level-0 region lattice.
struct CDArgs {
  int32_t c[3];       // lattice dims
  int32_t a, u, v;    // stacking axis and the slower / faster slice axes (3D)
  int64_t s_off[3];   // stream offsets of S1, S2, S3 in the decomposition code buffer
  int32_t s_idx[3];   // stream indices (for maxima)
  int32_t B[3], k[3]; // decode masks for S1..S3 (retrieve)
};

}  // namespace apc

// Kernel launchers (kernels.hip).  All return hipError_t of the launch.
namespace apc {
template <typename T>
hipError_t launch_range(const T* x, int64_t n, unsigned long long* acc4, hipStream_t s);
template <typename T>
hipError_t launch_subsample(const T* src, const int32_t* msrc, T* dst, const int32_t* mdst, hipStream_t s);
template <typename T, typename Q>
hipError_t launch_coef(const T* G, const RegionArgs& ra, int mode, unsigned long long* gmax, int64_t k_shift,
                       Q* codes, hipStream_t s);
template <typename T, typename Q>
hipError_t launch_coarse(const T* G, int64_t n, int mode, unsigned long long* gmax, int64_t k_shift, Q* codes,
                         hipStream_t s);
template <typename Q>
hipError_t launch_cd_forward(const Q* region_codes, const CDArgs& ca, Q* cd_codes, unsigned long long* smax,
                             hipStream_t s);
template <typename Q>
hipError_t launch_cd_inverse(const Q* cd_codes, const CDArgs& ca, Q* region_out, hipStream_t s);
template <typename Q>
hipError_t launch_encode(const Q* codes, const Q* cd_codes, const StreamDev* sd_dev, int nstreams,
                         int64_t total_chunks, const int64_t* chunk_begin_host, int B_max, uint64_t* mag,
                         uint32_t* cnt, uint64_t* stage, hipStream_t s);
hipError_t launch_scan(const StreamDev* sd_dev, const int32_t* job_stream, const int32_t* job_plane, int njobs,
                       const uint32_t* cnt, uint32_t* idx, int64_t* totals, hipStream_t s);
hipError_t launch_sign_move(const StreamDev* sd_dev, int nstreams, int64_t total_chunks, const uint32_t* cnt,
                            const uint32_t* idx, const int64_t* plane_sign_off, const uint64_t* stage,
                            uint64_t* sign, hipStream_t s);
template <typename Q>
hipError_t launch_decode(const StreamDev* sd_dev, int nstreams, int64_t total_chunks, const uint64_t* mag,
                         const uint32_t* idx, const uint64_t* sign, const int64_t* plane_sign_off, Q* codes,
                         Q* cd_codes, hipStream_t s);
template <typename Q>
hipError_t launch_coarsest_q(const Q* q, int64_t n, int32_t B, int32_t k, double delta, double* xc, hipStream_t s);
template <typename OutT, typename Q>
hipError_t launch_recon(const double* xc, const int32_t* cm, const RegionArgs& ra, const Q* q, int32_t B, int32_t k,
                        double delta, OutT* out, hipStream_t s);
template <typename OutT>
hipError_t launch_inject(const double* xc, const int32_t* cm, OutT* out, const int32_t* m, hipStream_t s);
template <typename OutT>
hipError_t launch_cast(const double* xc, int64_t n, OutT* out, hipStream_t s);
}  // namespace apc
