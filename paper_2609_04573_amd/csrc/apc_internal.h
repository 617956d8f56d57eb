// Internal declarations shared by the host orchestration and the gfx950
// kernels.  Fields are handled in a 3D embedding (leading axes of length 1).
// Every pass is one launch over a table of segments (one per field, level
// and region), so many fields of uneven shapes share each launch.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace apc {

constexpr int kChunk = 4096;        // codes per chunk (sign index granularity)
constexpr int kBlockElems = 4096;   // lattice elements per work block (16 per thread)
constexpr int kLvlCH = 128;  // per-level pass: longest run of planes along axis 0

enum AxisKind : int32_t { AX_ALL = 0, AX_ODD = 1, AX_EVEN = 2 };

// Division by a run-time constant: q = high64(M * n) with M = floor((2^64-1)/d)+1,
// exact for every 32-bit n (d = 1 is special-cased).
struct FastDiv {
  uint64_t M;
  uint32_t d;
  uint32_t one;
};

// One region of one level, as a lattice on that level's compact grid:
// node coordinate i = t (all), 2t+1 (odd) or 2t (even) on each axis.
struct Lattice {
  int32_t m[3];     // compact grid dims of the level
  int32_t c[3];     // lattice dims
  int32_t kind[3];  // AxisKind per axis
  int32_t ax;       // interpolation axis of the region (the odd one)
  FastDiv f2, f1;   // division by c[2] and by c[1]
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

// Coefficient pass over one (field, level, region).
struct CoefSeg {
  RegionArgs ra;
  const void* G;              // the level's compact grid of original values (T)
  void* codes;                // Q*, pass 2 output (lattice order)
  unsigned long long* gmax;   // pass 1: max |c| of the group (double bits)
  int64_t blk_begin;          // first global work block of this segment
  int32_t k_shift;            // pass 2: P - E of the group
  int32_t pad;
};

// Reconstruction of one (field, level, region).
struct ReconSeg {
  RegionArgs ra;
  const double* xc;     // reconstructed coarser level (float64 compact grid)
  int32_t cm1, cm2;     // its dims 1 and 2
  const void* q;        // codes of the region (Q*, lattice order)
  void* out;            // float64 grid of this level, or the output field (T) at level 0
  double delta;
  int64_t blk_begin;
  int32_t B, k;         // truncation of the codes to k of B planes
  int32_t final_out;    // 1: out is the T output field
  int32_t pad;
};

// Per-level tensor-product pass over one (field, level): tiles of
// (1024 / t2) x t2 points of (axis 1, axis 2) by runs of ch planes along axis 0.
struct LevelSeg {
  int32_t m[3];          // level grid dims
  int32_t mc[3];         // coarser level grid dims
  int32_t degree;
  int32_t nt1, nt2;      // tiles along axes 1 and 2
  int32_t final_out;     // reconstruction: out is the T output field
  int64_t blk_begin;     // first work block (tiles x runs) of this segment
  const void* src;       // refactor: the field (T), level grid at strides xs; reconstruction: coarser level (double)
  int64_t xs[3];         // refactor: element strides of the level grid in src
  unsigned long long* racc;  // max pass on level 0: range accumulators (min, max, max |x|, non-finite), or null
  void* out;             // reconstruction: level grid (double), or the T output field
  void* q[3];            // codes of regions 0, 1, 2 (Q*, lattice order)
  int32_t B[3], k[3];    // reconstruction: truncation of each region's codes
  double delta;          // reconstruction: quantization step
  unsigned long long* gmax;  // max pass: max |c| of the level (double bits)
  int32_t k_shift;       // quantization: P - E
  int32_t ch;            // planes per run along axis 0 (even)
};

// Flat segments: range pass, compact grids, coarsest level, injection.
struct FlatSeg {
  const void* src;
  void* dst;
  int64_t n;            // elements
  int64_t blk_begin;
  int64_t s[3];         // source strides (elements) per destination axis
  int32_t dm[3];        // destination-space dims (iteration space)
  FastDiv f2, f1;       // division by dm[2], dm[1]
  int32_t dst_m1, dst_m2;   // inject: fine grid dims 1, 2 (destination index 2i)
  int32_t final_out;        // inject / coarsest: destination is the T output field
  int32_t B, k;             // coarsest: truncation
  int32_t k_shift;          // coarse quantization: P - E
  double delta;             // coarsest: step
  unsigned long long* acc;  // range: 4 accumulators; coarse pass 1: group max
};

// Coefficient-decomposition view of one level-0 region lattice.
struct CDSeg {
  int32_t c[3];        // lattice dims
  int32_t pad;
  FastDiv f2, f1;
  const void* R;       // region codes (forward input)
  void* Rout;          // region codes (inverse output)
  void* S[3];          // S1, S2, S3 codes (stream order)
  unsigned long long* smax[3];
  int64_t blk_begin;
  int32_t B[3], k[3];  // decode masks (inverse)
  FastDiv ftv, ftu;    // row-tile inverse pass: division by the tiles along v and along u
};

// Device-side description of one bitplane stream for the codec kernels.
struct StreamDev {
  void* codes;          // Q*, stream order
  uint64_t* mag;        // magnitude section (B*M words)
  uint32_t* idx;        // index section (B*C entries)
  uint32_t* cnt;        // per-chunk counts scratch (C*B, chunk-major, refactor)
  uint32_t* zcnt;       // lossless stage: nonzero words per (chunk, plane), chunk-major (refactor), or null
  uint64_t* stage;      // sign staging scratch (64 words per chunk, refactor)
  uint64_t* sign;       // sign section
  const int64_t* pso;   // per plane: sign words before it
  int64_t n, M, C;
  int64_t chunk_begin;  // first global chunk id of this stream in the launch
  int64_t sign_n;       // sign words of the stream
  int32_t B;
  int32_t k0, k1;       // decode: planes [k0, k1) to add
  int32_t fresh;        // decode: resident codes are all zero (skip reading them)
  int32_t xor_chain;    // negabinary streams: stored digit planes XOR-chained
  int32_t pad;
};

// Lossless stage of one stream's magnitude planes (zero-word suppression):
// work items are (plane, chunk) pairs, item i of the stream = plane i / C,
// chunk i % C.  A suppressed plane's stored section is C presence words
// (bit i of word c: raw word 64c + i is nonzero), C uint32 counts of nonzero
// words before chunk c (padded to whole words) and the nonzero words; a raw
// plane's section is its M words.
struct ZwsSeg {
  const uint64_t* raw_in;    // pack: the raw planes (B x M words)
  uint64_t* raw_out;         // unpack: the raw planes
  uint32_t* zoff;            // pack: per-(plane, chunk) counts before the chunk (read); unpack: written
  uint64_t* comp_out;        // pack: the stored sections of every plane
  const uint64_t* comp_in;   // unpack: the stored sections
  const int64_t* pmo;        // pack, unpack: word offset of each plane's stored section
  uint64_t zmask;            // bit j: plane j is stored suppressed
  int64_t M, C;
  int64_t blk_begin;         // first global item of this stream
  int32_t B, pad;
};

// Sign-section layout, computed on the device from the per-(stream, plane)
// sign counts.  Jobs are the (stream, plane) pairs in stream order, planes
// most significant first; streams are the encode table's entries.
struct SignJob {
  int64_t* pso_dst;  // where the plane's word offset within its stream goes
  int32_t s_first;   // first job of the plane's stream
  int32_t pad;
};
struct SignStream {
  int32_t first, njob;  // its jobs
  int32_t f_first;      // first job of its field
  int32_t pad;
  int64_t ub;           // words of the field's sign arena
};

inline FastDiv make_fastdiv(uint32_t d) {
  FastDiv f;
  f.d = d;
  f.one = d <= 1 ? 1u : 0u;
  f.M = d <= 1 ? 0ull : (~0ull / d + 1ull);
  return f;
}

}  // namespace apc

// Kernel launchers (kernels.hip).  Segment tables live in device memory;
// nblk is the total number of 4096-element work blocks of the table.
namespace apc {
template <typename T>
hipError_t launch_range(const FlatSeg* segs, int nseg, int64_t nblk, hipStream_t s);
template <typename T>
hipError_t launch_gather(const FlatSeg* segs, int nseg, int64_t nblk, hipStream_t s);
template <typename T, typename Q>
hipError_t launch_coef(const CoefSeg* segs, int nseg, int64_t nblk, int mode, hipStream_t s);
template <typename T, typename Q>
hipError_t launch_level(const LevelSeg* segs, int nseg, int64_t nblk, int mode, int t2, hipStream_t s);
template <typename T, typename Q>
hipError_t launch_coarse(const FlatSeg* segs, int nseg, int64_t nblk, int mode, hipStream_t s);
template <typename Q>
hipError_t launch_cd_forward(const CDSeg* segs, int nseg, int64_t nblk, int a, int tiled, hipStream_t s);
template <typename Q>
hipError_t launch_cd_inverse(const CDSeg* segs, int nseg, int64_t nblk, int a, int phase, hipStream_t s);
template <typename Q>
hipError_t launch_encode(const StreamDev* sd, int ns, int64_t chunks, hipStream_t s);
hipError_t launch_scan(const StreamDev* sd, const int32_t* job_s, const int32_t* job_j, int njobs, int64_t* totals,
                       hipStream_t s);
hipError_t launch_sign_layout(const int64_t* totals, int njobs, const SignJob* jobs, int ns, const SignStream* ss,
                              StreamDev* sd, int64_t* prefix, int32_t* err, hipStream_t s);
hipError_t launch_sign_move(const StreamDev* sd, int ns, int64_t chunks, hipStream_t s);
template <typename Q>
hipError_t launch_decode(const StreamDev* sd, int ns, int64_t chunks, bool all_fresh, int max_planes, hipStream_t s);
// mode 1: pack the stored sections; 2: unpack them
hipError_t launch_zws(const ZwsSeg* segs, int nseg, int64_t items, int mode, hipStream_t s);
// Negabinary digit planes: encode (codes -> stored planes), decode (planes
// [k0, k1) OR-ed into resident digit words), and the truncated integers of
// resident digit words (FlatSeg: src words, dst codes, n, B, k).
template <typename Q>
hipError_t launch_encode_nb(const StreamDev* sd, int ns, int64_t chunks, hipStream_t s);
template <typename Q>
hipError_t launch_decode_nb(const StreamDev* sd, int ns, int64_t chunks, hipStream_t s);
template <typename Q>
hipError_t launch_nb_values(const FlatSeg* segs, int nseg, int64_t nblk, hipStream_t s);
// Zero the n 64-bit words at dst of every segment (FlatSeg: dst, n).
hipError_t launch_zero_words(const FlatSeg* segs, int nseg, int64_t nblk, hipStream_t s);
template <typename T, typename Q>
hipError_t launch_coarsest(const FlatSeg* segs, int nseg, int64_t nblk, hipStream_t s);
template <typename T>
hipError_t launch_inject(const FlatSeg* segs, int nseg, int64_t nblk, hipStream_t s);
template <typename T, typename Q>
hipError_t launch_recon(const ReconSeg* segs, int nseg, int64_t nblk, hipStream_t s);
}  // namespace apc
