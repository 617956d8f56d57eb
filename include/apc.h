/*
 * apc.h — C ABI of the MI355X (gfx950) adaptive progressive compressor.
 *
 * The method: a float field is refactored once into bitplane streams of
 * quantized multilevel-interpolation coefficients (Section IV: per-level and
 * per-region interpolation; Section V-B: coefficient decomposition;
 * Section VI-C: generic bitplane encoding, Algorithm 1), and later retrieved
 * progressively to a requested max-error bound or PSNR from only the planes
 * that target needs (Section III-A problem statements; Section V-C error
 * mapping and max ordering; Algorithm 2).
 *
 * Conventions for every entry point:
 *  - Every function returns apc_status (0 = APC_OK, negative = error) and
 *    never throws; apc_last_error() gives a message for the calling thread.
 *  - Device pointers are HIP device addresses on the current device; host
 *    pointers are plain host memory.  hip_stream is a hipStream_t (NULL =
 *    the null stream); work is ordered on that stream.  Entry points that
 *    return metadata synchronize the stream before returning.
 *  - Fields are row-major with the last axis fastest, ndim 1..3.
 *  - A handle is not thread-safe: callers serialize calls on one handle.
 */
#ifndef APC_H
#define APC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t apc_status;
enum {
  APC_OK = 0,
  APC_E_INVALID = -1,        /* bad argument (dims, scheme, stream index, size) */
  APC_E_DTYPE = -2,          /* dtype other than float32 / float64 */
  APC_E_NONFINITE = -3,      /* field holds NaN or Inf (refactor rejects it) */
  APC_E_BELOW_FLOOR = -4,    /* target tighter than the full representation */
  APC_E_OOM = -5,            /* device allocation failed */
  APC_E_HIP = -6,            /* HIP runtime error */
  APC_E_BUSY = -7,           /* server admission refused (budget or queue full) */
  APC_E_CORRUPT = -8,        /* serialized bytes fail their checks */
  APC_E_NODEVICE = -9        /* no HIP device visible */
};

enum { APC_F32 = 0, APC_F64 = 1 };                 /* dtype */
enum { APC_PER_LEVEL = 0, APC_PER_REGION = 1, APC_AUTO = 2, APC_AUTO_PSNR = 3 };  /* apc_scheme.kind */
enum { APC_EB_ABS = 0, APC_EB_REL = 1, APC_PSNR = 2, APC_RMSE_ABS = 3 };  /* apc_target.kind */
enum { APC_MODE_EB = 0, APC_MODE_PSNR = 1 };       /* select_pipeline mode */

/* Pipeline configuration (Table I: interpolation scheme, dimension order of
 * per-region interpolation, coefficient-decomposition direction or none). */
typedef struct {
  int32_t kind;      /* APC_PER_LEVEL or APC_PER_REGION; or, for the refactor
                        calls, APC_AUTO / APC_AUTO_PSNR: the field's kind,
                        order and decomposition direction are chosen first by
                        apc_select_pipeline in error-bound / PSNR mode
                        (Section VI-A), keeping this scheme's levels,
                        lossless and encoding fields; the handle's metadata
                        JSON names the scheme used */
  int32_t degree;    /* 1 = multilinear, 3 = cubic (Section IV) */
  int32_t order[3];  /* per-region pass order, a permutation of 0..ndim-1
                        (ignored for per-level, which goes fastest axis first) */
  int32_t cd_axis;   /* -1 = no coefficient decomposition, else stacking axis
                        0..ndim-1 (ndim >= 2) */
  int32_t levels;    /* 0 = default L = 1 + ceil(log2(max dim - 1)) */
  int32_t lossless;  /* 1 = lossless stage on the stored planes (Section V:
                        bitplanes followed by lossless compression): each
                        plane's magnitude words are stored zero-word
                        suppressed (C presence words, C uint32 counts of
                        nonzero words before each chunk padded to whole
                        words, the nonzero words) where that is smaller than
                        its M raw words, and plane sizes, plans and blobs use
                        the stored sizes; 0 = raw planes.  Reconstructions
                        for the same planes are identical either way. */
  int32_t encoding;  /* Table I encodings: 0 = generic bitplanes (sign and
                        magnitude, the error-bound mode's); 1 = negabinary
                        digit planes (base -2, B digits, no sign bits; a code
                        truncated to k planes is off by at most
                        floor((2^(B-k+1) - 1) / 3)); 2 = negabinary with XOR
                        chaining (every stored plane after the first is the
                        XOR of its digit plane and the one above; the PSNR
                        mode's).  Digit-plane blobs hold only the planes. */
} apc_scheme;

/* Retrieval target (Section III-A).  APC_EB_ABS: max|x - x'| <= value;
 * APC_EB_REL: max|x - x'| <= value * (max x - min x); APC_PSNR: PSNR in dB
 * (20 log10(range / RMSE)) at least value; APC_RMSE_ABS: RMSE <= value. */
typedef struct {
  int32_t kind;
  double value;
} apc_target;

typedef struct {
  int64_t bytes_total;    /* S_tau: planes of the plan plus metadata */
  int64_t bytes_fetched;  /* plane bytes this call decoded that earlier calls had not */
  double bound;           /* error-model bound the plan achieves (max error or RMSE) */
  double tau;             /* the absolute tolerance the plan was made for */
  double bitrate;         /* 8 * bytes_total / n */
  int32_t n_streams;
  int32_t nsteps;         /* greedy steps taken */
} apc_retrieve_info;

typedef struct apc_handle apc_handle;

/* Refactor a device-resident field (Algorithm 1).  field_dev: n elements of
 * dtype (caller owned, read only, must stay valid until the stream passes
 * this call).  On success *out owns every plane stream (device memory) and
 * the host metadata; release it with apc_free.  The call waits for the
 * coefficient maxima and plane counts (the quantization steps depend on
 * global group maxima, the metadata on the counts) and returns while its
 * last kernels (the sign placement) may still run on hip_stream: the handle
 * carries an event behind them, and retrieval, ladders, the server,
 * serialization and blob export on any stream wait for that event first.
 * Errors: APC_E_INVALID (dims/scheme), APC_E_DTYPE, APC_E_NONFINITE,
 * APC_E_OOM, APC_E_HIP; *out is untouched on error (queued work is waited
 * for before the call's temporaries are released). */
apc_status apc_refactor(const void* field_dev, int32_t dtype, const int64_t* dims, int32_t ndim,
                        const apc_scheme* scheme, void* hip_stream, apc_handle** out);

/* Refactor many fields of one dtype together (batching): every pass is one
 * launch over the segments of all fields, and the host synchronizes three
 * times for the whole batch instead of three times per field.  fields_dev[f]
 * has ndims[f] dims, read consecutively from dims; schemes[f] applies to
 * field f.  out[f] receives a handle identical (same streams, same metadata)
 * to apc_refactor of that field alone.  On error no handle is returned. */
apc_status apc_refactor_batch(const void* const* fields_dev, int32_t dtype, const int64_t* dims,
                              const int32_t* ndims, const apc_scheme* schemes, int32_t nfields,
                              void* hip_stream, apc_handle** out);

/* Plan only (Section V-C interpreter, host side, no device work): fills
 * planes_out[n_streams] (may be NULL) and info.  APC_E_BELOW_FLOOR if the
 * target cannot be met even with every plane. */
apc_status apc_plan(apc_handle* h, const apc_target* target, int32_t* planes_out,
                    apc_retrieve_info* info);

/* Retrieve (Algorithm 2) to a target: plans, decodes the planes not yet
 * decoded by earlier calls on this handle (incremental), recomposes and
 * reconstructs into out_dev (n elements of the handle's dtype, caller owned).
 * The result depends only on the plan, not on what earlier calls decoded.
 * APC_E_BELOW_FLOOR leaves out_dev unwritten. */
apc_status apc_retrieve(apc_handle* h, const apc_target* target, void* out_dev,
                        apc_retrieve_info* info, void* hip_stream);

/* Retrieve with an explicit plane count per stream (planes[n_streams], each
 * clamped to the stream's plane count). */
apc_status apc_retrieve_planes(apc_handle* h, const int32_t* planes, void* out_dev, void* hip_stream);

/* Many retrievals in shared launches (Algorithm 2 for each request; the
 * retrieval counterpart of apc_refactor_batch): request i retrieves handle
 * hs[i] to targets[i] into outs_dev[i] (caller owned, that handle's size and
 * dtype).  All handles hold one dtype; a handle may appear more than once.
 * Each handle decodes once, up to the largest plan among its requests
 * (incremental, as apc_retrieve); every request's recomposition and
 * reconstruction read the codes truncated to its own plan, so each output
 * equals apc_retrieve of that request alone.  infos (n entries, may be
 * NULL): each request's plan, bytes_fetched crediting the planes it adds in
 * request order.  Returns once the work is queued on hip_stream.
 * APC_E_BELOW_FLOOR (nothing queued, no output written) if any target is
 * below its handle's floor; APC_E_INVALID for null arguments or mixed
 * dtypes. */
apc_status apc_retrieve_batch(apc_handle* const* hs, int32_t n, const apc_target* targets, void* const* outs_dev,
                              apc_retrieve_info* infos, void* hip_stream);

/* Retrieval that allocates nothing, for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc).  Same plan and same output bytes as apc_retrieve with
 * the same target, but every plane of the plan is decoded from zero (the
 * handle's resident planes are neither used nor updated, so
 * info.bytes_fetched counts every plane of the plan), and every device
 * buffer the retrieval needs (decoded codes, float64 coarse grids, the
 * recomposition buffer, launch tables) is carved from one static device
 * array of 256 MiB per device, held from module load until the process
 * ends.  The call issues no hipMalloc, hipFree or other allocating routine;
 * its launch tables are copied from pageable host memory with
 * hipMemcpyAsync on hip_stream, and all work runs on hip_stream (no helper
 * stream).  The array keeps the last call's contents; nothing in it needs
 * to start at zero.  All calls on one device share the array: calls queued
 * on one stream are ordered, calls that overlap on different streams race.
 * Errors: APC_E_INVALID if the field's buffers exceed the array (float32
 * fields need about 13 bytes per point with a decomposition, so 256^3 fits
 * and 320^3 does not), APC_E_BELOW_FLOOR as apc_retrieve. */
apc_status apc_retrieve_static(apc_handle* h, const apc_target* target, void* out_dev, apc_retrieve_info* info,
                               void* hip_stream);

/* Retrieval ladder as one HIP graph: the plans of targets[0..n) are made
 * now, their decode / recompose / reconstruct launches are captured once,
 * and apc_ladder_launch replays them on any stream, writing step i to
 * outs_dev[i] (caller owned, n elements each).  Every replay starts from no
 * resident planes, so it gives the same bytes as n single apc_retrieve calls
 * on a fresh handle.  The ladder borrows the handle's work buffers: do not
 * run other retrievals on the same handle while a replay is in flight. */
typedef struct apc_ladder apc_ladder;
apc_status apc_ladder_create(apc_handle* h, const apc_target* targets, int32_t n, void* const* outs_dev,
                             void* hip_stream, apc_ladder** out);
apc_status apc_ladder_launch(apc_ladder* ladder, void* hip_stream);
void apc_ladder_free(apc_ladder* ladder);

/* Serving: a request loop over resident refactored fields with continuous
 * batching.  Requests queue in arrival order.  Whenever one of max_slots
 * slot streams is free, the server's worker thread takes the queued
 * requests (up to max_batch of them, in order, while their work buffers fit
 * in hbm_budget_bytes; the decoded-code buffers of the fields are resident
 * and not counted) as one batch: the planes no earlier batch decoded are
 * decoded for each field up to the largest plan of the batch on that field
 * (all fields in shared launches, on the server's decode stream), then the
 * recomposition and reconstruction of every request of the batch run as
 * merged launches on the slot stream.  Batches on different slots overlap
 * on the device, and requests that arrive meanwhile join the next batch.
 * Each request reads the resident codes truncated to its own plan, so its
 * output equals that of the same request made alone.  max_slots = 1 and
 * max_batch = 1 give a one-at-a-time (FIFO) server.  The server owns the
 * fields' retrieval state until apc_server_destroy (which lets queued work
 * finish); handles stay owned by the caller and must outlive the server.
 *   submit: plans on the calling thread and queues; APC_E_BELOW_FLOOR for an
 *           unreachable target; APC_E_BUSY if the queue is full or the
 *           request alone exceeds the budget.  out_dev (caller owned, n
 *           elements of the field's dtype) is written asynchronously and
 *           must not be shared with another request in flight.
 *   poll / wait: completion of a ticket (wait also returns the plan info,
 *           whose bytes_fetched counts the planes the request added in
 *           arrival order, and forgets the ticket).
 *   stats: latency from submit to completion over completed requests, and
 *           the most requests on the device at once. */
typedef struct apc_server apc_server;
apc_status apc_server_create(apc_handle* const* fields, int32_t nfields, int64_t hbm_budget_bytes,
                             int32_t max_slots, int32_t max_batch, apc_server** out);
apc_status apc_server_submit(apc_server* sv, int32_t field, const apc_target* target, void* out_dev,
                             int64_t* ticket);
apc_status apc_server_poll(apc_server* sv, int64_t ticket, int32_t* done);
apc_status apc_server_wait(apc_server* sv, int64_t ticket, apc_retrieve_info* info);
apc_status apc_server_stats(apc_server* sv, double* p50_ms, double* p99_ms, double* mean_ms, int64_t* completed,
                            int64_t* max_running);
apc_status apc_server_reset_stats(apc_server* sv);
void apc_server_destroy(apc_server* sv);

/* Target-driven pipeline selection (Section VI-A): regular ~1% sample
 * blocks, every candidate of Table I refactored on the sample, plan sizes at
 * the nine tuning tolerances, majority vote (interpolation first, then the
 * decomposition direction).  mode: APC_MODE_EB or APC_MODE_PSNR. */
apc_status apc_select_pipeline(const void* field_dev, int32_t dtype, const int64_t* dims, int32_t ndim,
                               int32_t mode, apc_scheme* out, void* hip_stream);

/* Sweep-tile autotuner for batched per-level passes.  The per-level
 * interpolation sweep (the tensor-product refinement of Section IV) runs on
 * tiles of t2 columns (the fastest axis) by 1024/t2 rows, t2 in {32, 64,
 * 128}.  apc_tune_tiles times the level's max and quantization passes
 * (together) with each width on the given device field (dims and dtype as
 * apc_refactor; degree 1 or 3) for every level of at least 2^18 points with
 * more than one plane along axis 0, and records the width for that level
 * shape (the fastest, or a wider one within 3% of it; dtype, log2 of the
 * axis-1 and axis-2 extents) in a
 * process-wide table that later refactors and retrievals of any field use.
 * It allocates a scratch buffer of one code per point while it runs.
 * Outputs (optional): the width chosen for level 0 (0 if no level was
 * timed) and the level-0 times in microseconds for widths 32, 64, 128
 * (us0: 3 doubles).  The field is only read.  Tile widths never change
 * results, only speed; levels with one plane along axis 0 (2D and 1D
 * fields) always take one-column tiles.
 * apc_tile_override forces one width for every pass (0 restores the table);
 * APC_E_INVALID for other values.  apc_tile_width reports the width used
 * for a level of extents m1 x m2. */
apc_status apc_tune_tiles(const void* field_dev, int32_t dtype, const int64_t* dims, int32_t ndim, int32_t degree,
                          void* hip_stream, int32_t* tile0, double* us0);
apc_status apc_tile_override(int32_t t2);
apc_status apc_tile_width(int32_t dtype, int64_t m1, int64_t m2, int32_t* t2);

void apc_free(apc_handle* h);
const char* apc_strerror(apc_status s);
const char* apc_last_error(void);

/* ---- introspection (tests, benchmarks, storage) ---------------------- */

int32_t apc_num_streams(const apc_handle* h);
int32_t apc_num_groups(const apc_handle* h);
int64_t apc_num_points(const apc_handle* h);

/* Stream s: code count, plane count B, max |code|, and its serialized size
 * in bytes (index + magnitude + sign sections, as the format below). */
apc_status apc_stream_info(const apc_handle* h, int32_t s, int64_t* n, int32_t* B, int64_t* maxabs,
                           int64_t* blob_bytes);

/* Copy stream s, serialized, to host memory (cap >= blob_bytes).  Layout:
 * B*C uint32 index entries (C = ceil(n/4096)) padded to 8 bytes, then B*M
 * uint64 magnitude words (M = ceil(n/64)), then the sign words of each
 * plane, all little endian, planes most significant first. */
apc_status apc_stream_blob(const apc_handle* h, int32_t s, void* host_dst, int64_t cap);

/* Metadata as a JSON text (groups, streams, staircase, bounds). */
apc_status apc_metadata_json(const apc_handle* h, char* buf, int64_t cap, int64_t* len);

/* Retrieval interpreters (Section V-C; Algorithm 2 "RetrievalInterpreter").
 * APC_INTERP_GREEDY (the default): steps taken in order of weighted error
 *   decrease per byte; plans for tighter targets contain looser ones.
 * APC_INTERP_DP: the fewest bytes within the target by dynamic programming
 *   over the error budget split into 2048 parts (each unit's error term
 *   rounded up to whole parts), never more bytes than the greedy plan.
 * APC_INTERP_BEST_FIRST: for per-level interpolation with decomposition,
 *   the level-0 staircase's step counts searched cheapest first with pruning,
 *   the other units by the dynamic program; otherwise APC_INTERP_DP.
 * APC_INTERP_PAPER: the paper's choice, APC_INTERP_DP for per-region and
 *   APC_INTERP_BEST_FIRST for per-level interpolation.
 * The last three are invoked incrementally: planes already decoded on the
 * handle (and, in a ladder, by its earlier steps) cost nothing.  The server
 * plans every request as for a fresh handle.  Every interpreter's plan
 * satisfies the target.  APC_E_INVALID for other values. */
enum { APC_INTERP_GREEDY = 0, APC_INTERP_DP = 1, APC_INTERP_BEST_FIRST = 2, APC_INTERP_PAPER = 3 };
apc_status apc_set_interpreter(apc_handle* h, int32_t interp);

/* Shape and dtype of a handle's field: dims (3 int64, the first ndim set),
 * ndim, dtype (APC_F32 / APC_F64); any output may be NULL. */
apc_status apc_field_info(const apc_handle* h, int64_t* dims, int32_t* ndim, int32_t* dtype);

/* Serialization of the refactored representation (Section III-B: the data
 * are refactored once and stored; retrievals happen later from what was
 * stored).  The byte string holds the geometry and scheme, the metadata the
 * interpreter needs (range, group maxima, per-stream plane counts and
 * new-significant counts) and every stream's blob in the apc_stream_blob
 * layout, each section with its length and a 64-bit checksum:
 *   [0,8) magic "APCREP01"; [8,16) total length; [16,24) metadata length;
 *   [24,32) metadata checksum; metadata (int32 dtype, ndim; int64 dims[3];
 *   int32 kind, degree, order[3], cd_axis, levels, L, P, lossless,
 *   encoding, 0; float64 xmin, xmax, A; uint32 group and stream counts;
 *   float64 M per group; per stream int64 n, maxabs, int32 B, 0, int64
 *   nsig[B], and with the lossless stage int64 nnz[B]); then per stream
 *   uint64 blob length, uint64 blob checksum, blob.  Little endian.
 * apc_serialize: with host_dst NULL only *len is set (the size needed);
 *   otherwise host_dst (caller owned, cap >= *len bytes) receives the
 *   bytes.  Waits for the handle's refactor to finish.  APC_E_INVALID if
 *   cap is too small.
 * apc_deserialize: checks every field (magic, lengths, checksums, the
 *   geometry and layout they imply, plane and index counts) and returns
 *   APC_E_CORRUPT, with a message naming the first failed check, for
 *   truncated, padded or altered bytes.  With out NULL it only checks (host
 *   only, no device needed).  Otherwise *out is a new handle (release with
 *   apc_free) whose streams are uploaded on hip_stream; the call returns
 *   after the upload.  The handle retrieves exactly as the serialized one. */
apc_status apc_serialize(const apc_handle* h, void* host_dst, int64_t cap, int64_t* len);
apc_status apc_deserialize(const void* src, int64_t len, void* hip_stream, apc_handle** out);
/* The same checks, and a handle that holds only the host metadata (no device
 * needed): apc_plan, apc_set_interpreter and the introspection calls work on
 * it; retrieval, ladders, the server, blob export and serialization return
 * APC_E_INVALID.  For planning services away from the data. */
apc_status apc_deserialize_host(const void* src, int64_t len, apc_handle** out);

/* Out-of-core blocks (the paper refactors fixed-size blocks independently,
 * one per core, and stores them: the end-to-end transfer use case).  The
 * field is host memory (row-major, dims as apc_refactor, caller owned, read
 * only); it is split into blocks of extents `block` (ragged at the far
 * edges), each refactored with `scheme` as an independent field and kept
 * serialized (apc_serialize layout) in host memory owned by the set.  The
 * device holds one group of at most group_bytes of field at a time (plus
 * its refactoring buffers), so the field may exceed device memory.
 * apc_blocks_retrieve turns the target into one absolute bound every block
 * meets (a relative bound or PSNR uses the range of the whole field; per
 * block max error <= tau gives max error <= tau overall, per block RMSE <= r
 * gives RMSE <= r overall), plans each block on host metadata with the
 * set's interpreter, uploads only the planned planes of each block (the
 * stored sections' prefixes), reconstructs it on the device and copies it
 * into out_host (caller owned, the field's size).  info: bytes over all
 * blocks, the largest block bound (max error) or the pooled RMSE bound.
 * The set's own blobs are not re-verified against their stream checksums
 * (they are computed when the set writes them; apc_deserialize of a block's
 * bytes verifies them).  Both calls synchronize hip_stream.  apc_blocks_blob returns block b's
 * serialized bytes (owned by the set; blocks in row-major block order). */
typedef struct apc_blockset apc_blockset;
apc_status apc_blocks_refactor(const void* field_host, int32_t dtype, const int64_t* dims, int32_t ndim,
                               const int64_t* block, const apc_scheme* scheme, int64_t group_bytes, void* hip_stream,
                               apc_blockset** out);
apc_status apc_blocks_retrieve(apc_blockset* bs, const apc_target* target, void* out_host, apc_retrieve_info* info,
                               void* hip_stream);
apc_status apc_blocks_set_interpreter(apc_blockset* bs, int32_t interp);
apc_status apc_blocks_info(const apc_blockset* bs, int64_t* nblocks, int64_t* stored_bytes, double* xmin,
                           double* xmax);
apc_status apc_blocks_blob(const apc_blockset* bs, int64_t b, const void** bytes, int64_t* len);
void apc_blocks_free(apc_blockset* bs);

/* Host-only helper (no device needed): exact chain norms of the 1D
 * interpolation chain on an axis of length n for levels 0..L-1, rounded to
 * float64 (max row / column abs sums).  inf_out, one_out: L doubles. */
apc_status apc_axis_norms(int64_t n, int32_t L, int32_t degree, double* inf_out, double* one_out);

/* Launch profiling (measurement only).  While enabled, every kernel launch
 * is bracketed by HIP events recorded on the stream it runs on.
 * apc_profile_report waits for the recorded events and returns, per kernel,
 * {"count", "ms" (summed event time), "bytes" (data the launches must read
 * and write)} as JSON, then clears the records.  Launches may come from
 * several threads while it is enabled (the server's worker, the caller);
 * launches captured into a graph are not timed. */
apc_status apc_profile_enable(int32_t on);
apc_status apc_profile_report(char* buf, int64_t cap, int64_t* len);
/* Restrict profiling to launches of one kernel name (as reported above);
 * NULL or "" profiles every launch. */
apc_status apc_profile_only(const char* name);

#ifdef __cplusplus
}
#endif
#endif /* APC_H */
