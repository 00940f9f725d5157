/*
 * lpcc.h - C ABI of the gfx950 (MI355X) implementation of the integer-only
 * octree context model and range coder of "Towards Practical Lossless Neural
 * Compression for LiDAR Point Clouds" (arXiv 2603.25260).
 *
 * What the library computes
 *   A point cloud of int32 voxel coordinates in [0, 2^D)^3 is turned into an
 *   octree (Sec. S3.2, "Implementation of Octree Operations": Morton sort,
 *   halve and de-duplicate, 8-bit occupancy codes).  Coding it losslessly is
 *   the problem of Sec. 3.1, Eq. 1-3: the codes of each level are coded
 *   under a distribution predicted from the levels before it.  Depth by depth, from the root, an integer-only network predicts
 *   each node's distribution over the 255 non-empty occupancy codes
 *   (Eq. 2-3): shallow depths propagate the previous depth's features through
 *   a ResBlock and one upsample/prune step (Eq. 8-9); deep depths re-densify
 *   the last coded level down to the dense depth k0 = D - n_deep - 1 and
 *   upsample/prune back (GRED and XFP, Eq. 4-7 and 10-11).  Every layer uses
 *   int8 weights and activations, int32 accumulation and multiply-shift
 *   requantisation (Sec. 3.3, Eq. 12-14); the softmax uses an exponent table
 *   on the non-positive domain and integer normalisation (Eq. 15).  The
 *   resulting 16-bit CDF drives a byte-oriented range coder, in chunks of 2^c
 *   nodes per depth.  Nothing is computed in floating point.
 *
 * Conventions
 *   - All functions return an int status: LPCC_OK (0) or a negative code.
 *   - Pointers to point data and streams may be host or device memory of the
 *     context's device; the kind is detected per call.  The library copies
 *     what it needs and keeps no caller pointer after a call returns.
 *   - Coordinates: int32 [n][3] (x, y, z).  Duplicates are allowed and removed.
 *     n = 0 is a valid (empty) frame.
 *   - Decoded coordinates are the unique voxels in Morton order (x is the most
 *     significant bit of every bit triple).
 *   - A context is used by one host thread at a time; a model may be shared by
 *     several contexts of the same device.
 *   - Calls are synchronous: outputs are complete when the call returns.
 *
 * Bitstream (little-endian; the paper leaves the entropy coder and the stream
 *   layout open, Sec. 3.1 "Prediction & Coding"): u32 "LPC1", u8 version
 *   (1: every depth modelled; 2: base geometry, see lpcc_ctx_set_base_depth),
 *   u8 D, u8 n_deep, u8 c (log2 of the chunk size), u32 blob id (FNV-1a of
 *   the weight blob), u32 N_D, u32 N_d for d = 0..D-1, [version 2: the base
 *   tables], u16 payload length of every chunk (depth ascending, chunk
 *   ascending), then the payloads.  Chunk k of depth d codes nodes
 *   [k 2^c, min((k+1) 2^c, N_d)) of that depth.
 */
#ifndef LPCC_H
#define LPCC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define LPCC_OK 0
#define LPCC_E_INVAL (-1)    /* null pointer, coordinate outside [0,2^D), bad level / chunk size */
#define LPCC_E_CAPACITY (-2) /* output too small; the required size is written back            */
#define LPCC_E_CORRUPT (-3)  /* malformed or inconsistent bitstream                             */
#define LPCC_E_MODEL (-4)    /* malformed weight blob, or stream made with another model       */
#define LPCC_E_DEVICE (-5)   /* HIP runtime error; text via lpcc_last_error                     */
#define LPCC_E_NOMEM (-6)    /* device allocation failed, or workspace over the context's budget  */

typedef struct lpcc_model lpcc_model; /* weights resident on one device, read-only  */
typedef struct lpcc_ctx lpcc_ctx;     /* device, stream, workspace of one caller     */

/*
 * Seeded random-init weight blob (the model of Sec. S2 with the schedule of
 * Sec. 3.1-3.2; every layer int8 weights, int32 bias and the multiply-shift
 * requantisation of Eq. 12-14).  Host only, integer arithmetic only,
 * deterministic: the same arguments always give the same bytes.
 *   seed         SplitMix64 seed (counter form) of every draw
 *   C            channel width: 16, 32 or 64
 *   D, n_deep    octree levels and number of re-densified deep depths
 *                (0 <= n_deep <= D - 1; the dense fusion depth is D - n_deep - 1)
 *   flags        LPCC_W_NO_XFP: the ablation schedule without cross-scale
 *                propagation (blob version 2); LPCC_W_ZERO_POINTS: activation
 *                zero points in [-8, 8] on every layer (Eq. 13-14);
 *                LPCC_W_SHARED: level-aware parameter sharing (the future work
 *                named in the last paragraph of Sec. S2): the layers of one
 *                role share one weight tensor across depths (the predictor's
 *                two layers at every depth; per kind the shallow depths
 *                d <= k0 and the deep depths apart), every layer keeps its own
 *                bias and requantisation (version flag 0x100)
 *   blob, cap    output buffer (host); may be NULL with cap = 0 to query
 *   len          bytes of the blob (also with LPCC_E_CAPACITY)
 * Layout: u32 "LPCW", u32 version, u32 C, u32 D, u32 n_deep, u32 n_layers,
 * u64 seed; per layer u32 kind, depth, j, taps, cin, cout, i32 m_pos, m_neg,
 * u32 r, i32 z_in, z_out, [shared: u32 owner, the index of the layer whose
 * weights it uses], i32 bias[cout], i8 W[taps][cin][cout] (shared: only in
 * the owner's record), zero padding to 4 bytes.  The draws do not depend on
 * sharing: a shared blob is the unshared one with every layer's weights
 * replaced by its owner's.  W = (u >> 33) mod 255 - 127, bias = (u >> 33) mod 8193
 * - 4096, r = 24, m_pos = floor(2^24 / (73.6 sqrt(taps cin))) (3/4 of it for
 * the logit layer), m_neg = 0 (ReLU), m_pos (identity) or m_pos / 4 (PReLU).
 * Errors: LPCC_E_INVAL (bad argument), LPCC_E_CAPACITY (cap < len).
 */
#define LPCC_W_NO_XFP 1
#define LPCC_W_ZERO_POINTS 2
#define LPCC_W_SHARED 4
int lpcc_make_weights(uint64_t seed, int C, int D, int n_deep, int flags, void* blob, size_t cap, size_t* len);

/*
 * Weight blob -> device model (the per-depth layers of Sec. S2).  The blob is
 * parsed, validated (layer order, shapes, |bias| < 2^24, 0 <= m < 2^31,
 * 0 <= r <= 62, zero points in int8; in a shared blob every owner index
 * points at an earlier or the same layer of equal shape that owns its
 * weights) and copied to `device`, each shared weight tensor once; the caller
 * keeps ownership of `blob`.
 * Errors: LPCC_E_INVAL (null), LPCC_E_MODEL (bad blob), LPCC_E_DEVICE / NOMEM.
 */
int lpcc_model_load(const void* blob, size_t len, int device, lpcc_model** out);
void lpcc_model_free(lpcc_model* m);
/* Channel width C, octree depth D, number of deep (re-densified) depths, blob id. */
int lpcc_model_info(const lpcc_model* m, int* C, int* D, int* n_deep, uint32_t* blob_id);

/*
 * Context on `device` (the execution state of the level-by-level pipeline of
 * Sec. 3.1-3.3 for one caller).  `hip_stream` (a hipStream_t) is where all
 * work of the context is enqueued; the context does not own it.  With NULL
 * the context creates a stream of its own (default priority, blocking:
 * ordered with the null stream, so inputs written there are complete when its
 * work starts) and destroys it in lpcc_ctx_free.  Every call returns after
 * its work on the stream has finished.  Device workspace grows on demand and
 * is reused between calls; `hbm_budget` (bytes, 0 = no limit) caps the
 * workspace the context may hold: a call that would need more fails with
 * LPCC_E_NOMEM and leaves the context usable.
 */
int lpcc_ctx_create(int device, void* hip_stream, size_t hbm_budget, lpcc_ctx** out);
void lpcc_ctx_free(lpcc_ctx* c);
/* Device workspace bytes the context holds now and at most so far. */
int lpcc_ctx_workspace(const lpcc_ctx* c, size_t* held, size_t* peak);
/* Text of the last error of this context (valid until the next call). */
const char* lpcc_last_error(const lpcc_ctx* c);

/*
 * Encode one frame: octree construction (Sec. S3.2), per depth the features
 * of the shallow (Eq. 8-9) or re-densified deep path (Eq. 4-7, 10-11), the
 * predictor and integer softmax (Eq. 7, 15) and range coding of the codes
 * under the predicted distribution (Eq. 2-3).
 *   xyz        int32 [n][3], host or device
 *   chunk_log2 c in [4, 14]: nodes per range-coder chunk = 2^c
 *   out        bitstream buffer (host or device) of `cap` bytes
 *   out_len    bytes written, or the required size on LPCC_E_CAPACITY
 * Errors: LPCC_E_INVAL (bad coordinate / argument), LPCC_E_CAPACITY.  On
 * LPCC_E_CAPACITY no byte at or past `cap` is written (the bytes below it
 * are unspecified).
 */
int lpcc_encode_frame(lpcc_ctx* c, const lpcc_model* m, const int32_t* xyz, int64_t n, int chunk_log2,
                      uint8_t* out, size_t cap, size_t* out_len);

/*
 * Allocation-free form of lpcc_encode_frame, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops and
 * harnesses that forbid hipMalloc.  Same arguments, same bytes out as
 * lpcc_encode_frame on the same context (its stream, base depth and tiling),
 * but no call into a device or pinned-host allocator: every intermediate
 * buffer of the encode is carved from a static block of 256 MiB that the
 * library holds on each device it runs on (from the first context created on
 * the device until the process ends), and host read-backs go through a 4 MiB
 * pageable buffer made with the context.  The caller passes inputs and
 * outputs as for lpcc_encode_frame (host or device).
 * Every call on a device shares that device's block, which keeps the last
 * call's contents (each call clears what it needs cleared itself); calls that
 * overlapped on one device would race on it, so the library holds a per-device
 * lock for the whole (synchronous) call and concurrent callers run one after
 * another.
 * Errors: as lpcc_encode_frame; LPCC_E_NOMEM when the frame's workspace does
 * not fit the block or its host staging the buffer (checked before any work
 * is enqueued for that phase; lpcc_last_error gives the sizes);
 * LPCC_E_DEVICE when the block's device address could not be looked up.
 */
int lpcc_encode_frame_noalloc(lpcc_ctx* c, const lpcc_model* m, const int32_t* xyz, int64_t n, int chunk_log2,
                              uint8_t* out, size_t cap, size_t* out_len);

/*
 * Decode one frame, depth by depth: the model of every depth reads only the
 * depths decoded before it (Eq. 2), so the decoder rebuilds the same
 * distributions and the geometry progressively (Sec. 3.1, S3.2 child
 * expansion in Morton order).
 *   bs, len    bitstream, host or device
 *   xyz_out    int32 [cap][3] (host or device): unique voxels in Morton order
 *   n_out      number of voxels, also returned with LPCC_E_CAPACITY
 * Errors: LPCC_E_CORRUPT (bad header, counts, lengths, or coder state),
 *         LPCC_E_MODEL (stream made with another model), LPCC_E_CAPACITY.
 */
int lpcc_decode_frame(lpcc_ctx* c, const lpcc_model* m, const uint8_t* bs, size_t len, int32_t* xyz_out,
                      int64_t cap, int64_t* n_out);

/*
 * CDF rows of one depth: the predicted distribution of Eq. 3 / Eq. 7 after
 * the integer softmax of Eq. 15, as the coder uses it, for `level` (0..D-1),
 * int32 [N_level][256] with cdf[0] = 0, cdf[255] = 65536 and
 * cdf[s+1] - cdf[s] >= 1 the frequency of occupancy code s + 1.
 *   cdf_out    host or device; n_nodes = N_level (also with LPCC_E_CAPACITY)
 */
int lpcc_level_probs(lpcc_ctx* c, const lpcc_model* m, const int32_t* xyz, int64_t n, int level,
                     int32_t* cdf_out, int64_t cap, int64_t* n_nodes);

/*
 * Depth and point count from the first 16 bytes of a stream (host memory
 * only; the stream layout above).  max_workspace (may be NULL): device
 * workspace bytes a fresh context needs to decode this stream with any model
 * it may have been made with (C <= 64), computed from the depth counts, so it
 * needs len >= 16 + 4 D (base-geometry streams: their tables too); with fewer
 * bytes it is 0.  Errors: LPCC_E_INVAL (null), LPCC_E_CORRUPT (bad header).
 */
int lpcc_peek_header(const uint8_t* bs, size_t len, int* D, int64_t* n_points, size_t* max_workspace);

/*
 * Batched forms of the calls above (the same computation per frame): `nf`
 * frames of one model share every launch of a depth
 * (one launch per depth and layer over the rows of all frames).  Results are
 * identical, byte for byte, to the per-frame calls.  Per-frame status codes
 * go to status[nf]; the return value is LPCC_OK if every frame succeeded,
 * otherwise the first failing frame's code.  Pointers follow the per-frame
 * rules; every xyz[i] / out[i] / bs[i] / xyz_out[i] is a separate buffer.
 */
int lpcc_encode_batch(lpcc_ctx* c, const lpcc_model* m, int nf, const int32_t* const* xyz, const int64_t* n,
                      int chunk_log2, uint8_t* const* out, const size_t* cap, size_t* out_len, int* status);
int lpcc_decode_batch(lpcc_ctx* c, const lpcc_model* m, int nf, const uint8_t* const* bs, const size_t* len,
                      int32_t* const* xyz_out, const int64_t* cap, int64_t* n_out, int* status);

/*
 * Serving: continuous batching of encode / decode requests from many
 * sensors on one device (callers that stream frames from live sensors; the
 * per-frame computation is the one of lpcc_encode_frame / lpcc_decode_frame).
 *
 * The server runs `n_slots` slots concurrently, each with its own stream and
 * workspace (a frame's octree and features stay resident on the device while
 * it is processed).  Admission is by device memory: the slots' workspace is
 * counted as allocated, and a job is admitted when the growth its slot needs
 * for it (an upper bound from its point count or its stream header) fits in
 * `hbm_budget` (0 = 7/8 of the free memory) beside what the slots hold and
 * what running jobs were granted; idle slots release their workspace when a
 * waiting job needs it.  Each slot's context is capped at what it was
 * granted, so the device workspace of the server never exceeds the budget
 * (bytes_peak).  A free slot takes the oldest admissible job and up to
 * `max_batch - 1` queued jobs of the same model and kind, which share every
 * launch (lpcc_encode_batch / lpcc_decode_batch).  Results are byte-
 * identical to the per-frame calls.  Job buffers belong to the caller and must
 * stay valid until the job is reported by lpcc_server_poll.  Timestamps are
 * CLOCK_MONOTONIC nanoseconds.
 */
typedef struct lpcc_server lpcc_server;
typedef struct {
  int kind;             /* 0 = encode, 1 = decode                                   */
  int model;            /* index into the server's model list                       */
  const void* in;       /* encode: int32 [n][3]; decode: stream bytes (host/device)  */
  int64_t n_points;     /* encode: n                                                 */
  size_t in_len;        /* decode: stream length in bytes                            */
  void* out;            /* encode: stream buffer; decode: int32 [cap][3]             */
  size_t out_cap;       /* encode: bytes; decode: points                             */
  int64_t t_arrival_ns; /* arrival time (0 = at submission)                          */
  int chunk_log2;       /* encode: nodes per coder chunk = 2^c                        */
} lpcc_job;
typedef struct {
  uint64_t ticket;
  int status;           /* LPCC_OK or the per-frame error                            */
  int kind;
  size_t out_len;       /* encode: stream bytes; decode: points                      */
  int64_t n_points;     /* points of the frame                                       */
  int64_t t_arrival_ns, t_start_ns, t_done_ns;
  int batch;            /* number of jobs that shared this job's launches            */
} lpcc_done;
typedef struct {
  double p50_ms, p99_ms, mean_ms; /* arrival -> completion latency                  */
  double mpts_per_s;              /* points of completed jobs / (last done - first arrival) */
  int64_t completed, admitted, queued, running;
  size_t bytes_in_use;            /* workspace held by the slots + growth granted to running jobs */
  size_t bytes_budget;
  size_t bytes_peak;              /* largest bytes_in_use so far (bounds the device workspace)    */
} lpcc_stats;

int lpcc_server_create(int device, const lpcc_model* const* models, int n_models, int n_slots, int max_batch,
                       size_t hbm_budget, lpcc_server** out);
/* Queue a job; returns at once with its ticket.  LPCC_E_INVAL for bad fields,
 * LPCC_E_CORRUPT for a decode job whose stream header is unreadable. */
int lpcc_server_submit(lpcc_server* s, const lpcc_job* job, uint64_t* ticket);
/* Completed jobs (up to `max`), waiting up to `wait_ms` when none is ready. */
int lpcc_server_poll(lpcc_server* s, lpcc_done* done, int max, int* n_done, int wait_ms);
/* Block until every submitted job has completed. */
int lpcc_server_drain(lpcc_server* s);
int lpcc_server_stats(lpcc_server* s, lpcc_stats* st);
void lpcc_server_free(lpcc_server* s);

/*
 * Kernel timing (measurement, no part of the method): when enabled, the context records HIP events around every
 * launch of the kernel family named `name` ("predict", "conv", "up", ...) on
 * its stream and accumulates their durations.  lpcc_timing_read returns the
 * number of launches and the summed milliseconds since the last reset.
 */
int lpcc_timing_enable(lpcc_ctx* c, const char* name);
int lpcc_timing_read(lpcc_ctx* c, int64_t* launches, double* total_ms, int64_t* units);

/*
 * Kernel variants of the gather-GEMM, child-convolution and upsampling
 * launches (the indexed linear transforms of the sparse convolutions,
 * Sec. 3.3, the stride-2 steps of Eq. 4 and the upsampling of Eq. 6).  Each
 * kind has a compacted variant, which works only on the present taps of a
 * wave's rows or the occupied children of a block's parents (wave ballot
 * and prefix count), and a dense one over every tap or child slot (absent
 * ones contribute zeros); a wave computes rb blocks of 16 rows.  rb = 0 (the
 * default) autotunes: the first launch of every (kernel, widths, log2 rows)
 * class on this context runs each candidate, timed with HIP events on the
 * context's stream, and later launches of the class use the fastest.  rb =
 * 1, 2 or 4 fixes the compacted variants (that many row blocks per wave for
 * the gather-GEMMs), 11, 12 or 14 the dense variants with rb - 10 row blocks
 * per wave.  Every choice computes identical outputs.  Returns LPCC_E_INVAL
 * for other values.
 *
 * lpcc_ctx_tuning reports the table: 6 ints per class (kind 0 gemm / 1 up,
 * mode, cin, cout, log2 rows, chosen variant or 0 while undecided) into out
 * (host, 6 * cap ints), the number of classes into *n; LPCC_E_CAPACITY when
 * cap is too small (the first cap rows are written).  Variant codes: rb (1,
 * 2, 4) and 10 + rb for the gather-GEMMs, 101/102 (compacted, 64/128 parents
 * per block) and 110 + rb for the child convolution, 201/202 (compacted,
 * 128/512 parents per block) and 210 + rb for the upsampling.
 *
 * lpcc_ctx_set_tuning imports such a table (host, 6 * n ints, the format
 * lpcc_ctx_tuning writes): each row's class then uses the row's variant
 * without timing candidates, so runs in separate processes (a profiler's
 * counter passes, say) launch the same kernels.  Rows with variant 0 are
 * skipped.  A fixed tiling (lpcc_ctx_set_tiling) still takes precedence.
 * Returns LPCC_E_INVAL, with nothing applied, for a kind other than 0 or 1,
 * widths <= 0, log2 rows outside [0, 62] or a variant code the kind does not
 * have.
 */
int lpcc_ctx_set_tiling(lpcc_ctx* c, int rb);
int lpcc_ctx_set_tuning(lpcc_ctx* c, const int32_t* rows, int n);

/*
 * Graph mode (off by default; launch mechanics only, the computation is that
 * of the calls above).  When on, each launch batch of a call (the
 * level loop of a decode; the model, coder and packing stages of an encode)
 * is captured on the context's stream into a HIP graph and launched as one
 * graph.  The context keeps one executable graph per batch position and call
 * kind and updates it in place (hipGraphExecUpdate) when the next call has
 * the same launch sequence, else instantiates a new one.  Batches that time
 * kernels (autotuning, lpcc_timing_enable) run directly.  Outputs are
 * identical in both modes.  lpcc_ctx_graph_stats counts instantiations and
 * in-place updates since the context was created.
 */
int lpcc_ctx_set_graphs(lpcc_ctx* c, int on);
int lpcc_ctx_graph_stats(lpcc_ctx* c, int64_t* instantiated, int64_t* updated);
int lpcc_ctx_tuning(lpcc_ctx* c, int32_t* out, int cap, int* n);

/*
 * Base geometry (the paper codes the geometry of the levels it does not
 * model directly from the frequencies of their symbols, Sec. S2).  With
 * base depth B > 0 the streams this context encodes code the occupancy codes
 * of depths 0..B-1 with a static table per depth built from the counts of
 * that depth's codes (the integer-softmax rule with counts in place of the
 * exponentials: f_s = 1 + floor(n_s 65281 / N), the rest of 2^16 to the most
 * frequent code), and the model runs from depth B on, with zero features at
 * depth B.  Such streams are version 2: after the depth counts they carry
 * u8 B and, per base depth, u8 m and m pairs (u8 code, u32 count) of the
 * codes present, ascending.  B = 0 (the default) models every depth and
 * writes version 1 streams.  Decoding reads B from each stream.
 * LPCC_E_INVAL for B outside [0, 21); an encode call whose model has its
 * dense fusion depth k0 = D - n_deep - 1 below B fails with LPCC_E_INVAL.
 * lpcc_level_probs always evaluates the model from depth 0.
 */
int lpcc_ctx_set_base_depth(lpcc_ctx* c, int base);

/*
 * How the 3x3x3 neighbour tables of the convolved depths are built (Sec. 3.3
 * runs the sparse convolutions over such tables, built from a coordinate
 * hash).  Both modes give the same tables, entry for entry, hence the same
 * streams and decodes.
 *   mode 0 (default): a coordinate hash (open addressing, linear probing,
 *     2^k >= 2N slots of {u64 key, i32 row}) at the first convolved depth
 *     (an encode also hashes its depths below 32768 nodes, in the two
 *     launches it shares across depths); every other depth derives its
 *     table from its parent depth's table, occupancy codes and first-child
 *     rows (the neighbour at offset delta of the child in slot o of parent p
 *     is child slot (o + delta) mod 2 of the parent-level cell
 *     p + floor((o + delta) / 2), per axis).
 *   mode 1: a coordinate hash and 27 probes per node at every convolved
 *     depth.
 * Applies to the calls made on this context after it returns.  LPCC_E_INVAL
 * for another mode or a null context.
 */
int lpcc_ctx_set_kmap_mode(lpcc_ctx* c, int mode);

/*
 * The integer exponent table of the softmax (Eq. 15; the table covers the
 * non-positive domain, Sec. 3.3 "Integer softmax") as the library builds
 * it: out[i] = round(2^15 e^{-i/16}), i = 0..255, computed on the host with
 * an integer recurrence.  Host memory; needs no device.
 */
int lpcc_softmax_table(int32_t* out);

/*
 * The form in which the kernels evaluate one layer's requantisation (Eq. 14):
 * q(a) = ((a m + 2^(r-1)) >> r) + z_out, m = m_pos for a >= 0 else m_neg,
 * clamped to [-128, 127].  The kernels clamp the int32 accumulator to
 * [a_lo, a_hi] first: a_hi is the smallest a >= 0 with q(a) >= 127 (INT32_MAX
 * if none), a_lo the largest a < 0 with q(a) <= -128 (INT32_MIN if none), so
 * no output changes and the shifted product stays below 2^31.  With r = 0 a
 * multiplier above 256 is replaced by 256 (the same function).
 * out[0..4] = {m_pos, m_neg, a_lo, a_hi, rq24} as used, where rq24 = 1 when
 * a m + 2^(r-1) over the clamped range is an exact 24-bit signed
 * multiply-add inside int32 (the kernels then skip the 64-bit product); host
 * memory (5 int32), needs no device.  LPCC_E_INVAL for parameters a weight blob may not hold (negative
 * multipliers, r outside [0, 62], z_out outside int8).
 */
int lpcc_requant_bounds(int32_t m_pos, int32_t m_neg, int r, int z_out, int32_t* out);

#ifdef __cplusplus
}
#endif
#endif /* LPCC_H */
