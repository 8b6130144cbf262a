/*
 * pmc.h -- C-ABI of the MI355X progressive multi-component compression library.
 *
 * Method: Magri & Lindstrom, "A General Framework for Progressive Data
 * Compression and Retrieval".  A field x is stored as components y_1..y_n,
 * y_i = C(x - x~_{i-1}, tau_i), x~_i = x~_{i-1} + D(y_i), for a strictly
 * decreasing tolerance sequence (Sec. 4.1, Alg. 1).  The sum of the first k
 * decoded components, added left to right in the precision of x (Sec. 3), is
 * the progressive reconstruction x~_k (Sec. 4.2, Alg. 2) and satisfies
 * max|x - x~_k| <= tau_k (Sec. 4.3, Eq. (1)).  The codec C / D is a zfp-style
 * fixed-accuracy codec on 4x4x4 blocks (stream format version 1).
 *
 * Conventions for every call:
 *  - Device pointers (d_*) are allocated by the caller (e.g. PyTorch); the
 *    library never allocates device memory.  Host pointers are plain memory.
 *  - Work is enqueued on the HIP stream given to pmc_ctx_create; calls return
 *    once their kernels are enqueued unless stated otherwise.
 *  - Fields are dense, C order, x fastest: element (x, y, z) is at
 *    x + nx * (y + ny * z).  Lower-dimensional data use extents of 1.
 *    Field pointers given to pmc_compress, pmc_batch_compress, pmc_retrieve,
 *    pmc_refine and pmc_server_submit must be 16-byte aligned (every PyTorch
 *    allocation is):
 *    rows move as 16-byte pieces; others give PMC_E_ARG.
 *  - Return value: PMC_OK (0) or a negative pmc_status; the context keeps a
 *    message for pmc_last_error.  On error no output is valid.
 *  - One context per host thread.
 */
#ifndef PMC_H
#define PMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PMC_OK = 0,
  PMC_E_ARG = -1,         /* bad argument: dims, n, tau not strictly decreasing (Alg. 1 input) or not > 0 */
  PMC_E_NONFINITE = -2,   /* NaN or Inf in the input; the method does not handle them (Sec. 6.1) */
  PMC_E_NOMEM = -3,       /* workspace or stream capacity too small; the size needed is reported */
  PMC_E_CORRUPT = -4,     /* malformed stream */
  PMC_E_UNREACHABLE = -5, /* requested tolerance is below the last component's */
  PMC_E_BOUND = -6,       /* an Eq. (1) bound was missed (not expected; see the acceptance rule) */
  PMC_E_DEVICE = -7,      /* HIP runtime error */
  PMC_E_CANCELLED = -8    /* a served query was cancelled (pmc_server_cancel) */
} pmc_status;

typedef enum { PMC_F32 = 1, PMC_F64 = 2 } pmc_dtype;

/* A 3-D field: extents (x fastest) and element type.  Every call accepts at
 * most 2^36 values and 2^32 blocks of 4x4x4 (PMC_E_ARG beyond). */
typedef struct {
  uint64_t nx, ny, nz;
  int32_t dtype; /* pmc_dtype */
  int32_t reserved;
} pmc_field;

typedef struct pmc_ctx pmc_ctx;
typedef struct pmc_store pmc_store;

/* ---- context ------------------------------------------------------------ */
/* Bind to HIP device `device` and stream `hip_stream` (a hipStream_t; NULL for
 * the default stream). */
pmc_status pmc_ctx_create(int device, void* hip_stream, pmc_ctx** out);
void pmc_ctx_destroy(pmc_ctx* ctx);
/* Message of the last failed call on this context ("" if none). */
const char* pmc_last_error(const pmc_ctx* ctx);

/* Options:
 *  PMC_OPT_FUSED_DECODE (default 1): retrieval decodes all requested
 *    components of a chunk in one pass and writes x~_k once; 0 runs one pass
 *    per component (x~ read and written each time), the literal Alg. 2 loop.
 *    Both give bit-identical results.
 *  PMC_OPT_SYNC_CHECK (default 0): decode calls synchronise the stream and
 *    report PMC_E_CORRUPT when a kernel found a malformed stream.  With 0 the
 *    calls only enqueue work and return PMC_OK; a block whose stream does
 *    not parse is then written as quiet NaNs instead of being left as it
 *    was. */
/*  PMC_OPT_PROFILE (default 0): bracket every kernel launch with HIP events
 *    on the context stream; pmc_prof_read returns the per-kernel totals.
 *  PMC_OPT_CODEC (default 0): the compressor C / D that pmc_compress and
 *    pmc_compress_static put behind the multi-component driver, which works
 *    with any error-bounded lossy compressor (Sec. 6.2):
 *      0  the zfp-style block-transform codec (stream format version 1),
 *      1  prediction and uniform quantisation on the same 4x4x4 blocks (a
 *         prediction-based compressor, Sec. 5): residuals quantised to
 *         multiples of 2 tau (halved per escalation step), a block-local
 *         Lorenzo predictor where it narrows the code, zigzag values at one
 *         width per block; tolerances must lie in [2^-960, 2^1000].
 *    The codec is recorded in every stream header (byte 5) and in the
 *    store; retrieval, refinement, region retrieval, serialisation and the
 *    server follow it.  Batches (pmc_batch_*) use codec 0. */
enum { PMC_OPT_FUSED_DECODE = 1, PMC_OPT_SYNC_CHECK = 2, PMC_OPT_PROFILE = 3, PMC_OPT_CODEC = 4 };
pmc_status pmc_ctx_set_option(pmc_ctx* ctx, int option, int value);

/* Per-kernel launch count and summed duration (milliseconds, from HIP events)
 * since the last reset.  Synchronises the stream.  Fills up to cap entries,
 * sets *n to the number of kernels seen; reset != 0 clears the totals. */
typedef struct {
  char name[32];
  uint64_t launches;
  double ms;
} pmc_prof_entry;
pmc_status pmc_prof_read(pmc_ctx* ctx, pmc_prof_entry* out, int cap, int* n, int reset);

/* ---- range (tau_0 of the tolerance schedule, Sec. 5.1) --------------------
 * min and max of the field in float64 and the number of non-finite values.
 * d_ws: at least 256 bytes of device scratch.  Synchronises the stream. */
pmc_status pmc_range(pmc_ctx* ctx, const pmc_field* f, const void* d_x, void* d_ws, size_t ws_bytes,
                     double* vmin, double* vmax, uint64_t* nonfinite);

/* ---- accuracy gain of a reconstruction (Sec. 5.1.1, its defining equation) -
 * gain = log2(sigma / rmse) - rate: sigma is the standard deviation of x
 * (over all values, float64), rmse the root-mean-square of x - xt, rate the
 * caller's bits per value (for x~_k: all bytes of components 1..k times 8,
 * over the value count).  out[0] = sigma, out[1] = rmse, out[2] = gain
 * (+inf when rmse = 0, -inf when sigma = 0 < rmse).  d_x and d_xt are device
 * fields of the same shape and type (f); d_ws: at least pmc_stats_ws_bytes()
 * bytes of device scratch.  Sums are float64 in a fixed order, so a result
 * repeats bit for bit.  Synchronises the context's stream.  Errors:
 * PMC_E_ARG (null pointer, bad field), PMC_E_NOMEM (workspace too small),
 * PMC_E_DEVICE. */
size_t pmc_stats_ws_bytes(void);
pmc_status pmc_accuracy_gain(pmc_ctx* ctx, const pmc_field* f, const void* d_x, const void* d_xt, double rate,
                             void* d_ws, size_t ws_bytes, double out[3]);

/* ---- a second compressor: the float32 cast of Sec. 3 ------------------------
 * The multi-component driver with C(e) = fl32(e) (round to nearest even
 * float32) and D(y) = y in the field's type; tolerances play no part.  For a
 * float64 field the components form a floating-point expansion: three
 * reproduce every double x with 2^-97 <= |x| < 2^128 (and zero); below that
 * the last component's bits fall under the float32 subnormal spacing, above
 * it the first cast overflows.  pmc_cast_compress runs all n components
 * (1 <= n <= 32) of Alg. 1: component i (i = 0..n-1) goes to d_comps + i * N
 * (N = values of the field; the caller owns the n * N floats), and linf[i]
 * (host, optional) receives max |x - x~_{i+1}| in float64 (synchronises).
 * d_ws: at least 256 bytes of device scratch.  pmc_cast_retrieve writes
 * x~_k = (...((+0 + y_1) + y_2) ...) + y_k, 0 <= k <= 32, in the field's type
 * (enqueued only).  Non-finite input gives unspecified errors.  Errors:
 * PMC_E_ARG, PMC_E_NOMEM, PMC_E_DEVICE. */
pmc_status pmc_cast_compress(pmc_ctx* ctx, const pmc_field* f, const void* d_x, int n, float* d_comps, void* d_ws,
                             size_t ws_bytes, double* linf);
pmc_status pmc_cast_retrieve(pmc_ctx* ctx, const pmc_field* f, const float* d_comps, int k, void* d_out);

/* ---- multi-component compression (Alg. 1, Sec. 4.1) ----------------------
 * Sizes for pmc_compress: device workspace bytes, and the capacity one
 * component's stream can need in the worst case (all blocks raw).  The total
 * stream capacity is at most n * stream_cap_per_comp (each stream starts on a
 * 256-byte boundary). */
pmc_status pmc_compress_sizes(const pmc_field* f, int n, size_t* ws_bytes, size_t* stream_cap_per_comp);

/* Compress d_x into n components with tolerances tau[0] > tau[1] > ... > 0
 * (absolute, pointwise).  Streams are written one after another into d_streams
 * (capacity streams_cap bytes), which must stay alive as long as the store.
 * On success *out holds per-component metadata: prescribed tau and measured
 * max|x - x~_i| in float64 (Sec. 4.3, last paragraph), stream bytes, block
 * counts.  Synchronises the stream once at the end to read the sizes.
 * PMC_E_BOUND still returns the store (valid streams; some blocks exceed
 * their tolerance, counted as misses); the caller frees it. */
pmc_status pmc_compress(pmc_ctx* ctx, const pmc_field* f, const void* d_x, int n, const double* tau,
                        void* d_ws, size_t ws_bytes, void* d_streams, size_t streams_cap, pmc_store** out);

/* ---- compression for callers that cannot allocate device memory ----------
 * For callers that cannot call hipMalloc or run an allocator (code under HIP
 * graph capture, tight serving or simulation loops, harnesses that forbid
 * allocation): pmc_compress with its workspace taken from a static device
 * buffer of PMC_STATIC_WS_BYTES that the library holds on each GPU until the
 * process ends (located by pmc_ctx_create, once per device).  Inputs, outputs
 * and results as for pmc_compress; the caller still passes d_streams.  A
 * field whose workspace (pmc_compress_sizes) exceeds PMC_STATIC_WS_BYTES is
 * refused with PMC_E_NOMEM and the size it needs (about 12 bytes per value
 * for float32 and 24 for float64 with three or more components, so up to
 * about 5.5 M float32 or 2.7 M float64 values).  No device memory is
 * allocated or freed.  Every call on one GPU uses that GPU's one buffer:
 * calls that overlap on a GPU (from other threads or on other streams) race,
 * and the caller must serialise them. */
#define PMC_STATIC_WS_BYTES ((size_t)64 << 20)
pmc_status pmc_compress_static(pmc_ctx* ctx, const pmc_field* f, const void* d_x, int n, const double* tau,
                               void* d_streams, size_t streams_cap, pmc_store** out);

/* Per-component metadata (arrays of store n entries; any may be NULL). */
pmc_status pmc_store_info(const pmc_store* s, int* n, double* tau, double* linf, uint64_t* bytes,
                          uint64_t* nraw, uint64_t* nesc);
/* The codec of a store's components (PMC_OPT_CODEC's values). */
pmc_status pmc_store_codec(const pmc_store* s, int* codec);
/* Block counts of component i (0-based): counts[0..4] = empty, coded, raw,
 * escalated (coded with more planes than the tolerance alone asks for) and
 * tolerance misses. */
pmc_status pmc_store_counts(const pmc_store* s, int i, uint64_t counts[5]);
/* Decode layout of component i (0-based): *max_span_words = the largest
 * number of payload words in four consecutive chunks (the 64 blocks one
 * decode wavefront handles), and *staged = 1 when that span fits the LDS
 * staging buffer of the decoder (those components are read from LDS; larger
 * spans, e.g. streams of mostly raw blocks, are read from device memory).
 * Either pointer may be NULL.  PMC_E_ARG on a bad index. */
pmc_status pmc_store_span(const pmc_store* s, int i, uint64_t* max_span_words, int* staged);
/* Decode route of component i (0-based): *high_half = 1 when the store is
 * float32 with the block-transform codec and every coded block of the
 * component codes its planes in the top ten bit positions of a coefficient
 * with an exponent inside float32's fast dequantisation.  Retrievals whose
 * residual components (index > 0) all qualify run those components' inverse
 * transforms on the coefficients' high 16-bit halves, two per register (the
 * same results).  Found by the encoder, and again from the payload when a
 * store is deserialised.  PMC_E_ARG on a bad index or a NULL pointer. */
pmc_status pmc_store_decode_route(const pmc_store* s, int i, int* high_half);
/* Field of a store. */
pmc_status pmc_store_field(const pmc_store* s, pmc_field* f);
/* Device address and byte size of component i's stream (0-based). */
pmc_status pmc_store_stream(const pmc_store* s, int i, const void** d_stream, uint64_t* bytes);

/* Smallest k with tau_k <= tol (use_measured = 0) or with the measured error
 * <= tol (use_measured = 1), following Sec. 6.2 (tolerances or measured
 * errors stored as per-component metadata).  PMC_E_UNREACHABLE if none. */
pmc_status pmc_select_k(const pmc_store* s, double tol, int use_measured, int* k);

/* ---- progressive reconstruction (Alg. 2, Sec. 4.2) ----------------------
 * Device scratch needed by the decode calls (status word). */
size_t pmc_decode_ws_bytes(void);
/* d_out <- x~_k = (...((+0 + x_1) + x_2) ...) + x_k, 1 <= k <= n. */
pmc_status pmc_retrieve(pmc_ctx* ctx, const pmc_store* s, int k, void* d_out, void* d_ws, size_t ws_bytes);
/* d_inout holds x~_{k_from}; add components k_from+1..k_to in order
 * (incremental refinement without decoder state, Sec. 4.2 last paragraph). */
pmc_status pmc_refine(pmc_ctx* ctx, const pmc_store* s, int k_from, int k_to, void* d_inout, void* d_ws,
                      size_t ws_bytes);
/* Region retrieval (Sec. 6.1: blocks decoded on demand while the components
 * stay compressed): x~_k restricted to the box lo[a] <= coordinate < hi[a]
 * (a = 0, 1, 2 for x, y, z; x fastest, as in pmc_field).  Only the blocks
 * meeting the box are decoded; d_out receives the box alone, dense, x
 * fastest: (hi[0]-lo[0]) * (hi[1]-lo[1]) * (hi[2]-lo[2]) values of the
 * field's type, bit-identical to the same samples of pmc_retrieve(k).
 * 1 <= k <= n; each axis needs lo < hi <= extent (else PMC_E_ARG).  d_ws as
 * for pmc_retrieve; enqueued on the context's stream. */
pmc_status pmc_retrieve_box(pmc_ctx* ctx, const pmc_store* s, int k, const uint64_t lo[3], const uint64_t hi[3],
                            void* d_out, void* d_ws, size_t ws_bytes);

/* ---- persistence --------------------------------------------------------
 * Serialise metadata and streams to host memory (synchronises).  With
 * host_buf == NULL only *used is set to the size needed. */
pmc_status pmc_store_serialize(pmc_ctx* ctx, const pmc_store* s, void* host_buf, size_t cap, size_t* used);
/* Rebuild a store from a serialised blob, uploading its streams into
 * d_streams (capacity cap, caller-owned).  pmc_store_device_bytes validates
 * the blob on the host (sizes with checked arithmetic, every stream header
 * and chunk index; PMC_E_CORRUPT otherwise) and reports the device bytes a
 * store needs: the per-block indexes, the streams and a 512-byte trailer (a
 * status word and per-component flags).  pmc_store_deserialize validates the
 * same way, uploads, rebuilds the per-block indexes on the device (finding
 * each component's decode route, pmc_store_decode_route) and synchronises; a
 * payload that does not parse gives PMC_E_CORRUPT and no store. */
pmc_status pmc_store_device_bytes(const void* host_buf, size_t size, size_t* need);
pmc_status pmc_store_deserialize(pmc_ctx* ctx, const void* host_buf, size_t size, void* d_streams, size_t cap,
                                 pmc_store** out);
void pmc_store_free(pmc_store* s);

/* ---- batches: many fields of uneven size and mixed type ---------------
 * Alg. 1 for nf fields at once.  All components of all fields run as one
 * captured HIP graph, replayed on every pmc_batch_compress: per component a
 * persistent encode kernel per element type walks a list of (field, 64-block
 * group) items, then a segmented chunk scan and a batched pack run.  The
 * schedule (persistent grid = grid_mult x compute units; item order 0 =
 * field-major, 1 = interleaved across fields, 2 = largest field first) never
 * changes the output bytes.  n[i] components for field i with tolerances
 * tau[i][0] > ... > tau[i][n[i]-1] > 0.  With the environment variable
 * PMC_TUNE_CACHE naming a file, plans reuse and pmc_batch_tune records the
 * schedule chosen for the same size class. */
typedef struct pmc_batch pmc_batch;
pmc_status pmc_batch_plan(pmc_ctx* ctx, int nf, const pmc_field* fields, const int* n, const double* const* tau,
                          pmc_batch** out);
/* device workspace and stream-buffer bytes a batch needs */
pmc_status pmc_batch_sizes(const pmc_batch* b, size_t* ws_bytes, size_t* streams_bytes);
pmc_status pmc_batch_schedule(pmc_batch* b, int grid_mult, int order);
pmc_status pmc_batch_get_schedule(const pmc_batch* b, int* grid_mult, int* order);
/* d_x[i]: field i on the device.  out[i] receives a store per field whose
 * streams live in d_streams.  Synchronises once to read the sizes. */
pmc_status pmc_batch_compress(pmc_batch* b, const void* const* d_x, void* d_ws, size_t ws_bytes, void* d_streams,
                              size_t streams_cap, pmc_store** out);
/* Autotuner: times every schedule (grid_mult 1, 2, 4, 8 x 3 orders) on these
 * inputs with HIP events, keeps the fastest and reports its graph time. */
pmc_status pmc_batch_tune(pmc_batch* b, const void* const* d_x, void* d_ws, size_t ws_bytes, void* d_streams,
                          size_t streams_cap, float* best_ms);
const char* pmc_batch_order_name(int order);
void pmc_batch_free(pmc_batch* b);

/* ---- serving progressive-retrieval queries ---------------------------
 * A request loop on a host thread serves queries "field f at tolerance tau"
 * with k = the smallest component count whose prescribed tolerance is <= tau
 * (Sec. 6.2).  Decoded partial sums x~_k stay resident on the device in a
 * (field, k) cache inside the caller's arena, so a query is served by copying
 * a cached x~_k, by refining the cached x~_j with the largest j < k
 * (components j+1..k, Sec. 4.2), or by decoding from scratch.  Continuous
 * batching: every step admits waiting queries in arrival order while batch
 * slots (max_batch) and the HBM budget allow and decodes all of them in one
 * launch per element type; steps are enqueued while earlier steps run.  The
 * budget bounds the arena bytes in use (cache entries and result slots) plus
 * the caller outputs of running queries; least-recently-used cache entries
 * that no running step touches are evicted to admit a query.  Results are
 * bit-identical alone or in a mix.  The stores added must outlive the server.
 * A query with d_out == NULL gets a result slot in the arena, readable via
 * pmc_server_result until pmc_server_release.  Internally synchronised. */
typedef struct pmc_server pmc_server;
typedef struct {
  uint64_t submitted, completed, hits, partial, misses, steps, batched_queries, max_queue;
  uint64_t cache_entries, cache_bytes, arena_peak, pending, running;
  uint64_t cancelled;
} pmc_server_stats;
pmc_status pmc_server_create(pmc_ctx* ctx, size_t hbm_budget, void* d_arena, size_t arena_bytes, int max_batch,
                             pmc_server** out);
pmc_status pmc_server_add(pmc_server* s, const pmc_store* store, int* field_id);
/* PMC_E_UNREACHABLE when tol is below the field's last tolerance */
pmc_status pmc_server_submit(pmc_server* s, int field_id, double tol, void* d_out, uint64_t* ticket);
/* Seconds on the monotonic clock the server measures latencies with. */
double pmc_clock(void);
/* As pmc_server_submit, with the query's arrival time given on pmc_clock()'s
 * clock (e.g. its scheduled time in an arrival trace): the latency counts
 * from there, so time spent before the call (a submitter running late) is
 * included.  arrival <= 0, or later than the call, means the call itself. */
pmc_status pmc_server_submit_at(pmc_server* s, int field_id, double tol, void* d_out, double arrival,
                                uint64_t* ticket);
/* latency_s = completion - arrival in seconds (-1 while running); arrival is
 * the submission, or the time given to pmc_server_submit_at */
pmc_status pmc_server_poll(pmc_server* s, uint64_t ticket, int* done, pmc_status* st, double* latency_s);
/* device address of a finished query's x~_k; source: 0 decoded from scratch,
 * 1 refined from a cached partial sum, 2 copied from the cache */
pmc_status pmc_server_result(pmc_server* s, uint64_t ticket, const void** d_result, int* k, int* source);
pmc_status pmc_server_release(pmc_server* s, uint64_t ticket);
/* Cancels a query.  One still waiting is removed from the queue and never
 * runs.  One already admitted to a running step finishes on the device, and
 * its result slot is returned when that step ends (a caller's d_out may be
 * written until then).  Either way pmc_server_poll then reports it done with
 * status PMC_E_CANCELLED (for a running one: once its step has ended),
 * pmc_server_result refuses it and pmc_server_release is a no-op.  PMC_OK,
 * also for a query cancelled before; PMC_E_ARG for an unknown ticket or a
 * query that has already finished (release it instead). */
pmc_status pmc_server_cancel(pmc_server* s, uint64_t ticket);
pmc_status pmc_server_get_stats(pmc_server* s, pmc_server_stats* out);
/* finishes every submitted query, then stops the request loop */
void pmc_server_destroy(pmc_server* s);

#ifdef __cplusplus
}
#endif
#endif /* PMC_H */
