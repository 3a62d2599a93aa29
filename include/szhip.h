/*
 * szhip.h -- C ABI of the MI355X (gfx950) error-bounded lossy compressor
 * implementing the method of arXiv 1706.03791 (SZ-1.4):
 *   - multilayer prediction of every point from preceding *decompressed*
 *     neighbours along all dimensions (Sec. III-A, Eq. predmodel; the
 *     1-layer case is the Lorenzo predictor);
 *   - error-controlled linear-scaling quantization into 2^m codes, code 0
 *     marking unpredictable points (Sec. IV-A), with the adaptive choice of
 *     m (Sec. IV-B);
 *   - storage of unpredictable points by binary-representation reduction
 *     (Sec. IV-B, Algorithm 1);
 *   - Huffman coding of the codes over any alphabet size (Sec. IV-A);
 *   - the matching decompressor.
 *
 * All pointers named d_* are device pointers (HIP device memory on the
 * context's GPU) and must be 16-byte aligned; h_* are host pointers.  Every
 * buffer is owned by the caller; the library never frees caller memory.  A
 * context owns its scratch memory, which grows on demand and is released by
 * sz_ctx_destroy.  Work is enqueued on the given HIP stream (hipStream_t
 * passed as void*; NULL = the null stream).
 *
 * Errors are negative return codes, never exceptions:
 *   SZ_EINVAL     invalid parameters or misaligned pointer;
 *   SZ_ECAPACITY  output capacity too small (output contents undefined);
 *   SZ_ECORRUPT   container fails its consistency checks;
 *   SZ_ENONFINITE range-relative bound requested on data with NaN/Inf;
 *   SZ_ENOMEM     scratch allocation failed;
 *   SZ_EHIP       a HIP runtime call failed.
 * One context per host thread; several streams may be used with one context
 * only if calls on it are serialised by the caller.
 */
#ifndef SZHIP_H
#define SZHIP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SZ_OK 0
#define SZ_EINVAL (-1)
#define SZ_ECAPACITY (-2)
#define SZ_ECORRUPT (-3)
#define SZ_ENONFINITE (-4)
#define SZ_ENOMEM (-5)
#define SZ_EHIP (-6)
#define SZ_ESTALL (-7) /* internal dataflow wait exceeded its bound (a bug) */
#define SZ_ETIMEDOUT (-8) /* sz_server_wait: the request did not finish in time */
#define SZ_ESCRATCH (-9)  /* sz_compress_async_noalloc: workspace beyond its static scratch */

typedef enum { SZ_F32 = 0, SZ_F64 = 1 } sz_dtype;

/* Metric 1 (Sec. II): absolute bound, value-range-relative bound
 * (eb_rel * (max - min)), or both (the smaller of the two applies). */
typedef enum { SZ_EB_ABS = 0, SZ_EB_REL = 1, SZ_EB_ABS_AND_REL = 2 } sz_eb_mode;

/* Parameters of one field (Sec. II states the problem: a d-dimensional
 * floating-point array compressed under a user bound; Sec. III-A the layer
 * count n; Sec. IV-A/IV-B the interval count 2^m and its adaptive choice). */
typedef struct {
  uint32_t struct_size; /* sizeof(sz_params), checked by every entry point that
                           takes parameters (SZ_EINVAL on a mismatch): the ABI
                           version of the caller's struct */
  uint32_t dtype;      /* sz_dtype */
  uint32_t ndim;       /* 1..3 */
  uint64_t dims[3];    /* C order, slowest first; dims[ndim-1] is contiguous
                          (the paper's lowest dimension n^(1), Algorithm 1) */
  uint64_t block[3];   /* independent-block extents; 0 = default (whole
                          extent for ndim >= 2, 2048 points for ndim == 1) */
  uint32_t layers;     /* n in [1,4] (Sec. III; the paper's default is 1) */
  uint32_t quant_bits; /* m in [1,16]: 2^m codes, 2^m - 1 intervals; 0 = adaptive */
  uint32_t eb_mode;    /* sz_eb_mode */
  uint32_t chunk;      /* Huffman symbols per decode chunk: 0 = 1024, else a
                          multiple of 256 in [256, 4096] */
  double eb_abs;       /* absolute bound (>= 0) */
  double eb_rel;       /* value-range-relative bound (>= 0) */
  double theta;        /* hit-rate threshold of the adaptive rule, 0 = 0.9 */
  uint32_t unpred_coding; /* storage of unpredictable values (Sec. IV-B, Algorithm 1):
                             0 = binary-representation reduction: sign and
                             exponent, then the kept mantissa bits of each value;
                             1 = the same reduced values, each XORed with the
                             previous one of its decode chunk, storing the count
                             of identical leading bytes and the bits after them */
  uint32_t reserved;   /* 0 */
} sz_params;

typedef struct {
  uint64_t n_points, n_unpred, huff_bits, tail_bits, compressed_bytes;
  uint64_t ebT_bits;   /* bit pattern of the bound used, in the element type */
  double eb_used;      /* that bound as a double */
  double hit_rate;     /* R_PH = 1 - unpredictable / N (Sec. III-B) */
  double value_min, value_max; /* range (relative modes only) */
  uint32_t m_used, m_suggested, raw_fallback, n_used_syms;
} sz_stats;

typedef struct sz_ctx sz_ctx;

/* Create a context on HIP device `device`.  Returns SZ_OK and *ctx
 * (SZ_EHIP for a bad device, SZ_ENOMEM if its small device plan cannot be
 * allocated).  The context owns its scratch arena and device plan; it holds
 * no caller memory.  Not a method of the paper: the state of the library. */
int sz_ctx_create(sz_ctx** ctx, int device);
/* Wait for the context's device, then free everything the context owns.
 * NULL is a no-op.  The context must not be used afterwards. */
void sz_ctx_destroy(sz_ctx* ctx);

/* Worst-case container size: the 192-byte header plus the raw field.  The
 * paper does not say what happens when coding expands the data; here a
 * container never exceeds the raw field plus its header, because
 * compression falls back to a raw copy (a lossless verbatim store).  Returns
 * 0 for invalid parameters. */
size_t sz_compress_bound(const sz_params* p);

/* Compress d_in (dims of p, dtype of p, row-major with dims[ndim-1]
 * contiguous) into the container d_out (capacity `cap` bytes), so that every
 * decompressed value lies strictly within the bound of the original (Sec. II,
 * Metric 1): range and bound resolution, then Algorithm 1 -- multilayer
 * prediction from decompressed neighbours (Sec. III-A, Eq. predmodel),
 * error-controlled quantization into 2^m codes (Sec. IV-A) with the adaptive
 * choice of m when quant_bits is 0 (Sec. IV-B), unpredictable values by
 * binary-representation reduction (Sec. IV-B), Huffman coding of the codes
 * (Sec. IV-A).  Synchronises `stream`; writes the container size to
 * *out_size and, if non-NULL, statistics to *stats.  Errors: SZ_EINVAL
 * (parameters, alignment), SZ_ENONFINITE (relative bound on NaN/Inf),
 * SZ_ECAPACITY (cap < container size; d_out contents undefined), SZ_ENOMEM,
 * SZ_EHIP. */
int sz_compress(sz_ctx* ctx, const sz_params* p, const void* d_in, void* d_out,
                size_t cap, size_t* out_size, sz_stats* stats, void* stream);

/* The pipeline of sz_compress (Sec. II, Algorithm 1) without any host
 * synchronisation, so it can be captured into a HIP graph: the container size
 * is written to device memory *d_out_size (uint64) and a status word (SZ_OK
 * or a negative code: SZ_ECAPACITY, SZ_ENONFINITE) to *d_status (int32) when
 * the stream reaches them.  The return value reports only what the host can
 * see (parameters, alignment, allocation of the context's scratch, which
 * happens on the first call of a size and must not happen under capture). */
int sz_compress_async(sz_ctx* ctx, const sz_params* p, const void* d_in, void* d_out,
                      size_t cap, uint64_t* d_out_size, int32_t* d_status, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * pipeline and the same bytes as sz_compress_async, with every piece of
 * workspace (codes, tile boundary records, histograms, chunk tables, the
 * device plan) taken from a static device array of
 * SZ_NOALLOC_SCRATCH_BYTES that the library holds on each GPU until the
 * process ends.  Nothing is allocated: no hipMalloc, hipFree or allocating
 * library call.  The context only names the device (its own scratch is not
 * used).  Fields whose workspace exceeds the static array fail with
 * SZ_ESCRATCH before anything is enqueued; the 512^3 f32 field at m <= 8
 * fits.  Every call on one GPU shares that GPU's array, and the array keeps
 * the last call's contents (each call clears what it needs cleared), so
 * calls whose executions overlap on one GPU race and must be serialised by
 * the caller (one stream, or events). */
#define SZ_NOALLOC_SCRATCH_BYTES (256u << 20)
int sz_compress_async_noalloc(sz_ctx* ctx, const sz_params* p, const void* d_in, void* d_out,
                              size_t cap, uint64_t* d_out_size, int32_t* d_status, void* stream);

/* Read the parameters and statistics stored in a container header (host
 * memory, n >= 192 bytes; the container format is this library's, not the
 * paper's).  The header is fully checked first: every count within its
 * bounds and every section offset equal to the layout the compressor writes;
 * SZ_ECORRUPT otherwise.  No device work. */
int sz_inspect(const void* h_hdr, size_t n, sz_params* p, sz_stats* stats);

/* Decompress the container d_comp (comp_size bytes) into d_out (capacity
 * cap bytes): Huffman decoding of the codes (Sec. IV-A), the stored
 * unpredictable values (Sec. IV-B), and the reconstruction of every point
 * from the same prediction the compressor made from decompressed neighbours
 * (Sec. III-A, Eq. predmodel): x' = prediction + (code - 2^(m-1)) * 2eb.
 * Synchronises `stream` (it reads and checks the header first).  Errors:
 * SZ_ECORRUPT (header or content inconsistent), SZ_ECAPACITY (cap smaller
 * than the field), SZ_EINVAL, SZ_ENOMEM, SZ_EHIP. */
int sz_decompress(sz_ctx* ctx, const void* d_comp, size_t comp_size, void* d_out,
                  size_t cap, void* stream);

/* Debug entry of the prediction + quantization sweep alone: writes the
 * codes (uint16, raster order) of one traversal at fixed m = p->quant_bits
 * (1..16) and, if d_xprime is non-NULL, the decompressed values the
 * compressor records (dtype of p).  Synchronises `stream`. */
int sz_quantize(sz_ctx* ctx, const sz_params* p, const void* d_in, uint16_t* d_codes,
                void* d_xprime, sz_stats* stats, void* stream);

const char* sz_strerror(int code);

/* Instrumentation (for benchmarks; not needed by callers of the codec).
 * sz_ctx_profile(ctx, 1) resets and enables per-stage HIP-event timing of
 * the synchronous calls sz_compress / sz_decompress on their stream;
 * sz_ctx_profile(ctx, SZ_PROFILE_STAGES | mask) times only the stages whose
 * bits (in the order below) are set in mask, since every timed stage adds
 * two event records to the stream; 0 disables; other values: SZ_EINVAL.
 * sz_ctx_profile_read fills up to n accumulated milliseconds and call
 * counts, in the order: value range + bound, compression sweep, codebook,
 * encoding + container, decode tables, Huffman decode, unpredictable values,
 * reconstruction sweep, code histogram (when it is a kernel of its own).
 * Returns the number of stages. */
#define SZ_PROFILE_STAGES 0x10000
int sz_ctx_profile(sz_ctx* ctx, int enable);
/* Schedule-invariance check (for tests; not needed by callers of the codec).
 * Later calls on the context run their prediction and reconstruction sweeps
 * (Algorithm 1's traversal, kept in the dependence order Sec. III-A fixes)
 * with another schedule: `schedule` 0 = default tiles, 1 = row-per-thread
 * tiles for every field; `claim_order` 0..2 = the order in which workgroups
 * claim the tiles (0 = default; 1 = another dependence order within each
 * block; 2 = that, with the independent blocks in reverse).  Every schedule
 * must produce the same bytes.  SZ_EINVAL for values out of range. */
int sz_ctx_debug_sweep(sz_ctx* ctx, int schedule, int claim_order);
int sz_ctx_profile_read(sz_ctx* ctx, double* ms, uint64_t* calls, int n);

/* ---------------------------------------------------------------- analysis
 * Error metrics of a reconstruction (Sec. II, Metric 2: RMSE, NRMSE, PSNR;
 * Metric 3: Pearson correlation coefficient) and the autocorrelation of the
 * compression errors (Sec. V), computed on the device in double precision
 * with a fixed reduction order.  e_i = x_i - x'_i in double; value range R_X
 * = max - min of the original; rmse = sqrt(mean e^2); nrmse = rmse / R_X;
 * psnr = 20 log10(R_X / rmse); pearson = cov(X, X') / (sigma_X sigma_X').
 * Autocorrelation at lag k (raster order): sum_{i+k<N} d_i d_{i+k} / sum d_i^2
 * with d = e - mean(e). */
typedef struct {
  uint64_t n;
  double value_min, value_max, value_range;
  double max_abs_err, mean_err;
  double rmse, nrmse, psnr, pearson;
} sz_quality_t;

/* d_orig and d_recon hold n (>= 2) elements of dtype; max_lag in [0, 255]
 * autocorrelation coefficients (lags 1..max_lag) go to h_autocorr (host,
 * may be NULL when max_lag is 0).  Synchronises `stream`; uses the
 * context's scratch. */
int sz_quality(sz_ctx* ctx, uint32_t dtype, uint64_t n, const void* d_orig, const void* d_recon,
               uint32_t max_lag, double* h_autocorr, sz_quality_t* out, void* stream);

/* Best-layer study (Sec. III-B, Table II): for n = 1..4 layers, the
 * prediction hitting rate R_PH of a centred sub-block of the field (extents
 * sample[d], slowest first; NULL or 0 = whole extent) with one interval
 * around the prediction (the quantizer at m = 1: a point is predictable when
 * it lies within the bound of its prediction), predicting from decompressed
 * values (rph_decomp[n-1], the compressor's case) and from original values
 * (rph_orig[n-1]).  The bound is that of the whole field under p's mode and
 * values; p->layers and p->quant_bits are ignored.  *best_n is the n with the
 * highest rph_decomp (the smallest such n on ties).  Synchronises `stream`. */
int sz_layer_survey(sz_ctx* ctx, const sz_params* p, const void* d_in, const uint64_t* sample,
                    double* rph_decomp, double* rph_orig, uint32_t* best_n, void* stream);

/* ------------------------------------------------------------ batched form
 * Many fields of uneven shape compressed together (not a method of the
 * paper: a throughput form of the same per-field computation).  Every stage
 * runs as one launch for the whole batch and the prediction sweep is one
 * persistent launch over the tiles of all fields; the sequence can be
 * captured into a HIP graph and replayed.  The container of field i is
 * byte-identical to what sz_compress produces for params[i] and input i.
 *
 * sz_batch_create plans a batch of n (1..65535) fields of one dtype for the
 * context's device.  `schedule` selects a tile schedule (0..3, see
 * sz_batch_info) or -1 to time all schedules on the first sz_batch_compress
 * and keep the fastest (cached per batch signature for the process).  The
 * batch owns its workspace and per-field plans; the context is only used
 * for its device and must outlive the batch.
 *
 * sz_batch_compress enqueues the compression of d_in[i] (dims of params[i])
 * into d_out[i] (capacity caps[i], >= sz_compress_bound(params[i]) to avoid
 * SZ_ECAPACITY) without host synchronisation (autotuning, when pending,
 * synchronises).  Container sizes go to device uint64 d_sizes[i] and status
 * words (SZ_OK or a negative code) to device int32 d_status[i].  With
 * use_graph != 0 the sequence is captured once per set of buffers into a HIP
 * graph (on a stream of the batch, ordered after and before `stream`) and
 * replayed.  Calls on one batch must not overlap in time on different
 * streams. */
typedef struct sz_batch sz_batch;
int sz_batch_create(sz_ctx* ctx, uint32_t n, const sz_params* params, int schedule, sz_batch** batch);
int sz_batch_compress(sz_batch* batch, const void* const* d_in, void* const* d_out, const size_t* caps,
                      uint64_t* d_sizes, int32_t* d_status, int use_graph, void* stream);
/* Schedule in use (-1 before tuning), sweep tiles of the batch, threads per
 * sweep workgroup, and the tuned time (ms) of each candidate (0 if not
 * measured).  Returns the number of candidate schedules. */
int sz_batch_info(const sz_batch* batch, int* schedule, uint32_t* tiles, int* threads, double* tune_ms, int n_ms);
void sz_batch_destroy(sz_batch* batch);

/* ------------------------------------------------------------- served form
 * A request server with continuous batching (not a method of the paper: a
 * serving form of the same per-request work).  A native scheduler thread
 * admits submitted requests, in arrival order, as execution slots (one HIP
 * stream each) and HBM free up, so requests arriving while others run
 * overlap with them on the device.  Every request's workspace is carved from
 * one device pool of `hbm_budget` bytes allocated by sz_server_create, and
 * nothing is allocated while serving.  Admission is by HBM footprint: the
 * request's input, its output capacity and its workspace all count against
 * `hbm_budget` while it is in flight.  A request that does not fit in what is
 * left lets later requests pass for at most 50 ms, then admission waits for
 * it; a request whose footprint exceeds the whole budget fails with
 * SZ_ENOMEM.  Results equal those of sz_compress /
 * sz_decompress on the same input.  Input and output buffers belong to the
 * client and must stay valid until sz_server_wait returns for the request. */
#define SZ_REQ_COMPRESS 0
#define SZ_REQ_DECOMPRESS 1

typedef struct {
  uint32_t op;          /* SZ_REQ_COMPRESS or SZ_REQ_DECOMPRESS */
  uint32_t reserved;
  sz_params params;     /* compress: the field; decompress: ignored */
  const void* d_in;     /* compress: field (device); decompress: container (device) */
  size_t in_bytes;      /* decompress: container size in bytes */
  const void* h_header; /* decompress: optional host copy of the container's first
                           192 bytes (NULL: the server reads it from d_in) */
  void* d_out;          /* compress: container buffer; decompress: field buffer (device) */
  size_t out_cap;       /* capacity of d_out in bytes */
} sz_request;

typedef struct {
  int32_t status;       /* SZ_OK or a negative code */
  uint32_t slot;        /* execution slot that ran the request */
  uint64_t out_size;    /* container bytes (compress) or field bytes (decompress) */
  uint64_t workspace_bytes;
  double t_submit, t_admit, t_done; /* seconds on the server's steady clock */
} sz_result;

typedef struct {
  uint64_t submitted, admitted, completed;
  uint32_t in_flight, max_in_flight;
  uint64_t pool_bytes, pool_peak_bytes; /* the budget, and the peak footprint in flight */
  double clock_s;       /* the server clock now */
} sz_server_stats_t;

typedef struct sz_server sz_server;
/* Start a server on `device` with a workspace pool of hbm_budget bytes
 * (>= 1 MiB) and `slots` (1..64) concurrent requests. */
int sz_server_create(int device, size_t hbm_budget, uint32_t slots, sz_server** server);
/* Queue a request (thread-safe, never blocks on the GPU); *id names it. */
int sz_server_submit(sz_server* server, const sz_request* req, uint64_t* id);
/* Wait for request `id` (timeout_ms < 0: no limit) and release its record:
 * SZ_OK with *res filled, SZ_ETIMEDOUT, or SZ_EINVAL for an unknown id. */
int sz_server_wait(sz_server* server, uint64_t id, sz_result* res, int timeout_ms);
int sz_server_stats(sz_server* server, sz_server_stats_t* stats);
/* Finish every queued request, then stop the scheduler and free the pool. */
void sz_server_destroy(sz_server* server);

#ifdef __cplusplus
}
#endif
#endif
