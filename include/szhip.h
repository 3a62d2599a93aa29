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

typedef enum { SZ_F32 = 0, SZ_F64 = 1 } sz_dtype;

/* Metric 1 (Sec. II): absolute bound, value-range-relative bound
 * (eb_rel * (max - min)), or both (the smaller of the two applies). */
typedef enum { SZ_EB_ABS = 0, SZ_EB_REL = 1, SZ_EB_ABS_AND_REL = 2 } sz_eb_mode;

typedef struct {
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

/* Create a context on HIP device `device`.  Returns SZ_OK and *ctx. */
int sz_ctx_create(sz_ctx** ctx, int device);
void sz_ctx_destroy(sz_ctx* ctx);

/* Worst-case container size: the 192-byte header plus the raw field (a
 * container never exceeds it: compression falls back to a raw copy). */
size_t sz_compress_bound(const sz_params* p);

/* Compress d_in (dims of p, dtype of p) into d_out (capacity `cap` bytes).
 * Synchronises `stream`; writes the container size to *out_size and, if
 * non-NULL, statistics to *stats.  SZ_ECAPACITY if cap < needed. */
int sz_compress(sz_ctx* ctx, const sz_params* p, const void* d_in, void* d_out,
                size_t cap, size_t* out_size, sz_stats* stats, void* stream);

/* Same pipeline without any host synchronisation (capturable into a HIP
 * graph): the container size is written to device memory *d_out_size
 * (uint64), and a status word (SZ_OK or a negative code) to *d_status
 * (int32).  `cap` must be >= sz_compress_bound(p). */
int sz_compress_async(sz_ctx* ctx, const sz_params* p, const void* d_in, void* d_out,
                      size_t cap, uint64_t* d_out_size, int32_t* d_status, void* stream);

/* Read the parameters and statistics stored in a container header (host
 * memory, at least 192 bytes). */
int sz_inspect(const void* h_hdr, size_t n, sz_params* p, sz_stats* stats);

/* Decompress the container d_comp (comp_size bytes) into d_out (capacity
 * cap bytes).  Synchronises `stream` (it reads the header first). */
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
 * sz_ctx_profile_read fills up to n accumulated milliseconds and call
 * counts, in the order: value range + bound, compression sweep, codebook,
 * encoding + container, decode tables, Huffman decode, unpredictable values,
 * reconstruction sweep.  Returns the number of stages. */
int sz_ctx_profile(sz_ctx* ctx, int enable);
int sz_ctx_profile_read(sz_ctx* ctx, double* ms, uint64_t* calls, int n);

#ifdef __cplusplus
}
#endif
#endif
