/*
 * szref.h -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow, sequential CPU oracle of the error-bounded lossy compressor of
 * arXiv 1706.03791 (SZ-1.4): multilayer prediction (Sec. III-A, Eq. predmodel),
 * error-controlled linear-scaling quantization into 2^m codes (Sec. IV-A),
 * storage of unpredictable points by binary-representation truncation
 * (Sec. IV-B, Algorithm 1), Huffman coding of the codes (Sec. IV-A) and the
 * matching decompressor.
 *
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library.  It shares no code, header or table with the GPU
 * library; the container layout and the arithmetic rules are re-implemented
 * here from their written definition.
 *
 * Error codes (negative ints): 0 ok, -1 invalid argument, -2 capacity too
 * small, -3 corrupt stream, -4 non-finite data in a range-relative mode,
 * -5 out of memory.
 */
#ifndef SZREF_H
#define SZREF_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define SZREF_OK 0
#define SZREF_EINVAL -1
#define SZREF_ECAPACITY -2
#define SZREF_ECORRUPT -3
#define SZREF_ENONFINITE -4
#define SZREF_ENOMEM -5

typedef struct {
  uint32_t dtype;      /* 0 = float32, 1 = float64 */
  uint32_t ndim;       /* 1..3 */
  uint64_t dims[3];    /* slowest first; dims[ndim-1] is contiguous */
  uint64_t block[3];   /* independent block extents, 0 = default */
  uint32_t layers;     /* n in [1,4] */
  uint32_t quant_bits; /* m in [1,16]; 0 = adaptive */
  uint32_t eb_mode;    /* 0 abs, 1 value-range relative, 2 both (minimum) */
  uint32_t chunk;      /* symbols per decode chunk: 0 = 1024, else a multiple of 256 in [256, 4096] */
  double eb_abs;
  double eb_rel;
  double theta;        /* hit-rate threshold for the adaptive rule, 0 = 0.9 */
  uint32_t unpred_coding; /* 0: unpredictable values as sign+exponent heads and
                             kept-bit tails; 1: each value of a chunk XORed
                             with the chunk's previous one, leading zero bytes
                             counted, the remaining kept bits stored */
  uint32_t reserved;
} szref_params;

typedef struct {
  uint64_t n_points, n_unpred, huff_bits, tail_bits, compressed_bytes;
  uint64_t ebT_bits;   /* bit pattern of the error bound used, in the element type */
  double eb_used, hit_rate, value_min, value_max;
  uint32_t m_used, m_suggested, raw_fallback, n_used_syms;
} szref_stats;

/* Resolved error bound, all in the element type's arithmetic. */
typedef struct {
  double eb;           /* bound before rounding into the element type */
  double ebT, twoeb, inv2eb; /* values of the element-type quantities */
  uint64_t ebT_bits, twoeb_bits, inv2eb_bits;
  double vmin, vmax;
} szref_eb;

int szref_resolve_eb(const szref_params* p, const void* data, szref_eb* out);

/* (n+1)^d - 1 prediction coefficients in lexicographic order of k (slowest
 * dimension outermost).  Writes the offsets k (d entries per term) into
 * `koff` when non-NULL.  Returns the number of terms or a negative error. */
int szref_coefficients(uint32_t ndim, uint32_t n, int64_t* coef, int32_t* koff, int cap);

/* Prediction from the ORIGINAL values (the R_PH^orig variant of Sec. III-B),
 * evaluated in the element type; used to pin the predictor. */
int szref_predict_original(const szref_params* p, const void* data, void* pred_out);

/* One traversal at a fixed m: codes (u16, raster order) and the decompressed
 * values the compressor records for later predictions.  n_unpred counts
 * code-0 points. */
int szref_quantize(const szref_params* p, const void* data, uint32_t m,
                   uint16_t* codes, void* xprime, uint64_t* n_unpred);

/* Huffman code lengths over `nsym` frequencies (zero = unused).  Returns the
 * maximum length or a negative error. */
int szref_huffman_lengths(const uint64_t* freq, uint32_t nsym, uint8_t* len);

size_t szref_compress_bound(const szref_params* p);

/* Full compressor.  *out is malloc'd (free with szref_free). */
int szref_compress(const szref_params* p, const void* data, uint8_t** out,
                   size_t* out_size, szref_stats* stats);

/* Same, also returning the codes and recorded decompressed values. */
int szref_compress_debug(const szref_params* p, const void* data, uint8_t** out,
                         size_t* out_size, szref_stats* stats, uint16_t* codes,
                         void* xprime);

int szref_decompress(const uint8_t* comp, size_t size, void* out, size_t cap);

/* Header fields: fills params (dims, dtype, ...) from a container. */
int szref_inspect(const uint8_t* comp, size_t size, szref_params* p, szref_stats* s);

void szref_free(void* ptr);

#ifdef __cplusplus
}
#endif
#endif
