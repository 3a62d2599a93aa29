/*
 * szref.c -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain sequential CPU oracle of the SZ-1.4 compressor (arXiv 1706.03791).
 * Written for checking by eye against the paper, not for speed: one point
 * at a time in raster order, one bit at a time in the Huffman coder.
 * Only the test suite, the smoke check and the benchmark's CPU-baseline leg
 * may load it.  Build: gcc -O2 -ffp-contract=off -fno-fast-math.
 *
 * Readings taken where the paper is silent:
 *  - memory is row-major, last index contiguous (the paper's lowest dimension);
 *  - neighbours outside the independent block read as zero;
 *  - eb in the element type is the double bound rounded toward zero;
 *    k = round-half-even((x - p) * (1 / 2eb)); accept iff |x - x_q| < eb;
 *  - unpredictable values keep sign, exponent and the top e(x) - e(eb)
 *    mantissa bits (binary-representation truncation);
 *  - Huffman: two-queue merge over leaves sorted by (frequency, symbol),
 *    leaf preferred on equal weights, code lengths <= 27 enforced by halving
 *    frequencies, canonical codes in (length, symbol) order, MSB-first bits;
 *  - adaptive m: run at m = 16, take the smallest m whose 2^m - 1 intervals
 *    cover theta = 0.9 of the points, rerun at that m.
 */
#include "szref.h"

#include <math.h>
#include <float.h>
#include <stdlib.h>
#include <string.h>

#define DEFAULT_CHUNK 1024u
#define DEFAULT_BLOCK_1D 2048u
#define LMAX 27
#define HDR_SIZE 192u
#define SECTION_ALIGN 64u
#define MAGIC 0x31485A53u /* bytes "SZH1" */
#define VERSION 2u

/* ------------------------------------------------------------------ layout */

struct layout {
  uint64_t dims[3];   /* padded to 3 dims: leading 1s */
  uint64_t block[3];
  uint64_t stride[3];
  uint64_t n;
};

struct stencil {
  int nterms;
  int64_t coef[124];
  int32_t koff[124 * 3]; /* offsets per padded dimension */
};

static int make_layout(const szref_params* p, struct layout* L) {
  if (p->ndim < 1 || p->ndim > 3) return SZREF_EINVAL;
  int pad = 3 - (int)p->ndim;
  for (int d = 0; d < 3; d++) { L->dims[d] = 1; L->block[d] = 1; }
  uint64_t n = 1;
  for (uint32_t d = 0; d < p->ndim; d++) {
    /* N < 2^40, tested before the product so that it cannot wrap */
    if (p->dims[d] == 0 || p->dims[d] > ((1ull << 40) - 1) / n) return SZREF_EINVAL;
    L->dims[pad + d] = p->dims[d];
    n *= p->dims[d];
  }
  for (uint32_t d = 0; d < p->ndim; d++) {
    uint64_t b = p->block[d];
    if (b == 0) b = (p->ndim == 1) ? DEFAULT_BLOCK_1D : p->dims[d];
    if (b > p->dims[d]) b = p->dims[d];
    L->block[pad + d] = b;
  }
  L->stride[2] = 1;
  L->stride[1] = L->dims[2];
  L->stride[0] = L->dims[1] * L->dims[2];
  L->n = n;
  return SZREF_OK;
}

static int64_t binom(int n, int k) {
  int64_t r = 1;
  for (int i = 1; i <= k; i++) r = r * (n - k + i) / i;
  return r;
}

/* Eq. predmodel: c_k = -prod_j (-1)^{k_j} C(n, k_j) over k in [0,n]^d \ {0}. */
int szref_coefficients(uint32_t ndim, uint32_t n, int64_t* coef, int32_t* koff, int cap) {
  if (ndim < 1 || ndim > 3 || n < 1 || n > 4) return SZREF_EINVAL;
  int count = 0;
  int32_t k[3] = {0, 0, 0};
  int total = 1;
  for (uint32_t d = 0; d < ndim; d++) total *= (int)(n + 1);
  for (int idx = 0; idx < total; idx++) {
    /* decode idx into k with the slowest dimension most significant */
    int rem = idx;
    for (int d = (int)ndim - 1; d >= 0; d--) { k[d] = rem % (int)(n + 1); rem /= (int)(n + 1); }
    int allzero = 1;
    for (uint32_t d = 0; d < ndim; d++) if (k[d]) allzero = 0;
    if (allzero) continue;
    int64_t prod = 1;
    for (uint32_t d = 0; d < ndim; d++) {
      int64_t b = binom((int)n, k[d]);
      prod *= (k[d] & 1) ? -b : b;
    }
    if (count >= cap) return SZREF_EINVAL;
    if (coef) coef[count] = -prod;
    if (koff) for (uint32_t d = 0; d < ndim; d++) koff[count * (int)ndim + (int)d] = k[d];
    count++;
  }
  return count;
}

static int make_stencil(uint32_t ndim, uint32_t n, struct stencil* S) {
  int32_t kd[124 * 3];
  int c = szref_coefficients(ndim, n, S->coef, kd, 124);
  if (c < 0) return c;
  S->nterms = c;
  int pad = 3 - (int)ndim;
  for (int t = 0; t < c; t++) {
    for (int d = 0; d < 3; d++) S->koff[t * 3 + d] = 0;
    for (uint32_t d = 0; d < ndim; d++) S->koff[t * 3 + pad + (int)d] = kd[t * (int)ndim + (int)d];
  }
  return SZREF_OK;
}

/* ------------------------------------------------------------------- bits */

struct bitwriter {
  uint32_t* words;
  uint64_t nbits;
  uint64_t cap_words;
};

static int bw_init(struct bitwriter* w) {
  w->cap_words = 1024;
  w->nbits = 0;
  w->words = (uint32_t*)calloc(w->cap_words, 4);
  return w->words ? SZREF_OK : SZREF_ENOMEM;
}

/* Stream bit b lives in word b/32 at bit position 31 - b%32 (MSB first). */
static void bw_put(struct bitwriter* w, uint64_t value, int nbits) {
  for (int i = nbits - 1; i >= 0; i--) {
    uint64_t b = w->nbits;
    if ((b >> 5) >= w->cap_words) {
      uint64_t nc = w->cap_words * 2;
      uint32_t* nw = (uint32_t*)realloc(w->words, nc * 4);
      if (!nw) abort();
      memset(nw + w->cap_words, 0, (nc - w->cap_words) * 4);
      w->words = nw;
      w->cap_words = nc;
    }
    if ((value >> i) & 1) w->words[b >> 5] |= 1u << (31 - (b & 31));
    w->nbits++;
  }
}

struct bitreader {
  const uint32_t* words;
  uint64_t nbits;
  uint64_t pos;
};

static int br_bit(struct bitreader* r, int* bit) {
  if (r->pos >= r->nbits) return 1;
  uint64_t b = r->pos++;
  *bit = (int)((r->words[b >> 5] >> (31 - (b & 31))) & 1u);
  return 0;
}

static int br_get(struct bitreader* r, int nbits, uint64_t* out) {
  uint64_t v = 0;
  for (int i = 0; i < nbits; i++) {
    int bit;
    if (br_bit(r, &bit)) return 1;
    v = (v << 1) | (uint64_t)bit;
  }
  *out = v;
  return 0;
}

/* ------------------------------------------------- element-type instances */

static float rint_f32(float v) { return rintf(v); }
static double rint_f64(double v) { return rint(v); }

#define ET float
#define UT uint32_t
#define SFX(name) name##_f32
#define rint_et_f32 rint_f32
#define MANT 23
#define EXPB 8
#define EMAX 255
#include "szref_traverse.inc"
#undef ET
#undef UT
#undef SFX
#undef MANT
#undef EXPB
#undef EMAX

#define ET double
#define UT uint64_t
#define SFX(name) name##_f64
#define rint_et_f64 rint_f64
#define MANT 52
#define EXPB 11
#define EMAX 2047
#include "szref_traverse.inc"
#undef ET
#undef UT
#undef SFX
#undef MANT
#undef EXPB
#undef EMAX

/* --------------------------------------------------------------- eb (Metric 1) */

int szref_resolve_eb(const szref_params* p, const void* data, szref_eb* E) {
  struct layout L;
  int rc = make_layout(p, &L);
  if (rc) return rc;
  if (p->dtype > 1 || p->eb_mode > 2) return SZREF_EINVAL;
  if (!isfinite(p->eb_abs) || !isfinite(p->eb_rel) || p->eb_abs < 0 || p->eb_rel < 0)
    return SZREF_EINVAL;
  E->vmin = E->vmax = 0;
  double eb = p->eb_abs;
  if (p->eb_mode != 0) {
    rc = (p->dtype == 0) ? minmax_f32((const float*)data, L.n, &E->vmin, &E->vmax)
                         : minmax_f64((const double*)data, L.n, &E->vmin, &E->vmax);
    if (rc) return rc;
    double range = E->vmax - E->vmin;
    double rel = p->eb_rel * range;
    eb = (p->eb_mode == 1) ? rel : (p->eb_abs < rel ? p->eb_abs : rel);
  }
  double tmax = (p->dtype == 0) ? (double)FLT_MAX : DBL_MAX;
  if (!(eb <= tmax / 4)) return SZREF_EINVAL;
  E->eb = eb;
  if (p->dtype == 0) eb_to_et_f32(eb, E); else eb_to_et_f64(eb, E);
  return SZREF_OK;
}

static int check_params(const szref_params* p) {
  if (p->dtype > 1 || p->ndim < 1 || p->ndim > 3) return SZREF_EINVAL;
  if (p->layers < 1 || p->layers > 4) return SZREF_EINVAL;
  if (p->quant_bits > 16) return SZREF_EINVAL;
  if (p->eb_mode > 2) return SZREF_EINVAL;
  if (p->chunk != 0 && (p->chunk < 256 || p->chunk > 4096 || p->chunk % 256)) return SZREF_EINVAL;
  if (p->theta < 0 || p->theta > 1 || p->theta != p->theta) return SZREF_EINVAL;
  if (p->unpred_coding > 1) return SZREF_EINVAL;
  return SZREF_OK;
}

int szref_predict_original(const szref_params* p, const void* data, void* pred) {
  struct layout L;
  struct stencil S;
  int rc = check_params(p);
  if (rc) return rc;
  if ((rc = make_layout(p, &L))) return rc;
  if ((rc = make_stencil(p->ndim, p->layers, &S))) return rc;
  if (p->dtype == 0) predict_all_original_f32(&L, &S, (const float*)data, (float*)pred);
  else predict_all_original_f64(&L, &S, (const double*)data, (double*)pred);
  return SZREF_OK;
}

int szref_quantize(const szref_params* p, const void* data, uint32_t m,
                   uint16_t* codes, void* xprime, uint64_t* n_unpred) {
  struct layout L;
  struct stencil S;
  szref_eb E;
  int rc = check_params(p);
  if (rc) return rc;
  if (m < 1 || m > 16) return SZREF_EINVAL;
  if ((rc = make_layout(p, &L))) return rc;
  if ((rc = make_stencil(p->ndim, p->layers, &S))) return rc;
  if ((rc = szref_resolve_eb(p, data, &E))) return rc;
  if (p->dtype == 0) traverse_f32(&L, &S, (const float*)data, &E, m, codes, (float*)xprime, n_unpred);
  else traverse_f64(&L, &S, (const double*)data, &E, m, codes, (double*)xprime, n_unpred);
  return SZREF_OK;
}

/* ----------------------------------------------------------------- Huffman */

struct leaf { uint64_t f; uint32_t sym; };

static int leaf_cmp(const void* a, const void* b) {
  const struct leaf* x = (const struct leaf*)a;
  const struct leaf* y = (const struct leaf*)b;
  if (x->f != y->f) return x->f < y->f ? -1 : 1;
  return x->sym < y->sym ? -1 : (x->sym > y->sym);
}

/* One two-queue construction (van Leeuwen): leaves sorted by (f, sym) form
 * the first queue, internal nodes the second in creation order; each step
 * removes the two lightest fronts, the leaf queue winning ties. */
static int two_queue_depths(const struct leaf* lv, uint32_t s, uint8_t* depth_out) {
  uint64_t* w = (uint64_t*)malloc(sizeof(uint64_t) * (2 * s));
  uint32_t* parent = (uint32_t*)malloc(sizeof(uint32_t) * (2 * s));
  uint32_t* depth = (uint32_t*)malloc(sizeof(uint32_t) * (2 * s));
  if (!w || !parent || !depth) { free(w); free(parent); free(depth); return SZREF_ENOMEM; }
  for (uint32_t i = 0; i < s; i++) w[i] = lv[i].f;
  uint32_t i = 0, j = s, next = s;
  for (uint32_t step = 0; step + 1 < s; step++) {
    uint32_t pick[2];
    for (int q = 0; q < 2; q++) {
      if (i < s && (j >= next || w[i] <= w[j])) pick[q] = i++;
      else pick[q] = j++;
    }
    w[next] = w[pick[0]] + w[pick[1]];
    parent[pick[0]] = next;
    parent[pick[1]] = next;
    next++;
  }
  uint32_t root = 2 * s - 2;
  depth[root] = 0;
  int maxd = 0;
  for (int64_t nd = (int64_t)root - 1; nd >= 0; nd--) {
    depth[nd] = depth[parent[nd]] + 1;
  }
  for (uint32_t q = 0; q < s; q++) {
    uint32_t d = depth[q];
    depth_out[q] = (uint8_t)(d > 255 ? 255 : d);
    if ((int)d > maxd) maxd = (int)d;
  }
  free(w); free(parent); free(depth);
  return maxd;
}

int szref_huffman_lengths(const uint64_t* freq, uint32_t nsym, uint8_t* len) {
  if (nsym == 0) return SZREF_EINVAL;
  memset(len, 0, nsym);
  uint32_t s = 0;
  for (uint32_t q = 0; q < nsym; q++) if (freq[q]) s++;
  if (s == 0) return 0;
  struct leaf* lv = (struct leaf*)malloc(sizeof(struct leaf) * s);
  uint8_t* d = (uint8_t*)malloc(s);
  if (!lv || !d) { free(lv); free(d); return SZREF_ENOMEM; }
  s = 0;
  for (uint32_t q = 0; q < nsym; q++) if (freq[q]) { lv[s].f = freq[q]; lv[s].sym = q; s++; }
  if (s == 1) {
    len[lv[0].sym] = 1;
    free(lv); free(d);
    return 1;
  }
  int maxd;
  for (;;) {
    qsort(lv, s, sizeof(struct leaf), leaf_cmp);
    maxd = two_queue_depths(lv, s, d);
    if (maxd < 0) { free(lv); free(d); return maxd; }
    if (maxd <= LMAX) break;
    for (uint32_t q = 0; q < s; q++) {
      uint64_t h = lv[q].f >> 1;
      lv[q].f = h ? h : 1;
    }
  }
  for (uint32_t q = 0; q < s; q++) len[lv[q].sym] = d[q];
  free(lv); free(d);
  return maxd;
}

/* Canonical codes: symbols ordered by (length, symbol) get consecutive
 * values, the value shifted left whenever the length grows. */
static void canonical_codes(const uint8_t* len, uint32_t nsym, uint32_t* code) {
  uint32_t next = 0;
  for (int l = 1; l <= LMAX; l++) {
    for (uint32_t q = 0; q < nsym; q++)
      if (len[q] == l) code[q] = next++;
    next <<= 1;
  }
}

/* ------------------------------------------------------------- container */

static void put_u16(uint8_t* b, uint16_t v) { b[0] = (uint8_t)v; b[1] = (uint8_t)(v >> 8); }
static void put_u32(uint8_t* b, uint32_t v) { for (int i = 0; i < 4; i++) b[i] = (uint8_t)(v >> (8 * i)); }
static void put_u64(uint8_t* b, uint64_t v) { for (int i = 0; i < 8; i++) b[i] = (uint8_t)(v >> (8 * i)); }
static uint16_t get_u16(const uint8_t* b) { return (uint16_t)(b[0] | (b[1] << 8)); }
static uint32_t get_u32(const uint8_t* b) { uint32_t v = 0; for (int i = 3; i >= 0; i--) v = (v << 8) | b[i]; return v; }
static uint64_t get_u64(const uint8_t* b) { uint64_t v = 0; for (int i = 7; i >= 0; i--) v = (v << 8) | b[i]; return v; }
static void put_f64(uint8_t* b, double d) { uint64_t u; memcpy(&u, &d, 8); put_u64(b, u); }
static double get_f64(const uint8_t* b) { uint64_t u = get_u64(b); double d; memcpy(&d, &u, 8); return d; }
static uint64_t align_up(uint64_t v, uint64_t a) { return (v + a - 1) / a * a; }

size_t szref_compress_bound(const szref_params* p) {
  struct layout L;
  if (check_params(p) || make_layout(p, &L)) return 0;
  uint64_t es = p->dtype ? 8 : 4;
  return (size_t)(HDR_SIZE + L.n * es);
}

struct hdr {
  uint32_t flags, dtype, ndim, layers, m, eb_mode, m_req;
  uint64_t dims[3], block[3];
  double eb_abs, eb_rel;
  uint64_t ebT_bits, n_points, n_unpred, huff_bits, tail_bits;
  uint32_t chunk, n_used;
  uint64_t n_chunks, off_cb, off_ch, off_bs, off_hd, off_tl, total;
};

static void write_hdr(uint8_t* b, const struct hdr* h) {
  memset(b, 0, HDR_SIZE);
  put_u32(b + 0, MAGIC);
  put_u16(b + 4, VERSION);
  put_u16(b + 6, (uint16_t)h->flags);
  b[8] = (uint8_t)h->dtype; b[9] = (uint8_t)h->ndim; b[10] = (uint8_t)h->layers; b[11] = (uint8_t)h->m;
  b[12] = (uint8_t)h->eb_mode; b[13] = (uint8_t)h->m_req;
  for (int d = 0; d < 3; d++) put_u64(b + 16 + 8 * d, h->dims[d]);
  for (int d = 0; d < 3; d++) put_u64(b + 40 + 8 * d, h->block[d]);
  put_f64(b + 64, h->eb_abs);
  put_f64(b + 72, h->eb_rel);
  put_u64(b + 80, h->ebT_bits);
  put_u64(b + 88, h->n_points);
  put_u64(b + 96, h->n_unpred);
  put_u64(b + 104, h->huff_bits);
  put_u64(b + 112, h->tail_bits);
  put_u32(b + 120, h->chunk);
  put_u32(b + 124, h->n_used);
  put_u64(b + 128, h->n_chunks);
  put_u64(b + 136, h->off_cb);
  put_u64(b + 144, h->off_ch);
  put_u64(b + 152, h->off_bs);
  put_u64(b + 160, h->off_hd);
  put_u64(b + 168, h->off_tl);
  put_u64(b + 176, h->total);
}

static int read_hdr(const uint8_t* b, size_t size, struct hdr* h) {
  if (size < HDR_SIZE) return SZREF_ECORRUPT;
  if (get_u32(b) != MAGIC || get_u16(b + 4) != VERSION) return SZREF_ECORRUPT;
  h->flags = get_u16(b + 6);
  h->dtype = b[8]; h->ndim = b[9]; h->layers = b[10]; h->m = b[11];
  h->eb_mode = b[12]; h->m_req = b[13];
  for (int d = 0; d < 3; d++) h->dims[d] = get_u64(b + 16 + 8 * d);
  for (int d = 0; d < 3; d++) h->block[d] = get_u64(b + 40 + 8 * d);
  h->eb_abs = get_f64(b + 64);
  h->eb_rel = get_f64(b + 72);
  h->ebT_bits = get_u64(b + 80);
  h->n_points = get_u64(b + 88);
  h->n_unpred = get_u64(b + 96);
  h->huff_bits = get_u64(b + 104);
  h->tail_bits = get_u64(b + 112);
  h->chunk = get_u32(b + 120);
  h->n_used = get_u32(b + 124);
  h->n_chunks = get_u64(b + 128);
  h->off_cb = get_u64(b + 136);
  h->off_ch = get_u64(b + 144);
  h->off_bs = get_u64(b + 152);
  h->off_hd = get_u64(b + 160);
  h->off_tl = get_u64(b + 168);
  h->total = get_u64(b + 176);
  if (h->dtype > 1 || h->ndim < 1 || h->ndim > 3 || h->layers < 1 || h->layers > 4) return SZREF_ECORRUPT;
  if (h->flags > 3 || h->flags == 3) return SZREF_ECORRUPT; /* raw copy, or the XOR coding of unpredictable values */
  if (h->total > size) return SZREF_ECORRUPT;
  return SZREF_OK;
}

/* Adaptive interval count (Sec. IV-B): smallest m whose intervals
 * |k| <= 2^(m-1) - 1 hold at least theta * N points of the m = 16 run. */
static uint32_t pick_m(const uint64_t* h16, uint64_t n, double theta) {
  for (uint32_t m = 1; m <= 16; m++) {
    int32_t lim = (1 << (m - 1)) - 1;
    uint64_t cov = 0;
    for (int32_t k = -lim; k <= lim; k++) cov += h16[k + 32768];
    if ((double)cov >= theta * (double)n) return m;
  }
  return 16;
}

static int compress_impl(const szref_params* p, const void* data, uint8_t** out,
                         size_t* out_size, szref_stats* st, uint16_t* codes_dbg,
                         void* xp_dbg) {
  struct layout L;
  struct stencil S;
  szref_eb E;
  int rc = check_params(p);
  if (rc) return rc;
  if ((rc = make_layout(p, &L))) return rc;
  if ((rc = make_stencil(p->ndim, p->layers, &S))) return rc;
  if ((rc = szref_resolve_eb(p, data, &E))) return rc;
  const uint64_t n = L.n;
  const uint64_t es = p->dtype ? 8 : 4;
  const uint32_t C = p->chunk ? p->chunk : DEFAULT_CHUNK;
  const double theta = (p->theta > 0) ? p->theta : 0.9;

  struct bitwriter bs = {0}, hd = {0}, tl = {0};
  uint32_t* chunk_bits = NULL;
  uint16_t* chunk_mid = NULL;
  uint32_t* uchunk = NULL;
  uint8_t* len = NULL;
  uint32_t* cw = NULL;
  uint16_t* codes = (uint16_t*)malloc(n * 2);
  void* xp = malloc(n * es);
  uint64_t* hist = (uint64_t*)calloc(65536, 8);
  if (!codes || !xp || !hist) { rc = SZREF_ENOMEM; goto done; }

  uint32_t m = p->quant_bits;
  uint64_t nu = 0;
  if (m == 0) {
    if (p->dtype == 0) traverse_f32(&L, &S, (const float*)data, &E, 16, codes, (float*)xp, &nu);
    else traverse_f64(&L, &S, (const double*)data, &E, 16, codes, (double*)xp, &nu);
    for (uint64_t i = 0; i < n; i++) hist[codes[i]]++;
    m = pick_m(hist, n, theta);
    if (m < 16) {
      memset(hist, 0, 65536 * 8);
      if (p->dtype == 0) traverse_f32(&L, &S, (const float*)data, &E, m, codes, (float*)xp, &nu);
      else traverse_f64(&L, &S, (const double*)data, &E, m, codes, (double*)xp, &nu);
      for (uint64_t i = 0; i < n; i++) hist[codes[i]]++;
    }
  } else {
    if (p->dtype == 0) traverse_f32(&L, &S, (const float*)data, &E, m, codes, (float*)xp, &nu);
    else traverse_f64(&L, &S, (const double*)data, &E, m, codes, (double*)xp, &nu);
    for (uint64_t i = 0; i < n; i++) hist[codes[i]]++;
  }
  const uint32_t nsym = 1u << m;

  /* Huffman over the 2^m codes (Sec. IV-A). */
  len = (uint8_t*)malloc(nsym);
  cw = (uint32_t*)calloc(nsym, 4);
  if (!len || !cw) { rc = SZREF_ENOMEM; goto done; }
  rc = szref_huffman_lengths(hist, nsym, len);
  if (rc < 0) goto done;
  canonical_codes(len, nsym, cw);

  if (bw_init(&bs) || bw_init(&hd) || bw_init(&tl)) { rc = SZREF_ENOMEM; goto done; }
  uint64_t n_chunks = (n + C - 1) / C;
  chunk_bits = (uint32_t*)calloc(n_chunks, 4);
  chunk_mid = (uint16_t*)calloc(n_chunks, 2);
  if (!chunk_bits || !chunk_mid) { rc = SZREF_ENOMEM; goto done; }
  for (uint64_t i = 0; i < n; i++) {
    uint64_t before = bs.nbits;
    bw_put(&bs, cw[codes[i]], len[codes[i]]);
    chunk_bits[i / C] += (uint32_t)(bs.nbits - before);
    /* reading A17: the bits of a chunk's first half, where a second decoder
     * of the chunk starts (at most C/2 * LMAX < 2^16 bits) */
    if (i % C < C / 2) chunk_mid[i / C] += (uint16_t)(bs.nbits - before);
  }
  const int xor_coding = p->unpred_coding == 1;
  if (xor_coding) {
    /* records in the tails section, their per-chunk bit counts in the heads section */
    uchunk = (uint32_t*)calloc(n_chunks, 4);
    if (!uchunk) { rc = SZREF_ENOMEM; goto done; }
    if (p->dtype == 0) pack_unpred_xor_f32(codes, (const float*)xp, n, C, (uint32_t)E.ebT_bits, &tl, uchunk);
    else pack_unpred_xor_f64(codes, (const double*)xp, n, C, E.ebT_bits, &tl, uchunk);
    for (uint64_t c = 0; c < n_chunks; c++) bw_put(&hd, uchunk[c], 32);
  } else if (p->dtype == 0) {
    pack_unpred_f32(codes, (const float*)xp, n, (uint32_t)E.ebT_bits, &hd, &tl);
  } else {
    pack_unpred_f64(codes, (const double*)xp, n, E.ebT_bits, &hd, &tl);
  }

  uint32_t n_used = 0;
  for (uint32_t q = 0; q < nsym; q++) if (len[q]) n_used++;

  struct hdr h;
  memset(&h, 0, sizeof h);
  h.flags = xor_coding ? 2 : 0;
  h.dtype = p->dtype; h.ndim = p->ndim; h.layers = p->layers; h.m = m;
  h.eb_mode = p->eb_mode; h.m_req = p->quant_bits;
  for (int d = 0; d < 3; d++) { h.dims[d] = 1; h.block[d] = 1; }
  for (uint32_t d = 0; d < p->ndim; d++) {
    h.dims[d] = p->dims[d];
    h.block[d] = L.block[3 - p->ndim + d];
  }
  h.eb_abs = p->eb_abs; h.eb_rel = p->eb_rel; h.ebT_bits = E.ebT_bits;
  h.n_points = n; h.n_unpred = nu; h.huff_bits = bs.nbits; h.tail_bits = tl.nbits;
  h.chunk = C; h.n_used = n_used; h.n_chunks = n_chunks;
  h.off_cb = HDR_SIZE;
  h.off_ch = align_up(h.off_cb + 3ull * n_used, SECTION_ALIGN);
  h.off_bs = align_up(h.off_ch + 6ull * n_chunks, SECTION_ALIGN);
  h.off_hd = align_up(h.off_bs + 4ull * ((bs.nbits + 31) / 32), SECTION_ALIGN);
  h.off_tl = align_up(h.off_hd + 4ull * ((hd.nbits + 31) / 32), SECTION_ALIGN);
  h.total = h.off_tl + 4ull * ((tl.nbits + 31) / 32);

  uint64_t raw_total = HDR_SIZE + n * es;
  int raw = h.total >= raw_total;
  uint8_t* buf;
  if (raw) {
    struct hdr r;
    memset(&r, 0, sizeof r);
    r.flags = 1; r.dtype = h.dtype; r.ndim = h.ndim; r.layers = h.layers; r.m = m;
    r.eb_mode = h.eb_mode; r.m_req = h.m_req;
    memcpy(r.dims, h.dims, sizeof r.dims); memcpy(r.block, h.block, sizeof r.block);
    r.eb_abs = h.eb_abs; r.eb_rel = h.eb_rel; r.ebT_bits = h.ebT_bits; r.n_points = n;
    r.chunk = C;
    r.off_cb = r.off_ch = r.off_bs = r.off_hd = r.off_tl = HDR_SIZE;
    r.total = raw_total;
    buf = (uint8_t*)calloc(raw_total, 1);
    if (!buf) { rc = SZREF_ENOMEM; goto done; }
    write_hdr(buf, &r);
    memcpy(buf + HDR_SIZE, data, n * es);
    *out_size = raw_total;
  } else {
    buf = (uint8_t*)calloc(h.total, 1);
    if (!buf) { rc = SZREF_ENOMEM; goto done; }
    write_hdr(buf, &h);
    uint8_t* cb = buf + h.off_cb;
    for (uint32_t q = 0; q < nsym; q++) {
      if (!len[q]) continue;
      put_u16(cb, (uint16_t)q);
      cb[2] = len[q];
      cb += 3;
    }
    for (uint64_t c = 0; c < n_chunks; c++) put_u32(buf + h.off_ch + 4 * c, chunk_bits[c]);
    for (uint64_t c = 0; c < n_chunks; c++) put_u16(buf + h.off_ch + 4 * n_chunks + 2 * c, chunk_mid[c]);
    for (uint64_t wd = 0; wd < (bs.nbits + 31) / 32; wd++) put_u32(buf + h.off_bs + 4 * wd, bs.words[wd]);
    for (uint64_t wd = 0; wd < (hd.nbits + 31) / 32; wd++) put_u32(buf + h.off_hd + 4 * wd, hd.words[wd]);
    for (uint64_t wd = 0; wd < (tl.nbits + 31) / 32; wd++) put_u32(buf + h.off_tl + 4 * wd, tl.words[wd]);
    *out_size = h.total;
  }
  *out = buf;
  if (st) {
    memset(st, 0, sizeof *st);
    st->n_points = n; st->n_unpred = nu; st->huff_bits = bs.nbits; st->tail_bits = tl.nbits;
    st->compressed_bytes = *out_size; st->ebT_bits = E.ebT_bits; st->eb_used = E.ebT;
    st->hit_rate = 1.0 - (double)hist[0] / (double)n;
    st->value_min = E.vmin; st->value_max = E.vmax;
    st->m_used = m;
    st->m_suggested = (st->hit_rate < theta && m < 16) ? m + 1 : m;
    st->raw_fallback = (uint32_t)raw; st->n_used_syms = n_used;
  }
  if (codes_dbg) memcpy(codes_dbg, codes, n * 2);
  if (xp_dbg) memcpy(xp_dbg, xp, n * es);
  rc = SZREF_OK;
done:
  free(chunk_bits);
  free(chunk_mid);
  free(uchunk);
  free(bs.words); free(hd.words); free(tl.words);
  free(codes); free(xp); free(hist); free(len); free(cw);
  return rc;
}

int szref_compress(const szref_params* p, const void* data, uint8_t** out,
                   size_t* out_size, szref_stats* st) {
  return compress_impl(p, data, out, out_size, st, NULL, NULL);
}

int szref_compress_debug(const szref_params* p, const void* data, uint8_t** out,
                         size_t* out_size, szref_stats* st, uint16_t* codes, void* xp) {
  return compress_impl(p, data, out, out_size, st, codes, xp);
}

int szref_inspect(const uint8_t* comp, size_t size, szref_params* p, szref_stats* s) {
  struct hdr h;
  int rc = read_hdr(comp, size, &h);
  if (rc) return rc;
  if (p) {
    memset(p, 0, sizeof *p);
    p->dtype = h.dtype; p->ndim = h.ndim; p->layers = h.layers; p->quant_bits = h.m_req;
    p->eb_mode = h.eb_mode; p->chunk = h.chunk; p->eb_abs = h.eb_abs; p->eb_rel = h.eb_rel;
    p->unpred_coding = (h.flags >> 1) & 1;
    for (uint32_t d = 0; d < h.ndim; d++) { p->dims[d] = h.dims[d]; p->block[d] = h.block[d]; }
  }
  if (s) {
    memset(s, 0, sizeof *s);
    s->n_points = h.n_points; s->n_unpred = h.n_unpred; s->huff_bits = h.huff_bits;
    s->tail_bits = h.tail_bits; s->compressed_bytes = h.total; s->ebT_bits = h.ebT_bits;
    s->m_used = h.m; s->raw_fallback = h.flags & 1; s->n_used_syms = h.n_used;
  }
  return SZREF_OK;
}

/* Does a section of len bytes at offset off lie within the first total bytes? */
static int section_fits(uint64_t off, uint64_t len, uint64_t total) {
  return off <= total && len <= total - off;
}

int szref_decompress(const uint8_t* comp, size_t size, void* out, size_t cap) {
  struct hdr h;
  int rc = read_hdr(comp, size, &h);
  if (rc) return rc;
  szref_params p;
  memset(&p, 0, sizeof p);
  p.dtype = h.dtype; p.ndim = h.ndim; p.layers = h.layers;
  for (uint32_t d = 0; d < h.ndim; d++) { p.dims[d] = h.dims[d]; p.block[d] = h.block[d]; }
  struct layout L;
  struct stencil S;
  if (make_layout(&p, &L)) return SZREF_ECORRUPT;
  if (L.n != h.n_points) return SZREF_ECORRUPT;
  const uint64_t es = h.dtype ? 8 : 4;
  if (cap < L.n * es) return SZREF_ECAPACITY;
  if (h.flags & 1) {
    if (h.total != HDR_SIZE + L.n * es) return SZREF_ECORRUPT;
    memcpy(out, comp + HDR_SIZE, L.n * es);
    return SZREF_OK;
  }
  if (h.m < 1 || h.m > 16 || h.chunk == 0) return SZREF_ECORRUPT;
  if (make_stencil(h.ndim, h.layers, &S)) return SZREF_ECORRUPT;
  const uint32_t nsym = 1u << h.m;
  const uint64_t n = L.n;
  if (h.n_chunks != (n + h.chunk - 1) / h.chunk) return SZREF_ECORRUPT;
  /* Section bounds.  The counts are bounded first so that no section
   * length below can wrap around, and each check is written so that a huge
   * offset cannot wrap either. */
  /* With the XOR coding (flag bit 1) the heads section holds one u32 bit
   * count per chunk and a record takes at most LZB + W bits. */
  const int xor_coding = (h.flags & 2) != 0;
  const uint64_t head_bits = xor_coding ? 32ull * h.n_chunks : h.n_unpred * (h.dtype ? 12 : 9);
  const uint64_t max_tail = xor_coding ? (h.dtype ? 3 + 64 : 2 + 32) : (h.dtype ? 52 : 23);
  if (h.n_used > nsym || h.n_unpred > n || h.huff_bits > n * LMAX || h.tail_bits > h.n_unpred * max_tail)
    return SZREF_ECORRUPT;
  if (!section_fits(h.off_cb, 3ull * h.n_used, h.total) || !section_fits(h.off_ch, 6ull * h.n_chunks, h.total) ||
      !section_fits(h.off_bs, 4ull * ((h.huff_bits + 31) / 32), h.total) ||
      !section_fits(h.off_hd, 4ull * ((head_bits + 31) / 32), h.total) ||
      !section_fits(h.off_tl, 4ull * ((h.tail_bits + 31) / 32), h.total))
    return SZREF_ECORRUPT;

  uint8_t* len = (uint8_t*)calloc(nsym, 1);
  uint32_t* cw = (uint32_t*)calloc(nsym, 4);
  uint16_t* codes = (uint16_t*)malloc(n * 2);
  void* uv = malloc((h.n_unpred ? h.n_unpred : 1) * es);
  uint32_t* bsw = (uint32_t*)malloc(4 * (((h.huff_bits + 31) / 32) + 1));
  uint32_t* hdw = (uint32_t*)malloc(4 * (((head_bits + 31) / 32) + 1));
  uint32_t* tlw = (uint32_t*)malloc(4 * (((h.tail_bits + 31) / 32) + 1));
  rc = SZREF_ENOMEM;
  if (!len || !cw || !codes || !uv || !bsw || !hdw || !tlw) goto out;
  rc = SZREF_ECORRUPT;
  for (uint32_t e = 0; e < h.n_used; e++) {
    const uint8_t* cb = comp + h.off_cb + 3ull * e;
    uint16_t sym = get_u16(cb);
    if (sym >= nsym || cb[2] == 0 || cb[2] > LMAX || len[sym]) goto out;
    len[sym] = cb[2];
  }
  canonical_codes(len, nsym, cw);
  for (uint64_t wd = 0; wd < (h.huff_bits + 31) / 32; wd++) bsw[wd] = get_u32(comp + h.off_bs + 4 * wd);
  for (uint64_t wd = 0; wd < (head_bits + 31) / 32; wd++) hdw[wd] = get_u32(comp + h.off_hd + 4 * wd);
  for (uint64_t wd = 0; wd < (h.tail_bits + 31) / 32; wd++) tlw[wd] = get_u32(comp + h.off_tl + 4 * wd);

  /* Sequential canonical decode, one bit at a time: extend the bit string
   * until it equals the code of some symbol of that length. */
  {
    struct bitreader br = {bsw, h.huff_bits, 0};
    uint64_t nz = 0, want = 0, cstart = 0;
    for (uint64_t i = 0; i < n; i++) {
      if (i % h.chunk == 0) {
        if (want != br.pos) goto out;
        cstart = br.pos;
        want += get_u32(comp + h.off_ch + 4 * (i / h.chunk));
      }
      /* reading A17: the stored start of the chunk's second half */
      if (i % h.chunk == h.chunk / 2 &&
          br.pos != cstart + get_u16(comp + h.off_ch + 4 * h.n_chunks + 2 * (i / h.chunk)))
        goto out;
      uint32_t v = 0;
      int l = 0, found = -1;
      while (found < 0) {
        int bit;
        if (br_bit(&br, &bit)) goto out;
        v = (v << 1) | (uint32_t)bit;
        l++;
        if (l > LMAX) goto out;
        for (uint32_t q = 0; q < nsym; q++)
          if (len[q] == l && cw[q] == v) { found = (int)q; break; }
      }
      codes[i] = (uint16_t)found;
      if (found == 0) nz++;
    }
    if (br.pos != h.huff_bits || want != h.huff_bits || nz != h.n_unpred) goto out;
  }
  if (xor_coding) {
    struct bitreader tr = {tlw, h.tail_bits, 0};
    int urc = h.dtype ? unpack_unpred_xor_f64(codes, n, h.chunk, h.ebT_bits, &tr, hdw, (double*)uv)
                      : unpack_unpred_xor_f32(codes, n, h.chunk, (uint32_t)h.ebT_bits, &tr, hdw, (float*)uv);
    if (urc || tr.pos != h.tail_bits) goto out;
  } else {
    struct bitreader hr = {hdw, head_bits, 0};
    struct bitreader tr = {tlw, h.tail_bits, 0};
    int urc = h.dtype ? unpack_unpred_f64(&hr, &tr, h.n_unpred, h.ebT_bits, (double*)uv)
                      : unpack_unpred_f32(&hr, &tr, h.n_unpred, (uint32_t)h.ebT_bits, (float*)uv);
    if (urc || tr.pos != h.tail_bits) goto out;
  }
  {
    szref_eb E;
    memset(&E, 0, sizeof E);
    if (h.dtype == 0) {
      float ebT; uint32_t u = (uint32_t)h.ebT_bits; memcpy(&ebT, &u, 4);
      eb_to_et_f32((double)ebT, &E);
      reconstruct_f32(&L, &S, codes, (const float*)uv, &E, h.m, (float*)out);
    } else {
      double ebT; memcpy(&ebT, &h.ebT_bits, 8);
      eb_to_et_f64(ebT, &E);
      reconstruct_f64(&L, &S, codes, (const double*)uv, &E, h.m, (double*)out);
    }
  }
  rc = SZREF_OK;
out:
  free(len); free(cw); free(codes); free(uv); free(bsw); free(hdw); free(tlw);
  return rc;
}

void szref_free(void* ptr) { free(ptr); }
