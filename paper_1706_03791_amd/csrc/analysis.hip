// Analysis entry points beside the codec:
//  * sz_quality: the error metrics of Sec. II (Metric 2: RMSE, NRMSE, PSNR;
//    Metric 3: Pearson correlation) and the autocorrelation of the
//    compression errors studied in Sec. V, computed on the device in double
//    precision with a fixed reduction order (deterministic results);
//  * sz_layer_survey: the best-layer study of Sec. III-B (Table II): the
//    prediction hitting rate R_PH for n = 1..4 layers on a centred sample of
//    the field, predicting from decompressed values (the compressor's case,
//    R_PH^decomp) and from original values (R_PH^orig), with one interval
//    around the prediction (m = 1: a point is predictable when it lies within
//    the error bound of its prediction).
#include <vector>

#include "runtime.hpp"

using namespace szh;

namespace szh {
namespace {

constexpr int kQNT = 256;
constexpr int kSeg = 4096;     // elements per block in the autocorrelation pass
constexpr int kMaxLag = 255;   // lags per call

template <int NT>
__device__ __forceinline__ double block_sum_d(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0;
  if (threadIdx.x == 0)
    for (int i = 0; i < NT / 64; i++) s += red[i];
  __syncthreads();
  return s;
}
template <int NT>
__device__ __forceinline__ double block_max_d(double v, double* red) {
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = -__builtin_huge_val();
  if (threadIdx.x == 0)
    for (int i = 0; i < NT / 64; i++) s = fmax(s, red[i]);
  __syncthreads();
  return s;
}

// Pass 1, per block: sum x, sum x', sum e, min x, max x, max |e| (e = x - x').
template <typename T>
__global__ void __launch_bounds__(kQNT) q_pass1(const T* __restrict__ x, const T* __restrict__ y, uint64_t n,
                                                double* part) {
  __shared__ double red[kQNT / 64];
  double sx = 0, sy = 0, se = 0, mn = __builtin_huge_val(), mx = -__builtin_huge_val(), mae = 0;
  for (uint64_t i = (uint64_t)blockIdx.x * kQNT + threadIdx.x; i < n; i += (uint64_t)gridDim.x * kQNT) {
    const double a = (double)x[i], b = (double)y[i], e = a - b;
    sx += a;
    sy += b;
    se += e;
    mn = fmin(mn, a);
    mx = fmax(mx, a);
    mae = fmax(mae, fabs(e));
  }
  double* p = part + (size_t)blockIdx.x * 6;
  sx = block_sum_d<kQNT>(sx, red);
  sy = block_sum_d<kQNT>(sy, red);
  se = block_sum_d<kQNT>(se, red);
  mn = -block_max_d<kQNT>(-mn, red);
  mx = block_max_d<kQNT>(mx, red);
  mae = block_max_d<kQNT>(mae, red);
  if (threadIdx.x == 0) {
    p[0] = sx;
    p[1] = sy;
    p[2] = se;
    p[3] = mn;
    p[4] = mx;
    p[5] = mae;
  }
}

// Pass 2, per block, with the means of pass 1: centred sums of squares and
// products, and the sum of squared errors.
template <typename T>
__global__ void __launch_bounds__(kQNT) q_pass2(const T* __restrict__ x, const T* __restrict__ y, uint64_t n,
                                                const double* means, double* part) {
  __shared__ double red[kQNT / 64];
  const double mxv = means[0], myv = means[1], mev = means[2];
  double sxx = 0, syy = 0, sxy = 0, see = 0, se2 = 0;
  for (uint64_t i = (uint64_t)blockIdx.x * kQNT + threadIdx.x; i < n; i += (uint64_t)gridDim.x * kQNT) {
    const double a = (double)x[i], b = (double)y[i], e = a - b;
    const double da = a - mxv, db = b - myv, de = e - mev;
    sxx += da * da;
    syy += db * db;
    sxy += da * db;
    see += de * de;
    se2 += e * e;
  }
  double* p = part + (size_t)blockIdx.x * 5;
  sxx = block_sum_d<kQNT>(sxx, red);
  syy = block_sum_d<kQNT>(syy, red);
  sxy = block_sum_d<kQNT>(sxy, red);
  see = block_sum_d<kQNT>(see, red);
  se2 = block_sum_d<kQNT>(se2, red);
  if (threadIdx.x == 0) {
    p[0] = sxx;
    p[1] = syy;
    p[2] = sxy;
    p[3] = see;
    p[4] = se2;
  }
}

// Column reductions of a [rows][cols] array of partials: one block per
// column; thread t folds rows t, t + kQNT, ... in order, then a fixed tree
// folds the threads (a fixed order: deterministic).  op 1 takes the minimum,
// op 2 the maximum instead of the sum for that column.
__global__ void __launch_bounds__(kQNT) q_reduce(const double* part, uint64_t rows, int cols, const int* ops,
                                                 double* out) {
  __shared__ double red[kQNT / 64];
  const int c = blockIdx.x;
  const int op = ops ? ops[c] : 0;
  const double id = op == 1 ? __builtin_huge_val() : (op == 2 ? -__builtin_huge_val() : 0.0);
  double acc = id;
  for (uint64_t r = threadIdx.x; r < rows; r += kQNT) {
    const double v = part[r * cols + c];
    acc = op == 1 ? fmin(acc, v) : (op == 2 ? fmax(acc, v) : acc + v);
  }
  double t;
  if (op == 0) {
    t = block_sum_d<kQNT>(acc, red);
  } else {
    t = block_max_d<kQNT>(op == 1 ? -acc : acc, red);
    if (op == 1) t = -t;
  }
  if (threadIdx.x == 0) out[c] = t;
}

__global__ void q_means(const double* sums, uint64_t n, double* means) {
  if (threadIdx.x == 0) {
    means[0] = sums[0] / (double)n;
    means[1] = sums[1] / (double)n;
    means[2] = sums[2] / (double)n;
  }
}

// Pass 3, per block of kSeg positions i: for every lag k in 1..K the sum of
// d_i d_{i+k} with d = e - mean(e), over i + k < n.  The kQNT threads split
// into K lag groups of P = kQNT / K threads; thread p of lag k sums the
// positions of part p of the segment in order, and the P part sums of a lag
// are then added in part order (a fixed order: deterministic).
template <typename T>
__global__ void __launch_bounds__(kQNT) q_autocorr(const T* __restrict__ x, const T* __restrict__ y, uint64_t n,
                                                   const double* means, int K, double* part) {
  __shared__ double d[kSeg + kMaxLag];
  __shared__ double ps[kQNT];
  const double mev = means[2];
  const uint64_t s0 = (uint64_t)blockIdx.x * kSeg;
  for (int j = threadIdx.x; j < kSeg + K; j += kQNT) {
    const uint64_t i = s0 + (uint64_t)j;
    d[j] = i < n ? ((double)x[i] - (double)y[i]) - mev : 0.0;
  }
  __syncthreads();
  const int P = kQNT / K;               // threads per lag (>= 1 since K <= kMaxLag < kQNT)
  const int k = 1 + (int)threadIdx.x % K;
  const int pi = (int)threadIdx.x / K;  // part index, < P for the first P * K threads
  const uint64_t lim = n > s0 ? n - s0 : 0;  // positions of this block inside the array
  const int len = (int)(lim < (uint64_t)kSeg ? lim : (uint64_t)kSeg);
  double acc = 0;
  if (pi < P) {
    const int per = (kSeg + P - 1) / P;
    const int j0 = pi * per, j1 = min(len, j0 + per);
    for (int j = j0; j < j1; j++) acc += (s0 + j + k < n) ? d[j] * d[j + k] : 0.0;
  }
  ps[threadIdx.x] = acc;
  __syncthreads();
  if ((int)threadIdx.x < K) {
    double t = 0;
    for (int q = 0; q < P; q++) t += ps[q * K + threadIdx.x];
    part[(size_t)blockIdx.x * K + threadIdx.x] = t;
  }
}

// ---- layer survey
template <typename T>
__global__ void crop_kernel(const T* __restrict__ src, T* __restrict__ dst, int64_t Y, int64_t X, int64_t oz,
                            int64_t oy, int64_t ox, int64_t sz, int64_t sy, int64_t sx) {
  const uint64_t n = (uint64_t)sz * sy * sx;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (uint64_t)gridDim.x * blockDim.x) {
    const int64_t xx = (int64_t)(i % sx), yy = (int64_t)((i / sx) % sy), zz = (int64_t)(i / ((uint64_t)sx * sy));
    dst[i] = src[((zz + oz) * Y + (yy + oy)) * X + (xx + ox)];
  }
}

// Points predictable from *original* neighbours with one interval around the
// prediction (the quantizer of Sec. IV-A at m = 1 with the same IEEE steps as
// the sweep: t = (x - p) / (2eb), k = rint(t) must be 0, |x - (p + k 2eb)| < eb).
template <typename T, int DIM, int NL>
__global__ void __launch_bounds__(256) orig_hits_kernel(const T* __restrict__ x, Geom g, uint64_t ebT_bits,
                                                        uint64_t twoeb_bits, uint64_t inv2eb_bits,
                                                        unsigned long long* count) {
  using U = typename FTr<T>::U;
  constexpr Terms<DIM, NL> TT{};
  constexpr int NTERM = Terms<DIM, NL>::N;
  const T ebT = bits_to<T>((U)ebT_bits), twoeb = bits_to<T>((U)twoeb_bits), inv2eb = bits_to<T>((U)inv2eb_bits);
  const int64_t Z = g.dims[0], Y = g.dims[1], X = g.dims[2];
  unsigned long long hits = 0;
  for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < (uint64_t)g.n; i += (uint64_t)gridDim.x * 256) {
    const int64_t xi = (int64_t)(i % X), yi = (int64_t)((i / X) % Y), zi = (int64_t)(i / ((uint64_t)X * Y));
    // position inside its independent block
    const int64_t bz = zi % g.blk[0], by = yi % g.blk[1], bx = xi % g.blk[2];
    T p = T(0);
#pragma unroll
    for (int t = 0; t < NTERM; t++) {
      const bool in = bz >= TT.a[t] && by >= TT.b[t] && bx >= TT.c[t];
      const T v = in ? x[((zi - TT.a[t]) * Y + (yi - TT.b[t])) * X + (xi - TT.c[t])] : T(0);
      p = p + T(TT.coef[t]) * v;
    }
    const T xv = x[i];
    const T tq = (xv - p) * inv2eb;
    bool ok = fabs(tq) < T(1);
    const T rk = rint(tq);
    ok = ok && rk == T(0);
    const T xq = p + rk * twoeb;
    ok = ok && fabs(xv - xq) < ebT;
    hits += ok ? 1ull : 0ull;
    (void)Z;
  }
  for (int o = 32; o > 0; o >>= 1) hits += __shfl_xor(hits, o);
  if ((threadIdx.x & 63) == 0 && hits) atomicAdd(count, hits);
}

template <typename T>
void launch_orig_hits(int ndim, int nl, const T* x, const Geom& g, const DevPlan& h, unsigned long long* count,
                      hipStream_t st) {
  const unsigned grid = (unsigned)std::min<uint64_t>(ceil_div((uint64_t)g.n, 256), 4096);
  const uint64_t a = h.ebT_bits, b = h.twoeb_bits, c = h.inv2eb_bits;
#define SZ_OH(D, N)                                                                                       \
  if (ndim == D && nl == N)                                                                               \
    hipLaunchKernelGGL((orig_hits_kernel<T, D, N>), dim3(grid), dim3(256), 0, st, x, g, a, b, c, count);
  SZ_OH(1, 1) SZ_OH(1, 2) SZ_OH(1, 3) SZ_OH(1, 4)
  SZ_OH(2, 1) SZ_OH(2, 2) SZ_OH(2, 3) SZ_OH(2, 4)
  SZ_OH(3, 1) SZ_OH(3, 2) SZ_OH(3, 3) SZ_OH(3, 4)
#undef SZ_OH
}

template <typename T>
int quality_t(sz_ctx* ctx, uint64_t n, const void* d_x, const void* d_y, uint32_t K, double* h_ac, sz_quality_t* q,
              hipStream_t st) {
  const unsigned g12 = (unsigned)std::min<uint64_t>(ceil_div(n, kQNT * 8), 2048);
  const uint64_t nseg = K ? ceil_div(n, kSeg) : 0;
  const size_t bytes = 256 + 8 * ((size_t)g12 * 11 + 16 + (size_t)nseg * K + K);
  int rc = ensure_arena(ctx, bytes);
  if (rc) return rc;
  double* part = (double*)ctx->arena;
  double* sums = part + (size_t)g12 * 6;   // 6 totals of pass 1
  double* means = sums + 6;                 // 3
  double* sums2 = means + 3;                // 5 totals of pass 2
  int* ops = (int*)(sums2 + 5);             // 6 ints (in the space of 3 doubles)
  double* acpart = (double*)(ops + 8);
  double* ac = acpart + (size_t)nseg * K;
  const int h_ops[6] = {0, 0, 0, 1, 2, 2};
  HIPCHK(hipMemcpyAsync(ops, h_ops, sizeof h_ops, hipMemcpyHostToDevice, st));
  const T* x = (const T*)d_x;
  const T* y = (const T*)d_y;
  hipLaunchKernelGGL(q_pass1<T>, dim3(g12), dim3(kQNT), 0, st, x, y, n, part);
  hipLaunchKernelGGL(q_reduce, dim3(6), dim3(kQNT), 0, st, (const double*)part, (uint64_t)g12, 6, (const int*)ops, sums);
  hipLaunchKernelGGL(q_means, dim3(1), dim3(64), 0, st, (const double*)sums, n, means);
  double* part2 = part;  // pass 1 partials are no longer needed
  hipLaunchKernelGGL(q_pass2<T>, dim3(g12), dim3(kQNT), 0, st, x, y, n, (const double*)means, part2);
  hipLaunchKernelGGL(q_reduce, dim3(5), dim3(kQNT), 0, st, (const double*)part2, (uint64_t)g12, 5, (const int*)nullptr,
                     sums2);
  if (K) {
    hipLaunchKernelGGL(q_autocorr<T>, dim3((unsigned)nseg), dim3(kQNT), 0, st, x, y, n, (const double*)means, (int)K,
                       acpart);
    hipLaunchKernelGGL(q_reduce, dim3(K), dim3(kQNT), 0, st, (const double*)acpart, nseg, (int)K, (const int*)nullptr,
                       ac);
  }
  double h_sums[6], h_sums2[5];
  HIPCHK(hipMemcpyAsync(h_sums, sums, sizeof h_sums, hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(h_sums2, sums2, sizeof h_sums2, hipMemcpyDeviceToHost, st));
  std::vector<double> acv(K);
  if (K) HIPCHK(hipMemcpyAsync(acv.data(), ac, sizeof(double) * K, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  std::memset(q, 0, sizeof *q);
  const double N = (double)n;
  q->n = n;
  q->value_min = h_sums[3];
  q->value_max = h_sums[4];
  q->value_range = h_sums[4] - h_sums[3];
  q->max_abs_err = h_sums[5];
  q->mean_err = h_sums[2] / N;
  q->rmse = std::sqrt(h_sums2[4] / N);
  q->nrmse = q->rmse / q->value_range;
  q->psnr = 20.0 * std::log10(q->value_range / q->rmse);
  q->pearson = h_sums2[2] / std::sqrt(h_sums2[0] * h_sums2[1]);
  for (uint32_t k = 0; k < K; k++) h_ac[k] = acv[k] / h_sums2[3];
  return SZ_OK;
}

template <typename T>
int survey_t(sz_ctx* ctx, const sz_params* p, const Layout& Lf, const void* d_in, const uint64_t* sample,
             double* rph_decomp, double* rph_orig, uint32_t* best_n, hipStream_t st) {
  // 1. the bound of the whole field (value range in relative modes)
  DevPlan* P = ctx->plan;
  PlanInit I = {};
  I.m = 1;
  I.eb_mode = (uint32_t)Lf.eb_mode;
  I.eb_abs = p->eb_abs;
  I.eb_rel = p->eb_rel;
  I.dtype = (uint32_t)Lf.dtype;
  hipLaunchKernelGGL(plan_init_kernel, dim3(1), dim3(64), 0, st, P, I);
  if (Lf.eb_mode != SZ_EB_ABS) {
    const uint64_t g = std::min<uint64_t>(ceil_div((uint64_t)Lf.n, 256 * 16 / sizeof(T)) + 1, 512);
    hipLaunchKernelGGL(minmax_kernel<T>, dim3((unsigned)g), dim3(256), 0, st, (const T*)d_in, (uint64_t)Lf.n, P);
  }
  hipLaunchKernelGGL(eb_resolve_kernel<T>, dim3(1), dim3(64), 0, st, P, I);
  HIPCHK(hipMemcpyAsync(ctx->h_plan, P, sizeof(DevPlan), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  if (ctx->h_plan->status) return ctx->h_plan->status;
  const double eb = ctx->h_plan->eb;  // eb_T as a double: re-rounding it into T is exact
  // 2. the centred sample, contiguous
  const int pad = 3 - Lf.ndim;
  int64_t sdim[3] = {1, 1, 1}, off[3] = {0, 0, 0};
  uint64_t ns = 1;
  for (int d = 0; d < 3; d++) {
    const int64_t full = Lf.dims3[d];
    int64_t s = full;
    if (d >= pad && sample && sample[d - pad] && (int64_t)sample[d - pad] < full) s = (int64_t)sample[d - pad];
    sdim[d] = s;
    off[d] = (full - s) / 2;
    ns *= (uint64_t)s;
  }
  sz_params q = *p;
  for (int d = 0; d < Lf.ndim; d++) {
    q.dims[d] = (uint64_t)sdim[pad + d];
    q.block[d] = std::min<uint64_t>((uint64_t)Lf.blk3[pad + d], q.dims[d]);
  }
  q.eb_mode = SZ_EB_ABS;
  q.eb_abs = eb;
  q.quant_bits = 1;
  int rc;
  // one sample buffer ahead of the sweep workspace
  const size_t sbytes = ((ns * sizeof(T)) + 255) & ~size_t(255);
  size_t need = 0;
  for (uint32_t nl = 1; nl <= 4; nl++) {
    q.layers = nl;
    Layout L;
    if ((rc = resolve(&q, L))) return rc;
    need = std::max(need, carve_comp(L, nullptr, nullptr, true, xchg_reserve(ctx)));
  }
  // the sweep carves from ctx->arena; keep the sample in a buffer of its own
  T* samp = nullptr;
  if (hipMallocAsync((void**)&samp, sbytes + 64, st) != hipSuccess) return SZ_ENOMEM;
  {
    const unsigned g = (unsigned)std::min<uint64_t>(ceil_div(ns, 256), 8192);
    hipLaunchKernelGGL(crop_kernel<T>, dim3(g), dim3(256), 0, st, (const T*)d_in, samp, Lf.dims3[1], Lf.dims3[2],
                       off[0], off[1], off[2], sdim[0], sdim[1], sdim[2]);
  }
  if ((rc = ensure_arena(ctx, need + 256))) {
    (void)hipFreeAsync(samp, st);
    return rc;
  }
  unsigned long long* cnt = nullptr;
  if (hipMallocAsync((void**)&cnt, 64, st) != hipSuccess) {
    (void)hipFreeAsync(samp, st);
    return SZ_ENOMEM;
  }
  HIPCHK(hipMemsetAsync(cnt, 0, 64, st));
  double best = -1;
  *best_n = 1;
  for (uint32_t nl = 1; nl <= 4; nl++) {
    q.layers = nl;
    Layout L;
    resolve(&q, L);
    // decompressed neighbours: one sweep at m = 1, unpredictable count = H[0]
    if ((rc = enqueue_compress_t<T>(ctx, L, &q, samp, nullptr, 0, st, true))) break;
    CompWs W;
    carve_comp(L, (uint8_t*)ctx->arena, &W, true, ctx->xres_used);
    uint32_t h0 = 0;
    HIPCHK(hipMemcpyAsync(&h0, W.hist, 4, hipMemcpyDeviceToHost, st));
    HIPCHK(hipMemcpyAsync(ctx->h_plan, ctx->plan, sizeof(DevPlan), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    if ((rc = ctx->h_plan->status)) break;
    // original neighbours
    launch_orig_hits<T>(L.ndim, (int)nl, samp, L.g, *ctx->h_plan, cnt + nl, st);
    unsigned long long hits = 0;
    HIPCHK(hipMemcpyAsync(&hits, cnt + nl, 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    rph_decomp[nl - 1] = 1.0 - (double)h0 / (double)ns;
    rph_orig[nl - 1] = (double)hits / (double)ns;
    if (rph_decomp[nl - 1] > best) {
      best = rph_decomp[nl - 1];
      *best_n = nl;
    }
  }
  (void)hipFreeAsync(cnt, st);
  (void)hipFreeAsync(samp, st);
  (void)hipStreamSynchronize(st);
  return rc;
}

}  // namespace
}  // namespace szh

extern "C" {

int sz_quality(sz_ctx* ctx, uint32_t dtype, uint64_t n, const void* d_orig, const void* d_recon, uint32_t max_lag,
               double* h_autocorr, sz_quality_t* out, void* stream) {
  if (!ctx || !d_orig || !d_recon || !out || n < 2 || dtype > 1 || max_lag > (uint32_t)kMaxLag ||
      (max_lag && !h_autocorr))
    return SZ_EINVAL;
  if (hipSetDevice(ctx->device) != hipSuccess) return SZ_EHIP;
  hipStream_t st = (hipStream_t)stream;
  return dtype == SZ_F32 ? quality_t<float>(ctx, n, d_orig, d_recon, max_lag, h_autocorr, out, st)
                         : quality_t<double>(ctx, n, d_orig, d_recon, max_lag, h_autocorr, out, st);
}

int sz_layer_survey(sz_ctx* ctx, const sz_params* p, const void* d_in, const uint64_t* sample, double* rph_decomp,
                    double* rph_orig, uint32_t* best_n, void* stream) {
  if (!ctx || !p || !d_in || !rph_decomp || !rph_orig || !best_n) return SZ_EINVAL;
  Layout L;
  int rc = resolve(p, L);
  if (rc) return rc;
  if (check_align(d_in)) return SZ_EINVAL;
  if (hipSetDevice(ctx->device) != hipSuccess) return SZ_EHIP;
  hipStream_t st = (hipStream_t)stream;
  return L.dtype == SZ_F32 ? survey_t<float>(ctx, p, L, d_in, sample, rph_decomp, rph_orig, best_n, st)
                           : survey_t<double>(ctx, p, L, d_in, sample, rph_decomp, rph_orig, best_n, st);
}

}  // extern "C"
