// C ABI entry points of the single-field codec (include/szhip.h): context
// management, compress / decompress / inspect, and the stage profiler.  The
// kernel sequences themselves are in runtime.hpp.
#include "runtime.hpp"

using namespace szh;

// ------------------------------------------------- static no-allocation scratch
// Workspace of sz_compress_async_noalloc: a device array of fixed size in
// the library's code object, so that entry point never allocates.  Every GPU
// the library runs on holds its own copy until the process ends.  In host
// code the name `scratch` is only a stand-in for the symbol: its device
// address on each GPU comes from hipGetSymbolAddress, taken once per device
// when the first context on that device is created, and only that address is
// passed to kernels.
constexpr size_t kPlanBytes = 256;
static_assert(sizeof(DevPlan) <= kPlanBytes, "the plan must fit its slot of the static scratch");
constexpr size_t kStaticScratch = (size_t)SZ_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) uint8_t scratch[kStaticScratch];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

// With `device` current: the device address of its static scratch, looked up
// once per device.
void* scratch_address(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> g(g_scratch_mu);
  if (!g_scratch[device]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess) return nullptr;
    g_scratch[device] = ptr;
  }
  return g_scratch[device];
}
}  // namespace


// =================================================================== C ABI
extern "C" {

int sz_ctx_create(sz_ctx** out, int device) {
  if (!out) return SZ_EINVAL;
  *out = nullptr;
  if (hipSetDevice(device) != hipSuccess) return SZ_EHIP;
  sz_ctx* c = new sz_ctx();
  c->device = device;
  if (hipMalloc(&c->plan, sizeof(DevPlan)) != hipSuccess) {
    delete c;
    return SZ_ENOMEM;
  }
  if (hipHostMalloc(&c->h_plan, sizeof(DevPlan), hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc(&c->h_hdr, kHdr, hipHostMallocDefault) != hipSuccess) {
    (void)hipFree(c->plan);
    delete c;
    return SZ_ENOMEM;
  }
  c->scratch = scratch_address(device);
  if (!c->scratch) {
    (void)hipFree(c->plan);
    (void)hipHostFree(c->h_plan);
    (void)hipHostFree(c->h_hdr);
    delete c;
    return SZ_EHIP;
  }
  *out = c;
  return SZ_OK;
}

void sz_ctx_destroy(sz_ctx* c) {
  if (!c) return;
  (void)hipSetDevice(c->device);
  (void)hipDeviceSynchronize();
  if (c->arena) (void)hipFree(c->arena);
  if (c->plan) (void)hipFree(c->plan);
  if (c->h_plan) (void)hipHostFree(c->h_plan);
  if (c->h_hdr) (void)hipHostFree(c->h_hdr);
  for (int i = 0; i < 2 * ST_COUNT; i++)
    if (c->ev[i]) (void)hipEventDestroy(c->ev[i]);
  delete c;
}

int sz_ctx_profile(sz_ctx* c, int enable) {
  if (!c) return SZ_EINVAL;
  if (hipSetDevice(c->device) != hipSuccess) return SZ_EHIP;
  for (int i = 0; i < 2 * ST_COUNT; i++)
    if (!c->ev[i] && hipEventCreate(&c->ev[i]) != hipSuccess) return SZ_EHIP;
  for (int i = 0; i < ST_COUNT; i++) {
    c->prof_ms[i] = 0;
    c->prof_calls[i] = 0;
    c->ev_used[i] = false;
  }
  if ((enable & ~0x1FFFF) != 0 || (enable > 1 && !(enable & 0x10000))) return SZ_EINVAL;
  c->prof = enable != 0;
  c->prof_mask = (enable & 0x10000) ? (uint32_t)(enable & 0xFFFF) : 0xFFFFu;
  return SZ_OK;
}

int sz_ctx_debug_sweep(sz_ctx* c, int schedule, int claim_order) {
  if (!c || schedule < 0 || schedule > 1 || claim_order < 0 || claim_order > 2) return SZ_EINVAL;
  c->dbg_sched = schedule;
  c->dbg_claim = (uint32_t)claim_order;
  return SZ_OK;
}

int sz_ctx_profile_read(sz_ctx* c, double* ms, uint64_t* calls, int n) {
  if (!c) return SZ_EINVAL;
  for (int i = 0; i < n && i < ST_COUNT; i++) {
    if (ms) ms[i] = c->prof_ms[i];
    if (calls) calls[i] = c->prof_calls[i];
  }
  return ST_COUNT;
}

size_t sz_compress_bound(const sz_params* p) {
  Layout L;
  if (resolve(p, L)) return 0;
  return kHdr + (size_t)L.n * L.ts;
}

static int compress_common(sz_ctx* ctx, const sz_params* p, const void* d_in, void* d_out, size_t cap,
                           hipStream_t st, Layout& L, bool codes_only) {
  if (!ctx) return SZ_EINVAL;
  const Sched legacy = p ? default_sched((int)p->dtype, (int)p->ndim, (int)p->layers, true) : Sched{};
  int rc = resolve(p, L, ctx->dbg_sched == 1 ? &legacy : nullptr);
  if (rc) return rc;
  if (check_align(d_in) || (!codes_only && check_align(d_out))) return SZ_EINVAL;
  if (hipSetDevice(ctx->device) != hipSuccess) return SZ_EHIP;
  return L.dtype == SZ_F32 ? enqueue_compress_t<float>(ctx, L, p, d_in, d_out, cap, st, codes_only)
                           : enqueue_compress_t<double>(ctx, L, p, d_in, d_out, cap, st, codes_only);
}

int sz_compress(sz_ctx* ctx, const sz_params* p, const void* d_in, void* d_out, size_t cap, size_t* out_size,
                sz_stats* stats, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  Layout L;
  int rc = compress_common(ctx, p, d_in, d_out, cap, st, L, false);
  if (rc) return rc;
  HIPCHK(hipMemcpyAsync(ctx->h_plan, ctx->plan, sizeof(DevPlan), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  stage_collect(ctx);
  const DevPlan& P = *ctx->h_plan;
  if (P.status) return P.status;
  if (out_size) *out_size = P.total;
  if (stats) fill_stats(P, L, stats);
  return SZ_OK;
}

int sz_compress_async(sz_ctx* ctx, const sz_params* p, const void* d_in, void* d_out, size_t cap,
                      uint64_t* d_out_size, int32_t* d_status, void* stream) {
  hipStream_t st = (hipStream_t)stream;
  Layout L;
  const bool prof = ctx ? ctx->prof : false;
  if (ctx) ctx->prof = false;  // no event records inside a possible capture
  int rc = compress_common(ctx, p, d_in, d_out, cap, st, L, false);
  if (ctx) ctx->prof = prof;
  if (rc) return rc;
  hipLaunchKernelGGL(finish_kernel, dim3(1), dim3(64), 0, st, (const DevPlan*)ctx->plan, d_out_size, d_status);
  return hipGetLastError() == hipSuccess ? SZ_OK : SZ_EHIP;
}

int sz_compress_async_noalloc(sz_ctx* ctx, const sz_params* p, const void* d_in, void* d_out, size_t cap,
                              uint64_t* d_out_size, int32_t* d_status, void* stream) {
  if (!ctx || !ctx->scratch) return SZ_EINVAL;
  Layout L;
  int rc = resolve(p, L);
  if (rc) return rc;
  if (check_align(d_in) || check_align(d_out)) return SZ_EINVAL;
  // the whole workspace comes from the static scratch, behind the plan
  if (carve_comp(L, nullptr, nullptr) > kStaticScratch - kPlanBytes) return SZ_ESCRATCH;
  if (hipSetDevice(ctx->device) != hipSuccess) return SZ_EHIP;
  sz_ctx view;  // a context over the static scratch; owns nothing
  view.device = ctx->device;
  view.prof = false;
  view.plan = (DevPlan*)ctx->scratch;
  view.arena = (uint8_t*)ctx->scratch + kPlanBytes;
  view.arena_size = kStaticScratch - kPlanBytes;
  view.fixed_arena = true;
  hipStream_t st = (hipStream_t)stream;
  rc = L.dtype == SZ_F32 ? enqueue_compress_t<float>(&view, L, p, d_in, d_out, cap, st, false)
                         : enqueue_compress_t<double>(&view, L, p, d_in, d_out, cap, st, false);
  if (rc) return rc;
  hipLaunchKernelGGL(finish_kernel, dim3(1), dim3(64), 0, st, (const DevPlan*)view.plan, d_out_size, d_status);
  return hipGetLastError() == hipSuccess ? SZ_OK : SZ_EHIP;
}

int sz_quantize(sz_ctx* ctx, const sz_params* p, const void* d_in, uint16_t* d_codes, void* d_xprime,
                sz_stats* stats, void* stream) {
  if (!p || p->quant_bits < 1 || p->quant_bits > 16) return SZ_EINVAL;
  sz_params q = *p;
  q.quant_bits = 16;  // keep 16-bit codes in the intermediate array
  hipStream_t st = (hipStream_t)stream;
  Layout L;
  if (!ctx) return SZ_EINVAL;
  const Sched legacy = default_sched((int)p->dtype, (int)p->ndim, (int)p->layers, true);
  int rc = resolve(&q, L, ctx->dbg_sched == 1 ? &legacy : nullptr);
  if (rc) return rc;
  if (!ctx || check_align(d_in) || check_align(d_codes)) return SZ_EINVAL;
  if (hipSetDevice(ctx->device) != hipSuccess) return SZ_EHIP;
  L.m_req = (int)p->quant_bits;
  L.cw = 2;
  q.quant_bits = p->quant_bits;
  rc = L.dtype == SZ_F32 ? enqueue_compress_t<float>(ctx, L, &q, d_in, nullptr, 0, st, true)
                         : enqueue_compress_t<double>(ctx, L, &q, d_in, nullptr, 0, st, true);
  if (rc) return rc;
  CompWs W;
  carve_comp(L, (uint8_t*)ctx->arena, &W, true, ctx->xres_used);
  HIPCHK(hipMemcpyAsync(d_codes, W.codes, (size_t)L.n * 2, hipMemcpyDeviceToDevice, st));
  if (d_xprime) HIPCHK(hipMemcpyAsync(d_xprime, W.xs, (size_t)L.n * L.ts, hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(ctx->h_plan, ctx->plan, sizeof(DevPlan), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  const DevPlan& P = *ctx->h_plan;
  if (P.status) return P.status;
  if (stats) fill_stats(P, L, stats);
  return SZ_OK;
}

int sz_inspect(const void* h_hdr, size_t n, sz_params* p, sz_stats* s) {
  if (!h_hdr) return SZ_EINVAL;
  Hdr h;
  if (n < kHdr) return SZ_ECORRUPT;
  int rc = parse_header((const uint8_t*)h_hdr, n, h, false);
  if (!rc) rc = check_sections(h);
  if (rc) return rc;
  if (p) hdr_params(h, p);
  if (s) {
    std::memset(s, 0, sizeof *s);
    s->n_points = h.n;
    s->n_unpred = h.n_unpred;
    s->huff_bits = h.huff_bits;
    s->tail_bits = h.tail_bits;
    s->compressed_bytes = h.total;
    s->ebT_bits = h.ebT_bits;
    s->m_used = h.m;
    s->raw_fallback = h.flags & 1;
    s->n_used_syms = h.n_used;
  }
  return SZ_OK;
}

int sz_decompress(sz_ctx* ctx, const void* d_comp, size_t comp_size, void* d_out, size_t cap, void* stream) {
  if (!ctx || !d_comp || !d_out) return SZ_EINVAL;
  if (check_align(d_comp) || check_align(d_out)) return SZ_EINVAL;
  if (comp_size < kHdr) return SZ_ECORRUPT;
  hipStream_t st = (hipStream_t)stream;
  if (hipSetDevice(ctx->device) != hipSuccess) return SZ_EHIP;
  HIPCHK(hipMemcpyAsync(ctx->h_hdr, d_comp, kHdr, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  Hdr h;
  Layout L;
  int rc = prepare_decompress(ctx->h_hdr, comp_size, cap, h, L, ctx->dbg_sched == 1);
  if (rc) return rc;
  if ((rc = enqueue_decompress_any(ctx, L, h, d_comp, d_out, st))) return rc;
  HIPCHK(hipMemcpyAsync(ctx->h_plan, ctx->plan, sizeof(DevPlan), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  stage_collect(ctx);
  return ctx->h_plan->status;
}

const char* sz_strerror(int code) {
  switch (code) {
    case SZ_OK: return "ok";
    case SZ_EINVAL: return "invalid argument";
    case SZ_ECAPACITY: return "output capacity too small";
    case SZ_ECORRUPT: return "corrupt container";
    case SZ_ENONFINITE: return "non-finite value with a range-relative bound";
    case SZ_ENOMEM: return "out of device memory";
    case SZ_EHIP: return "HIP runtime error";
    case SZ_ESTALL: return "internal wavefront wait exceeded its bound";
    case SZ_ETIMEDOUT: return "request not finished within the timeout";
    case SZ_ESCRATCH: return "field needs more workspace than the static no-allocation scratch holds";
  }
  return "unknown error";
}

}  // extern "C"
