// Host runtime shared by the C ABI entry points (single-field calls, the
// batched form and the request server): parameter resolution, workspace
// carving, and the kernel sequences of compression and decompression.
// Every step of the method runs in the kernels; the host only validates,
// sizes buffers and enqueues.  The compress sequence is free of host
// synchronisation so it can be captured into a HIP graph.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <type_traits>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <mutex>

#include "common.hpp"
#include "kernels.hpp"
#include "sweep_launch.hpp"

// Stages timed by the optional event profiler (sz_ctx_profile).
enum Stage {
  ST_RANGE = 0,      // value range + error bound
  ST_SWEEP_C,        // prediction + quantization sweep (all passes)
  ST_CODEBOOK,       // Huffman code lengths and canonical codes
  ST_ENCODE,         // chunk totals, scans, layout, bit packing, header
  ST_DECTAB,         // decode tables + chunk offsets
  ST_DECODE,         // Huffman decode + row-segment offsets
  ST_UNPRED,         // unpredictable values
  ST_SWEEP_D,        // reconstruction sweep
  ST_HIST,           // code histogram (wave-tiled sweep with fixed m)
  ST_COUNT
};

struct sz_ctx {
  int device = 0;
  bool prof = false;
  uint32_t prof_mask = 0xFFFFu;  // stages the profiler times (bit = Stage)
  hipEvent_t ev[2 * ST_COUNT] = {};
  bool ev_used[ST_COUNT] = {};
  double prof_ms[ST_COUNT] = {};
  uint64_t prof_calls[ST_COUNT] = {};
  void* arena = nullptr;
  size_t arena_size = 0;
  bool fixed_arena = false;        // arena memory lent by someone else: never (re)allocated here
  // The first xclean_bytes of the arena at xclean hold nothing but zeros and
  // tagged exchange records of this context's launches (wave sweep).
  void* xclean = nullptr;
  size_t xclean_bytes = 0;
  size_t xres_used = 0;  // exchange reserve of the last workspace carve (carve again with it)
  void* scratch = nullptr;         // this device's static scratch (no-allocation entry point)
  int dbg_sched = 0;               // sz_ctx_debug_sweep: 1 = row-per-thread tiles for every field
  uint32_t dbg_claim = 0;          // sz_ctx_debug_sweep: tile claim order
  szh::DevPlan* plan = nullptr;    // device
  szh::DevPlan* h_plan = nullptr;  // pinned host mirror
  uint8_t* h_hdr = nullptr;   // pinned host header staging
};


namespace szh {
// Internal linkage: every translation unit that launches these kernels
// carries its own copy.
namespace {

#define HIPCHK(x)                              \
  do {                                         \
    if ((x) != hipSuccess) return SZ_EHIP;     \
  } while (0)

void stage_begin(sz_ctx* c, int id, hipStream_t st) {
  if (!c->prof || !((c->prof_mask >> id) & 1u)) return;
  (void)hipEventRecord(c->ev[2 * id], st);
  c->ev_used[id] = true;
}
void stage_end(sz_ctx* c, int id, hipStream_t st) {
  if (c->prof && ((c->prof_mask >> id) & 1u)) (void)hipEventRecord(c->ev[2 * id + 1], st);
}
// After the stream has been synchronised: accumulate the recorded stages.
void stage_collect(sz_ctx* c) {
  if (!c->prof) return;
  for (int i = 0; i < ST_COUNT; i++) {
    if (!c->ev_used[i]) continue;
    float ms = 0;
    if (hipEventElapsedTime(&ms, c->ev[2 * i], c->ev[2 * i + 1]) == hipSuccess) {
      c->prof_ms[i] += ms;
      c->prof_calls[i] += 1;
    }
    c->ev_used[i] = false;
  }
}

struct Layout {
  int dtype, ndim, nl, m_req, eb_mode;
  int64_t dims3[3], blk3[3];
  int64_t n;
  uint32_t chunk;
  uint64_t n_chunks;
  int ts;          // element size
  int cw;          // bytes per code in the intermediate array
  Geom g;
  int grid;        // sweep workgroups
  uint64_t nseg;   // row segments (decompress queues)
  uint32_t ne;     // exporter rows per tile
  uint32_t nsp;    // steps stored per exporter row
  uint64_t xchg_bytes;
  bool wave;        // wave-tiled sweep (3D, one layer)
  int nw, az;       // its waves per workgroup and z sub-rows per lane
  uint64_t xy_bytes;  // y-exchange part of the exchange buffer (wave sweep)
  double theta;
  int xorc;         // unpredictable values XOR-coded (flag bit 1)
  uint64_t out_dims[3], out_block[3];
};

uint64_t ceil_div(uint64_t a, uint64_t b) { return (a + b - 1) / b; }

// Tile schedule of the sweep: legacy tiles of rz x ry rows (one row per
// thread) or wave tiles of nw waves x az z-rows x 64 y-rows.  The schedule
// changes launch geometry only, never the bytes produced.
struct Sched {
  int wave;    // 1: wave-tiled sweep (3D, one layer)
  int rz, ry;  // legacy tile
  int nw, az;  // wave tile
};

inline Sched default_sched(int dtype, int ndim, int nl, bool legacy = false) {
  Sched s;
  tile_shape(dtype, ndim, s.rz, s.ry);
  s.wave = (ndim == 3 || ndim == 2) && nl == 1 && !legacy;
  s.nw = wave_nw(dtype, ndim);
  s.az = wave_az(dtype, ndim);
  return s;
}

int resolve(const sz_params* p, Layout& L, const Sched* sched_override = nullptr) {
  if (!p || p->struct_size != sizeof(sz_params)) return SZ_EINVAL;
  if (p->dtype > 1 || p->ndim < 1 || p->ndim > 3) return SZ_EINVAL;
  if (p->layers < 1 || p->layers > 4 || p->quant_bits > 16 || p->eb_mode > 2) return SZ_EINVAL;
  if (p->chunk != 0 && (p->chunk < 256 || p->chunk > (uint32_t)kMaxChunk || p->chunk % 256)) return SZ_EINVAL;
  if (!(p->theta >= 0 && p->theta <= 1)) return SZ_EINVAL;
  if (p->unpred_coding > 1 || p->reserved != 0) return SZ_EINVAL;
  if (!std::isfinite(p->eb_abs) || !std::isfinite(p->eb_rel) || p->eb_abs < 0 || p->eb_rel < 0) return SZ_EINVAL;
  L.dtype = (int)p->dtype;
  L.ndim = (int)p->ndim;
  L.nl = (int)p->layers;
  L.m_req = (int)p->quant_bits;
  L.eb_mode = (int)p->eb_mode;
  L.theta = p->theta > 0 ? p->theta : 0.9;
  L.xorc = (int)p->unpred_coding;
  L.ts = p->dtype == SZ_F32 ? 4 : 8;
  L.cw = (p->quant_bits >= 1 && p->quant_bits <= 8) ? 1 : 2;
  const int pad = 3 - L.ndim;
  uint64_t n = 1;
  for (int d = 0; d < 3; d++) {
    L.dims3[d] = 1;
    L.blk3[d] = 1;
    L.out_dims[d] = 1;
    L.out_block[d] = 1;
  }
  for (int d = 0; d < L.ndim; d++) {
    // n stays below 2^40; the test comes before the product, which cannot wrap
    if (p->dims[d] == 0 || p->dims[d] >= (1ull << 31) || n > ((1ull << 40) - 1) / p->dims[d]) return SZ_EINVAL;
    n *= p->dims[d];
    L.dims3[pad + d] = (int64_t)p->dims[d];
    uint64_t b = p->block[d];
    if (b == 0) b = (L.ndim == 1) ? kDefaultBlock1D : p->dims[d];
    if (b > p->dims[d]) b = p->dims[d];
    L.blk3[pad + d] = (int64_t)b;
    L.out_dims[d] = p->dims[d];
    L.out_block[d] = b;
  }
  L.n = (int64_t)n;
  L.chunk = p->chunk ? p->chunk : kDefaultChunk;
  L.n_chunks = ceil_div(n, L.chunk);
  const Sched sched = sched_override ? *sched_override : default_sched(L.dtype, L.ndim, L.nl);
  const int rz = sched.rz, ry = sched.ry;
  Geom& g = L.g;
  for (int d = 0; d < 3; d++) {
    g.dims[d] = L.dims3[d];
    g.blk[d] = L.blk3[d];
    g.nblk[d] = (int32_t)ceil_div(L.dims3[d], L.blk3[d]);
  }
  g.ndim = L.ndim;
  g.n = L.n;
  if (L.ndim == 1) {
    const uint64_t nb = ceil_div(n, L.blk3[2]);
    g.tz_per_blk = 1;
    g.ty_per_blk = 1;
    g.ntiles = (int32_t)ceil_div(nb, ry);
    L.nseg = nb;
  } else {
    g.tz_per_blk = (L.ndim == 3) ? (int32_t)ceil_div(L.blk3[0], rz) : 1;
    g.ty_per_blk = (int32_t)ceil_div(L.blk3[1], ry);
    const uint64_t nt = (uint64_t)g.nblk[0] * g.nblk[1] * g.nblk[2] * g.tz_per_blk * g.ty_per_blk;
    if (nt >= (1ull << 31)) return SZ_EINVAL;
    g.ntiles = (int32_t)nt;
    L.nseg = (uint64_t)L.dims3[0] * L.dims3[1] * g.nblk[2];
  }
  L.grid = g.ntiles;
  // exchange buffer of boundary rows: [tile][exporter row][step]
  const int span = (L.ndim == 1) ? 0 : (rz - 1) + (ry - 1);
  const uint64_t ngroups = ceil_div((uint64_t)L.blk3[2] + span, kG);
  L.ne = (L.ndim == 3) ? (uint32_t)(L.nl * ry + (rz - L.nl) * L.nl) : (L.ndim == 2 ? (uint32_t)L.nl : 0);
  L.nsp = (uint32_t)ceil_div(kG * ngroups + rz + ry + kG, kG) * kG;
  L.xchg_bytes = (uint64_t)g.ntiles * L.ne * L.nsp * L.ts;
  // Buffer-resource offsets are 32-bit: the exchange buffer and the input
  // span of one tile must stay below 2 GiB.
  const uint64_t tile_span = (L.ndim == 3) ? (uint64_t)rz * L.dims3[1] * L.dims3[2]
                                           : (L.ndim == 2 ? (uint64_t)ry * L.dims3[2] : (uint64_t)ry * L.blk3[2]);
  if (L.xchg_bytes >= 0x7FFFFF00ull || (tile_span + 64) * L.ts >= 0x7FFFFF00ull) return SZ_EINVAL;
  // 2D and 3D fields with the 1-layer predictor use the wave-tiled sweep:
  // tiles of nw * az z-rows by 64 y-rows, one workgroup of nw waves each (a
  // 2D field is the single z-row of a 1 x Y x X field).
  L.wave = sched.wave && (L.ndim == 3 || L.ndim == 2) && L.nl == 1;
  L.az = 0;
  L.nw = 0;
  L.xy_bytes = 0;
  if (L.wave) {
    const int az = sched.az, nw = sched.nw, tz = nw * az;
    g.tz_per_blk = (int32_t)ceil_div(L.blk3[0], tz);
    // the z-exchange is read in whole 16-byte pieces of records
    if (g.tz_per_blk > 1 && tz % (16 / L.ts) != 0) return SZ_EINVAL;
    g.ty_per_blk = (int32_t)ceil_div(L.blk3[1], kWLanes);
    const uint64_t nt = (uint64_t)g.nblk[0] * g.nblk[1] * g.nblk[2] * g.tz_per_blk * g.ty_per_blk;
    if (nt >= (1ull << 31)) return SZ_EINVAL;
    g.ntiles = (int32_t)nt;
    L.grid = g.ntiles;
    L.az = az;
    L.nw = nw;
    const uint64_t nsteps = (uint64_t)L.blk3[2] + (tz - 1) + (kWLanes - 1);
    L.nsp = (uint32_t)(ceil_div(nsteps + kWLanes + tz + 4 * kWG, 16) * 16);
    L.ne = 0;
    // tagged records: 16 bytes per step along y, 8 bytes per 32-bit word of
    // a value along z
    L.xy_bytes = (uint64_t)g.ntiles * nw * L.nsp * 16;
    // z-exchange records only when a block holds several tiles along z
    const uint64_t xz_bytes = g.tz_per_blk > 1 ? (uint64_t)g.ntiles * 2 * 64 * L.nsp * (2 * L.ts) : 0;
    L.xchg_bytes = L.xy_bytes + xz_bytes;
    // elements one tile's input and code descriptors span past their base
    const uint64_t rows = L.ndim == 2 ? (uint64_t)kWLanes + 1 : ((uint64_t)tz + 1) * L.dims3[1];
    const uint64_t span = rows * L.dims3[2] + 4 * (tz + kWLanes + kWG);
    if (L.xy_bytes >= 0x7FFFFF00ull || xz_bytes >= 0x7FFFFF00ull || span * L.ts >= 0x7FFFFF00ull ||
        span * L.cw >= 0x7FFFFF00ull)
      return SZ_EINVAL;
  }
  return SZ_OK;
}

// Bump allocator over the context arena.
struct Carve {
  uint8_t* base;
  size_t off = 0;
  template <typename P>
  P* take(size_t bytes) {
    off = (off + 255) & ~size_t(255);
    P* r = (P*)(base + off);
    off += bytes;
    return r;
  }
};

struct CompWs {
  uint8_t* codes;
  void* xs;        // every recorded value (sz_quantize only)
  void* xchg;
  uint32_t* hist;
  uint32_t* hpart;  // per-block histogram rows (1-byte codes)
  uint32_t* progress;
  uint32_t* ticket;
  uint32_t *cbits, *cu, *ctb;
  uint64_t *boff, *uoff, *toff;
  uint64_t *tsum_b, *tsum_u, *tsum_t, *tot;
  uint8_t* len;
  uint32_t* cw;
  uint64_t* gkeys;
  uint64_t* gw;
  uint32_t *gpar, *ganc, *gdep;
};

// Bytes of the exchange region the sweep of L uses, and those a workspace
// reserves for it: at least `reserve`, the part of the region an earlier
// call kept clean (xchg_reserve).  The region comes first in a workspace.
inline uint64_t xchg_need(const Layout& L) { return (L.xchg_bytes + 512 + 15) & ~(uint64_t)15; }
inline size_t xchg_reserve(const sz_ctx* ctx) { return ctx->fixed_arena ? 0 : ctx->xclean_bytes; }

size_t carve_comp(const Layout& L, uint8_t* base, CompWs* W, bool keep_values = false, size_t reserve = 0) {
  Carve c{base};
  const uint64_t nt = ceil_div(L.n_chunks, 4096) + 1;
  CompWs w;
  w.xchg = c.take<uint8_t>(std::max<uint64_t>(xchg_need(L), reserve));
  w.codes = c.take<uint8_t>((L.n + 64) * L.cw);
  w.xs = keep_values ? c.take<uint8_t>(L.n * L.ts) : nullptr;
  w.hist = c.take<uint32_t>(65536 * 4);
  w.hpart = L.cw == 1 ? c.take<uint32_t>(kHistBlocks * 256 * 4)
                       : c.take<uint32_t>((size_t)2 * hist2_blocks((uint64_t)L.n) * kHist2Half * 4);
  w.progress = c.take<uint32_t>((L.g.ntiles + 1) * 4);
  w.ticket = w.progress + L.g.ntiles;
  w.cbits = c.take<uint32_t>(L.n_chunks * 4);
  w.cu = c.take<uint32_t>(L.n_chunks * 4);
  w.ctb = c.take<uint32_t>(L.n_chunks * 4);
  w.boff = c.take<uint64_t>(L.n_chunks * 8);
  w.uoff = c.take<uint64_t>(L.n_chunks * 8);
  w.toff = c.take<uint64_t>(L.n_chunks * 8);
  w.tsum_b = c.take<uint64_t>(nt * 8);
  w.tsum_u = c.take<uint64_t>(nt * 8);
  w.tsum_t = c.take<uint64_t>(nt * 8);
  w.tot = c.take<uint64_t>(4 * 8);
  w.len = c.take<uint8_t>(65536);
  w.cw = c.take<uint32_t>(65536 * 4);
  w.gkeys = c.take<uint64_t>(65536 * 8);
  w.gw = c.take<uint64_t>(131072 * 8);
  w.gpar = c.take<uint32_t>(131072 * 4);
  w.ganc = c.take<uint32_t>(262144 * 4);
  w.gdep = c.take<uint32_t>(262144 * 4);
  if (W) *W = w;
  return c.off + 256;
}

int ensure_arena(sz_ctx* ctx, size_t bytes) {
  if (bytes <= ctx->arena_size) return SZ_OK;
  if (ctx->fixed_arena) return SZ_ENOMEM;
  if (ctx->arena) {
    if (hipDeviceSynchronize() != hipSuccess) return SZ_EHIP;
    (void)hipFree(ctx->arena);
    ctx->arena = nullptr;
    ctx->arena_size = 0;
  }
  ctx->xclean = nullptr;
  ctx->xclean_bytes = 0;
  size_t want = bytes + bytes / 8;
  if (hipMalloc(&ctx->arena, want) != hipSuccess) {
    ctx->arena = nullptr;
    return SZ_ENOMEM;
  }
  ctx->arena_size = want;
  return SZ_OK;
}

// Zero `bytes` (a multiple of 16) at p, on st (a fill kernel: no memset
// node in a captured graph).
void zero_bytes(void* p, uint64_t bytes, hipStream_t st) {
  const uint64_t n = bytes / 16;
  if (!n) return;
  const uint64_t g = std::min<uint64_t>(ceil_div(n, 256), 1024);
  hipLaunchKernelGGL(zero16_kernel, dim3((unsigned)g), dim3(256), 0, st, (uint4*)p, n);
}

// Before a sweep that uses the exchange region at xchg.  The wave sweep polls
// records its writer may not have stored yet and tells them by their tag, so
// the region must hold nothing but zeros and this plan's earlier records:
// the part the context knows to be clean is kept, the rest is cleared (all
// of it for a lent arena, whose earlier contents are unknown).  The other
// sweeps write untagged records, after which nothing is known to be clean.
void prepare_xchg(sz_ctx* ctx, const Layout& L, void* xchg, hipStream_t st) {
  if (!L.wave) {
    ctx->xclean = nullptr;
    ctx->xclean_bytes = 0;
    return;
  }
  const uint64_t need = xchg_need(L);
  const bool known = !ctx->fixed_arena && xchg == ctx->xclean;
  const uint64_t clean = known ? ctx->xclean_bytes : 0;
  if (need > clean) zero_bytes((uint8_t*)xchg + clean, need - clean, st);
  if (!ctx->fixed_arena) {
    // the workspace reserved max(need, clean) bytes for the region
    ctx->xclean = xchg;
    ctx->xclean_bytes = std::max<uint64_t>(need, clean);
  }
}

int launch_sweep(const Layout& L, bool comp, const SweepArgs& a, hipStream_t st) {
  hipError_t e;
  const int cw = L.cw;
  if (L.dtype == SZ_F32) {
    e = L.ndim == 1 ? sweep_f32_d1(L.nl, comp, cw, a, L.grid, st)
                    : (L.ndim == 2 ? sweep_f32_d2(L.nl, comp, cw, a, L.grid, st)
                                   : sweep_f32_d3(L.nl, comp, cw, a, L.grid, st));
  } else {
    e = L.ndim == 1 ? sweep_f64_d1(L.nl, comp, cw, a, L.grid, st)
                    : (L.ndim == 2 ? sweep_f64_d2(L.nl, comp, cw, a, L.grid, st)
                                   : sweep_f64_d3(L.nl, comp, cw, a, L.grid, st));
  }
  return e == hipSuccess ? SZ_OK : SZ_EHIP;
}

WArgs make_wargs(const Layout& L, const void* x, void* codes, void* xo, void* xchg, uint32_t* ticket,
                 DevPlan* P) {
  WArgs a;
  for (int d = 0; d < 3; d++) {
    a.dims[d] = L.dims3[d];
    a.blk[d] = L.blk3[d];
    a.nblk[d] = L.g.nblk[d];
  }
  a.tz_per_blk = L.g.tz_per_blk;
  a.ty_per_blk = L.g.ty_per_blk;
  a.ntiles = L.g.ntiles;
  a.nsp = L.nsp;
  a.x = x;
  a.codes = codes;
  a.xo = xo;
  a.xy = xchg;
  a.xz = (uint8_t*)xchg + ((L.xy_bytes + 255) & ~255ull);
  a.uvals = nullptr;
  a.useg = nullptr;
  a.n_unpred = 0;
  a.codes_cap = (uint64_t)L.n + 64;
  a.n = (uint64_t)L.n;
  a.ticket = ticket;
  a.plan = P;
  a.pass2 = 0;
  a.export_all = 0;
  return a;
}

int launch_wsweep(const Layout& L, bool comp, const WArgs& a, hipStream_t st) {
  const hipError_t e = L.dtype == SZ_F32 ? wsweep_f32(comp, L.cw, L.nw, L.az, a, L.grid, st)
                                         : wsweep_f64(comp, L.cw, L.nw, L.az, a, L.grid, st);
  return e == hipSuccess ? SZ_OK : SZ_EHIP;
}

void launch_hist(const Layout& L, const void* codes, uint32_t* hist, uint32_t* hpart, const DevPlan* P,
                 uint32_t pass2, hipStream_t st) {
  if (L.cw == 1 && hpart) {
    // per-block rows, then one block per bin; bins past 2^m come out zero
    const uint64_t g = std::min<uint64_t>(ceil_div((uint64_t)L.n, 1024 * 64), kHistBlocks);
    hipLaunchKernelGGL(hist_kernel<uint8_t>, dim3((unsigned)g), dim3(1024), 0, st, (const uint8_t*)codes,
                       (uint64_t)L.n, hist, P, pass2, hpart);
    hipLaunchKernelGGL(hist_reduce_kernel, dim3(256), dim3(256), 0, st, (const uint32_t*)hpart, (uint32_t)g, hist, P,
                       pass2);
    return;
  }
  if (L.cw == 2 && hpart) {
    // two halves of 32768 bins, each block with its half in LDS, then the rows
    const uint32_t nb = hist2_blocks((uint64_t)L.n);
    const int lds = (int)(kHist2Half * 4);
    (void)hipFuncSetAttribute((const void*)hist2_kernel, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    hipLaunchKernelGGL(hist2_kernel, dim3(nb, 2), dim3(1024), lds, st, (const uint16_t*)codes, (uint64_t)L.n, hpart,
                       P, pass2);
    hipLaunchKernelGGL(hist2_reduce_kernel, dim3(65536 / 256), dim3(1024), 0, st, (const uint32_t*)hpart, nb, hist,
                       P, pass2);
    return;
  }
  const uint64_t g = std::min<uint64_t>(ceil_div((uint64_t)L.n, 1024 * 16), 1024);
  if (L.cw == 1)
    hipLaunchKernelGGL(hist_kernel<uint8_t>, dim3((unsigned)g), dim3(1024), 0, st, (const uint8_t*)codes,
                       (uint64_t)L.n, hist, P, pass2, (uint32_t*)nullptr);
  else
    hipLaunchKernelGGL(hist_kernel<uint16_t>, dim3((unsigned)g), dim3(1024), 0, st, (const uint16_t*)codes,
                       (uint64_t)L.n, hist, P, pass2, (uint32_t*)nullptr);
}

void fill(uint32_t* p, uint32_t v, uint64_t n, hipStream_t st) {
  if (!n) return;
  const uint64_t g = std::min<uint64_t>(ceil_div(n, 256), 4096);
  hipLaunchKernelGGL(fill_u32_kernel, dim3((unsigned)g), dim3(256), 0, st, p, v, n);
}

void zero2(uint32_t* p, uint64_t n, uint32_t* q, uint64_t m, hipStream_t st) {
  const uint64_t g = std::min<uint64_t>(ceil_div(n + m, 256), 4096);
  hipLaunchKernelGGL(zero2_u32_kernel, dim3((unsigned)g), dim3(256), 0, st, p, n, q, m);
}

// A scan whose total must equal `want` (a corrupt container otherwise).
void scan_u32_check(const uint32_t* in, uint64_t n, uint64_t* out, uint64_t* tsum, uint64_t* total, uint64_t want,
                    DevPlan* P, hipStream_t st) {
  const uint64_t nt = ceil_div(n, 4096);
  hipLaunchKernelGGL(scan_tile_sums, dim3((unsigned)nt), dim3(1024), 0, st, in, n, tsum);
  hipLaunchKernelGGL(scan_tile_offsets_check, dim3(1), dim3(1024), 0, st, tsum, nt, total, want, P);
  hipLaunchKernelGGL(scan_apply, dim3((unsigned)nt), dim3(1024), 0, st, in, n, (const uint64_t*)tsum, out);
}

void scan_u32(const uint32_t* in, uint64_t n, uint64_t* out, uint64_t* tsum, uint64_t* total, hipStream_t st) {
  const uint64_t nt = ceil_div(n, 4096);
  hipLaunchKernelGGL(scan_tile_sums, dim3((unsigned)nt), dim3(1024), 0, st, in, n, tsum);
  hipLaunchKernelGGL(scan_tile_offsets, dim3(1), dim3(1024), 0, st, tsum, nt, total);
  hipLaunchKernelGGL(scan_apply, dim3((unsigned)nt), dim3(1024), 0, st, in, n, (const uint64_t*)tsum, out);
}
// Three scans of n elements each (one launch per phase).
void scan3_u32(const Scan3& S, uint64_t n, hipStream_t st) {
  const uint64_t nt = ceil_div(n, 4096);
  hipLaunchKernelGGL(scan3_tile_sums, dim3((unsigned)nt, 3), dim3(1024), 0, st, S, n);
  hipLaunchKernelGGL(scan3_tile_offsets, dim3(1, 3), dim3(1024), 0, st, S, nt);
  hipLaunchKernelGGL(scan3_apply, dim3((unsigned)nt, 3), dim3(1024), 0, st, S, n);
}

template <typename T>
int enqueue_compress_t(sz_ctx* ctx, const Layout& L, const sz_params* p, const void* d_in, void* d_out, size_t cap,
                       hipStream_t st, bool debug_codes_only) {
  CompWs W;
  const size_t need = carve_comp(L, nullptr, nullptr, debug_codes_only, xchg_reserve(ctx));
  int rc = ensure_arena(ctx, need);
  if (rc) return rc;
  ctx->xres_used = xchg_reserve(ctx);  // (none after a new arena)
  carve_comp(L, (uint8_t*)ctx->arena, &W, debug_codes_only, ctx->xres_used);
  DevPlan* P = ctx->plan;
  const bool adaptive = L.m_req == 0;
  PlanInit I;
  I.m = adaptive ? 16 : (uint32_t)L.m_req;
  I.eb_mode = (uint32_t)L.eb_mode;
  I.eb_abs = p->eb_abs;
  I.eb_rel = p->eb_rel;
  I.dtype = (uint32_t)L.dtype;
  I.cap = cap;
  I.xorc = (uint32_t)L.xorc;
  hipLaunchKernelGGL(plan_init_kernel, dim3(1), dim3(64), 0, st, P, I);
  stage_begin(ctx, ST_RANGE, st);
  if (L.eb_mode != SZ_EB_ABS) {
    // 512 blocks (four loads in flight per thread) reach the copy bandwidth;
    // more would only add same-address atomics at the end
    const uint64_t g = std::min<uint64_t>(ceil_div(L.n, 256 * 16 / sizeof(T)) + 1, 512);
    hipLaunchKernelGGL(minmax_kernel<T>, dim3((unsigned)g), dim3(256), 0, st, (const T*)d_in, (uint64_t)L.n, P);
  }
  hipLaunchKernelGGL(eb_resolve_kernel<T>, dim3(1), dim3(64), 0, st, P, I);
  stage_end(ctx, ST_RANGE, st);
  zero2(W.hist, 65536, W.progress, L.g.ntiles + 1, st);
  SweepArgs a;
  a.g = L.g;
  a.x = d_in;
  a.codes = W.codes;
  a.xo = W.xs;
  a.xchg = W.xchg;
  a.ne = L.ne;
  a.nsp = L.nsp;
  a.uvals = nullptr;
  a.useg = nullptr;
  a.n_unpred = 0;
  a.codes_cap = (uint64_t)L.n + 64;
  a.hist = W.hist;
  a.progress = W.progress;
  a.ticket = W.ticket;
  a.plan = P;
  a.pass2 = 0;
  a.export_all = debug_codes_only ? 1 : 0;
  a.claim = ctx->dbg_claim;
  prepare_xchg(ctx, L, W.xchg, st);
  stage_begin(ctx, ST_SWEEP_C, st);
  int sweep_stage_open = ST_SWEEP_C;
  if (L.wave) {
    WArgs wa = make_wargs(L, d_in, W.codes, W.xs, W.xchg, W.ticket, P);
    wa.export_all = a.export_all;
    wa.claim = ctx->dbg_claim;
    if ((rc = launch_wsweep(L, true, wa, st))) return rc;
    if (!adaptive) {
      // the sweep alone is timed; the histogram has a stage of its own
      stage_end(ctx, ST_SWEEP_C, st);
      stage_begin(ctx, ST_HIST, st);
      sweep_stage_open = ST_HIST;
    }
    launch_hist(L, W.codes, W.hist, W.hpart, P, 0, st);
    if (adaptive) {
      hipLaunchKernelGGL(pick_m_kernel, dim3(1), dim3(1024), 0, st, W.hist, P, (uint64_t)L.n, L.theta);
      fill(W.progress, 0, L.g.ntiles + 1, st);
      wa.pass2 = 1;
      if ((rc = launch_wsweep(L, true, wa, st))) return rc;
      launch_hist(L, W.codes, W.hist, W.hpart, P, 1, st);
    }
  } else {
    if ((rc = launch_sweep(L, true, a, st))) return rc;
    if (adaptive) {
      hipLaunchKernelGGL(pick_m_kernel, dim3(1), dim3(1024), 0, st, W.hist, P, (uint64_t)L.n, L.theta);
      fill(W.progress, 0, L.g.ntiles + 1, st);
      a.pass2 = 1;
      if ((rc = launch_sweep(L, true, a, st))) return rc;
    }
  }
  stage_end(ctx, sweep_stage_open, st);
  if (debug_codes_only) return SZ_OK;
  CodebookArgs cb;
  cb.hist = W.hist;
  cb.len = W.len;
  cb.cw = W.cw;
  cb.gkeys = W.gkeys;
  cb.gw = W.gw;
  cb.gpar = W.gpar;
  cb.ganc = W.ganc;
  cb.gdep = W.gdep;
  cb.plan = P;
  cb.n = (uint64_t)L.n;
  cb.theta = L.theta;
  stage_begin(ctx, ST_CODEBOOK, st);
  hipLaunchKernelGGL(codebook_kernel, dim3(1), dim3(kCbNT), 0, st, cb);
  stage_end(ctx, ST_CODEBOOK, st);
  stage_begin(ctx, ST_ENCODE, st);
  const unsigned nch = (unsigned)std::min<uint64_t>(ceil_div(L.n_chunks, 4), 8192);
  const unsigned cs_lds = 4u * L.chunk * (unsigned)L.cw;
  if (L.cw == 1)
    hipLaunchKernelGGL((chunk_stats_kernel<T, uint8_t>), dim3(nch), dim3(256), cs_lds, st, (const uint8_t*)W.codes,
                       (const T*)d_in, (const uint8_t*)W.len, (uint64_t)L.n, L.chunk, W.cbits, W.cu, W.ctb,
                       (const DevPlan*)P);
  else if (L.m_req != 0 && L.m_req <= 12)
    hipLaunchKernelGGL((chunk_stats_kernel<T, uint16_t>), dim3(nch), dim3(256), cs_lds, st, (const uint16_t*)W.codes,
                       (const T*)d_in, (const uint8_t*)W.len, (uint64_t)L.n, L.chunk, W.cbits, W.cu, W.ctb,
                       (const DevPlan*)P);
  else {
    // alphabets that may outgrow the LDS table: every code length in LDS as
    // a byte (two workgroups per CU, each over many chunks, so that few
    // workgroups load the 64 KiB of lengths)
    const unsigned lds8 = cs_lds + 65536u;
    const unsigned nch8 = (unsigned)std::min<uint64_t>(ceil_div(L.n_chunks, 4), 512);
    (void)hipFuncSetAttribute((const void*)chunk_stats_kernel<T, uint16_t, true>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds8);
    hipLaunchKernelGGL((chunk_stats_kernel<T, uint16_t, true>), dim3(nch8), dim3(256), lds8, st,
                       (const uint16_t*)W.codes, (const T*)d_in, (const uint8_t*)W.len, (uint64_t)L.n, L.chunk,
                       W.cbits, W.cu, W.ctb, (const DevPlan*)P);
  }
  {
    // bit, unpredictable and tail-bit offsets of every chunk
    const Scan3 S{{W.cbits, W.cu, W.ctb}, {W.boff, W.uoff, W.toff}, {W.tsum_b, W.tsum_u, W.tsum_t},
                  {W.tot + 0, W.tot + 1, W.tot + 2}};
    scan3_u32(S, L.n_chunks, st);
  }
  LayoutArgs la;
  la.plan = P;
  la.tot_bits = W.tot + 0;
  la.tot_u = W.tot + 1;
  la.tot_tb = W.tot + 2;
  la.n_chunks = L.n_chunks;
  la.raw_size = kHdr + (uint64_t)L.n * L.ts;
  la.head_bits = 1 + FTr<T>::EXPB;
  la.xorc = (uint32_t)L.xorc;
  hipLaunchKernelGGL(layout_kernel, dim3(1), dim3(64), 0, st, la);
  {
    // zeroed container body, or the raw field when the layout chose raw
    const uint64_t gz = std::min<uint64_t>(ceil_div(cap / 4 + 1, 256), 8192);
    const uint64_t gr = std::min<uint64_t>(ceil_div((uint64_t)L.n * L.ts / 16 + 1, 256), 8192);
    hipLaunchKernelGGL(container_prep_kernel<T>, dim3((unsigned)std::max(gz, gr)), dim3(256), 0, st, (const T*)d_in,
                       (uint8_t*)d_out, (uint64_t)L.n, (const DevPlan*)P);
  }
  const unsigned enc_lds = enc_lds_bytes(L.chunk, (uint32_t)L.cw, (uint32_t)L.ts, L.xorc != 0);
  // One encoder form per call: values of unpredictable-heavy chunks held in
  // registers (f64 always; f32 when the share found on the device asks for
  // it, the other form returning at once) or loaded by each pass (with the
  // code entries still kept in registers for chunks of up to 1024).  The f32
  // register form runs on a grid that fits the GPU at once (its waves loop
  // over the chunks), so that returning costs a single round of workgroups.
  auto launch_enc = [&](auto ct, auto pr, uint32_t by_share, unsigned grid) {
    using CT = std::remove_pointer_t<decltype(ct)>;
    constexpr int PR = decltype(pr)::value;
    (void)hipFuncSetAttribute((const void*)encode_kernel<T, CT, PR>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)enc_lds);
    hipLaunchKernelGGL((encode_kernel<T, CT, PR>), dim3(grid), dim3(kEncNT), enc_lds, st, (const CT*)W.codes,
                       (const T*)d_in, (const uint8_t*)W.len, (const uint32_t*)W.cw, (uint64_t)L.n, L.chunk,
                       (const uint32_t*)W.cbits, (const uint64_t*)W.boff, (const uint64_t*)W.uoff,
                       (const uint64_t*)W.toff, (uint8_t*)d_out, (const DevPlan*)P, by_share);
  };
  auto enc_forms = [&](auto ct) {
    if (L.chunk > 1024) {
      launch_enc(ct, std::integral_constant<int, 0>{}, 0u, nch);
    } else if (sizeof(T) == 8) {
      launch_enc(ct, std::integral_constant<int, 16>{}, 0u, nch);
    } else {
      launch_enc(ct, std::integral_constant<int, -16>{}, 1u, nch);
      launch_enc(ct, std::integral_constant<int, 16>{}, 1u, std::min(nch, 1024u));
    }
  };
  if (L.cw == 1)
    enc_forms((uint8_t*)nullptr);
  else
    enc_forms((uint16_t*)nullptr);
  HeaderArgs h;
  h.out = (uint8_t*)d_out;
  h.len = W.len;
  h.plan = P;
  h.dtype = (uint32_t)L.dtype;
  h.ndim = (uint32_t)L.ndim;
  h.layers = (uint32_t)L.nl;
  h.eb_mode = (uint32_t)L.eb_mode;
  h.m_req = (uint32_t)L.m_req;
  h.chunk = L.chunk;
  for (int d = 0; d < 3; d++) {
    h.dims[d] = L.out_dims[d];
    h.block[d] = L.out_block[d];
  }
  h.eb_abs = p->eb_abs;
  h.eb_rel = p->eb_rel;
  h.n = (uint64_t)L.n;
  h.n_chunks = L.n_chunks;
  hipLaunchKernelGGL(header_kernel, dim3(1), dim3(256), 0, st, h);
  stage_end(ctx, ST_ENCODE, st);
  return hipGetLastError() == hipSuccess ? SZ_OK : SZ_EHIP;
}

int check_align(const void* p) { return ((uintptr_t)p & 15) ? SZ_EINVAL : SZ_OK; }

void fill_stats(const DevPlan& P, const Layout& L, sz_stats* s) {
  std::memset(s, 0, sizeof *s);
  s->n_points = (uint64_t)L.n;
  s->n_unpred = P.n_unpred;
  s->huff_bits = P.huff_bits;
  s->tail_bits = P.tail_bits;
  s->compressed_bytes = P.total;
  s->ebT_bits = P.ebT_bits;
  s->eb_used = P.eb;
  s->hit_rate = L.n ? 1.0 - (double)P.n_unpred / (double)L.n : 0.0;
  s->value_min = L.eb_mode != SZ_EB_ABS ? P.vmin : 0.0;
  s->value_max = L.eb_mode != SZ_EB_ABS ? P.vmax : 0.0;
  s->m_used = P.m;
  s->m_suggested = P.m_suggested;
  s->raw_fallback = P.raw;
  s->n_used_syms = P.n_used;
}

// -------------------------------------------------------------- decompress
void hdr_params(const Hdr& h, sz_params* p) {
  std::memset(p, 0, sizeof *p);
  p->struct_size = sizeof(sz_params);
  p->dtype = h.dtype;
  p->ndim = h.ndim;
  for (uint32_t d = 0; d < h.ndim && d < 3; d++) {
    p->dims[d] = h.dims[d];
    p->block[d] = h.block[d];
  }
  p->layers = h.layers;
  p->quant_bits = h.m_req;
  p->eb_mode = h.eb_mode;
  p->chunk = h.chunk;
  p->eb_abs = h.eb_abs;
  p->eb_rel = h.eb_rel;
  p->unpred_coding = (h.flags >> 1) & 1;
}

struct DecWs {
  uint8_t* codes;
  uint64_t *boff, *tsum_b, *tot;
  DecTables* tabs;
  uint32_t* sorted;
  uint64_t* gkeys;
  uint32_t* segcnt;
  uint64_t *useg, *tsum_s;
  void* uvals;
  uint32_t* rsum;
  uint64_t *roff, *tsum_r;
  uint32_t* progress;
  uint32_t* ticket;
  void* xchg;
  uint32_t* xcz;            // XOR coding: zero codes per chunk
  uint64_t *xuoff, *xroff;  // their scan; the scan of the chunks' record bits
  uint64_t *xts_u, *xts_r;
};

size_t carve_dec(const Layout& L, uint64_t U, uint8_t* base, DecWs* W, size_t reserve = 0) {
  Carve c{base};
  DecWs w;
  w.xchg = c.take<uint8_t>(std::max<uint64_t>(xchg_need(L), reserve));
  const uint64_t ngr = ceil_div(U, 256) + 1;  // unpredictable-value blocks (256 threads, one value each at most)
  w.codes = c.take<uint8_t>((L.n + 64) * L.cw);
  w.boff = c.take<uint64_t>(L.n_chunks * 8);
  w.tsum_b = c.take<uint64_t>((ceil_div(L.n_chunks, 4096) + 1) * 8);
  w.tot = c.take<uint64_t>(4 * 8);
  w.tabs = c.take<DecTables>(sizeof(DecTables));
  w.sorted = c.take<uint32_t>(65536 * 4);
  w.gkeys = c.take<uint64_t>(65536 * 8);
  w.segcnt = c.take<uint32_t>(L.nseg * 4);
  w.useg = c.take<uint64_t>(L.nseg * 8);
  w.tsum_s = c.take<uint64_t>((ceil_div(L.nseg, 4096) + 1) * 8);
  w.uvals = c.take<uint8_t>((U + 1) * L.ts);
  w.rsum = c.take<uint32_t>(ngr * 4);
  w.roff = c.take<uint64_t>(ngr * 8);
  w.tsum_r = c.take<uint64_t>((ceil_div(ngr, 4096) + 1) * 8);
  w.progress = c.take<uint32_t>((L.g.ntiles + 1) * 4);
  w.ticket = w.progress + L.g.ntiles;
  w.xcz = nullptr;
  w.xuoff = w.xroff = w.xts_u = w.xts_r = nullptr;
  if (L.xorc) {
    const uint64_t nt = ceil_div(L.n_chunks, 4096) + 1;
    w.xcz = c.take<uint32_t>(L.n_chunks * 4);
    w.xuoff = c.take<uint64_t>(L.n_chunks * 8);
    w.xroff = c.take<uint64_t>(L.n_chunks * 8);
    w.xts_u = c.take<uint64_t>(nt * 8);
    w.xts_r = c.take<uint64_t>(nt * 8);
  }
  if (W) *W = w;
  return c.off + 256;
}

template <typename T>
__global__ void set_eb_kernel(DevPlan* P, uint64_t ebT_bits) {
  if (threadIdx.x) return;
  const T e = bits_to<T>((typename FTr<T>::U)ebT_bits);
  const T two = e + e;
  const T inv = T(1) / two;
  P->eb = (double)e;
  P->ebT_bits = ebT_bits;
  P->twoeb_bits = (uint64_t)to_bits<T>(two);
  P->inv2eb_bits = (uint64_t)to_bits<T>(inv);
}

template <typename T>
int enqueue_decompress_t(sz_ctx* ctx, const Layout& L, const Hdr& h, const void* d_comp, void* d_out,
                         hipStream_t st) {
  DecWs W;
  const uint64_t U = h.n_unpred;
  int rc = ensure_arena(ctx, carve_dec(L, U, nullptr, nullptr, xchg_reserve(ctx)));
  if (rc) return rc;
  ctx->xres_used = xchg_reserve(ctx);  // (none after a new arena)
  carve_dec(L, U, (uint8_t*)ctx->arena, &W, ctx->xres_used);
  DevPlan* P = ctx->plan;
  PlanInit I = {};
  I.m = h.m;
  hipLaunchKernelGGL(plan_init_kernel, dim3(1), dim3(64), 0, st, P, I);
  // eb, 2eb and 1/(2eb) in the element type from the stored bit pattern
  hipLaunchKernelGGL(set_eb_kernel<T>, dim3(1), dim3(64), 0, st, P, h.ebT_bits);
  const uint8_t* comp = (const uint8_t*)d_comp;
  stage_begin(ctx, ST_DECTAB, st);
  hipLaunchKernelGGL(dectab_kernel, dim3(1), dim3(1024), 0, st, comp, h.off_cb, h.n_used, h.m, W.tabs, W.gkeys,
                     W.sorted, P);
  scan_u32_check((const uint32_t*)(comp + h.off_ch), L.n_chunks, W.boff, W.tsum_b, W.tot + 0, h.huff_bits, P, st);
  zero2(W.segcnt, L.nseg, W.progress, L.g.ntiles + 1, st);
  stage_end(ctx, ST_DECTAB, st);
  stage_begin(ctx, ST_DECODE, st);
  const uint64_t nwords = (h.huff_bits + 31) / 32;
  const unsigned gdec8 = (unsigned)ceil_div(L.n_chunks * DecShape<uint8_t>::LPC, DecShape<uint8_t>::NT);
  const unsigned gdec16 = (unsigned)ceil_div(L.n_chunks * DecShape<uint16_t>::LPC, DecShape<uint16_t>::NT);
  const int64_t X = L.dims3[2], Bx = L.blk3[2];
  const int32_t nbx = L.g.nblk[2];
  if (L.cw == 1)
    hipLaunchKernelGGL(decode_kernel<uint8_t>, dim3(gdec8), dim3(DecShape<uint8_t>::NT), 0, st, comp, h.off_bs, nwords,
                       (uint64_t)L.n, L.chunk, L.n_chunks, (const uint32_t*)(comp + h.off_ch),
                       (const uint64_t*)W.boff, (const DecTables*)W.tabs, (const uint32_t*)W.sorted,
                       (uint8_t*)W.codes, W.segcnt, X, Bx, nbx, P);
  else
    hipLaunchKernelGGL(decode_kernel<uint16_t>, dim3(gdec16), dim3(DecShape<uint16_t>::NT), 0, st, comp, h.off_bs, nwords,
                       (uint64_t)L.n, L.chunk, L.n_chunks, (const uint32_t*)(comp + h.off_ch),
                       (const uint64_t*)W.boff, (const DecTables*)W.tabs, (const uint32_t*)W.sorted,
                       (uint16_t*)W.codes, W.segcnt, X, Bx, nbx, P);
  scan_u32_check(W.segcnt, L.nseg, W.useg, W.tsum_s, W.tot + 1, U, P, st);
  stage_end(ctx, ST_DECODE, st);
  stage_begin(ctx, ST_UNPRED, st);
  if (U && L.xorc) {
    // XOR-coded values: each chunk's first value index and first record bit,
    // then one thread per chunk
    const unsigned gz = (unsigned)std::min<uint64_t>(ceil_div(L.n_chunks, 4), 8192);
    if (L.cw == 1)
      hipLaunchKernelGGL(chunk_zeros_kernel<uint8_t>, dim3(gz), dim3(256), 0, st, (const uint8_t*)W.codes,
                         (uint64_t)L.n, L.chunk, W.xcz, (const DevPlan*)P);
    else
      hipLaunchKernelGGL(chunk_zeros_kernel<uint16_t>, dim3(gz), dim3(256), 0, st, (const uint16_t*)W.codes,
                         (uint64_t)L.n, L.chunk, W.xcz, (const DevPlan*)P);
    scan_u32_check(W.xcz, L.n_chunks, W.xuoff, W.xts_u, W.tot + 2, U, P, st);
    const uint32_t* table = (const uint32_t*)(comp + h.off_hd);
    scan_u32_check(table, L.n_chunks, W.xroff, W.xts_r, W.tot + 3, h.tail_bits, P, st);
    const uint64_t tlw = (h.tail_bits + 31) / 32;
    hipLaunchKernelGGL(unpred_xor_kernel<T>, dim3((unsigned)ceil_div(L.n_chunks, 256)), dim3(256), 0, st, comp,
                       h.off_tl, tlw, table, (const uint64_t*)W.xroff, (const uint32_t*)W.xcz,
                       (const uint64_t*)W.xuoff, L.n_chunks, h.ebT_bits, (T*)W.uvals, P);
  } else if (U) {
    constexpr int HB = 1 + FTr<T>::EXPB;
    const uint32_t upt = unpred_per_thread(U);
    const uint64_t ngr = ceil_div(U, 256ull * upt);
    const uint64_t hdw = (U * HB + 31) / 32, tlw = (h.tail_bits + 31) / 32;
    hipLaunchKernelGGL(unpred_sums_kernel<T>, dim3((unsigned)ngr), dim3(256), 0, st, comp, h.off_hd, hdw, U,
                       h.ebT_bits, upt, W.rsum, (const DevPlan*)P);
    scan_u32(W.rsum, ngr, W.roff, W.tsum_r, W.tot + 2, st);
    hipLaunchKernelGGL(unpred_values_kernel<T>, dim3((unsigned)ngr), dim3(256), 0, st, comp, h.off_hd, hdw,
                       h.off_tl, tlw, U, h.ebT_bits, upt, (const uint64_t*)W.roff, h.tail_bits, (T*)W.uvals, P);
  }
  stage_end(ctx, ST_UNPRED, st);
  stage_begin(ctx, ST_SWEEP_D, st);
  SweepArgs a;
  a.g = L.g;
  a.x = nullptr;
  a.codes = W.codes;
  a.xo = d_out;
  a.xchg = W.xchg;
  a.ne = L.ne;
  a.nsp = L.nsp;
  a.uvals = W.uvals;
  a.useg = W.useg;
  a.n_unpred = U;
  a.codes_cap = (uint64_t)L.n + 64;
  a.hist = nullptr;
  a.progress = W.progress;
  a.ticket = W.ticket;
  a.plan = P;
  a.pass2 = 0;
  a.export_all = 0;
  a.claim = ctx->dbg_claim;
  prepare_xchg(ctx, L, W.xchg, st);
  if (L.wave) {
    WArgs wa = make_wargs(L, nullptr, W.codes, d_out, W.xchg, W.ticket, P);
    wa.claim = ctx->dbg_claim;
    wa.uvals = W.uvals;
    wa.useg = W.useg;
    wa.n_unpred = U;
    rc = launch_wsweep(L, false, wa, st);
  } else {
    rc = launch_sweep(L, false, a, st);
  }
  stage_end(ctx, ST_SWEEP_D, st);
  return rc;
}

__global__ void raw_unpack_kernel(const uint8_t* comp, uint8_t* out, uint64_t bytes) {
  const uint8_t* src = comp + kHdr;
  const uint64_t nv = bytes / 16;
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += (uint64_t)gridDim.x * blockDim.x)
    ((uint4*)out)[i] = ((const uint4*)src)[i];
  for (uint64_t i = nv * 16 + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < bytes;
       i += (uint64_t)gridDim.x * blockDim.x)
    out[i] = src[i];
}




// Header checks of a container (host copy of its first kHdr bytes) against
// its size and the output capacity; fills the header and the layout the
// decompressor uses.
int prepare_decompress(const uint8_t* hdr, size_t comp_size, size_t cap, Hdr& h, Layout& L,
                       bool legacy_sweep = false) {
  int rc = parse_header(hdr, comp_size, h);
  if (rc) return rc;
  if ((rc = check_sections(h))) return rc;
  sz_params p;
  hdr_params(h, &p);
  p.quant_bits = (h.flags & 1) ? 0 : h.m;  // intermediate code width follows the stored m
  const Sched sched = default_sched((int)h.dtype, (int)h.ndim, (int)h.layers, legacy_sweep);
  if (resolve(&p, L, &sched)) return SZ_ECORRUPT;
  for (uint32_t d = 0; d < h.ndim; d++)
    if (h.block[d] != L.out_block[d]) return SZ_ECORRUPT;
  if ((uint64_t)L.n != h.n) return SZ_ECORRUPT;
  const uint64_t bytes = (uint64_t)L.n * L.ts;
  if (cap < bytes) return SZ_ECAPACITY;
  if (h.flags & 1) return SZ_OK;
  if (h.chunk != L.chunk || h.n_chunks != L.n_chunks) return SZ_ECORRUPT;
  if (L.cw == 1 && h.m > 8) return SZ_ECORRUPT;
  return SZ_OK;
}

// Workspace bytes of decompressing a checked container (0 for a raw copy).
size_t dec_footprint(const Layout& L, const Hdr& h) {
  return (h.flags & 1) ? 0 : carve_dec(L, h.n_unpred, nullptr, nullptr);
}

// Enqueue the decompression of a checked container (raw copies included).
int enqueue_decompress_any(sz_ctx* ctx, const Layout& L, const Hdr& h, const void* d_comp, void* d_out,
                           hipStream_t st) {
  if (h.flags & 1) {
    const uint64_t bytes = (uint64_t)L.n * L.ts;
    PlanInit I = {};
    I.m = 1;
    hipLaunchKernelGGL(plan_init_kernel, dim3(1), dim3(64), 0, st, ctx->plan, I);
    const uint64_t g = std::min<uint64_t>(ceil_div(bytes / 16 + 1, 256), 8192);
    hipLaunchKernelGGL(raw_unpack_kernel, dim3((unsigned)g), dim3(256), 0, st, (const uint8_t*)d_comp,
                       (uint8_t*)d_out, bytes);
    return hipGetLastError() == hipSuccess ? SZ_OK : SZ_EHIP;
  }
  return L.dtype == SZ_F32 ? enqueue_decompress_t<float>(ctx, L, h, d_comp, d_out, st)
                           : enqueue_decompress_t<double>(ctx, L, h, d_comp, d_out, st);
}
}  // namespace
}  // namespace szh
