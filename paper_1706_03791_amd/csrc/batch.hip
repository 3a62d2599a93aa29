// Batched form of the compressor: many fields of uneven shape compressed by
// one sequence of batched launches instead of one pipeline per field.
//
// Every stage of the single-field pipeline (value range, bound, sweep,
// histogram, codebook, chunk statistics, scans, layout, encoding, header) is
// launched once for the whole batch: blockIdx.y selects the field's job
// descriptor and blockIdx.x/gridDim.x keep their single-field meaning.  The
// sweep is one persistent launch whose workgroups claim tiles of all fields
// through one ticket, fields laid end to end in ticket order; a tile only
// waits on earlier tiles of its own field, which hold smaller tickets and are
// therefore resident, so the launch cannot deadlock.  The whole sequence is
// captured into a HIP graph and replayed while the buffers stay the same.
//
// The tile schedule (threads per workgroup, hence wave and legacy tile
// shapes) and the ticket order of the fields are chosen by timing the
// candidates on the batch itself; the choice is cached per batch signature.
// A schedule changes launch geometry only: every candidate produces the same
// bytes as the single-field path (checked by the tests).
#include <map>
#include <vector>

#include "runtime.hpp"

using namespace szh;

namespace szh {
namespace {

enum BKind : uint32_t { BK_SINGLE = 0, BK_LEG1 = 1, BK_LEG2 = 2, BK_WAVE3 = 3 };

// Everything the batched stages need for one field.
struct BJob {
  const void* x;
  uint8_t* out;
  uint64_t* d_size;
  int32_t* d_status;
  uint64_t n, n_chunks, ntiles;
  uint32_t chunk, eb_mode, kind, adaptive;
  double theta;
  DevPlan* plan;
  PlanInit init;
  CompWs w;
  CodebookArgs cb;
  LayoutArgs la;
  HeaderArgs hd;
  SweepArgs sa;
  WArgs wa;
};

// ------------------------------------------------------- batched stages
__global__ void b_plan_init(const BJob* J, uint32_t* ticket) {
  const BJob& j = J[blockIdx.y];
  plan_init_kernel_dev(j.plan, j.init);
  if (blockIdx.y == 0 && threadIdx.x == 0) *ticket = 0;
}

template <typename T>
__global__ void __launch_bounds__(256) b_minmax(const BJob* J) {
  const BJob& j = J[blockIdx.y];
  if (j.eb_mode != SZ_EB_ABS) minmax_kernel_dev<T>((const T*)j.x, j.n, j.plan);
}

template <typename T>
__global__ void b_eb_resolve(const BJob* J) {
  const BJob& j = J[blockIdx.y];
  eb_resolve_kernel_dev<T>(j.plan, j.init);
}

// Zero each field's histogram (pass 0 only) and tile progress words.
__global__ void __launch_bounds__(256) b_zero_ws(const BJob* J, uint32_t hist_too) {
  const BJob& j = J[blockIdx.y];
  const uint64_t stride = (uint64_t)gridDim.x * 256;
  const uint64_t i0 = (uint64_t)blockIdx.x * 256 + threadIdx.x;
  if (hist_too)
    for (uint64_t i = i0; i < 65536; i += stride) j.w.hist[i] = 0;
  for (uint64_t i = i0; i < j.ntiles + 1; i += stride) j.w.progress[i] = 0;
}
__global__ void b_reset_ticket(uint32_t* ticket) {
  if (threadIdx.x == 0) *ticket = 0;
}

// The persistent sweep: one workgroup per claimed tile of any field.
template <typename T, typename CT, int NT>
__global__ void __launch_bounds__(NT) b_sweep(const BJob* J, const uint32_t* tstart, uint32_t nf, uint32_t* ticket,
                                              uint32_t pass2) {
  extern __shared__ __align__(16) uint8_t sz_lds[];
  __shared__ uint32_t s_f, s_t;
  if (threadIdx.x == 0) {
    const uint32_t t = atomicAdd(ticket, 1u);
    uint32_t lo = 0, hi = nf;  // last field with tstart <= t
    while (hi - lo > 1) {
      const uint32_t mid = (lo + hi) / 2;
      if (tstart[mid] <= t) lo = mid; else hi = mid;
    }
    s_f = lo;
    s_t = t - tstart[lo];
  }
  __syncthreads();
  const uint32_t f = __builtin_amdgcn_readfirstlane(s_f);
  const int t = (int)__builtin_amdgcn_readfirstlane(s_t);
  const BJob& j = J[f];
  const DevPlan* P = j.plan;
  if (P->status != 0 || (pass2 && !P->rerun)) return;
  constexpr int AZ = WaveShape<T>::AZ;
  if (j.kind == BK_WAVE3)
    wsweep_body<T, CT, true, NT / 64, AZ, false>(j.wa, t, sz_lds, pass2);
  else if (j.kind == BK_LEG2)
    sweep_body<T, CT, 2, 1, true, 1, NT>(j.sa, t, sz_lds);
  else if (j.kind == BK_LEG1)
    sweep_body<T, CT, 1, 1, true, 1, NT>(j.sa, t, sz_lds);
}
template <typename T, typename CT, int NT>
constexpr size_t b_sweep_lds() {
  constexpr size_t a = WSweepLds<T, NT / 64, WaveShape<T>::AZ>::BYTES;
  constexpr size_t b = SweepLds<T, CT, 2, 1, true, 1, NT>::BYTES;
  constexpr size_t c = SweepLds<T, CT, 1, 1, true, 1, NT>::BYTES;
  return a > b ? (a > c ? a : c) : (b > c ? b : c);
}

template <typename CT>
__global__ void __launch_bounds__(1024) b_hist(const BJob* J, uint32_t pass2) {
  const BJob& j = J[blockIdx.y];
  if (j.kind == BK_WAVE3) hist_kernel_dev<CT>((const CT*)j.w.codes, j.n, j.w.hist, j.plan, pass2, nullptr);
}

__global__ void __launch_bounds__(1024) b_pick_m(const BJob* J) {
  const BJob& j = J[blockIdx.y];
  if (j.adaptive) pick_m_kernel_dev(j.w.hist, j.plan, j.n, j.theta);
}

__global__ void __launch_bounds__(kCbNT) b_codebook(const BJob* J) { codebook_kernel_dev(J[blockIdx.y].cb); }

template <typename T, typename CT>
__global__ void __launch_bounds__(256) b_chunk_stats(const BJob* J) {
  const BJob& j = J[blockIdx.y];
  chunk_stats_kernel_dev<T, CT>((const CT*)j.w.codes, (const T*)j.x, j.w.len, j.n, j.chunk, j.w.cbits, j.w.cu,
                                j.w.ctb, j.plan);
}

// The three chunk arrays (Huffman bits, unpredictable counts, tail bits) are
// scanned together: blockIdx.z picks the array.
__device__ __forceinline__ const uint32_t* scan_in(const BJob& j, int z) {
  return z == 0 ? j.w.cbits : (z == 1 ? j.w.cu : j.w.ctb);
}
__device__ __forceinline__ uint64_t* scan_out(const BJob& j, int z) {
  return z == 0 ? j.w.boff : (z == 1 ? j.w.uoff : j.w.toff);
}
__device__ __forceinline__ uint64_t* scan_tsum(const BJob& j, int z) {
  return z == 0 ? j.w.tsum_b : (z == 1 ? j.w.tsum_u : j.w.tsum_t);
}
__global__ void __launch_bounds__(1024) b_scan_tile_sums(const BJob* J) {
  const BJob& j = J[blockIdx.y];
  if (j.plan->status || (uint64_t)blockIdx.x * 4096 >= j.n_chunks) return;
  scan_tile_sums_dev(scan_in(j, blockIdx.z), j.n_chunks, scan_tsum(j, blockIdx.z));
}
__global__ void __launch_bounds__(1024) b_scan_tile_offsets(const BJob* J) {
  const BJob& j = J[blockIdx.y];
  if (j.plan->status) return;
  scan_tile_offsets_dev(scan_tsum(j, blockIdx.z), (j.n_chunks + 4095) / 4096, j.w.tot + blockIdx.z);
}
__global__ void __launch_bounds__(1024) b_scan_apply(const BJob* J) {
  const BJob& j = J[blockIdx.y];
  if (j.plan->status || (uint64_t)blockIdx.x * 4096 >= j.n_chunks) return;
  scan_apply_dev(scan_in(j, blockIdx.z), j.n_chunks, scan_tsum(j, blockIdx.z), scan_out(j, blockIdx.z));
}

__global__ void b_layout(const BJob* J) { layout_kernel_dev(J[blockIdx.y].la); }

__global__ void __launch_bounds__(256) b_zero_container(const BJob* J) {
  const BJob& j = J[blockIdx.y];
  zero_container_kernel_dev((uint32_t*)j.out, j.plan);
}

template <typename T, typename CT>
__global__ void __launch_bounds__(kEncNT) b_encode(const BJob* J) {
  const BJob& j = J[blockIdx.y];
  encode_kernel_dev<T, CT>((const CT*)j.w.codes, (const T*)j.x, j.w.len, j.w.cw, j.n, j.chunk, j.w.cbits, j.w.boff,
                           j.w.uoff, j.w.toff, j.out, j.plan);
}

__global__ void __launch_bounds__(256) b_header(const BJob* J) { header_kernel_dev(J[blockIdx.y].hd); }

template <typename T>
__global__ void __launch_bounds__(256) b_raw_copy(const BJob* J) {
  const BJob& j = J[blockIdx.y];
  raw_copy_kernel_dev<T>((const T*)j.x, j.out, j.n, j.plan);
}

__global__ void b_finish(const BJob* J) {
  const BJob& j = J[blockIdx.y];
  finish_kernel_dev(j.plan, j.d_size, j.d_status);
}

// ------------------------------------------------------------ host side
struct Cand {
  int nt;    // threads per sweep workgroup
  int lpt;   // 1: fields in ticket order longest first; 0: as given
};
// Candidate schedules per element type.
const Cand kCandF32[] = {{512, 1}, {512, 0}, {256, 1}, {256, 0}};
const Cand kCandF64[] = {{256, 1}, {256, 0}, {128, 1}, {128, 0}};
constexpr int kNCand = 4;

struct BPlan {
  int cand = -1;
  Cand c{};
  std::vector<Layout> L;         // per field (caller order)
  std::vector<uint32_t> kind;    // per field
  std::vector<size_t> off;       // workspace offset per field
  std::vector<uint32_t> order;   // ticket order -> field
  std::vector<uint32_t> tstart;  // first ticket of each position in ticket order
  uint32_t tiles = 0;
  size_t arena = 0;
  bool any_adaptive = false, any_single = false;
  unsigned gx_mm = 1, gx_zero = 1, gx_hist = 1, gx_ch = 1, gx_scan = 1, gx_raw = 1, gx_zc = 1;
  size_t lds_sweep = 0, lds_cs = 0, lds_enc = 0;
};

std::mutex g_tune_mu;
std::map<std::vector<uint64_t>, int> g_tune_cache;  // batch signature -> candidate

}  // namespace
}  // namespace szh

struct sz_batch {
  sz_ctx* ctx = nullptr;
  uint32_t n = 0;
  int dtype = 0, cw = 1;
  uint32_t cmax = 0;
  std::vector<sz_params> p;
  std::vector<uint64_t> sig;
  int forced = -1;
  BPlan plan;
  double tune_ms[kNCand] = {};
  void* arena = nullptr;
  size_t arena_size = 0;
  DevPlan* plans = nullptr;  // n device plans
  BJob* d_jobs = nullptr;
  BJob* h_jobs = nullptr;    // pinned staging
  uint32_t* d_tstart = nullptr;
  uint32_t* d_ticket = nullptr;
  hipStream_t gstream = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  hipEvent_t ev_staged = nullptr;  // the last upload of h_jobs has been read
  bool staged_pending = false;
  hipGraphExec_t exec = nullptr;
  std::vector<const void*> key;  // buffers the captured graph was built for
  int key_cand = -1;
};

namespace szh {
namespace {

uint32_t kind_of(const Layout& L) {
  if (L.nl != 1) return BK_SINGLE;
  return L.ndim == 3 ? BK_WAVE3 : (L.ndim == 2 ? BK_LEG2 : BK_LEG1);
}

int build_plan(sz_batch* b, int cand, BPlan& P) {
  const Cand c = b->dtype == SZ_F32 ? kCandF32[cand] : kCandF64[cand];
  P = BPlan();
  P.cand = cand;
  P.c = c;
  const uint32_t n = b->n;
  P.L.resize(n);
  P.kind.resize(n);
  P.off.resize(n);
  std::vector<double> cost(n);
  size_t off = 0;
  for (uint32_t i = 0; i < n; i++) {
    sz_params q = b->p[i];
    Layout tmp;
    int rc = resolve(&q, tmp);
    if (rc) return rc;
    const uint32_t k = kind_of(tmp);
    Layout& L = P.L[i];
    if (k == BK_SINGLE) {
      L = tmp;
    } else {
      Sched s;
      s.wave = k == BK_WAVE3;
      s.rz = 1;
      s.ry = c.nt;
      s.nw = c.nt / 64;
      s.az = wave_az(b->dtype, 3);
      if ((rc = resolve(&q, L, &s))) return rc;
    }
    L.cw = b->cw;  // one code width for the whole batch (bytes do not depend on it)
    P.kind[i] = k;
    P.any_single |= k == BK_SINGLE;
    P.any_adaptive |= L.m_req == 0;
    off = (off + 255) & ~size_t(255);
    P.off[i] = off;
    off += carve_comp(L, nullptr, nullptr);
    // dependence chain of the sweep, in steps: the longest raster path
    cost[i] = (double)(L.dims3[0] + L.dims3[1] + L.dims3[2]) + 1e-9 * (double)L.n;
    const uint64_t ts = (uint64_t)L.ts;
    P.gx_mm = std::max<unsigned>(P.gx_mm, (unsigned)std::min<uint64_t>(ceil_div(L.n, 256 * 16 / ts) + 1, 512));
    P.gx_zero = std::max<unsigned>(P.gx_zero, (unsigned)std::min<uint64_t>(ceil_div(65536 + L.g.ntiles, 256), 512));
    P.gx_hist = std::max<unsigned>(P.gx_hist, (unsigned)std::min<uint64_t>(ceil_div(L.n, 1024 * 16), 1024));
    P.gx_ch = std::max<unsigned>(P.gx_ch, (unsigned)std::min<uint64_t>(ceil_div(L.n_chunks, 4), 8192));
    P.gx_scan = std::max<unsigned>(P.gx_scan, (unsigned)ceil_div(L.n_chunks, 4096));
    P.gx_raw = std::max<unsigned>(P.gx_raw, (unsigned)std::min<uint64_t>(ceil_div(L.n * ts / 16 + 1, 256), 8192));
    P.gx_zc = std::max<unsigned>(P.gx_zc, (unsigned)std::min<uint64_t>(ceil_div((kHdr + L.n * ts) / 4 + 1, 256), 8192));
  }
  P.arena = off + 256;
  P.order.resize(n);
  for (uint32_t i = 0; i < n; i++) P.order[i] = i;
  if (c.lpt)
    std::stable_sort(P.order.begin(), P.order.end(), [&](uint32_t a, uint32_t q) { return cost[a] > cost[q]; });
  P.tstart.resize(n + 1);
  uint32_t t = 0;
  for (uint32_t k = 0; k < n; k++) {
    P.tstart[k] = t;
    const uint32_t f = P.order[k];
    if (P.kind[f] != BK_SINGLE) t += (uint32_t)P.L[f].g.ntiles;
  }
  P.tstart[n] = t;
  P.tiles = t;
  P.lds_cs = 4u * b->cmax * (unsigned)b->cw;
  P.lds_enc = enc_lds_bytes(b->cmax, (uint32_t)b->cw, b->dtype == SZ_F32 ? 4u : 8u, true);
  if (b->dtype == SZ_F32)
    P.lds_sweep = c.nt == 512 ? (b->cw == 1 ? b_sweep_lds<float, uint8_t, 512>() : b_sweep_lds<float, uint16_t, 512>())
                              : (b->cw == 1 ? b_sweep_lds<float, uint8_t, 256>() : b_sweep_lds<float, uint16_t, 256>());
  else
    P.lds_sweep = c.nt == 256 ? (b->cw == 1 ? b_sweep_lds<double, uint8_t, 256>() : b_sweep_lds<double, uint16_t, 256>())
                              : (b->cw == 1 ? b_sweep_lds<double, uint8_t, 128>() : b_sweep_lds<double, uint16_t, 128>());
  return SZ_OK;
}

int ensure_batch_arena(sz_batch* b, size_t bytes) {
  if (bytes <= b->arena_size) return SZ_OK;
  if (b->arena) {
    if (hipDeviceSynchronize() != hipSuccess) return SZ_EHIP;
    (void)hipFree(b->arena);
    b->arena = nullptr;
    b->arena_size = 0;
  }
  if (hipMalloc(&b->arena, bytes) != hipSuccess) {
    b->arena = nullptr;
    return SZ_ENOMEM;
  }
  b->arena_size = bytes;
  return SZ_OK;
}

// Fill the host job array (in ticket order) for the given buffers.
void fill_jobs(sz_batch* b, const BPlan& P, const void* const* d_in, void* const* d_out, const size_t* caps,
               uint64_t* d_sizes, int32_t* d_status) {
  for (uint32_t k = 0; k < b->n; k++) {
    const uint32_t i = P.order[k];
    const Layout& L = P.L[i];
    const sz_params& p = b->p[i];
    BJob& j = b->h_jobs[k];
    std::memset(&j, 0, sizeof j);
    j.x = d_in[i];
    j.out = (uint8_t*)d_out[i];
    j.d_size = d_sizes + i;
    j.d_status = d_status + i;
    j.n = (uint64_t)L.n;
    j.n_chunks = L.n_chunks;
    j.ntiles = (uint64_t)L.g.ntiles;
    j.chunk = L.chunk;
    j.eb_mode = (uint32_t)L.eb_mode;
    j.kind = P.kind[i];
    j.adaptive = L.m_req == 0;
    j.theta = L.theta;
    j.plan = b->plans + i;
    carve_comp(L, (uint8_t*)b->arena + P.off[i], &j.w);
    j.init.m = j.adaptive ? 16 : (uint32_t)L.m_req;
    j.init.eb_mode = (uint32_t)L.eb_mode;
    j.init.eb_abs = p.eb_abs;
    j.init.eb_rel = p.eb_rel;
    j.init.dtype = (uint32_t)L.dtype;
    j.init.cap = caps[i];
    j.init.xorc = (uint32_t)L.xorc;
    CodebookArgs& cb = j.cb;
    cb.hist = j.w.hist;
    cb.len = j.w.len;
    cb.cw = j.w.cw;
    cb.gkeys = j.w.gkeys;
    cb.gw = j.w.gw;
    cb.gpar = j.w.gpar;
    cb.ganc = j.w.ganc;
    cb.gdep = j.w.gdep;
    cb.plan = j.plan;
    cb.n = j.n;
    cb.theta = L.theta;
    LayoutArgs& la = j.la;
    la.plan = j.plan;
    la.tot_bits = j.w.tot + 0;
    la.tot_u = j.w.tot + 1;
    la.tot_tb = j.w.tot + 2;
    la.n_chunks = L.n_chunks;
    la.raw_size = kHdr + (uint64_t)L.n * L.ts;
    la.head_bits = L.dtype == SZ_F32 ? 1 + FTr<float>::EXPB : 1 + FTr<double>::EXPB;
    la.xorc = (uint32_t)L.xorc;
    HeaderArgs& h = j.hd;
    h.out = j.out;
    h.len = j.w.len;
    h.plan = j.plan;
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
    h.eb_abs = p.eb_abs;
    h.eb_rel = p.eb_rel;
    h.n = (uint64_t)L.n;
    h.n_chunks = L.n_chunks;
    SweepArgs& a = j.sa;
    a.g = L.g;
    a.x = d_in[i];
    a.codes = j.w.codes;
    a.xo = nullptr;
    a.xchg = j.w.xchg;
    a.ne = L.ne;
    a.nsp = L.nsp;
    a.uvals = nullptr;
    a.useg = nullptr;
    a.n_unpred = 0;
    a.codes_cap = (uint64_t)L.n + 64;
    a.hist = j.w.hist;
    a.progress = j.w.progress;
    a.ticket = j.w.ticket;
    a.plan = j.plan;
    a.pass2 = 0;
    a.export_all = 0;
    if (L.wave) j.wa = make_wargs(L, d_in[i], j.w.codes, nullptr, j.w.xchg, j.w.ticket, j.plan);
  }
}

// Fill the pinned job array for these buffers and copy it to the device on
// `st`.  The previous copy is waited for first, so a copy still queued never
// reads a job array meant for a later call.
int upload_jobs(sz_batch* b, const BPlan& P, const void* const* d_in, void* const* d_out, const size_t* caps,
                uint64_t* d_sizes, int32_t* d_status, hipStream_t st) {
  if (b->staged_pending && hipEventSynchronize(b->ev_staged) != hipSuccess) return SZ_EHIP;
  fill_jobs(b, P, d_in, d_out, caps, d_sizes, d_status);
  HIPCHK(hipMemcpyAsync(b->d_jobs, b->h_jobs, sizeof(BJob) * b->n, hipMemcpyHostToDevice, st));
  HIPCHK(hipEventRecord(b->ev_staged, st));
  b->staged_pending = true;
  return SZ_OK;
}

template <typename T, typename CT, int NT>
void launch_b_sweep(const sz_batch* b, const BPlan& P, uint32_t pass2, hipStream_t st) {
  auto k = b_sweep<T, CT, NT>;
  hipLaunchKernelGGL(k, dim3(P.tiles), dim3(NT), P.lds_sweep, st, (const BJob*)b->d_jobs, (const uint32_t*)b->d_tstart,
                     b->n, b->d_ticket, pass2);
}
template <typename T, typename CT>
void set_b_sweep_attr(const BPlan& P) {
  if (P.c.nt == (sizeof(T) == 4 ? 512 : 256))
    (void)hipFuncSetAttribute((const void*)b_sweep<T, CT, (sizeof(T) == 4 ? 512 : 256)>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)P.lds_sweep);
  else
    (void)hipFuncSetAttribute((const void*)b_sweep<T, CT, (sizeof(T) == 4 ? 256 : 128)>,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)P.lds_sweep);
}
template <typename T, typename CT>
void sweep_all(const sz_batch* b, const BPlan& P, uint32_t pass2, hipStream_t st) {
  if (P.tiles) {
    if (P.c.nt == (sizeof(T) == 4 ? 512 : 256))
      launch_b_sweep<T, CT, (sizeof(T) == 4 ? 512 : 256)>(b, P, pass2, st);
    else
      launch_b_sweep<T, CT, (sizeof(T) == 4 ? 256 : 128)>(b, P, pass2, st);
  }
  if (P.any_single) {
    // fields outside the persistent kernel (more than one layer) keep their
    // own launches, on the same stream
    for (uint32_t k = 0; k < b->n; k++) {
      const uint32_t i = P.order[k];
      if (P.kind[i] != BK_SINGLE) continue;
      SweepArgs a = b->h_jobs[k].sa;
      a.pass2 = pass2;
      (void)launch_sweep(P.L[i], true, a, st);
    }
  }
}

// The whole batched compression, enqueued on `st` (no host synchronisation).
template <typename T, typename CT>
void enqueue_batch(sz_batch* b, const BPlan& P, hipStream_t st) {
  const uint32_t n = b->n;
  const BJob* J = b->d_jobs;
  hipLaunchKernelGGL(b_plan_init, dim3(1, n), dim3(64), 0, st, J, b->d_ticket);
  hipLaunchKernelGGL(b_minmax<T>, dim3(P.gx_mm, n), dim3(256), 0, st, J);
  hipLaunchKernelGGL(b_eb_resolve<T>, dim3(1, n), dim3(64), 0, st, J);
  hipLaunchKernelGGL(b_zero_ws, dim3(P.gx_zero, n), dim3(256), 0, st, J, 1u);
  sweep_all<T, CT>(b, P, 0, st);
  hipLaunchKernelGGL(b_hist<CT>, dim3(P.gx_hist, n), dim3(1024), 0, st, J, 0u);
  if (P.any_adaptive) {
    hipLaunchKernelGGL(b_pick_m, dim3(1, n), dim3(1024), 0, st, J);
    hipLaunchKernelGGL(b_zero_ws, dim3(P.gx_zero, n), dim3(256), 0, st, J, 0u);
    hipLaunchKernelGGL(b_reset_ticket, dim3(1), dim3(64), 0, st, b->d_ticket);
    sweep_all<T, CT>(b, P, 1, st);
    hipLaunchKernelGGL(b_hist<CT>, dim3(P.gx_hist, n), dim3(1024), 0, st, J, 1u);
  }
  hipLaunchKernelGGL(b_codebook, dim3(1, n), dim3(kCbNT), 0, st, J);
  hipLaunchKernelGGL((b_chunk_stats<T, CT>), dim3(P.gx_ch, n), dim3(256), P.lds_cs, st, J);
  hipLaunchKernelGGL(b_scan_tile_sums, dim3(P.gx_scan, n, 3), dim3(1024), 0, st, J);
  hipLaunchKernelGGL(b_scan_tile_offsets, dim3(1, n, 3), dim3(1024), 0, st, J);
  hipLaunchKernelGGL(b_scan_apply, dim3(P.gx_scan, n, 3), dim3(1024), 0, st, J);
  hipLaunchKernelGGL(b_layout, dim3(1, n), dim3(64), 0, st, J);
  hipLaunchKernelGGL(b_zero_container, dim3(P.gx_zc, n), dim3(256), 0, st, J);
  hipLaunchKernelGGL((b_encode<T, CT>), dim3(P.gx_ch, n), dim3(kEncNT), P.lds_enc, st, J);
  hipLaunchKernelGGL(b_header, dim3(1, n), dim3(256), 0, st, J);
  hipLaunchKernelGGL(b_raw_copy<T>, dim3(P.gx_raw, n), dim3(256), 0, st, J);
  hipLaunchKernelGGL(b_finish, dim3(1, n), dim3(64), 0, st, J);
}

template <typename T, typename CT>
void set_attrs(const BPlan& P) {
  set_b_sweep_attr<T, CT>(P);
  (void)hipFuncSetAttribute((const void*)b_encode<T, CT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)P.lds_enc);
  (void)hipFuncSetAttribute((const void*)b_chunk_stats<T, CT>, hipFuncAttributeMaxDynamicSharedMemorySize,
                            (int)P.lds_cs);
}

void dispatch_enqueue(sz_batch* b, const BPlan& P, hipStream_t st) {
  if (b->dtype == SZ_F32) {
    if (b->cw == 1) enqueue_batch<float, uint8_t>(b, P, st);
    else enqueue_batch<float, uint16_t>(b, P, st);
  } else {
    if (b->cw == 1) enqueue_batch<double, uint8_t>(b, P, st);
    else enqueue_batch<double, uint16_t>(b, P, st);
  }
}
void dispatch_attrs(const sz_batch* b, const BPlan& P) {
  if (b->dtype == SZ_F32) {
    if (b->cw == 1) set_attrs<float, uint8_t>(P);
    else set_attrs<float, uint16_t>(P);
  } else {
    if (b->cw == 1) set_attrs<double, uint8_t>(P);
    else set_attrs<double, uint16_t>(P);
  }
}

// Make plan `cand` current: workspace, tile table, launch attributes.
int activate(sz_batch* b, int cand) {
  if (b->plan.cand == cand) return SZ_OK;
  BPlan P;
  int rc = build_plan(b, cand, P);
  if (rc) return rc;
  if (hipDeviceSynchronize() != hipSuccess) return SZ_EHIP;
  if ((rc = ensure_batch_arena(b, P.arena))) return rc;
  // The wave sweep tells the exchange records of a launch by their tag: a new
  // layout starts from an arena holding none of anything else.
  if (hipMemset(b->arena, 0, P.arena) != hipSuccess) return SZ_EHIP;
  if (b->d_tstart) (void)hipFree(b->d_tstart);
  b->d_tstart = nullptr;
  if (hipMalloc(&b->d_tstart, sizeof(uint32_t) * (b->n + 1)) != hipSuccess) return SZ_ENOMEM;
  if (hipMemcpy(b->d_tstart, P.tstart.data(), sizeof(uint32_t) * (b->n + 1), hipMemcpyHostToDevice) != hipSuccess)
    return SZ_EHIP;
  dispatch_attrs(b, P);
  b->plan = std::move(P);
  return SZ_OK;
}

// Time every candidate on the batch's own buffers and keep the fastest.
int autotune(sz_batch* b, const void* const* d_in, void* const* d_out, const size_t* caps, uint64_t* d_sizes,
             int32_t* d_status, hipStream_t st) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return SZ_EHIP;
  int best = 0;
  double best_ms = 1e300;
  for (int c = 0; c < kNCand; c++) {
    int rc = activate(b, c);
    if (rc) return rc;
    if ((rc = upload_jobs(b, b->plan, d_in, d_out, caps, d_sizes, d_status, st))) return rc;
    dispatch_enqueue(b, b->plan, st);  // warm-up
    (void)hipEventRecord(e0, st);
    for (int r = 0; r < 2; r++) dispatch_enqueue(b, b->plan, st);
    (void)hipEventRecord(e1, st);
    if (hipEventSynchronize(e1) != hipSuccess) return SZ_EHIP;
    float ms = 0;
    (void)hipEventElapsedTime(&ms, e0, e1);
    b->tune_ms[c] = ms / 2;
    if (ms / 2 < best_ms) {
      best_ms = ms / 2;
      best = c;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune_cache[b->sig] = best;
  }
  return activate(b, best);
}

}  // namespace
}  // namespace szh

// =================================================================== C ABI
extern "C" {

int sz_batch_create(sz_ctx* ctx, uint32_t n, const sz_params* params, int schedule, sz_batch** out) {
  if (!ctx || !params || !out || n == 0 || n > 65535 || schedule >= kNCand) return SZ_EINVAL;
  *out = nullptr;
  if (hipSetDevice(ctx->device) != hipSuccess) return SZ_EHIP;
  sz_batch* b = new sz_batch();
  b->ctx = ctx;
  b->n = n;
  b->p.assign(params, params + n);
  b->dtype = (int)params[0].dtype;
  b->cw = 1;
  b->forced = schedule;
  b->sig.push_back(n);
  for (uint32_t i = 0; i < n; i++) {
    Layout L;
    int rc = resolve(&params[i], L);
    if (rc || (int)params[i].dtype != b->dtype) {
      delete b;
      return rc ? rc : SZ_EINVAL;
    }
    if (L.cw == 2) b->cw = 2;
    b->cmax = std::max(b->cmax, L.chunk);
    b->sig.push_back(((uint64_t)L.dtype << 60) | ((uint64_t)L.ndim << 56) | ((uint64_t)L.nl << 52) |
                     ((uint64_t)L.m_req << 44));
    for (int d = 0; d < 3; d++) b->sig.push_back(((uint64_t)L.dims3[d] << 32) | (uint64_t)L.blk3[d]);
  }
  bool ok = hipMalloc(&b->plans, sizeof(DevPlan) * n) == hipSuccess &&
            hipMalloc(&b->d_jobs, sizeof(BJob) * n) == hipSuccess &&
            hipMalloc(&b->d_ticket, 256) == hipSuccess &&
            hipHostMalloc(&b->h_jobs, sizeof(BJob) * n, hipHostMallocDefault) == hipSuccess &&
            hipStreamCreateWithFlags(&b->gstream, hipStreamNonBlocking) == hipSuccess &&
            hipEventCreateWithFlags(&b->ev_in, hipEventDisableTiming) == hipSuccess &&
            hipEventCreateWithFlags(&b->ev_out, hipEventDisableTiming) == hipSuccess &&
            hipEventCreateWithFlags(&b->ev_staged, hipEventDisableTiming) == hipSuccess;
  if (!ok) {
    sz_batch_destroy(b);
    return SZ_ENOMEM;
  }
  int cand = schedule;
  if (cand < 0) {
    std::lock_guard<std::mutex> g(g_tune_mu);
    auto it = g_tune_cache.find(b->sig);
    if (it != g_tune_cache.end()) cand = it->second;
  }
  if (cand >= 0) {
    int rc = activate(b, cand);
    if (rc) {
      sz_batch_destroy(b);
      return rc;
    }
  }
  *out = b;
  return SZ_OK;
}

void sz_batch_destroy(sz_batch* b) {
  if (!b) return;
  (void)hipSetDevice(b->ctx->device);
  (void)hipDeviceSynchronize();
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->arena) (void)hipFree(b->arena);
  if (b->plans) (void)hipFree(b->plans);
  if (b->d_jobs) (void)hipFree(b->d_jobs);
  if (b->d_ticket) (void)hipFree(b->d_ticket);
  if (b->d_tstart) (void)hipFree(b->d_tstart);
  if (b->h_jobs) (void)hipHostFree(b->h_jobs);
  if (b->ev_in) (void)hipEventDestroy(b->ev_in);
  if (b->ev_out) (void)hipEventDestroy(b->ev_out);
  if (b->ev_staged) (void)hipEventDestroy(b->ev_staged);
  if (b->gstream) (void)hipStreamDestroy(b->gstream);
  delete b;
}

int sz_batch_compress(sz_batch* b, const void* const* d_in, void* const* d_out, const size_t* caps,
                      uint64_t* d_sizes, int32_t* d_status, int use_graph, void* stream) {
  if (!b || !d_in || !d_out || !caps || !d_sizes || !d_status) return SZ_EINVAL;
  for (uint32_t i = 0; i < b->n; i++) {
    if (!d_in[i] || !d_out[i] || ((uintptr_t)d_in[i] & 15) || ((uintptr_t)d_out[i] & 15)) return SZ_EINVAL;
    if (caps[i] < kHdr) return SZ_ECAPACITY;
  }
  hipStream_t st = (hipStream_t)stream;
  if (hipSetDevice(b->ctx->device) != hipSuccess) return SZ_EHIP;
  int rc;
  if (b->plan.cand < 0 && (rc = autotune(b, d_in, d_out, caps, d_sizes, d_status, st))) return rc;
  const BPlan& P = b->plan;
  if (!use_graph) {
    if ((rc = upload_jobs(b, P, d_in, d_out, caps, d_sizes, d_status, st))) return rc;
    dispatch_enqueue(b, P, st);
    return hipGetLastError() == hipSuccess ? SZ_OK : SZ_EHIP;
  }
  // Graph mode: the captured sequence is reused while the buffers are the
  // same; it runs on the batch's own stream, ordered after and before `st`.
  std::vector<const void*> key;
  key.reserve(3 * b->n + 2);
  for (uint32_t i = 0; i < b->n; i++) {
    key.push_back(d_in[i]);
    key.push_back(d_out[i]);
    key.push_back((const void*)(uintptr_t)caps[i]);
  }
  key.push_back(d_sizes);
  key.push_back(d_status);
  if (!b->exec || key != b->key || b->key_cand != P.cand) {
    if (b->exec) {
      (void)hipStreamSynchronize(b->gstream);
      (void)hipGraphExecDestroy(b->exec);
      b->exec = nullptr;
    }
    (void)hipStreamSynchronize(b->gstream);
    fill_jobs(b, P, d_in, d_out, caps, d_sizes, d_status);  // host copies of the sweep arguments
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamBeginCapture(b->gstream, hipStreamCaptureModeThreadLocal));
    dispatch_enqueue(b, P, b->gstream);
    HIPCHK(hipStreamEndCapture(b->gstream, &g));
    const hipError_t e = hipGraphInstantiate(&b->exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      b->exec = nullptr;
      return SZ_EHIP;
    }
    b->key = key;
    b->key_cand = P.cand;
  }
  HIPCHK(hipEventRecord(b->ev_in, st));
  HIPCHK(hipStreamWaitEvent(b->gstream, b->ev_in, 0));
  if ((rc = upload_jobs(b, P, d_in, d_out, caps, d_sizes, d_status, b->gstream))) return rc;
  HIPCHK(hipGraphLaunch(b->exec, b->gstream));
  HIPCHK(hipEventRecord(b->ev_out, b->gstream));
  HIPCHK(hipStreamWaitEvent(st, b->ev_out, 0));
  return SZ_OK;
}

int sz_batch_info(const sz_batch* b, int* schedule, uint32_t* tiles, int* threads, double* tune_ms, int n_ms) {
  if (!b) return SZ_EINVAL;
  if (schedule) *schedule = b->plan.cand;
  if (tiles) *tiles = b->plan.tiles;
  if (threads) *threads = b->plan.cand >= 0 ? b->plan.c.nt : 0;
  for (int i = 0; tune_ms && i < n_ms && i < kNCand; i++) tune_ms[i] = b->tune_ms[i];
  return kNCand;
}

}  // extern "C"
