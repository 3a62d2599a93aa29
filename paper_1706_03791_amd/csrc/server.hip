// Served form of the compressor: a request loop with continuous batching
// (not a method of the paper: a serving form of the same per-field work).
//
// Clients submit compress and decompress requests of any size from any host
// thread; a native scheduler thread admits them as execution slots and HBM
// free up and runs every admitted request on its slot's stream, so requests
// that arrive while others are on the GPU overlap with them on the device.
// Workspaces (codes, exchange rows, histograms, code tables, scan arrays)
// are carved from one device pool allocated at start-up, whose size is the
// HBM budget, and nothing is allocated while serving.  Admission is by HBM
// footprint: a request's input, its output capacity and its workspace all
// count against the budget while it is in flight (the client owns the first
// two, the pool holds the third).  Requests are admitted in arrival order; a request that does
// not fit in the free pool lets later, smaller requests pass for a bounded
// time (then admission waits for it).  Each result is the same as that of a
// single sz_compress / sz_decompress call: a request runs the same kernel
// sequence on its own workspace, whatever else is in flight.
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <thread>
#include <unordered_map>
#include <vector>

#include "runtime.hpp"

using namespace szh;

namespace szh {
namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// First-fit allocator over [0, size) with coalescing of free blocks.
struct Pool {
  size_t size = 0;
  std::map<size_t, size_t> free_;  // offset -> length
  size_t used = 0, peak = 0;
  void init(size_t n) {
    size = n;
    free_.clear();
    free_[0] = n;
  }
  static constexpr size_t kNone = ~size_t(0);
  size_t alloc(size_t n) {
    n = (n + 255) & ~size_t(255);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < n) continue;
      const size_t off = it->first, len = it->second;
      free_.erase(it);
      if (len > n) free_[off + n] = len - n;
      used += n;
      peak = std::max(peak, used);
      return off;
    }
    return kNone;
  }
  void release(size_t off, size_t n) {
    n = (n + 255) & ~size_t(255);
    used -= n;
    auto it = free_.emplace(off, n).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }
};

struct Req {
  uint64_t id = 0;
  sz_request r{};
  double t_submit = 0, t_admit = 0, t_done = 0;
  int32_t status = 0;
  uint64_t out_size = 0;
  int state = 0;  // 0 pending, 1 running, 2 done
  bool prepared = false;
  Layout L{};
  Hdr h{};
  size_t fp = 0, off = 0;
  size_t fp_total = 0;  // fp + input bytes + output capacity
  int slot = -1;
};

struct Slot {
  sz_ctx ctx;  // plan, pinned mirrors; arena points into the pool while busy
  hipStream_t st = nullptr;
  hipEvent_t done = nullptr;
  Req* req = nullptr;
};

}  // namespace
}  // namespace szh

struct sz_server {
  int device = 0;
  size_t budget = 0;
  void* pool_mem = nullptr;
  Pool pool;
  std::vector<Slot> slots;
  hipStream_t ctl = nullptr;  // header reads
  uint8_t* h_hdr = nullptr;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<Req*> submitted;
  std::deque<Req*> pending;  // scheduler thread only
  std::unordered_map<uint64_t, Req*> reqs;
  uint64_t next_id = 1;
  bool stop = false;
  std::thread th;
  // statistics
  uint64_t n_done = 0, n_admitted = 0;
  uint32_t max_inflight = 0, inflight = 0;
  size_t pool_peak = 0;
  size_t accounted = 0;  // fp_total of the requests in flight
  double backfill_s = 0.05;
};

namespace szh {
namespace {

// Validate a request and compute its workspace footprint (scheduler thread).
int prepare(sz_server* s, Req* q) {
  const sz_request& r = q->r;
  if (r.op == SZ_REQ_COMPRESS) {
    if (!r.d_in || !r.d_out || check_align(r.d_in) || check_align(r.d_out)) return SZ_EINVAL;
    int rc = resolve(&r.params, q->L);
    if (rc) return rc;
    q->fp = carve_comp(q->L, nullptr, nullptr);
    q->fp_total = q->fp + (size_t)q->L.n * q->L.ts + r.out_cap;
    return SZ_OK;
  }
  if (r.op != SZ_REQ_DECOMPRESS) return SZ_EINVAL;
  if (!r.d_in || !r.d_out || check_align(r.d_in) || check_align(r.d_out)) return SZ_EINVAL;
  if (r.in_bytes < kHdr) return SZ_ECORRUPT;
  const uint8_t* hdr = (const uint8_t*)r.h_header;
  if (!hdr) {
    HIPCHK(hipMemcpyAsync(s->h_hdr, r.d_in, kHdr, hipMemcpyDeviceToHost, s->ctl));
    HIPCHK(hipStreamSynchronize(s->ctl));
    hdr = s->h_hdr;
  }
  int rc = prepare_decompress(hdr, r.in_bytes, r.out_cap, q->h, q->L);
  if (rc) return rc;
  q->fp = dec_footprint(q->L, q->h);
  q->fp_total = q->fp + r.in_bytes + r.out_cap;
  return SZ_OK;
}

void finish(sz_server* s, Req* q, int32_t status, uint64_t size) {
  std::lock_guard<std::mutex> g(s->mu);
  q->status = status;
  q->out_size = status ? 0 : size;
  q->t_done = now_s();
  q->state = 2;
  s->n_done++;
  s->cv_done.notify_all();
}

int launch(sz_server* s, Slot& sl, Req* q) {
  sz_ctx& c = sl.ctx;
  c.arena = (uint8_t*)s->pool_mem + q->off;
  c.arena_size = q->fp ? q->fp : 0;
  c.fixed_arena = true;  // the carve from the pool is all this request may use
  const sz_request& r = q->r;
  int rc;
  if (r.op == SZ_REQ_COMPRESS)
    rc = q->L.dtype == SZ_F32
             ? enqueue_compress_t<float>(&c, q->L, &r.params, r.d_in, r.d_out, r.out_cap, sl.st, false)
             : enqueue_compress_t<double>(&c, q->L, &r.params, r.d_in, r.d_out, r.out_cap, sl.st, false);
  else
    rc = enqueue_decompress_any(&c, q->L, q->h, r.d_in, r.d_out, sl.st);
  if (rc) return rc;
  HIPCHK(hipMemcpyAsync(c.h_plan, c.plan, sizeof(DevPlan), hipMemcpyDeviceToHost, sl.st));
  HIPCHK(hipEventRecord(sl.done, sl.st));
  return SZ_OK;
}

void scheduler(sz_server* s) {
  (void)hipSetDevice(s->device);
  for (;;) {
    bool progress = false;
    {
      std::unique_lock<std::mutex> g(s->mu);
      while (!s->submitted.empty()) {
        s->pending.push_back(s->submitted.front());
        s->submitted.pop_front();
      }
      if (s->stop && s->pending.empty() && s->inflight == 0) break;
    }
    // completions
    for (Slot& sl : s->slots) {
      if (!sl.req || hipEventQuery(sl.done) != hipSuccess) continue;
      Req* q = sl.req;
      const DevPlan& P = *sl.ctx.h_plan;
      const uint64_t size = q->r.op == SZ_REQ_COMPRESS ? P.total : (uint64_t)q->L.n * q->L.ts;
      if (q->fp) s->pool.release(q->off, q->fp);
      s->accounted -= q->fp_total;
      sl.req = nullptr;
      sl.ctx.arena = nullptr;
      sl.ctx.arena_size = 0;
      {
        std::lock_guard<std::mutex> g(s->mu);
        s->inflight--;
      }
      finish(s, q, P.status, size);
      progress = true;
    }
    // admissions, in arrival order; a request that does not fit lets later
    // ones pass until it has waited backfill_s
    const double t = now_s();
    bool head_blocked = false;
    for (auto it = s->pending.begin(); it != s->pending.end();) {
      int free_slot = -1;
      for (size_t k = 0; k < s->slots.size(); k++)
        if (!s->slots[k].req) {
          free_slot = (int)k;
          break;
        }
      if (free_slot < 0) break;
      Req* q = *it;
      if (!q->prepared) {
        const int rc = prepare(s, q);
        q->prepared = true;
        if (!rc && q->fp_total > s->budget) {
          it = s->pending.erase(it);
          finish(s, q, SZ_ENOMEM, 0);
          progress = true;
          continue;
        }
        if (rc) {
          it = s->pending.erase(it);
          finish(s, q, rc, 0);
          progress = true;
          continue;
        }
      }
      if (head_blocked) {
        // behind a blocked request: only while it has not waited too long
        if (t - s->pending.front()->t_submit > s->backfill_s) break;
      }
      const bool fits = s->accounted + q->fp_total <= s->budget;
      const size_t off = !fits ? Pool::kNone : (q->fp ? s->pool.alloc(q->fp) : 0);
      if (off == Pool::kNone) {
        head_blocked = true;
        ++it;
        continue;
      }
      q->off = off;
      s->accounted += q->fp_total;
      {
        std::lock_guard<std::mutex> g(s->mu);
        s->pool_peak = std::max(s->pool_peak, s->accounted);
      }
      Slot& sl = s->slots[(size_t)free_slot];
      sl.req = q;
      q->slot = free_slot;
      q->t_admit = now_s();
      q->state = 1;
      const int rc = launch(s, sl, q);
      {
        std::lock_guard<std::mutex> g(s->mu);
        s->inflight++;
        s->n_admitted++;
        s->max_inflight = std::max(s->max_inflight, s->inflight);
      }
      if (rc) {
        // nothing usable was enqueued: release at once
        (void)hipStreamSynchronize(sl.st);
        if (q->fp) s->pool.release(q->off, q->fp);
        s->accounted -= q->fp_total;
        sl.req = nullptr;
        {
          std::lock_guard<std::mutex> g(s->mu);
          s->inflight--;
        }
        finish(s, q, rc, 0);
      }
      it = s->pending.erase(it);
      progress = true;
    }
    if (!progress) {
      std::unique_lock<std::mutex> g(s->mu);
      if (s->submitted.empty() && !(s->stop && s->pending.empty() && s->inflight == 0))
        s->cv_work.wait_for(g, std::chrono::microseconds(s->inflight ? 20 : 2000));
    }
  }
}

}  // namespace
}  // namespace szh

// =================================================================== C ABI
extern "C" {

int sz_server_create(int device, size_t hbm_budget, uint32_t slots, sz_server** out) {
  if (!out || slots == 0 || slots > 64 || hbm_budget < (1u << 20)) return SZ_EINVAL;
  *out = nullptr;
  if (hipSetDevice(device) != hipSuccess) return SZ_EHIP;
  sz_server* s = new sz_server();
  s->device = device;
  s->budget = hbm_budget;
  bool ok = hipMalloc(&s->pool_mem, hbm_budget) == hipSuccess &&
            hipStreamCreateWithFlags(&s->ctl, hipStreamNonBlocking) == hipSuccess &&
            hipHostMalloc(&s->h_hdr, kHdr, hipHostMallocDefault) == hipSuccess;
  s->slots.resize(slots);
  for (Slot& sl : s->slots) {
    sl.ctx.device = device;
    ok = ok && hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking) == hipSuccess &&
         hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) == hipSuccess &&
         hipMalloc(&sl.ctx.plan, sizeof(DevPlan)) == hipSuccess &&
         hipHostMalloc(&sl.ctx.h_plan, sizeof(DevPlan), hipHostMallocDefault) == hipSuccess &&
         hipHostMalloc(&sl.ctx.h_hdr, kHdr, hipHostMallocDefault) == hipSuccess;
  }
  if (!ok) {
    sz_server_destroy(s);
    return SZ_ENOMEM;
  }
  s->pool.init(hbm_budget);
  s->th = std::thread(scheduler, s);
  *out = s;
  return SZ_OK;
}

int sz_server_submit(sz_server* s, const sz_request* r, uint64_t* id) {
  if (!s || !r || !id) return SZ_EINVAL;
  Req* q = new Req();
  q->r = *r;
  q->t_submit = now_s();
  {
    std::lock_guard<std::mutex> g(s->mu);
    if (s->stop) {
      delete q;
      return SZ_EINVAL;
    }
    q->id = s->next_id++;
    s->reqs[q->id] = q;
    s->submitted.push_back(q);
  }
  s->cv_work.notify_one();
  *id = q->id;
  return SZ_OK;
}

int sz_server_wait(sz_server* s, uint64_t id, sz_result* res, int timeout_ms) {
  if (!s) return SZ_EINVAL;
  std::unique_lock<std::mutex> g(s->mu);
  auto it = s->reqs.find(id);
  if (it == s->reqs.end()) return SZ_EINVAL;
  Req* q = it->second;
  auto pred = [&] { return q->state == 2; };
  if (timeout_ms < 0)
    s->cv_done.wait(g, pred);
  else if (!s->cv_done.wait_for(g, std::chrono::milliseconds(timeout_ms), pred))
    return SZ_ETIMEDOUT;
  if (res) {
    res->status = q->status;
    res->slot = (uint32_t)q->slot;
    res->out_size = q->out_size;
    res->workspace_bytes = q->fp;
    res->t_submit = q->t_submit;
    res->t_admit = q->t_admit;
    res->t_done = q->t_done;
  }
  s->reqs.erase(it);
  delete q;
  return SZ_OK;
}

int sz_server_stats(sz_server* s, sz_server_stats_t* out) {
  if (!s || !out) return SZ_EINVAL;
  std::lock_guard<std::mutex> g(s->mu);
  out->submitted = s->next_id - 1;
  out->admitted = s->n_admitted;
  out->completed = s->n_done;
  out->in_flight = s->inflight;
  out->max_in_flight = s->max_inflight;
  out->pool_bytes = s->budget;
  out->pool_peak_bytes = s->pool_peak;
  out->clock_s = now_s();
  return SZ_OK;
}

void sz_server_destroy(sz_server* s) {
  if (!s) return;
  if (s->th.joinable()) {
    {
      std::lock_guard<std::mutex> g(s->mu);
      s->stop = true;
    }
    s->cv_work.notify_all();
    s->th.join();
  }
  (void)hipSetDevice(s->device);
  for (Slot& sl : s->slots) {
    if (sl.st) (void)hipStreamSynchronize(sl.st);
    if (sl.st) (void)hipStreamDestroy(sl.st);
    if (sl.done) (void)hipEventDestroy(sl.done);
    if (sl.ctx.plan) (void)hipFree(sl.ctx.plan);
    if (sl.ctx.h_plan) (void)hipHostFree(sl.ctx.h_plan);
    if (sl.ctx.h_hdr) (void)hipHostFree(sl.ctx.h_hdr);
    sl.ctx.plan = nullptr;
    sl.ctx.h_plan = nullptr;
    sl.ctx.h_hdr = nullptr;
  }
  if (s->ctl) (void)hipStreamDestroy(s->ctl);
  if (s->h_hdr) (void)hipHostFree(s->h_hdr);
  if (s->pool_mem) (void)hipFree(s->pool_mem);
  for (auto& kv : s->reqs) delete kv.second;
  delete s;
}

}  // extern "C"
