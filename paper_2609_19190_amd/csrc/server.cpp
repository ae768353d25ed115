// Served spatial mapping (C ABI fr_server_*): a continuous-batching request
// loop for map jobs that arrive over time.
//
// One device arena of a fixed HBM budget is allocated at creation; every
// admitted job takes one block of it holding its own copies of the raw
// volume and mask, its level volume and mask-voxel list, its staging rows,
// its map-major output and its small tables (the job's footprint).  A worker
// thread admits queued jobs in arrival order as soon as a block of the
// job's footprint and one of the execution slots (HIP streams) are free,
// enqueues the job's whole pipeline on that slot's stream (copies,
// discretisation, map kernel, transpose, status read-back, event) without a
// host synchronisation, and retires jobs whose event has completed.  Jobs
// in flight on different slots overlap on the device: their map kernels are
// launched with one workgroup per work item, so the dispatcher interleaves
// the workgroups of every running job instead of running jobs one after
// another.  Outputs stay resident in the arena until the client releases
// them.  Every job is computed by the same kernels as fr_map, so its maps do
// not depend on what else is running.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/fr.h"
#include "fr_internal.h"

namespace {

thread_local std::string g_serr;

fr_status sfail(fr_status code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
fr_status sfail(fr_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_serr = buf;
  return code;
}

// CLOCK_MONOTONIC seconds (libstdc++'s steady_clock reads that clock).
double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

constexpr int64_t kAlign = 256;
int64_t align_up(int64_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// First-fit allocator over [0, size) with address-ordered free blocks that
// coalesce on release.
class Arena {
 public:
  void init(int64_t size) {
    size_ = size;
    free_.clear();
    free_[0] = size;
    used_ = peak_ = 0;
  }
  int64_t alloc(int64_t bytes) {
    bytes = align_up(bytes);
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      const int64_t off = it->first, rest = it->second - bytes;
      free_.erase(it);
      if (rest > 0) free_[off + bytes] = rest;
      used_ += bytes;
      peak_ = std::max(peak_, used_);
      return off;
    }
    return -1;
  }
  void release(int64_t off, int64_t bytes) {
    bytes = align_up(bytes);
    used_ -= bytes;
    auto next = free_.lower_bound(off);
    if (next != free_.end() && off + bytes == next->first) {
      bytes += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {
      auto prev = std::prev(next);
      if (prev->first + prev->second == off) {
        prev->second += bytes;
        return;
      }
    }
    free_[off] = bytes;
  }
  int64_t size() const { return size_; }
  int64_t used() const { return used_; }
  int64_t peak() const { return peak_; }

 private:
  int64_t size_ = 0, used_ = 0, peak_ = 0;
  std::map<int64_t, int64_t> free_;
};

// Workgroups (and scratch slices) of a served job's generic-kernel launch.
constexpr int kServeGenericGrid = 64;

// Byte offsets of a job's parts inside its arena block.
struct Layout {
  int64_t vol, mask, levels, list, stage, out, bcount, boff, bmin, bmax, job, params, over0, over1,
      gscratch, total;
};

// The job needs the generic kernel: radius above 3, or neighbourhoods that
// may hold more than 64 present levels.
bool needs_generic(const fr::BatchJob& B) { return B.radius > 3 || (B.radius >= 2 && B.lcap > 64); }

Layout layout_of(const fr::BatchJob& B) {
  Layout L;
  int64_t o = 0;
  auto take = [&](int64_t bytes) {
    const int64_t at = o;
    o = align_up(o + bytes);
    return at;
  };
  const int64_t esize = B.dtype == FR_I16 ? 2 : 4;
  L.vol = take(B.nvox * esize);
  L.mask = take(B.nvox);
  L.levels = take(B.nvox);
  L.list = take(4 * B.n_mask);
  L.stage = take((int64_t)sizeof(float) * fr::kStageStride * B.n_mask);
  L.out = take((int64_t)sizeof(float) * B.count * B.n_mask);
  L.bcount = take(4 * (int64_t)B.nseg);
  L.boff = take(8 * (int64_t)B.nseg);
  L.bmin = take(8 * (int64_t)B.nseg);
  L.bmax = take(8 * (int64_t)B.nseg);
  L.job = take(sizeof(fr::BatchJob));
  L.params = take(sizeof(fr::DiscParams));
  L.over0 = take((int64_t)sizeof(int2) * B.n_mask);
  L.over1 = take((int64_t)sizeof(int2) * B.n_mask);
  L.gscratch = take(needs_generic(B) ? (int64_t)kServeGenericGrid * (int64_t)fr::generic_scratch_bytes(B.lcap) : 0);
  L.total = o;
  return L;
}

struct SJob {
  fr_job spec;
  fr::BatchJob bj;
  int lcap = 32;
  Layout lay;
  int64_t off = -1;
  int state = 0;  // 0 queued, 1 running, 2 done
  int32_t status = FR_OK, ng = 0;
  double t_submit = 0, t_admit = 0, t_done = 0;
  const float* out = nullptr;
};

struct Slot {
  hipStream_t st = nullptr;
  hipEvent_t ev = nullptr;
  fr::BatchJob* h_job = nullptr;     // pinned upload of the job record
  fr::DiscParams* h_params = nullptr;  // pinned read-back of the job status
  int64_t ticket = -1;
};

}  // namespace

struct fr_server_s {
  int device = 0;
  int n_cu = 0;
  char* base = nullptr;
  Arena arena;
  std::vector<Slot> slots;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::deque<int64_t> pending;
  std::unordered_map<int64_t, SJob> jobs;
  std::deque<int64_t> done_unpolled;
  std::vector<double> latencies_ms;
  int64_t next_ticket = 1;
  int64_t submitted = 0, completed = 0, failed = 0, voxels = 0;
  int32_t inflight = 0, max_inflight = 0;
  bool stop = false;
  std::thread worker;
};

namespace {

int32_t map_status(int32_t err) {
  switch (err) {
    case fr::kJobOk: return FR_OK;
    case fr::kJobEmpty: return FR_E_EMPTY_MASK;
    case fr::kJobCount: return FR_E_ARG;
    default: return FR_E_RANGE;
  }
}

// Enqueue one admitted job on its slot; called with the server lock held.
hipError_t launch_job(fr_server_s* s, SJob& J, Slot& sl) {
  char* blk = s->base + J.off;
  const Layout& L = J.lay;
  fr::BatchJob B = J.bj;
  B.vol = blk + L.vol;
  B.mask = (const uint8_t*)(blk + L.mask);
  B.levels = (uint8_t*)(blk + L.levels);
  B.list = (int32_t*)(blk + L.list);
  B.stage = (float*)(blk + L.stage);
  B.out = (float*)(blk + L.out);
  B.seg_base = 0;
  J.out = B.out;
  *sl.h_job = B;
  const int64_t esize = B.dtype == FR_I16 ? 2 : 4;
  hipError_t e;
  if ((e = hipMemcpyAsync((void*)B.vol, J.spec.volume, B.nvox * esize, hipMemcpyDefault, sl.st)) !=
      hipSuccess)
    return e;
  if ((e = hipMemcpyAsync((void*)B.mask, J.spec.mask, B.nvox, hipMemcpyDefault, sl.st)) != hipSuccess)
    return e;
  fr::BatchJob* djob = (fr::BatchJob*)(blk + L.job);
  fr::DiscParams* dpar = (fr::DiscParams*)(blk + L.params);
  if ((e = hipMemcpyAsync(djob, sl.h_job, sizeof(fr::BatchJob), hipMemcpyHostToDevice, sl.st)) !=
      hipSuccess)
    return e;
  fr::DiscScratch sc;
  sc.nblocks = B.nseg;
  sc.block_count = (int32_t*)(blk + L.bcount);
  sc.block_offset = (int64_t*)(blk + L.boff);
  sc.block_min = (double*)(blk + L.bmin);
  sc.block_max = (double*)(blk + L.bmax);
  sc.params = dpar;
  if ((e = fr::launch_discretise_batch(djob, 1, nullptr, B.nseg, sc, sl.st)) != hipSuccess) return e;
  int2* over0 = (int2*)(blk + L.over0);
  int2* over1 = (int2*)(blk + L.over1);
  fr::MapArgs none;
  memset(&none, 0, sizeof none);
  if (B.radius <= 3) {
    int vpw, mult, klmax;
    fr::tuned_settings(B.dtype, B.radius, J.lcap, &vpw, &mult, &klmax);
    const int32_t n_items = (int32_t)((B.n_mask + vpw - 1) / vpw);
    // one workgroup per work item: workgroups of concurrent jobs interleave
    if ((e = fr::launch_map_batch(djob, dpar, nullptr, n_items, nullptr, vpw, B.dtype, B.radius, klmax,
                                  n_items, over0, &dpar->n_over[0], nullptr, sl.st)) != hipSuccess)
      return e;
    if (B.radius >= 2 && klmax == 32 && B.lcap > 32) {
      const int grid64 = s->n_cu * fr::map_batch_blocks_per_cu(B.dtype, B.radius, 64);
      // a persistent grid over a list known only on the device: a work queue,
      // so jobs running beside it do not leave it a long tail
      if ((e = fr::launch_map_batch(djob, dpar, over0, 0, &dpar->n_over[0], 1, B.dtype, B.radius, 64,
                                    grid64, over1, &dpar->n_over[1], &dpar->queue[1], sl.st)) != hipSuccess)
        return e;
    }
    if (needs_generic(B)) {
      const int list = klmax == 32 ? 1 : 0;
      if ((e = fr::launch_map_generic(none, djob, dpar, list ? over1 : over0, &dpar->n_over[list], 0,
                                      B.dtype, blk + L.gscratch, B.lcap, kServeGenericGrid,
                                      sl.st)) != hipSuccess)
        return e;
    }
  } else if ((e = fr::launch_map_generic(none, djob, dpar, nullptr, nullptr, (int32_t)B.n_mask, B.dtype,
                                         blk + L.gscratch, B.lcap, kServeGenericGrid, sl.st)) !=
             hipSuccess) {
    return e;
  }
  if ((e = fr::launch_transpose_batch(djob, dpar, nullptr, (int32_t)((B.n_mask + 63) / 64), sl.st)) !=
      hipSuccess)
    return e;
  if ((e = hipMemcpyAsync(sl.h_params, dpar, sizeof(fr::DiscParams), hipMemcpyDeviceToHost, sl.st)) !=
      hipSuccess)
    return e;
  return hipEventRecord(sl.ev, sl.st);
}

void finish_job(fr_server_s* s, SJob& J, int64_t ticket, int32_t status, int32_t ng) {
  J.t_done = now_s();
  J.state = 2;
  J.status = status;
  J.ng = ng;
  s->completed++;
  if (status != FR_OK)
    s->failed++;
  else
    s->voxels += J.bj.n_mask;
  s->latencies_ms.push_back((J.t_done - J.t_submit) * 1e3);
  s->done_unpolled.push_back(ticket);
  s->inflight--;
  s->cv_done.notify_all();
}

void worker_main(fr_server_s* s) {
  (void)hipSetDevice(s->device);
  std::unique_lock<std::mutex> lk(s->mu);
  for (;;) {
    bool progress = false;
    for (auto& sl : s->slots) {
      if (sl.ticket < 0) continue;
      const hipError_t q = hipEventQuery(sl.ev);
      if (q == hipErrorNotReady) continue;
      SJob& J = s->jobs[sl.ticket];
      if (q == hipSuccess)
        finish_job(s, J, sl.ticket, map_status(sl.h_params->err), sl.h_params->ng);
      else
        finish_job(s, J, sl.ticket, FR_E_DEVICE, 0);
      sl.ticket = -1;
      progress = true;
    }
    while (!s->stop && !s->pending.empty()) {
      Slot* free_slot = nullptr;
      for (auto& sl : s->slots)
        if (sl.ticket < 0) {
          free_slot = &sl;
          break;
        }
      if (!free_slot) break;
      const int64_t t = s->pending.front();
      SJob& J = s->jobs[t];
      const int64_t off = s->arena.alloc(J.lay.total);
      if (off < 0) break;  // arrival order: wait until the head job fits
      s->pending.pop_front();
      J.off = off;
      J.state = 1;
      J.t_admit = now_s();
      free_slot->ticket = t;
      s->inflight++;
      s->max_inflight = std::max(s->max_inflight, s->inflight);
      if (launch_job(s, J, *free_slot) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipStreamSynchronize(free_slot->st);
        finish_job(s, J, t, FR_E_DEVICE, 0);
        free_slot->ticket = -1;
      }
      progress = true;
    }
    if (s->stop && s->inflight == 0) break;
    if (!progress) {
      if (s->inflight > 0) {  // poll the running jobs' events
        lk.unlock();
        std::this_thread::sleep_for(std::chrono::microseconds(20));
        lk.lock();
      } else {
        s->cv_work.wait(lk);  // new job, a release, or stop
      }
    }
  }
}

void free_server(fr_server_s* s) {
  for (auto& sl : s->slots) {
    if (sl.ev) (void)hipEventDestroy(sl.ev);
    if (sl.st) (void)hipStreamDestroy(sl.st);
    if (sl.h_job) (void)hipHostFree(sl.h_job);
    if (sl.h_params) (void)hipHostFree(sl.h_params);
  }
  if (s->base) (void)hipFree(s->base);
  delete s;
}

}  // namespace

extern "C" {

fr_status fr_server_create(const fr_server_config* cfg, fr_server* out) {
  g_serr.clear();
  if (!cfg || !out) return sfail(FR_E_ARG, "cfg and out are required");
  if (cfg->hbm_budget_bytes < (1 << 20)) return sfail(FR_E_ARG, "hbm_budget_bytes must be >= 1 MiB");
  if (cfg->slots < 1 || cfg->slots > 16) return sfail(FR_E_ARG, "slots must be in 1..16");
  if (cfg->reserved != 0) return sfail(FR_E_ARG, "reserved must be 0");
  fr_server_s* s = new (std::nothrow) fr_server_s();
  if (!s) return sfail(FR_E_NOMEM, "host allocation failed");
  if (hipGetDevice(&s->device) != hipSuccess ||
      hipDeviceGetAttribute(&s->n_cu, hipDeviceAttributeMultiprocessorCount, s->device) != hipSuccess) {
    delete s;
    return sfail(FR_E_DEVICE, "hipGetDevice failed");
  }
  const int64_t budget = cfg->hbm_budget_bytes / kAlign * kAlign;
  if (hipMalloc((void**)&s->base, budget) != hipSuccess) {
    (void)hipGetLastError();
    s->base = nullptr;
    free_server(s);
    return sfail(FR_E_NOMEM, "arena of %lld bytes could not be allocated", (long long)budget);
  }
  s->arena.init(budget);
  s->slots.resize(cfg->slots);
  for (auto& sl : s->slots) {
    if (hipStreamCreateWithFlags(&sl.st, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming) != hipSuccess ||
        hipHostMalloc((void**)&sl.h_job, sizeof(fr::BatchJob), hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc((void**)&sl.h_params, sizeof(fr::DiscParams), hipHostMallocDefault) != hipSuccess) {
      free_server(s);
      return sfail(FR_E_DEVICE, "slot streams/events/pinned memory could not be created");
    }
  }
  s->worker = std::thread(worker_main, s);
  *out = s;
  return FR_OK;
}

fr_status fr_server_footprint(const fr_job* job, int64_t* bytes) {
  g_serr.clear();
  if (!job || !bytes) return sfail(FR_E_ARG, "job and bytes are required");
  fr::BatchJob B;
  int lcap;
  char msg[256];
  const fr_status st = fr::validate_job(*job, 0, &B, &lcap, msg, sizeof msg, false);
  if (st != FR_OK) return sfail(st, "%s", msg);
  *bytes = align_up(layout_of(B).total);
  return FR_OK;
}

fr_status fr_server_submit(fr_server s, const fr_job* job, int64_t* ticket) {
  g_serr.clear();
  if (!s || !job || !ticket) return sfail(FR_E_ARG, "server, job and ticket are required");
  SJob J;
  J.spec = *job;
  char msg[256];
  const fr_status st = fr::validate_job(*job, 0, &J.bj, &J.lcap, msg, sizeof msg, false);
  if (st != FR_OK) return sfail(st, "%s", msg);
  if (job->out_maps || job->out_capacity_floats)
    return sfail(FR_E_ARG, "served jobs write into the server's arena: out_maps must be NULL");
  J.lay = layout_of(J.bj);
  std::lock_guard<std::mutex> lk(s->mu);
  if (align_up(J.lay.total) > s->arena.size())
    return sfail(FR_E_CAPACITY, "job footprint %lld bytes exceeds the arena (%lld bytes)",
                 (long long)J.lay.total, (long long)s->arena.size());
  if (s->stop) return sfail(FR_E_ARG, "server is shutting down");
  J.t_submit = now_s();
  const int64_t t = s->next_ticket++;
  s->jobs.emplace(t, J);
  s->pending.push_back(t);
  s->submitted++;
  *ticket = t;
  s->cv_work.notify_one();
  return FR_OK;
}

fr_status fr_server_poll(fr_server s, int64_t* tickets, int32_t max_tickets, int32_t* n_done) {
  g_serr.clear();
  if (!s || !n_done || (max_tickets > 0 && !tickets)) return sfail(FR_E_ARG, "bad arguments");
  std::lock_guard<std::mutex> lk(s->mu);
  int32_t n = 0;
  while (n < max_tickets && !s->done_unpolled.empty()) {
    tickets[n++] = s->done_unpolled.front();
    s->done_unpolled.pop_front();
  }
  *n_done = n;
  return FR_OK;
}

fr_status fr_server_wait(fr_server s, int64_t ticket, double timeout_ms) {
  g_serr.clear();
  if (!s) return sfail(FR_E_ARG, "server is NULL");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) return sfail(FR_E_ARG, "unknown ticket %lld", (long long)ticket);
  const auto pred = [&] {
    auto j = s->jobs.find(ticket);
    return j == s->jobs.end() || j->second.state == 2;
  };
  if (timeout_ms < 0) {
    s->cv_done.wait(lk, pred);
  } else if (!s->cv_done.wait_for(lk, std::chrono::duration<double, std::milli>(timeout_ms), pred)) {
    return sfail(FR_E_TIMEOUT, "ticket %lld not finished after %.1f ms", (long long)ticket, timeout_ms);
  }
  return FR_OK;
}

fr_status fr_server_result(fr_server s, int64_t ticket, fr_result* r) {
  g_serr.clear();
  if (!s || !r) return sfail(FR_E_ARG, "server and result are required");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) return sfail(FR_E_ARG, "unknown ticket %lld", (long long)ticket);
  const SJob& J = it->second;
  memset(r, 0, sizeof *r);
  r->done = J.state == 2;
  r->status = J.status;
  r->ng = J.ng;
  r->count = J.bj.count;
  r->n_mask = J.bj.n_mask;
  r->maps = (J.state == 2 && J.status == FR_OK) ? J.out : nullptr;
  r->footprint_bytes = align_up(J.lay.total);
  r->t_submit = J.t_submit;
  r->t_admit = J.t_admit;
  r->t_done = J.t_done;
  return FR_OK;
}

fr_status fr_server_copy(fr_server s, int64_t ticket, float* dst, int64_t capacity_floats,
                         void* hip_stream) {
  g_serr.clear();
  if (!s || !dst) return sfail(FR_E_ARG, "server and dst are required");
  const float* src;
  int64_t n;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->jobs.find(ticket);
    if (it == s->jobs.end()) return sfail(FR_E_ARG, "unknown ticket %lld", (long long)ticket);
    const SJob& J = it->second;
    if (J.state != 2 || J.status != FR_OK)
      return sfail(FR_E_ARG, "ticket %lld has no maps (state %d, status %d)", (long long)ticket,
                   J.state, J.status);
    src = J.out;
    n = (int64_t)J.bj.count * J.bj.n_mask;
  }
  if (capacity_floats < n)
    return sfail(FR_E_CAPACITY, "dst holds %lld floats, %lld needed", (long long)capacity_floats,
                 (long long)n);
  const hipError_t e =
      hipMemcpyAsync(dst, src, sizeof(float) * n, hipMemcpyDefault, (hipStream_t)hip_stream);
  if (e != hipSuccess) return sfail(FR_E_DEVICE, "copy failed: %s", hipGetErrorString(e));
  return FR_OK;
}

fr_status fr_server_release(fr_server s, int64_t ticket) {
  g_serr.clear();
  if (!s) return sfail(FR_E_ARG, "server is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) return sfail(FR_E_ARG, "unknown ticket %lld", (long long)ticket);
  if (it->second.state != 2) return sfail(FR_E_ARG, "ticket %lld has not finished", (long long)ticket);
  if (it->second.off >= 0) s->arena.release(it->second.off, it->second.lay.total);
  s->jobs.erase(it);
  auto u = std::find(s->done_unpolled.begin(), s->done_unpolled.end(), ticket);
  if (u != s->done_unpolled.end()) s->done_unpolled.erase(u);
  s->cv_work.notify_one();
  return FR_OK;
}

fr_status fr_server_stats(fr_server s, fr_server_info* out) {
  g_serr.clear();
  if (!s || !out) return sfail(FR_E_ARG, "server and stats are required");
  std::lock_guard<std::mutex> lk(s->mu);
  memset(out, 0, sizeof *out);
  out->submitted = s->submitted;
  out->completed = s->completed;
  out->failed = s->failed;
  out->mapped_voxels = s->voxels;
  out->arena_bytes = s->arena.size();
  out->arena_used_bytes = s->arena.used();
  out->arena_peak_bytes = s->arena.peak();
  out->slots = (int32_t)s->slots.size();
  out->max_inflight = s->max_inflight;
  out->queued = (int32_t)s->pending.size();
  out->inflight = s->inflight;
  if (!s->latencies_ms.empty()) {
    std::vector<double> v = s->latencies_ms;
    std::sort(v.begin(), v.end());
    auto rank = [&](double q) {  // nearest-rank percentile
      size_t k = (size_t)ceil(q * v.size());
      return v[k == 0 ? 0 : k - 1];
    };
    out->p50_ms = rank(0.50);
    out->p99_ms = rank(0.99);
    double sum = 0;
    for (double x : v) sum += x;
    out->mean_ms = sum / v.size();
  }
  return FR_OK;
}

fr_status fr_server_destroy(fr_server s) {
  g_serr.clear();
  if (!s) return FR_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->pending.clear();
    s->cv_work.notify_one();
  }
  if (s->worker.joinable()) s->worker.join();
  free_server(s);
  return FR_OK;
}

const char* fr_server_last_error(void) { return g_serr.c_str(); }

}  // extern "C"
