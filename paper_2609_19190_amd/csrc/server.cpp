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
#include "fr_error.h"
#include "fr_internal.h"

namespace {


fr_status sfail(fr_status code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
fr_status sfail(fr_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  fr::set_error(buf);
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

// The admission policy, shared by the live server and the host replay.
// Queued jobs wait in submission order; when slots are free the head job
// takes the first free arena block that fits it; if none does, later jobs
// that fit may pass it, at most max_bypass of them per head (then the head
// waits for running jobs to free space).  Jobs whose deadline has passed
// leave the queue first.  Injected failures turn the next admissions into
// allocation failures (nothing kept).  All of it is host bookkeeping.
struct Queued {
  int64_t ticket;
  int64_t bytes;
  double deadline;  // absolute seconds; 0: none
};
struct Decision {
  int64_t ticket;
  int kind;  // FR_ADMITTED, FR_ADMIT_EXPIRED, FR_ADMIT_ALLOC_FAILED
  int64_t off;
};

class Admission {
 public:
  void init(int64_t budget, int max_bypass) {
    arena_.init(budget);
    max_bypass_ = max_bypass;
    q_.clear();
    head_ = -1;
    passed_ = 0;
    fail_next_ = 0;
  }
  bool fits_ever(int64_t bytes) const { return align_up(bytes) <= arena_.size(); }
  void push(const Queued& j) { q_.push_back(j); }
  bool cancel_queued(int64_t ticket) {
    for (auto it = q_.begin(); it != q_.end(); ++it)
      if (it->ticket == ticket) {
        q_.erase(it);
        return true;
      }
    return false;
  }
  void inject(int n) { fail_next_ = n; }
  void release(int64_t off, int64_t bytes) { arena_.release(off, bytes); }
  // Admits into at most free_slots slots at time now; appends the outcomes.
  void step(int free_slots, double now, std::vector<Decision>* out) {
    for (auto it = q_.begin(); it != q_.end();) {
      if (it->deadline > 0.0 && now >= it->deadline) {
        out->push_back({it->ticket, FR_ADMIT_EXPIRED, -1});
        it = q_.erase(it);
      } else {
        ++it;
      }
    }
    while (free_slots > 0 && !q_.empty()) {
      if (q_.front().ticket != head_) {  // a new head: its bypass count starts
        head_ = q_.front().ticket;
        passed_ = 0;
      }
      size_t pick = 0;
      int64_t off = arena_.alloc(q_[0].bytes);
      if (off < 0 && passed_ < max_bypass_) {
        for (size_t i = 1; i < q_.size() && off < 0; ++i) {
          off = arena_.alloc(q_[i].bytes);
          if (off >= 0) pick = i;
        }
      }
      if (off < 0) break;  // nothing fits until running jobs free space
      const Queued j = q_[pick];
      q_.erase(q_.begin() + (std::ptrdiff_t)pick);
      if (pick > 0) ++passed_;
      if (fail_next_ > 0) {
        --fail_next_;
        arena_.release(off, j.bytes);
        out->push_back({j.ticket, FR_ADMIT_ALLOC_FAILED, -1});
        continue;
      }
      out->push_back({j.ticket, FR_ADMITTED, off});
      --free_slots;
    }
  }
  // Earliest deadline of a queued job (0: none).
  double next_deadline() const {
    double d = 0.0;
    for (const auto& j : q_)
      if (j.deadline > 0.0 && (d == 0.0 || j.deadline < d)) d = j.deadline;
    return d;
  }
  size_t queued() const { return q_.size(); }
  int64_t size() const { return arena_.size(); }
  int64_t used() const { return arena_.used(); }
  int64_t peak() const { return arena_.peak(); }

 private:
  Arena arena_;
  std::deque<Queued> q_;
  int max_bypass_ = 0;
  int64_t head_ = -1;
  int passed_ = 0;
  int fail_next_ = 0;
};

// Workgroups (and scratch slices) of a served job's generic-kernel launch.
constexpr int kServeGenericGrid = 64;

// Byte offsets of a job's parts inside its arena block.
// The output comes first: [0, keep) stays until the client releases the
// job; the working part [keep, total) is freed as soon as the job ends.
struct Layout {
  int64_t vol, mask, levels, list, stage, out, bcount, boff, bmin, bmax, job, params, over0, over1,
      gscratch, keep, total;
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
  L.out = take((int64_t)sizeof(float) * B.count * B.n_mask);
  L.keep = o;
  L.vol = take(B.nvox * esize);
  L.mask = take(B.nvox);
  L.levels = take(B.nvox);
  L.list = take(4 * B.n_mask);
  L.stage = take((int64_t)sizeof(float) * fr::kStageStride * B.n_mask);
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
  int64_t held = 0;  // bytes of the block still held (total, then keep once done)
  int state = 0;  // 0 queued, 1 running, 2 done
  bool cancel = false;  // cancelled while running: no maps at completion
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
  Admission adm;
  std::vector<Slot> slots;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
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
    // one workgroup per work item: workgroups of concurrent jobs interleave.
    // Served jobs solve their MCC problems inside the map kernel: a job's own
    // MCC kernel would take every CU for its short run and stall the jobs
    // beside it (measured: served throughput fell below the plain path's).
    if ((e = fr::launch_map_batch(djob, dpar, nullptr, n_items, nullptr, vpw, B.dtype, B.radius, klmax,
                                  n_items, over0, &dpar->n_over[0], nullptr, nullptr, 0, nullptr,
                                  sl.st)) != hipSuccess)
      return e;
    if (B.radius >= 2 && klmax == 32 && B.lcap > 32) {
      const int grid64 = s->n_cu * fr::map_batch_blocks_per_cu(B.dtype, B.radius, 64, false);
      // a persistent grid over a list known only on the device: a work queue,
      // so jobs running beside it do not leave it a long tail
      if ((e = fr::launch_map_batch(djob, dpar, over0, 0, &dpar->n_over[0], 1, B.dtype, B.radius, 64,
                                    grid64, over1, &dpar->n_over[1], &dpar->queue[1], nullptr, 0, nullptr,
                                    sl.st)) != hipSuccess)
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

// A job ends (ran = it held a slot).  Latencies count the jobs that
// produced maps.
void finish_job(fr_server_s* s, SJob& J, int64_t ticket, int32_t status, int32_t ng, bool ran) {
  J.t_done = now_s();
  J.state = 2;
  J.status = status;
  J.ng = ng;
  s->completed++;
  if (status != FR_OK) {
    s->failed++;
    J.out = nullptr;
    if (J.off >= 0) {  // a failed or cancelled job keeps no block
      s->adm.release(J.off, J.held);
      J.off = -1;
      J.held = 0;
    }
  } else {
    s->voxels += J.bj.n_mask;
    s->latencies_ms.push_back((J.t_done - J.t_submit) * 1e3);
    // the working buffers go back to the arena now; the output stays
    if (J.held > J.lay.keep) {
      s->adm.release(J.off + J.lay.keep, J.held - J.lay.keep);
      J.held = J.lay.keep;
    }
  }
  s->done_unpolled.push_back(ticket);
  if (ran) s->inflight--;
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
      if (J.cancel)
        finish_job(s, J, sl.ticket, FR_E_CANCELLED, 0, true);
      else if (q == hipSuccess)
        finish_job(s, J, sl.ticket, map_status(sl.h_params->err), sl.h_params->ng, true);
      else
        finish_job(s, J, sl.ticket, FR_E_DEVICE, 0, true);
      sl.ticket = -1;
      progress = true;
    }
    if (!s->stop) {
      int free_slots = 0;
      for (auto& sl : s->slots) free_slots += sl.ticket < 0;
      std::vector<Decision> dec;
      s->adm.step(free_slots, now_s(), &dec);
      for (const Decision& d : dec) {
        SJob& J = s->jobs[d.ticket];
        progress = true;
        if (d.kind == FR_ADMIT_EXPIRED) {
          finish_job(s, J, d.ticket, FR_E_TIMEOUT, 0, false);
          continue;
        }
        if (d.kind == FR_ADMIT_ALLOC_FAILED) {
          finish_job(s, J, d.ticket, FR_E_NOMEM, 0, false);
          continue;
        }
        Slot* free_slot = nullptr;
        for (auto& sl : s->slots)
          if (sl.ticket < 0) {
            free_slot = &sl;
            break;
          }
        J.off = d.off;
        J.held = J.lay.total;
        J.state = 1;
        J.t_admit = now_s();
        free_slot->ticket = d.ticket;
        s->inflight++;
        s->max_inflight = std::max(s->max_inflight, s->inflight);
        if (launch_job(s, J, *free_slot) != hipSuccess) {
          (void)hipGetLastError();
          (void)hipStreamSynchronize(free_slot->st);
          finish_job(s, J, d.ticket, FR_E_DEVICE, 0, true);
          free_slot->ticket = -1;
        }
      }
    }
    if (s->stop && s->inflight == 0) break;
    if (!progress) {
      if (s->inflight > 0) {  // poll the running jobs' events
        lk.unlock();
        std::this_thread::sleep_for(std::chrono::microseconds(20));
        lk.lock();
      } else if (const double dl = s->adm.next_deadline(); dl > 0.0) {
        // a queued job's deadline, a new job, a release, or stop
        s->cv_work.wait_for(lk, std::chrono::duration<double>(std::max(dl - now_s(), 0.0) + 1e-4));
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
  fr::clear_error();
  if (!cfg || !out) return sfail(FR_E_ARG, "cfg and out are required");
  if (cfg->hbm_budget_bytes < (1 << 20)) return sfail(FR_E_ARG, "hbm_budget_bytes must be >= 1 MiB");
  if (cfg->slots < 1 || cfg->slots > 16) return sfail(FR_E_ARG, "slots must be in 1..16");
  if (cfg->max_bypass < 0 || cfg->max_bypass > 1024)
    return sfail(FR_E_ARG, "max_bypass must be in 0..1024");
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
  s->adm.init(budget, cfg->max_bypass);
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
  fr::clear_error();
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
  return fr_server_submit_ex(s, job, nullptr, ticket);
}

fr_status fr_server_submit_ex(fr_server s, const fr_job* job, const fr_submit_options* options,
                              int64_t* ticket) {
  fr::clear_error();
  if (!s || !job || !ticket) return sfail(FR_E_ARG, "server, job and ticket are required");
  double deadline_ms = 0.0;
  if (options) {
    if (!(options->deadline_ms >= 0.0) || options->reserved[0] || options->reserved[1])
      return sfail(FR_E_ARG, "deadline_ms must be >= 0 and reserved 0");
    deadline_ms = options->deadline_ms;
  }
  SJob J;
  J.spec = *job;
  char msg[256];
  const fr_status st = fr::validate_job(*job, 0, &J.bj, &J.lcap, msg, sizeof msg, false);
  if (st != FR_OK) return sfail(st, "%s", msg);
  if (job->out_maps || job->out_capacity_floats)
    return sfail(FR_E_ARG, "served jobs write into the server's arena: out_maps must be NULL");
  J.lay = layout_of(J.bj);
  std::lock_guard<std::mutex> lk(s->mu);
  if (!s->adm.fits_ever(J.lay.total))
    return sfail(FR_E_CAPACITY, "job footprint %lld bytes exceeds the arena (%lld bytes)",
                 (long long)J.lay.total, (long long)s->adm.size());
  if (s->stop) return sfail(FR_E_ARG, "server is shutting down");
  J.t_submit = now_s();
  const int64_t t = s->next_ticket++;
  s->jobs.emplace(t, J);
  s->adm.push({t, J.lay.total, deadline_ms > 0.0 ? J.t_submit + deadline_ms * 1e-3 : 0.0});
  s->submitted++;
  *ticket = t;
  s->cv_work.notify_one();
  return FR_OK;
}

fr_status fr_server_poll(fr_server s, int64_t* tickets, int32_t max_tickets, int32_t* n_done) {
  fr::clear_error();
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
  fr::clear_error();
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
  fr::clear_error();
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
  fr::clear_error();
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
  fr::clear_error();
  if (!s) return sfail(FR_E_ARG, "server is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) return sfail(FR_E_ARG, "unknown ticket %lld", (long long)ticket);
  if (it->second.state != 2) return sfail(FR_E_ARG, "ticket %lld has not finished", (long long)ticket);
  if (it->second.off >= 0) s->adm.release(it->second.off, it->second.held);
  s->jobs.erase(it);
  auto u = std::find(s->done_unpolled.begin(), s->done_unpolled.end(), ticket);
  if (u != s->done_unpolled.end()) s->done_unpolled.erase(u);
  s->cv_work.notify_one();
  return FR_OK;
}

fr_status fr_server_stats(fr_server s, fr_server_info* out) {
  fr::clear_error();
  if (!s || !out) return sfail(FR_E_ARG, "server and stats are required");
  std::lock_guard<std::mutex> lk(s->mu);
  memset(out, 0, sizeof *out);
  out->submitted = s->submitted;
  out->completed = s->completed;
  out->failed = s->failed;
  out->mapped_voxels = s->voxels;
  out->arena_bytes = s->adm.size();
  out->arena_used_bytes = s->adm.used();
  out->arena_peak_bytes = s->adm.peak();
  out->slots = (int32_t)s->slots.size();
  out->max_inflight = s->max_inflight;
  out->queued = (int32_t)s->adm.queued();
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
  fr::clear_error();
  if (!s) return FR_OK;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->cv_work.notify_one();
  }
  if (s->worker.joinable()) s->worker.join();
  free_server(s);
  return FR_OK;
}

fr_status fr_server_cancel(fr_server s, int64_t ticket) {
  fr::clear_error();
  if (!s) return sfail(FR_E_ARG, "server is NULL");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->jobs.find(ticket);
  if (it == s->jobs.end()) return sfail(FR_E_ARG, "unknown ticket %lld", (long long)ticket);
  SJob& J = it->second;
  if (J.state == 2) return sfail(FR_E_ARG, "ticket %lld has already finished", (long long)ticket);
  if (J.state == 0) {
    if (s->adm.cancel_queued(ticket)) finish_job(s, J, ticket, FR_E_CANCELLED, 0, false);
  } else {
    J.cancel = true;  // its kernels complete; the worker then ends it
  }
  s->cv_work.notify_one();
  return FR_OK;
}

fr_status fr_server_inject_alloc_failures(fr_server s, int32_t n) {
  fr::clear_error();
  if (!s || n < 0) return sfail(FR_E_ARG, "server is NULL or n < 0");
  std::lock_guard<std::mutex> lk(s->mu);
  s->adm.inject(n);
  return FR_OK;
}

fr_status fr_admission_replay(int64_t budget_bytes, int32_t slots, int32_t max_bypass,
                              const fr_admit_event* events, int32_t n_events,
                              fr_admit_record* records, int32_t max_records, int32_t* n_records) {
  fr::clear_error();
  if (budget_bytes < kAlign || slots < 1 || max_bypass < 0 || n_events < 0 ||
      (n_events > 0 && !events) || max_records < 0 || (max_records > 0 && !records) || !n_records)
    return sfail(FR_E_ARG, "bad arguments");
  Admission adm;
  adm.init(budget_bytes / kAlign * kAlign, max_bypass);
  struct Run {
    int64_t off = -1, bytes = 0;
  };
  std::unordered_map<int64_t, int> state;  // 0 queued, 1 running, 2 ended
  std::unordered_map<int64_t, Run> running;
  std::unordered_map<int64_t, bool> cancelled_running;  // cancelled after admission
  int free_slots = slots;
  int32_t n = 0;
  double t_prev = -INFINITY;
  auto emit = [&](double t, int64_t ticket, int64_t off, int outcome) {
    if (n >= max_records) return false;
    records[n].t = t;
    records[n].ticket = ticket;
    records[n].offset = off;
    records[n].outcome = outcome;
    records[n].reserved = 0;
    ++n;
    return true;
  };
  std::unordered_map<int64_t, int64_t> bytes_of;
  for (int32_t i = 0; i < n_events; ++i) {
    const fr_admit_event& e = events[i];
    if (!(e.t >= t_prev)) return sfail(FR_E_ARG, "event %d: time goes back", i);
    t_prev = e.t;
    switch (e.kind) {
      case FR_ADMIT_SUBMIT:
        if (state.count(e.ticket) || e.bytes <= 0 || !(e.deadline_ms >= 0.0))
          return sfail(FR_E_ARG, "event %d: repeated ticket, bad size or deadline", i);
        if (!adm.fits_ever(e.bytes)) {
          state[e.ticket] = 2;
          if (!emit(e.t, e.ticket, -1, FR_ADMIT_REJECTED)) return sfail(FR_E_CAPACITY, "records full");
          break;
        }
        state[e.ticket] = 0;
        bytes_of[e.ticket] = e.bytes;
        adm.push({e.ticket, e.bytes, e.deadline_ms > 0.0 ? e.t + e.deadline_ms * 1e-3 : 0.0});
        break;
      case FR_ADMIT_CANCEL: {
        auto st = state.find(e.ticket);
        if (st == state.end() || st->second == 2)
          return sfail(FR_E_ARG, "event %d: cancel of an unknown or ended job", i);
        if (st->second == 0) {
          adm.cancel_queued(e.ticket);
          st->second = 2;
          if (!emit(e.t, e.ticket, -1, FR_ADMIT_CANCELLED)) return sfail(FR_E_CAPACITY, "records full");
        } else {
          cancelled_running[e.ticket] = true;
        }
        break;
      }
      case FR_ADMIT_COMPLETE: {
        auto st = state.find(e.ticket);
        if (st == state.end() || st->second != 1)
          return sfail(FR_E_ARG, "event %d: complete of a job that is not running", i);
        st->second = 2;
        adm.release(running[e.ticket].off, running[e.ticket].bytes);
        running.erase(e.ticket);
        ++free_slots;
        if (cancelled_running.count(e.ticket) &&
            !emit(e.t, e.ticket, -1, FR_ADMIT_CANCELLED))  // ends cancelled, without maps
          return sfail(FR_E_CAPACITY, "records full");
        break;
      }
      case FR_ADMIT_FAIL_NEXT:
        if (e.value < 0) return sfail(FR_E_ARG, "event %d: negative count", i);
        adm.inject(e.value);
        break;
      default:
        return sfail(FR_E_ARG, "event %d: unknown kind %d", i, e.kind);
    }
    std::vector<Decision> dec;
    adm.step(free_slots, e.t, &dec);
    for (const Decision& d : dec) {
      state[d.ticket] = d.kind == FR_ADMITTED ? 1 : 2;
      if (d.kind == FR_ADMITTED) {
        running[d.ticket] = Run{d.off, bytes_of[d.ticket]};
        --free_slots;
      }
      if (!emit(e.t, d.ticket, d.off, d.kind)) return sfail(FR_E_CAPACITY, "records full");
    }
  }
  *n_records = n;
  return FR_OK;
}

const char* fr_server_last_error(void) { return fr::last_error(); }

}  // extern "C"
