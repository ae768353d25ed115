// Batched spatial mapping (C ABI fr_batch_*): many VOIs of different sizes,
// radii and gray-level counts mapped by one enqueue with no host round trip.
//
// prepare  host validation; plans the batch-wide discretisation segment
//          table and, per variant (raw type, radius, level class: at most
//          32 or up to 255 present levels; radii above 3 form generic
//          variants), the (job, first voxel) work items; allocates
//          the batch's own device workspace and uploads the tables
//          (synchronous, once).
// launch   enqueues batched discretisation, then every variant's passes
//          (the 32-level instance over all its voxels, the 64-level instance
//          over the neighbourhoods with more present levels; both take their
//          items from a work queue) on 1..n branches: streams forked from
//          the caller's, variants packed longest-first by estimated work,
//          so kernels of different variants run side by side and fill each
//          other's tails; after the join, the generic kernel over what
//          remains and a batched transpose.  Optionally captured once into a
//          hipGraph (the fork and join become graph edges) and replayed.
//          Allocates nothing.
// status   per-job errors found on the device (mask count, Ng range), read
//          after the stream has synchronised.
// autotune times work-item size, grid size and the first pass's instance
//          (32 or 64 levels) per variant on the prepared batch and keeps the
//          fastest (cached per process for later batches of the variant),
//          then the number of concurrent branches of the whole batch.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "../../include/fr.h"
#include "fr_internal.h"

namespace {

thread_local std::string g_berr;

fr_status bfail(fr_status code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
fr_status bfail(fr_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_berr = buf;
  return code;
}

#define BHIP(expr)                                                                      \
  do {                                                                                  \
    hipError_t e_ = (expr);                                                             \
    if (e_ != hipSuccess)                                                               \
      return bfail(FR_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));         \
  } while (0)

struct Tuning {
  int vpw = 4;        // voxels per work item (four fill an MCC flush)
  int grid_mult = 1;  // persistent grid = resident workgroups x grid_mult
  // local-level capacity of the first pass's instance: 32 (the 64-level
  // instance then takes the neighbourhoods with 33..64 present levels) or
  // 64 (one pass; one wave per SIMD at radius 3, no register spills);
  // array sizes only, so the maps do not change
  int kernel_lmax = 32;
};

// Tuned settings per (dtype, radius, level class 32 / 64), shared by every
// batch, and the tuned number of concurrent branches (0: not tuned).
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int>, Tuning> g_tuned;
int g_branches_tuned = 0;

struct Variant {
  int dtype = 0, radius = 0;
  bool generic = false;  // radius above 3: the generic kernel maps every voxel
  int lcap = 1;          // largest present-level bound of its jobs
  int lclass = 32;       // 32 or 64: the tuning key's level class
  Tuning tune;
  std::vector<int> jobs;  // job indices
  int64_t n_vox = 0;      // mask voxels of its jobs
  int2* d_items = nullptr;
  int32_t n_items = 0;
  int32_t cap_items = 0;
  int grid = 0;
  int2* d_over[2] = {nullptr, nullptr};  // overflow lists (n_vox entries each)
  int branch = 0;                        // concurrent branch it runs on
};

// Forked streams a batch may use.
constexpr int kMaxBranches = 4;

int32_t map_count_of(uint32_t fam) {
  static const int cnt[6] = {18, 24, 16, 16, 14, 5};
  int32_t n = 0;
  for (int q = 0; q < 6; ++q)
    if (fam & (1u << q)) n += cnt[q];
  return n;
}

int level_class(int lcap) { return lcap <= 32 ? 32 : 64; }

}  // namespace

struct fr_batch_s {
  int device = 0;
  int n_cu = 0;
  std::vector<fr_job> jobs;
  std::vector<fr::BatchJob> bj;
  std::vector<Variant> variants;
  std::vector<int2> tr_items;
  int64_t n_seg = 0;
  int lcap_generic = 0;  // level bound of the generic launches (0: none)
  // device workspace
  fr::BatchJob* d_jobs = nullptr;
  fr::DiscParams* d_params = nullptr;
  fr::DiscParams* h_params = nullptr;  // pinned
  int32_t* d_seg_job = nullptr;
  int32_t* d_bcount = nullptr;
  int64_t* d_boff = nullptr;
  double* d_bmin = nullptr;
  double* d_bmax = nullptr;
  uint8_t* d_levels = nullptr;
  int32_t* d_lists = nullptr;
  float* d_stage = nullptr;
  int2* d_tr_items = nullptr;
  // per variant: two overflow counts, then the work-queue heads of the two
  // fixed-radius passes; after the last variant, the two MCC stash counts
  int32_t* d_counters = nullptr;
  void* d_gscratch = nullptr;     // generic-kernel scratch
  // MCC problems of the 32-level passes (one per voxel of the fast
  // variants at most), solved by one k_mcc launch after the join
  unsigned char* d_mcc = nullptr;
  int64_t cap_mcc = 0;
  hipEvent_t fork = nullptr;
  int branches = 2;               // concurrent branches of the fixed-radius passes
  hipStream_t aux[kMaxBranches] = {};
  hipEvent_t done[kMaxBranches] = {};
  // graph
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipStream_t graph_stream = nullptr;
  bool prepared = false;
};

namespace {

void free_workspace(fr_batch_s* b) {
  (void)hipFree(b->d_jobs);
  (void)hipFree(b->d_params);
  if (b->h_params) (void)hipHostFree(b->h_params);
  (void)hipFree(b->d_seg_job);
  (void)hipFree(b->d_bcount);
  (void)hipFree(b->d_boff);
  (void)hipFree(b->d_bmin);
  (void)hipFree(b->d_bmax);
  (void)hipFree(b->d_levels);
  (void)hipFree(b->d_lists);
  (void)hipFree(b->d_stage);
  (void)hipFree(b->d_tr_items);
  (void)hipFree(b->d_counters);
  (void)hipFree(b->d_gscratch);
  (void)hipFree(b->d_mcc);
  if (b->fork) (void)hipEventDestroy(b->fork);
  for (int k = 0; k < kMaxBranches; ++k) {
    if (b->done[k]) (void)hipEventDestroy(b->done[k]);
    if (b->aux[k]) (void)hipStreamDestroy(b->aux[k]);
    b->done[k] = nullptr;
    b->aux[k] = nullptr;
  }
  for (auto& v : b->variants) {
    (void)hipFree(v.d_items);
    (void)hipFree(v.d_over[0]);
    (void)hipFree(v.d_over[1]);
  }
  b->d_jobs = nullptr;
  b->d_params = nullptr;
  b->h_params = nullptr;
  b->d_seg_job = nullptr;
  b->d_bcount = nullptr;
  b->d_boff = nullptr;
  b->d_bmin = b->d_bmax = nullptr;
  b->d_levels = nullptr;
  b->d_lists = nullptr;
  b->d_stage = nullptr;
  b->d_tr_items = nullptr;
  b->d_counters = nullptr;
  b->d_mcc = nullptr;
  b->cap_mcc = 0;
  b->d_gscratch = nullptr;
  b->fork = nullptr;
  b->lcap_generic = 0;
  b->variants.clear();
}

void drop_graph(fr_batch_s* b) {
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  b->exec = nullptr;
  b->graph = nullptr;
  b->graph_stream = nullptr;
}

// Work items of one variant with its current work-item size (fast
// variants: (job, first voxel) per vpw voxels; generic ones: one per
// voxel); uploads them.
fr_status build_items(fr_batch_s* b, Variant& v) {
  std::vector<int2> items;
  const int step = v.generic ? 1 : v.tune.vpw;
  for (int j : v.jobs) {
    const int64_t n = b->jobs[j].n_mask;
    for (int64_t m = 0; m < n; m += step) items.push_back(make_int2(j, (int)m));
  }
  // job-major order: workgroups resident at the same time map neighbouring
  // voxels of one job and share its cache lines
  v.n_items = (int32_t)items.size();
  if (v.n_items > v.cap_items) {
    (void)hipFree(v.d_items);
    v.d_items = nullptr;
    if (hipMalloc((void**)&v.d_items, items.size() * sizeof(int2)) != hipSuccess)
      return bfail(FR_E_NOMEM, "work-item table allocation failed");
    v.cap_items = v.n_items;
  }
  BHIP(hipMemcpy(v.d_items, items.data(), items.size() * sizeof(int2), hipMemcpyHostToDevice));
  if (v.generic) {
    v.grid = fr::kGenericGrid;
  } else {
    const int per_cu =
        fr::map_batch_blocks_per_cu(v.dtype, v.radius, v.tune.kernel_lmax, v.tune.kernel_lmax == 32);
    int64_t grid = (int64_t)b->n_cu * per_cu * v.tune.grid_mult;
    if (grid > v.n_items) grid = v.n_items;
    v.grid = (int)std::max<int64_t>(grid, 1);
  }
  return FR_OK;
}

constexpr int kCountersPerVariant = 4;

// The two MCC stash counts, after every variant's counters.
int32_t* mcc_counts(fr_batch_s* b) {
  return b->d_counters + kCountersPerVariant * (int64_t)b->variants.size();
}

// The fixed-radius passes of a fast variant on stream s: the first
// instance over all items (the 32-level one stashing its MCC problems),
// the 64-level one over its overflow; both take their items from a work
// queue, so variants running side by side balance.
fr_status enqueue_fast(fr_batch_s* b, const Variant& v, int vi, hipStream_t s) {
  int32_t* c0 = b->d_counters + kCountersPerVariant * vi;
  const int kl = v.tune.kernel_lmax;
  const bool stash = kl == 32;
  BHIP(fr::launch_map_batch(b->d_jobs, b->d_params, v.d_items, v.n_items, nullptr, v.tune.vpw,
                            v.dtype, v.radius, kl, v.grid, v.d_over[0], c0, c0 + 2,
                            stash ? b->d_mcc : nullptr, b->cap_mcc, mcc_counts(b), s));
  if (v.radius >= 2 && kl == 32 && v.lcap > 32) {
    const int grid64 = b->n_cu * fr::map_batch_blocks_per_cu(v.dtype, v.radius, 64, false);
    BHIP(fr::launch_map_batch(b->d_jobs, b->d_params, v.d_over[0], 0, c0, 1, v.dtype, v.radius, 64,
                              grid64, v.d_over[1], c0 + 1, c0 + 3, nullptr, 0, nullptr, s));
  }
  return FR_OK;
}

// The generic passes of a variant (after the join): what the fixed-radius
// passes handed on, or every voxel of a generic variant.
fr_status enqueue_generic(fr_batch_s* b, const Variant& v, int vi, hipStream_t s) {
  fr::MapArgs none;
  memset(&none, 0, sizeof none);
  if (v.generic) {
    BHIP(fr::launch_map_generic(none, b->d_jobs, b->d_params, v.d_items, nullptr, v.n_items, v.dtype,
                                b->d_gscratch, b->lcap_generic, fr::kGenericGrid, s));
  } else if (v.radius >= 2 && v.lcap > 64) {
    const int list = v.tune.kernel_lmax == 32 ? 1 : 0;
    BHIP(fr::launch_map_generic(none, b->d_jobs, b->d_params, v.d_over[list],
                                b->d_counters + kCountersPerVariant * vi + list, 0, v.dtype, b->d_gscratch,
                                b->lcap_generic, fr::kGenericGrid, s));
  }
  return FR_OK;
}

// Pack the fast variants longest-first into b->branches branches by an
// estimate of their work (mask voxels x cube size, doubled when more than
// 32 levels may be present).
void assign_branches(fr_batch_s* b) {
  std::vector<int> order;
  for (int vi = 0; vi < (int)b->variants.size(); ++vi)
    if (!b->variants[vi].generic) order.push_back(vi);
  auto cost = [&](int vi) {
    const Variant& v = b->variants[vi];
    const double S = 2.0 * v.radius + 1.0;
    return (double)v.n_vox * S * S * S * (v.lcap > 32 ? 2.0 : 1.0);
  };
  std::sort(order.begin(), order.end(), [&](int x, int y) { return cost(x) > cost(y); });
  std::vector<double> load(b->branches, 0.0);
  for (int vi : order) {
    const int k = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    b->variants[vi].branch = k;
    load[k] += cost(vi);
  }
}

fr_status enqueue(fr_batch_s* b, hipStream_t st) {
  fr::DiscScratch s;
  s.nblocks = b->n_seg;
  s.block_count = b->d_bcount;
  s.block_offset = b->d_boff;
  s.block_min = b->d_bmin;
  s.block_max = b->d_bmax;
  s.params = b->d_params;
  const int nv = (int)b->variants.size();
  BHIP(fr::launch_zero_i32(b->d_counters, kCountersPerVariant * nv + 2, st));
  BHIP(fr::launch_discretise_batch(b->d_jobs, (int32_t)b->jobs.size(), b->d_seg_job, b->n_seg, s, st));
  // fork: the fast variants on b->branches streams (one branch: the
  // caller's stream itself), joined before the generic passes
  const bool fork = b->branches > 1;
  if (fork) {
    BHIP(hipEventRecord(b->fork, st));
    for (int k = 0; k < b->branches; ++k) BHIP(hipStreamWaitEvent(b->aux[k], b->fork, 0));
  }
  for (int vi = 0; vi < nv; ++vi) {
    const Variant& v = b->variants[vi];
    if (v.generic) continue;
    fr_status e = enqueue_fast(b, v, vi, fork ? b->aux[v.branch] : st);
    if (e != FR_OK) return e;
  }
  if (fork) {
    for (int k = 0; k < b->branches; ++k) {
      BHIP(hipEventRecord(b->done[k], b->aux[k]));
      BHIP(hipStreamWaitEvent(st, b->done[k], 0));
    }
  }
  BHIP(fr::launch_mcc(mcc_counts(b), nullptr, b->d_mcc, b->cap_mcc, st));
  for (int vi = 0; vi < nv; ++vi) {
    fr_status e = enqueue_generic(b, b->variants[vi], vi, st);
    if (e != FR_OK) return e;
  }
  BHIP(fr::launch_transpose_batch(b->d_jobs, b->d_params, b->d_tr_items, (int32_t)b->tr_items.size(),
                                  st));
  return FR_OK;
}

// Upper bound of the present levels of one of the job's neighbourhoods.
int job_level_cap(const fr_job& J) {
  const int S = 2 * J.kernel_radius + 1;
  const int C = S * S * S;
  const int ngb = J.disc_mode == FR_FBN ? (int)J.disc_value : 255;
  return std::min(ngb, C);
}

}  // namespace

namespace fr {

int32_t validate_job(const ::fr_job& J, int j, BatchJob* bj, int* lcap_out, char* msg,
                     size_t msg_len, bool need_out) {
#define VFAIL(code, ...)                      \
  do {                                        \
    snprintf(msg, msg_len, __VA_ARGS__);      \
    return code;                              \
  } while (0)
  if (J.nx <= 0 || J.ny <= 0 || J.nz <= 0) VFAIL(FR_E_ARG, "job %d: dims must be positive", j);
  const int64_t n = (int64_t)J.nx * J.ny * J.nz;
  if (n > INT32_MAX) VFAIL(FR_E_RANGE, "job %d: volume exceeds 2^31-1 voxels", j);
  if (J.dtype != FR_I16 && J.dtype != FR_F32) VFAIL(FR_E_ARG, "job %d: dtype %d unknown", j, J.dtype);
  if (J.disc_mode != FR_FBW && J.disc_mode != FR_FBN)
    VFAIL(FR_E_ARG, "job %d: discretisation mode unknown", j);
  if (!(J.disc_value > 0.0) || !isfinite(J.disc_value))
    VFAIL(FR_E_ARG, "job %d: bin value must be finite and > 0", j);
  if (J.disc_mode == FR_FBN && (J.disc_value != floor(J.disc_value) || J.disc_value > 255.0))
    VFAIL(FR_E_RANGE, "job %d: bin count must be an integer in 1..255", j);
  for (int i = 0; i < 3; ++i)
    if (!(J.spacing_mm[i] > 0.0) || !isfinite(J.spacing_mm[i]))
      VFAIL(FR_E_ARG, "job %d: spacing_mm[%d] must be finite and > 0", j, i);
  if (J.kernel_radius < 1 || J.kernel_radius > FR_MAX_RADIUS)
    VFAIL(FR_E_RANGE, "job %d: kernel_radius %d outside 1..%d", j, J.kernel_radius, FR_MAX_RADIUS);
  if (J.reserved != 0) VFAIL(FR_E_ARG, "job %d: reserved field must be 0", j);
  if (J.families == 0 || (J.families & ~(uint32_t)FR_ALL))
    VFAIL(FR_E_RANGE, "job %d: families mask 0x%x invalid", j, J.families);
  if (J.n_mask <= 0 || J.n_mask > n) VFAIL(FR_E_ARG, "job %d: n_mask out of range", j);
  if (!J.volume || !J.mask) VFAIL(FR_E_ARG, "job %d: volume and mask are required", j);
  const int32_t count = map_count_of(J.families);
  if (need_out) {
    if (J.out_capacity_floats < (int64_t)count * J.n_mask)
      VFAIL(FR_E_CAPACITY, "job %d: out_maps holds %lld floats, %lld needed", j,
            (long long)J.out_capacity_floats, (long long)count * J.n_mask);
    const void* ptrs[3] = {J.volume, J.mask, J.out_maps};
    const char* names[3] = {"volume", "mask", "out_maps"};
    for (int q = 0; q < 3; ++q) {
      if (!ptrs[q]) VFAIL(FR_E_ARG, "job %d: %s is NULL", j, names[q]);
      hipPointerAttribute_t at;
      if (hipPointerGetAttributes(&at, ptrs[q]) != hipSuccess) {
        (void)hipGetLastError();
        VFAIL(FR_E_ARG, "job %d: %s is not a HIP device pointer", j, names[q]);
      }
      if (at.type != hipMemoryTypeDevice && at.type != hipMemoryTypeManaged)
        VFAIL(FR_E_ARG, "job %d: %s is not device memory", j, names[q]);
    }
  }
#undef VFAIL
  BatchJob& B = *bj;
  B = BatchJob{};
  B.vol = J.volume;
  B.mask = J.mask;
  B.out = J.out_maps;
  B.nvox = n;
  B.n_mask = J.n_mask;
  B.nx = J.nx;
  B.ny = J.ny;
  B.nz = J.nz;
  B.dtype = J.dtype;
  B.mode = J.disc_mode;
  B.radius = J.kernel_radius;
  B.lcap = job_level_cap(J);
  B.count = count;
  B.value = J.disc_value;
  B.lower = J.disc_lower;
  B.voxel_volume = J.spacing_mm[0] * J.spacing_mm[1] * J.spacing_mm[2];
  B.families = J.families;
  B.seg_base = 0;
  B.nseg = (int32_t)((n + kDiscSeg - 1) / kDiscSeg);
  B.opt.glcm_dist = 1;
  B.opt.gldm_alpha = 0;
  B.opt.averaged = 0;
  B.opt.reserved = 0;
  *lcap_out = B.lcap;
  return FR_OK;
}

void tuned_settings(int dtype, int radius, int lcap, int* vpw, int* grid_mult, int* kernel_lmax) {
  Tuning t;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_tuned.find(std::make_tuple(dtype, radius, level_class(lcap)));
    if (it != g_tuned.end()) t = it->second;
  }
  *vpw = t.vpw;
  *grid_mult = t.grid_mult;
  *kernel_lmax = radius == 1 ? 32 : t.kernel_lmax;
}

}  // namespace fr

extern "C" {

fr_status fr_batch_create(fr_batch* out) {
  g_berr.clear();
  if (!out) return bfail(FR_E_ARG, "out is NULL");
  fr_batch_s* b = new (std::nothrow) fr_batch_s();
  if (!b) return bfail(FR_E_NOMEM, "host allocation failed");
  if (hipGetDevice(&b->device) != hipSuccess) {
    delete b;
    return bfail(FR_E_DEVICE, "hipGetDevice failed");
  }
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, b->device) != hipSuccess) {
    delete b;
    return bfail(FR_E_DEVICE, "hipGetDeviceProperties failed");
  }
  b->n_cu = prop.multiProcessorCount;
  *out = b;
  return FR_OK;
}

fr_status fr_batch_destroy(fr_batch b) {
  g_berr.clear();
  if (!b) return FR_OK;
  drop_graph(b);
  free_workspace(b);
  delete b;
  return FR_OK;
}

fr_status fr_batch_prepare(fr_batch b, const fr_job* jobs, int32_t n_jobs) {
  g_berr.clear();
  if (!b || !jobs || n_jobs <= 0) return bfail(FR_E_ARG, "batch, jobs and n_jobs > 0 are required");
  drop_graph(b);
  free_workspace(b);
  b->prepared = false;
  b->jobs.assign(jobs, jobs + n_jobs);
  b->bj.assign(n_jobs, fr::BatchJob{});
  int64_t seg = 0, vox = 0, mvox = 0;
  std::map<std::tuple<int, int, int>, int> vindex;
  fr_status st;
  for (int j = 0; j < n_jobs; ++j) {
    const fr_job& J = jobs[j];
    fr::BatchJob& B = b->bj[j];
    int lcap = 0;
    char msg[256];
    if ((st = fr::validate_job(J, j, &B, &lcap, msg, sizeof msg, true)) != FR_OK)
      return bfail(st, "%s", msg);
    const int64_t n = B.nvox;
    // offsets into the batch buffers (pointers set after allocation)
    B.levels = (uint8_t*)(uintptr_t)vox;
    B.list = (int32_t*)(uintptr_t)mvox;
    B.seg_base = (int32_t)seg;
    seg += B.nseg;
    vox += n;
    mvox += J.n_mask;
    // the level class separates jobs whose neighbourhoods may hold more than
    // 32 levels, so each class gets its own first-pass instance
    const int lclass = J.kernel_radius > 3 ? 0 : level_class(lcap);
    const auto key = std::make_tuple(J.dtype, J.kernel_radius, lclass);
    auto it = vindex.find(key);
    if (it == vindex.end()) {
      Variant v;
      v.dtype = J.dtype;
      v.radius = J.kernel_radius;
      v.generic = J.kernel_radius > 3;
      vindex[key] = (int)b->variants.size();
      b->variants.push_back(v);
      it = vindex.find(key);
    }
    Variant& v = b->variants[it->second];
    v.jobs.push_back(j);
    v.lcap = std::max(v.lcap, lcap);
    v.n_vox += J.n_mask;
  }
  for (auto& v : b->variants) {
    v.lclass = v.generic ? 0 : level_class(v.lcap);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto t = g_tuned.find(std::make_tuple(v.dtype, v.radius, v.lclass));
    if (t != g_tuned.end()) v.tune = t->second;
    if (v.radius == 1) v.tune.kernel_lmax = 32;
    if (v.generic || (v.radius >= 2 && v.lcap > 64)) b->lcap_generic = std::max(b->lcap_generic, v.lcap);
  }
  b->n_seg = seg;
  if (seg > INT32_MAX) return bfail(FR_E_RANGE, "batch too large");
  // device workspace
  auto dal = [&](void** p, size_t bytes) { return hipMalloc(p, bytes ? bytes : 1) == hipSuccess; };
  const int nv = (int)b->variants.size();
  if (!dal((void**)&b->d_jobs, sizeof(fr::BatchJob) * n_jobs) ||
      !dal((void**)&b->d_params, sizeof(fr::DiscParams) * n_jobs) ||
      !dal((void**)&b->d_seg_job, sizeof(int32_t) * seg) || !dal((void**)&b->d_bcount, sizeof(int32_t) * seg) ||
      !dal((void**)&b->d_boff, sizeof(int64_t) * seg) || !dal((void**)&b->d_bmin, sizeof(double) * seg) ||
      !dal((void**)&b->d_bmax, sizeof(double) * seg) || !dal((void**)&b->d_levels, (size_t)vox) ||
      !dal((void**)&b->d_lists, sizeof(int32_t) * mvox) ||
      !dal((void**)&b->d_stage, sizeof(float) * fr::kStageStride * mvox) ||
      !dal((void**)&b->d_counters, sizeof(int32_t) * (kCountersPerVariant * nv + 2)) ||
      (b->lcap_generic > 0 &&
       !dal(&b->d_gscratch, (size_t)fr::kGenericGrid * fr::generic_scratch_bytes(b->lcap_generic)))) {
    free_workspace(b);
    return bfail(FR_E_NOMEM, "batch workspace allocation failed (%lld voxels, %lld mask voxels)",
                 (long long)vox, (long long)mvox);
  }
  for (auto& v : b->variants) {
    if (v.generic) continue;
    if (!dal((void**)&v.d_over[0], sizeof(int2) * v.n_vox) || !dal((void**)&v.d_over[1], sizeof(int2) * v.n_vox)) {
      free_workspace(b);
      return bfail(FR_E_NOMEM, "overflow-list allocation failed");
    }
    b->cap_mcc += v.n_vox;
  }
  if (!dal((void**)&b->d_mcc, (size_t)b->cap_mcc * fr::kMccProblemBytes)) {
    free_workspace(b);
    return bfail(FR_E_NOMEM, "MCC stash allocation failed (%lld problems)", (long long)b->cap_mcc);
  }
  for (int k = 0; k < kMaxBranches; ++k) {
    if (hipStreamCreateWithFlags(&b->aux[k], hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&b->done[k], hipEventDisableTiming) != hipSuccess) {
      free_workspace(b);
      return bfail(FR_E_DEVICE, "branch stream/event creation failed");
    }
  }
  {
    int fast = 0;
    for (auto& v : b->variants) fast += !v.generic;
    b->branches = std::max(1, std::min({b->branches, fast, kMaxBranches}));
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      if (g_branches_tuned > 0) b->branches = std::max(1, std::min({g_branches_tuned, fast, kMaxBranches}));
    }
    assign_branches(b);
  }
  if (hipEventCreateWithFlags(&b->fork, hipEventDisableTiming) != hipSuccess) {
    free_workspace(b);
    return bfail(FR_E_DEVICE, "event creation failed");
  }
  if (hipHostMalloc((void**)&b->h_params, sizeof(fr::DiscParams) * n_jobs, hipHostMallocDefault) != hipSuccess) {
    free_workspace(b);
    return bfail(FR_E_NOMEM, "pinned allocation failed");
  }
  std::vector<int32_t> seg_job(seg);
  b->tr_items.clear();
  int64_t mstage = 0;
  for (int j = 0; j < n_jobs; ++j) {
    fr::BatchJob& B = b->bj[j];
    B.levels = b->d_levels + (int64_t)(uintptr_t)B.levels;
    B.list = b->d_lists + (int64_t)(uintptr_t)B.list;
    B.stage = b->d_stage + mstage * fr::kStageStride;
    mstage += B.n_mask;
    for (int s2 = 0; s2 < B.nseg; ++s2) seg_job[B.seg_base + s2] = j;
    for (int64_t m = 0; m < B.n_mask; m += 64) b->tr_items.push_back(make_int2(j, (int)m));
  }
  BHIP(hipMemcpy(b->d_jobs, b->bj.data(), sizeof(fr::BatchJob) * n_jobs, hipMemcpyHostToDevice));
  BHIP(hipMemcpy(b->d_seg_job, seg_job.data(), sizeof(int32_t) * seg, hipMemcpyHostToDevice));
  if (!dal((void**)&b->d_tr_items, sizeof(int2) * b->tr_items.size())) {
    free_workspace(b);
    return bfail(FR_E_NOMEM, "transpose table allocation failed");
  }
  BHIP(hipMemcpy(b->d_tr_items, b->tr_items.data(), sizeof(int2) * b->tr_items.size(),
                 hipMemcpyHostToDevice));
  for (auto& v : b->variants)
    if ((st = build_items(b, v)) != FR_OK) return st;
  b->prepared = true;
  return FR_OK;
}

fr_status fr_batch_launch(fr_batch b, void* hip_stream, int32_t use_graph) {
  g_berr.clear();
  if (!b || !b->prepared) return bfail(FR_E_ARG, "batch not prepared");
  hipStream_t st = (hipStream_t)hip_stream;
  if (!use_graph) return enqueue(b, st);
  if (!st) return bfail(FR_E_ARG, "graph replay needs a non-null stream");
  if (b->exec && b->graph_stream != st) drop_graph(b);
  if (!b->exec) {
    BHIP(hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal));
    fr_status e = enqueue(b, st);
    hipGraph_t g = nullptr;
    hipError_t he = hipStreamEndCapture(st, &g);
    if (e != FR_OK) {
      if (g) (void)hipGraphDestroy(g);
      return e;
    }
    if (he != hipSuccess) return bfail(FR_E_DEVICE, "stream capture failed: %s", hipGetErrorString(he));
    b->graph = g;
    BHIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
    b->graph_stream = st;
  }
  BHIP(hipGraphLaunch(b->exec, st));
  return FR_OK;
}

fr_status fr_batch_status(fr_batch b, int32_t* job_status, int32_t* ng, void* hip_stream) {
  g_berr.clear();
  if (!b || !b->prepared) return bfail(FR_E_ARG, "batch not prepared");
  const int n = (int)b->jobs.size();
  hipStream_t st = (hipStream_t)hip_stream;
  BHIP(hipMemcpyAsync(b->h_params, b->d_params, sizeof(fr::DiscParams) * n, hipMemcpyDeviceToHost, st));
  BHIP(hipStreamSynchronize(st));
  int bad = 0;
  for (int j = 0; j < n; ++j) {
    int32_t code = FR_OK;
    switch (b->h_params[j].err) {
      case fr::kJobOk: code = FR_OK; break;
      case fr::kJobEmpty: code = FR_E_EMPTY_MASK; break;
      case fr::kJobCount: code = FR_E_ARG; break;
      default: code = FR_E_RANGE; break;
    }
    if (code != FR_OK) bad++;
    if (job_status) job_status[j] = code;
    if (ng) ng[j] = b->h_params[j].ng;
  }
  if (bad) return bfail(FR_E_RANGE, "%d job(s) failed on the device (see job_status)", bad);
  return FR_OK;
}

fr_status fr_batch_autotune(fr_batch b, void* hip_stream) {
  g_berr.clear();
  if (!b || !b->prepared) return bfail(FR_E_ARG, "batch not prepared");
  hipStream_t st = (hipStream_t)hip_stream;
  drop_graph(b);
  fr_status e = enqueue(b, st);  // levels and lists for the timing runs
  // the item tables are rewritten below (on the null stream, which does not
  // wait for non-blocking streams): the batch must have finished first
  BHIP(hipStreamSynchronize(st));
  if (e != FR_OK) return e;
  struct Events {
    hipEvent_t a = nullptr, b = nullptr;
    ~Events() {
      if (a) (void)hipEventDestroy(a);
      if (b) (void)hipEventDestroy(b);
    }
  } ev;
  BHIP(hipEventCreate(&ev.a));
  BHIP(hipEventCreate(&ev.b));
  hipEvent_t e0 = ev.a, e1 = ev.b;
  const int nv = (int)b->variants.size();
  for (int vi = 0; vi < nv; ++vi) {
    Variant& v = b->variants[vi];
    if (v.generic) continue;
    Tuning best = v.tune;
    float best_ms = 1e30f;
    const int vpws[] = {2, 4, 8, 16};
    const int mults[] = {1, 2};
    const int caps[] = {32, 64};
    for (int cap : caps)
      for (int vpw : vpws)
        for (int mult : mults) {
          if (cap == 64 && v.radius == 1) continue;  // radius 1 has one instance
          v.tune.kernel_lmax = cap;
          v.tune.vpw = vpw;
          v.tune.grid_mult = mult;
          if ((e = build_items(b, v)) != FR_OK) return e;
          float ms = 0.f;
          for (int rep = 0; rep < 2; ++rep) {  // second run is the one kept
            BHIP(fr::launch_zero_i32(b->d_counters + kCountersPerVariant * vi, kCountersPerVariant, st));
            BHIP(fr::launch_zero_i32(mcc_counts(b), 2, st));
            BHIP(hipEventRecord(e0, st));
            if ((e = enqueue_fast(b, v, vi, st)) != FR_OK) return e;
            // the MCC problems this variant stashed belong to its time
            BHIP(fr::launch_mcc(mcc_counts(b), nullptr, b->d_mcc, b->cap_mcc, st));
            BHIP(hipEventRecord(e1, st));
            BHIP(hipEventSynchronize(e1));
            BHIP(hipEventElapsedTime(&ms, e0, e1));
          }
          if (ms < best_ms) {
            best_ms = ms;
            best = v.tune;
          }
        }
    v.tune = best;
    if ((e = build_items(b, v)) != FR_OK) return e;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[std::make_tuple(v.dtype, v.radius, v.lclass)] = best;
  }
  // the number of concurrent branches: the whole batch timed per choice
  {
    int fast = 0;
    for (auto& v : b->variants) fast += !v.generic;
    int best_k = b->branches;
    float best_ms = 1e30f;
    for (int k = 1; k <= std::min(fast, kMaxBranches); ++k) {
      b->branches = k;
      assign_branches(b);
      float ms = 0.f;
      for (int rep = 0; rep < 2; ++rep) {
        BHIP(hipEventRecord(e0, st));
        if ((e = enqueue(b, st)) != FR_OK) return e;
        BHIP(hipEventRecord(e1, st));
        BHIP(hipEventSynchronize(e1));
        BHIP(hipEventElapsedTime(&ms, e0, e1));
      }
      if (ms < best_ms) {
        best_ms = ms;
        best_k = k;
      }
    }
    b->branches = std::max(best_k, 1);
    assign_branches(b);
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_branches_tuned = b->branches;
  }
  // the outputs of the batch as tuned
  if ((e = enqueue(b, st)) != FR_OK) return e;
  BHIP(hipStreamSynchronize(st));
  return FR_OK;
}

fr_status fr_batch_describe(fr_batch b, int32_t* n_variants, int32_t* table, int32_t table_len) {
  g_berr.clear();
  if (!b || !b->prepared) return bfail(FR_E_ARG, "batch not prepared");
  if (n_variants) *n_variants = (int32_t)b->variants.size();
  if (table)
    for (size_t i = 0; i < b->variants.size() && (int32_t)(i * 8 + 7) < table_len; ++i) {
      const Variant& v = b->variants[i];
      int32_t* t = table + i * 8;
      t[0] = v.dtype;
      t[1] = v.radius;
      t[2] = v.lcap;
      t[3] = (int32_t)v.jobs.size();
      t[4] = v.n_items;
      t[5] = v.generic ? 1 : v.tune.vpw;
      t[6] = v.grid;
      t[7] = v.generic ? 0 : v.tune.kernel_lmax;
    }
  return FR_OK;
}

const char* fr_batch_last_error(void) { return g_berr.c_str(); }

}  // extern "C"
