// Batched spatial mapping (C ABI fr_batch_*): many VOIs of different sizes,
// radii and gray-level counts mapped by one enqueue with no host round trip.
//
// prepare  host validation; plans the batch-wide discretisation segment
//          table and the work items: per raw type, one list of (job, first
//          voxel) items over every job of radius 1..3, grouped by variant
//          (radius and level class) and ordered by estimated work, largest
//          first; generic variants (radii 4 and 5) keep lists of their own;
//          allocates the batch's own device workspace and uploads the
//          tables (synchronous, once).
// launch   enqueues, on the caller's stream: batched discretisation; per raw
//          type one fused persistent pass over all its items (every fixed
//          radius in one kernel, items from a work queue, the 32-level
//          instances, MCC problems stashed); per raw type one fused
//          64-level pass over the neighbourhoods with more present levels
//          (problems with <= 32 levels stashed too); one k_mcc over the
//          stash; the generic kernel over what remains and
//          over the generic variants; a batched transpose.  Optionally
//          captured once into a hipGraph and replayed.  Allocates nothing.
// status   per-job errors found on the device (mask count, Ng range), read
//          after the stream has synchronised.
// autotune times the voxels per work item of each variant on the prepared
//          batch and keeps the fastest (cached per process for later
//          batches and served jobs of the variant).
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
#include "fr_error.h"
#include "fr_internal.h"

namespace {


fr_status bfail(fr_status code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
fr_status bfail(fr_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  fr::set_error(buf);
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
  int grid_mult = 1;  // persistent grid = resident workgroups x grid_mult (served jobs)
  // local-level capacity of the first pass's instance (served jobs): 32
  // (the 64-level instance then takes the neighbourhoods with 33..64
  // present levels) or 64; array sizes only, so the maps do not change
  int kernel_lmax = 32;
};

// Tuned settings per (dtype, radius, level class 32 / 64), shared by every
// batch and served job.
std::mutex g_tune_mu;
std::map<std::tuple<int, int, int>, Tuning> g_tuned;

struct Variant {
  int dtype = 0, radius = 0;
  bool generic = false;  // radius above 3: the generic kernel maps every voxel
  int lcap = 1;          // largest present-level bound of its jobs
  int lclass = 32;       // 32 or 64: the tuning key's level class
  Tuning tune;
  std::vector<int> jobs;  // job indices
  int64_t n_vox = 0;      // mask voxels of its jobs
  int32_t n_items = 0;    // its work items (in its group's list, or its own)
  int2* d_items = nullptr;  // generic variants: their own item list
};

// The fixed-radius jobs of one raw type: one fused list of work items and
// the overflow lists of its two passes (one entry per voxel at most).
struct Group {
  int dtype = 0;
  std::vector<int> variants;  // fast variants, largest estimated work first
  int64_t n_vox = 0;
  int2* d_items = nullptr;
  int32_t n_items = 0;
  int32_t cap_items = 0;
  int2* d_over[2] = {nullptr, nullptr};
  bool need64 = false;       // some job may hold 33..64 present levels
  bool need_generic = false;  // some job may hold more than 64
  int grid32 = 0, grid64 = 0;
};
constexpr int kGroupCounters = 4;  // two overflow counts, two work-queue heads

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
  // per group: two overflow counts and two work-queue heads; then the two
  // MCC stash counts
  int32_t* d_counters = nullptr;
  void* d_gscratch = nullptr;     // generic-kernel scratch
  // MCC problems of the 32-level passes (one per fixed-radius voxel at
  // most), solved by one k_mcc launch
  unsigned char* d_mcc = nullptr;
  int64_t cap_mcc = 0;
  Group groups[2];                // FR_I16, FR_F32
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
  for (auto& v : b->variants) (void)hipFree(v.d_items);
  for (auto& g : b->groups) {
    (void)hipFree(g.d_items);
    (void)hipFree(g.d_over[0]);
    (void)hipFree(g.d_over[1]);
    g = Group{};
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

// Estimated work of a variant: mask voxels x cube size, doubled when more
// than 32 levels may be present.
double variant_cost(const Variant& v) {
  const double S = 2.0 * v.radius + 1.0;
  return (double)v.n_vox * S * S * S * (v.lcap > 32 ? 2.0 : 1.0);
}

// Uploads a list of work items into *d (grown as needed).
fr_status upload_items(const std::vector<int2>& items, int2** d, int32_t* cap) {
  if ((int64_t)items.size() > INT32_MAX) return bfail(FR_E_RANGE, "too many work items");
  if ((int32_t)items.size() > *cap) {
    (void)hipFree(*d);
    *d = nullptr;
    *cap = 0;
    if (hipMalloc((void**)d, std::max<size_t>(items.size(), 1) * sizeof(int2)) != hipSuccess)
      return bfail(FR_E_NOMEM, "work-item table allocation failed");
    *cap = (int32_t)items.size();
  }
  if (!items.empty())
    BHIP(hipMemcpy(*d, items.data(), items.size() * sizeof(int2), hipMemcpyHostToDevice));
  return FR_OK;
}

// The work items of a fast variant's jobs, vpw voxels each, job-major (so
// workgroups resident together map neighbouring voxels of one job).
void variant_items(const fr_batch_s* b, const Variant& v, int vpw, std::vector<int2>* items) {
  for (int j : v.jobs)
    for (int64_t m = 0; m < b->jobs[j].n_mask; m += vpw) items->push_back(make_int2(j, (int)m));
}

// Every job's work-item size from its variant's tuning, uploaded with the
// job table; then each group's fused item list (its variants in order) and
// each generic variant's own list (one voxel per item).
fr_status build_items(fr_batch_s* b) {
  for (auto& v : b->variants)
    for (int j : v.jobs) b->bj[j].vpw = v.generic ? 1 : v.tune.vpw;
  BHIP(hipMemcpy(b->d_jobs, b->bj.data(), sizeof(fr::BatchJob) * b->bj.size(), hipMemcpyHostToDevice));
  fr_status e;
  for (auto& g : b->groups) {
    std::vector<int2> items;
    for (int vi : g.variants) {
      Variant& v = b->variants[vi];
      const size_t before = items.size();
      variant_items(b, v, v.tune.vpw, &items);
      v.n_items = (int32_t)(items.size() - before);
    }
    if ((e = upload_items(items, &g.d_items, &g.cap_items)) != FR_OK) return e;
    g.n_items = (int32_t)items.size();
  }
  for (auto& v : b->variants) {
    if (!v.generic) continue;
    std::vector<int2> items;
    variant_items(b, v, 1, &items);
    int32_t cap = 0;
    (void)hipFree(v.d_items);
    v.d_items = nullptr;
    if ((e = upload_items(items, &v.d_items, &cap)) != FR_OK) return e;
    v.n_items = (int32_t)items.size();
  }
  return FR_OK;
}

int32_t* group_counters(fr_batch_s* b, int gi) { return b->d_counters + kGroupCounters * gi; }
// The two MCC stash counts, after the groups' counters.
int32_t* mcc_counts(fr_batch_s* b) { return b->d_counters + kGroupCounters * 2; }
constexpr int kCounters = kGroupCounters * 2 + 2;

// The fused first pass of group gi over n items of its list.
fr_status enqueue_first(fr_batch_s* b, int gi, int32_t n, hipStream_t st) {
  Group& g = b->groups[gi];
  int32_t* c = group_counters(b, gi);
  BHIP(fr::launch_map_fused(b->d_jobs, b->d_params, g.d_items, n, nullptr, g.dtype, 32, g.grid32, g.d_over[0],
                            c, c + 2, b->d_mcc, b->cap_mcc, mcc_counts(b), st));
  return FR_OK;
}

fr_status enqueue(fr_batch_s* b, hipStream_t st) {
  fr::DiscScratch s;
  s.nblocks = b->n_seg;
  s.block_count = b->d_bcount;
  s.block_offset = b->d_boff;
  s.block_min = b->d_bmin;
  s.block_max = b->d_bmax;
  s.params = b->d_params;
  BHIP(fr::launch_zero_i32(b->d_counters, kCounters, st));
  BHIP(fr::launch_discretise_batch(b->d_jobs, (int32_t)b->jobs.size(), b->d_seg_job, b->n_seg, s, st));
  fr_status e;
  for (int gi = 0; gi < 2; ++gi)
    if (b->groups[gi].n_items > 0 && (e = enqueue_first(b, gi, b->groups[gi].n_items, st)) != FR_OK) return e;
  for (int gi = 0; gi < 2; ++gi) {  // neighbourhoods with 33..64 present levels
    Group& g = b->groups[gi];
    if (!g.need64) continue;
    int32_t* c = group_counters(b, gi);
    BHIP(fr::launch_map_fused(b->d_jobs, b->d_params, g.d_over[0], 0, c, g.dtype, 64, g.grid64, g.d_over[1],
                              c + 1, c + 3, b->d_mcc, b->cap_mcc, mcc_counts(b), st));
  }
  BHIP(fr::launch_mcc(mcc_counts(b), nullptr, b->d_mcc, b->cap_mcc, st));
  fr::MapArgs none;
  memset(&none, 0, sizeof none);
  for (int gi = 0; gi < 2; ++gi) {  // and more than 64
    Group& g = b->groups[gi];
    if (!g.need_generic) continue;
    BHIP(fr::launch_map_generic(none, b->d_jobs, b->d_params, g.d_over[1], group_counters(b, gi) + 1, 0,
                                g.dtype, b->d_gscratch, b->lcap_generic, fr::kGenericGrid, st));
  }
  for (auto& v : b->variants) {
    if (!v.generic) continue;
    BHIP(fr::launch_map_generic(none, b->d_jobs, b->d_params, v.d_items, nullptr, v.n_items, v.dtype,
                                b->d_gscratch, b->lcap_generic, fr::kGenericGrid, st));
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
  fr::clear_error();
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
  fr::clear_error();
  if (!b) return FR_OK;
  drop_graph(b);
  free_workspace(b);
  delete b;
  return FR_OK;
}

fr_status fr_batch_prepare(fr_batch b, const fr_job* jobs, int32_t n_jobs) {
  fr::clear_error();
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
    if (v.generic || (v.radius >= 2 && v.lcap > 64)) b->lcap_generic = std::max(b->lcap_generic, v.lcap);
  }
  // groups: the fast variants of each raw type, largest estimated work first
  for (int gi = 0; gi < 2; ++gi) b->groups[gi].dtype = gi == 0 ? FR_I16 : FR_F32;
  {
    std::vector<int> order;
    for (int vi = 0; vi < (int)b->variants.size(); ++vi)
      if (!b->variants[vi].generic) order.push_back(vi);
    std::stable_sort(order.begin(), order.end(), [&](int x, int y) {
      return variant_cost(b->variants[x]) > variant_cost(b->variants[y]);
    });
    for (int vi : order) {
      const Variant& v = b->variants[vi];
      Group& g = b->groups[v.dtype == FR_I16 ? 0 : 1];
      g.variants.push_back(vi);
      g.n_vox += v.n_vox;
      g.need64 = g.need64 || (v.radius >= 2 && v.lcap > 32);
      g.need_generic = g.need_generic || (v.radius >= 2 && v.lcap > 64);
      b->cap_mcc += v.n_vox;
    }
  }
  b->n_seg = seg;
  if (seg > INT32_MAX) return bfail(FR_E_RANGE, "batch too large");
  // device workspace
  auto dal = [&](void** p, size_t bytes) { return hipMalloc(p, bytes ? bytes : 1) == hipSuccess; };
  if (!dal((void**)&b->d_jobs, sizeof(fr::BatchJob) * n_jobs) ||
      !dal((void**)&b->d_params, sizeof(fr::DiscParams) * n_jobs) ||
      !dal((void**)&b->d_seg_job, sizeof(int32_t) * seg) || !dal((void**)&b->d_bcount, sizeof(int32_t) * seg) ||
      !dal((void**)&b->d_boff, sizeof(int64_t) * seg) || !dal((void**)&b->d_bmin, sizeof(double) * seg) ||
      !dal((void**)&b->d_bmax, sizeof(double) * seg) || !dal((void**)&b->d_levels, (size_t)vox) ||
      !dal((void**)&b->d_lists, sizeof(int32_t) * mvox) ||
      !dal((void**)&b->d_stage, sizeof(float) * fr::kStageStride * mvox) ||
      !dal((void**)&b->d_counters, sizeof(int32_t) * kCounters) ||
      !dal((void**)&b->d_mcc, (size_t)b->cap_mcc * fr::kMccProblemBytes) ||
      (b->lcap_generic > 0 &&
       !dal(&b->d_gscratch, (size_t)fr::kGenericGrid * fr::generic_scratch_bytes(b->lcap_generic)))) {
    free_workspace(b);
    return bfail(FR_E_NOMEM, "batch workspace allocation failed (%lld voxels, %lld mask voxels)",
                 (long long)vox, (long long)mvox);
  }
  for (auto& g : b->groups) {
    if (g.variants.empty()) continue;
    if (!dal((void**)&g.d_over[0], sizeof(int2) * g.n_vox) || !dal((void**)&g.d_over[1], sizeof(int2) * g.n_vox)) {
      free_workspace(b);
      return bfail(FR_E_NOMEM, "overflow-list allocation failed");
    }
    g.grid32 = b->n_cu * fr::map_fused_blocks_per_cu(g.dtype, 32);
    g.grid64 = b->n_cu * fr::map_fused_blocks_per_cu(g.dtype, 64);
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
  BHIP(hipMemcpy(b->d_seg_job, seg_job.data(), sizeof(int32_t) * seg, hipMemcpyHostToDevice));
  if (!dal((void**)&b->d_tr_items, sizeof(int2) * b->tr_items.size())) {
    free_workspace(b);
    return bfail(FR_E_NOMEM, "transpose table allocation failed");
  }
  BHIP(hipMemcpy(b->d_tr_items, b->tr_items.data(), sizeof(int2) * b->tr_items.size(),
                 hipMemcpyHostToDevice));
  if ((st = build_items(b)) != FR_OK) return st;  // uploads the job table too
  b->prepared = true;
  return FR_OK;
}

fr_status fr_batch_launch(fr_batch b, void* hip_stream, int32_t use_graph) {
  fr::clear_error();
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
  fr::clear_error();
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
  fr::clear_error();
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
  // each fast variant alone: the fused first pass over its items (vpw
  // voxels each) and the MCC of the problems it stashed
  for (int vi = 0; vi < (int)b->variants.size(); ++vi) {
    Variant& v = b->variants[vi];
    if (v.generic) continue;
    const int gi = v.dtype == FR_I16 ? 0 : 1;
    Group& g = b->groups[gi];
    Tuning best = v.tune;
    float best_ms = 1e30f;
    const int vpws[] = {2, 4, 8, 16};
    for (int vpw : vpws) {
      for (int j : v.jobs) b->bj[j].vpw = vpw;
      BHIP(hipMemcpy(b->d_jobs, b->bj.data(), sizeof(fr::BatchJob) * b->bj.size(), hipMemcpyHostToDevice));
      std::vector<int2> items;
      variant_items(b, v, vpw, &items);
      if ((e = upload_items(items, &g.d_items, &g.cap_items)) != FR_OK) return e;
      float ms = 0.f;
      for (int rep = 0; rep < 2; ++rep) {  // second run is the one kept
        BHIP(fr::launch_zero_i32(b->d_counters, kCounters, st));
        BHIP(hipEventRecord(e0, st));
        if ((e = enqueue_first(b, gi, (int32_t)items.size(), st)) != FR_OK) return e;
        BHIP(fr::launch_mcc(mcc_counts(b), nullptr, b->d_mcc, b->cap_mcc, st));
        BHIP(hipEventRecord(e1, st));
        BHIP(hipEventSynchronize(e1));
        BHIP(hipEventElapsedTime(&ms, e0, e1));
      }
      if (ms < best_ms) {
        best_ms = ms;
        best = v.tune;
        best.vpw = vpw;
      }
    }
    v.tune = best;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tuned[std::make_tuple(v.dtype, v.radius, v.lclass)] = best;
  }
  if ((e = build_items(b)) != FR_OK) return e;
  // the outputs of the batch as tuned
  if ((e = enqueue(b, st)) != FR_OK) return e;
  BHIP(hipStreamSynchronize(st));
  return FR_OK;
}

fr_status fr_batch_describe(fr_batch b, int32_t* n_variants, int32_t* table, int32_t table_len) {
  fr::clear_error();
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
      t[6] = v.generic ? fr::kGenericGrid : b->groups[v.dtype == FR_I16 ? 0 : 1].grid32;
      t[7] = v.generic ? 0 : 32;
    }
  return FR_OK;
}

const char* fr_batch_last_error(void) { return fr::last_error(); }

}  // extern "C"
