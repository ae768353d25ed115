// Host side of the C ABI declared in include/fr.h: argument validation,
// the per-device scratch pool, launches and the map-name table.
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <mutex>
#include <string>
#include <vector>

#include "../../include/fr.h"
#include "fr_error.h"
#include "fr_internal.h"

namespace {

thread_local std::string g_err;

fr_status fail(fr_status code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
fr_status fail(fr_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(expr)                                                                  \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(FR_E_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_));         \
  } while (0)

// ------------------------------------------------------------------------
// Per-device scratch pool: level volume, mask-voxel list, block tables and a
// pinned parameter block.  Grown on demand, reused across calls.
// ------------------------------------------------------------------------
struct Pool {
  uint8_t* levels = nullptr;
  int32_t* list = nullptr;
  int64_t cap_vox = 0;
  int32_t* block_count = nullptr;
  int64_t* block_offset = nullptr;
  double* block_min = nullptr;
  double* block_max = nullptr;
  int64_t cap_blocks = 0;
  fr::DiscParams* params = nullptr;
  fr::DiscParams* host_params = nullptr;  // pinned
  float* stage = nullptr;                 // voxel-major map staging rows
  int64_t cap_stage = 0;                  // rows
  int2* over[2] = {nullptr, nullptr};     // overflow lists of the 32- and 64-level passes
  int64_t cap_over = 0;                   // entries per list
  void* gscratch = nullptr;               // generic-kernel scratch slices
  size_t cap_gscratch = 0;                // bytes
  unsigned char* mcc = nullptr;           // MCC problem stash of the 32-level pass
  int64_t cap_mcc = 0;                    // problems
};

std::mutex g_pool_mu;
std::vector<Pool> g_pools;

// A pool buffer is replaced by a larger one only after the device has
// finished the enqueued calls that may still use it (fr_map returns before
// its kernels run).  Growth is monotone, so this wait is rare.
void pool_drain() { (void)hipDeviceSynchronize(); }

fr_status pool_get(int64_t nvox, Pool** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_pool_mu);
  if ((int)g_pools.size() <= dev) g_pools.resize(dev + 1);
  Pool& p = g_pools[dev];
  if (!p.params) {
    if (hipMalloc((void**)&p.params, sizeof(fr::DiscParams)) != hipSuccess)
      return fail(FR_E_NOMEM, "hipMalloc of the parameter block failed");
    if (hipHostMalloc((void**)&p.host_params, sizeof(fr::DiscParams), hipHostMallocDefault) !=
        hipSuccess)
      return fail(FR_E_NOMEM, "hipHostMalloc of the parameter block failed");
  }
  if (nvox > p.cap_vox) {
    pool_drain();
    if (p.levels) (void)hipFree(p.levels);
    if (p.list) (void)hipFree(p.list);
    p.levels = nullptr;
    p.list = nullptr;
    p.cap_vox = 0;
    if (hipMalloc((void**)&p.levels, (size_t)nvox) != hipSuccess ||
        hipMalloc((void**)&p.list, (size_t)nvox * sizeof(int32_t)) != hipSuccess)
      return fail(FR_E_NOMEM, "scratch allocation of %lld voxels failed", (long long)nvox);
    p.cap_vox = nvox;
  }
  const int64_t nb = (nvox + fr::kDiscSeg - 1) / fr::kDiscSeg;
  if (nb > p.cap_blocks) {
    pool_drain();
    (void)hipFree(p.block_count);
    (void)hipFree(p.block_offset);
    (void)hipFree(p.block_min);
    (void)hipFree(p.block_max);
    p.cap_blocks = 0;
    if (hipMalloc((void**)&p.block_count, nb * sizeof(int32_t)) != hipSuccess ||
        hipMalloc((void**)&p.block_offset, nb * sizeof(int64_t)) != hipSuccess ||
        hipMalloc((void**)&p.block_min, nb * sizeof(double)) != hipSuccess ||
        hipMalloc((void**)&p.block_max, nb * sizeof(double)) != hipSuccess)
      return fail(FR_E_NOMEM, "scratch allocation of %lld block entries failed", (long long)nb);
    p.cap_blocks = nb;
  }
  *out = &p;
  return FR_OK;
}

fr_status pool_over(Pool* p, int64_t n) {
  if (n <= p->cap_over) return FR_OK;
  pool_drain();
  for (auto& o : p->over) {
    if (o) (void)hipFree(o);
    o = nullptr;
  }
  p->cap_over = 0;
  for (auto& o : p->over)
    if (hipMalloc((void**)&o, (size_t)n * sizeof(int2)) != hipSuccess)
      return fail(FR_E_NOMEM, "overflow-list allocation of %lld entries failed", (long long)n);
  p->cap_over = n;
  return FR_OK;
}

fr_status pool_gscratch(Pool* p, size_t bytes) {
  if (bytes <= p->cap_gscratch) return FR_OK;
  pool_drain();
  if (p->gscratch) (void)hipFree(p->gscratch);
  p->gscratch = nullptr;
  p->cap_gscratch = 0;
  if (hipMalloc(&p->gscratch, bytes) != hipSuccess)
    return fail(FR_E_NOMEM, "generic-kernel scratch of %zu bytes could not be allocated", bytes);
  p->cap_gscratch = bytes;
  return FR_OK;
}

fr_status pool_mcc(Pool* p, int64_t n) {
  if (n <= p->cap_mcc) return FR_OK;
  pool_drain();
  if (p->mcc) (void)hipFree(p->mcc);
  p->mcc = nullptr;
  p->cap_mcc = 0;
  if (hipMalloc((void**)&p->mcc, (size_t)n * fr::kMccProblemBytes) != hipSuccess)
    return fail(FR_E_NOMEM, "MCC stash of %lld problems could not be allocated", (long long)n);
  p->cap_mcc = n;
  return FR_OK;
}

fr_status pool_stage(Pool* p, int64_t rows) {
  if (rows <= p->cap_stage) return FR_OK;
  pool_drain();
  if (p->stage) (void)hipFree(p->stage);
  p->stage = nullptr;
  p->cap_stage = 0;
  if (hipMalloc((void**)&p->stage, (size_t)rows * fr::kStageStride * sizeof(float)) != hipSuccess)
    return fail(FR_E_NOMEM, "staging allocation of %lld voxel rows failed", (long long)rows);
  p->cap_stage = rows;
  return FR_OK;
}

// ------------------------------------------------------------------------
// Canonical map names (Table 2's spatial families, IBSI feature names).
// ------------------------------------------------------------------------
const char* const kFamily[6] = {"firstorder", "glcm", "glrlm", "glszm", "gldm", "ngtdm"};
const int kCount[6] = {18, 24, 16, 16, 14, 5};
const char* const kFeat[6][24] = {
    {"Energy", "TotalEnergy", "Entropy", "Minimum", "10Percentile", "90Percentile", "Maximum",
     "Mean", "Median", "InterquartileRange", "Range", "MeanAbsoluteDeviation",
     "RobustMeanAbsoluteDeviation", "RootMeanSquared", "Skewness", "Kurtosis", "Variance",
     "Uniformity"},
    {"Autocorrelation", "JointAverage", "ClusterProminence", "ClusterShade", "ClusterTendency",
     "Contrast", "Correlation", "DifferenceAverage", "DifferenceEntropy", "DifferenceVariance",
     "JointEnergy", "JointEntropy", "Imc1", "Imc2", "Idm", "MCC", "Idmn", "Id", "Idn",
     "InverseVariance", "MaximumProbability", "SumAverage", "SumEntropy", "SumSquares"},
    {"ShortRunEmphasis", "LongRunEmphasis", "GrayLevelNonUniformity",
     "GrayLevelNonUniformityNormalized", "RunLengthNonUniformity",
     "RunLengthNonUniformityNormalized", "RunPercentage", "GrayLevelVariance", "RunVariance",
     "RunEntropy", "LowGrayLevelRunEmphasis", "HighGrayLevelRunEmphasis",
     "ShortRunLowGrayLevelEmphasis", "ShortRunHighGrayLevelEmphasis",
     "LongRunLowGrayLevelEmphasis", "LongRunHighGrayLevelEmphasis"},
    {"SmallAreaEmphasis", "LargeAreaEmphasis", "GrayLevelNonUniformity",
     "GrayLevelNonUniformityNormalized", "SizeZoneNonUniformity",
     "SizeZoneNonUniformityNormalized", "ZonePercentage", "GrayLevelVariance", "ZoneVariance",
     "ZoneEntropy", "LowGrayLevelZoneEmphasis", "HighGrayLevelZoneEmphasis",
     "SmallAreaLowGrayLevelEmphasis", "SmallAreaHighGrayLevelEmphasis",
     "LargeAreaLowGrayLevelEmphasis", "LargeAreaHighGrayLevelEmphasis"},
    {"SmallDependenceEmphasis", "LargeDependenceEmphasis", "GrayLevelNonUniformity",
     "DependenceNonUniformity", "DependenceNonUniformityNormalized", "GrayLevelVariance",
     "DependenceVariance", "DependenceEntropy", "LowGrayLevelEmphasis", "HighGrayLevelEmphasis",
     "SmallDependenceLowGrayLevelEmphasis", "SmallDependenceHighGrayLevelEmphasis",
     "LargeDependenceLowGrayLevelEmphasis", "LargeDependenceHighGrayLevelEmphasis"},
    {"Coarseness", "Contrast", "Busyness", "Complexity", "Strength"}};

std::once_flag g_names_once;
std::vector<std::string> g_names[64];

void build_names() {
  for (uint32_t fam = 1; fam < 64; ++fam)
    for (int q = 0; q < 6; ++q)
      if (fam & (1u << q))
        for (int k = 0; k < kCount[q]; ++k)
          g_names[fam].push_back(std::string(kFamily[q]) + "_" + kFeat[q][k]);
}

// ------------------------------------------------------------------------
// Validation helpers.
// ------------------------------------------------------------------------
fr_status check_device_ptr(const void* p, const char* what) {
  if (!p) return fail(FR_E_ARG, "%s is NULL", what);
  hipPointerAttribute_t at;
  if (hipPointerGetAttributes(&at, p) != hipSuccess) {
    (void)hipGetLastError();
    return fail(FR_E_ARG, "%s is not a HIP device pointer", what);
  }
  if (at.type != hipMemoryTypeDevice && at.type != hipMemoryTypeManaged)
    return fail(FR_E_ARG, "%s is not device memory", what);
  return FR_OK;
}

fr_status check_volume_args(const void* volume, int32_t dtype, int32_t nx, int32_t ny,
                            int32_t nz, const uint8_t* mask, int32_t mode, double value) {
  if (nx <= 0 || ny <= 0 || nz <= 0) return fail(FR_E_ARG, "dims must be positive");
  const int64_t n = (int64_t)nx * ny * nz;
  if (n > INT32_MAX) return fail(FR_E_RANGE, "volume of %lld voxels exceeds 2^31-1", (long long)n);
  if (dtype != FR_I16 && dtype != FR_F32) return fail(FR_E_ARG, "dtype %d unknown", dtype);
  if (mode != FR_FBW && mode != FR_FBN) return fail(FR_E_ARG, "discretisation mode %d unknown", mode);
  if (!(value > 0.0) || !isfinite(value)) return fail(FR_E_ARG, "bin value must be finite and > 0");
  if (mode == FR_FBN && (value != floor(value) || value > 255.0))
    return fail(FR_E_RANGE, "bin count must be an integer in 1..255");
  fr_status st;
  if ((st = check_device_ptr(volume, "volume")) != FR_OK) return st;
  if ((st = check_device_ptr(mask, "mask")) != FR_OK) return st;
  return FR_OK;
}

// Parameter block of the last map or discretisation enqueued per device
// (fr_map_status reads it).
std::mutex g_last_mu;
std::vector<fr::DiscParams*> g_last_params;

fr_status note_params(fr::DiscParams* params) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  std::lock_guard<std::mutex> lk(g_last_mu);
  if ((int)g_last_params.size() <= dev) g_last_params.resize(dev + 1, nullptr);
  g_last_params[dev] = params;
  return FR_OK;
}

// Enqueue discretisation into `levels` (device) with the segment tables and
// parameter block of s; expect_count >= 0 adds the device check of the
// mask-voxel count.
fr_status enqueue_discretise_into(const void* volume, int32_t dtype, int32_t nx, int32_t ny,
                                  int32_t nz, const uint8_t* mask, int32_t mode, double value,
                                  double lower, uint8_t* levels, int32_t* list,
                                  const fr::DiscScratch& s, int64_t expect_count, hipStream_t st) {
  const int64_t n = (int64_t)nx * ny * nz;
  HIP_TRY(fr::launch_discretise(volume, dtype, n, mask, mode, value, lower, levels, list, s,
                                expect_count, st));
  return note_params(s.params);
}

fr_status enqueue_discretise(const void* volume, int32_t dtype, int32_t nx, int32_t ny, int32_t nz,
                             const uint8_t* mask, int32_t mode, double value, double lower,
                             uint8_t* levels, Pool* p, int64_t expect_count, hipStream_t st) {
  const int64_t n = (int64_t)nx * ny * nz;
  fr::DiscScratch s;
  s.nblocks = (n + fr::kDiscSeg - 1) / fr::kDiscSeg;
  s.block_count = p->block_count;
  s.block_offset = p->block_offset;
  s.block_min = p->block_min;
  s.block_max = p->block_max;
  s.params = p->params;
  return enqueue_discretise_into(volume, dtype, nx, ny, nz, mask, mode, value, lower, levels,
                                 p->list, s, expect_count, st);
}

// The status a device parameter block reports (message in fr_last_error).
fr_status params_status(const fr::DiscParams& d) {
  switch (d.err) {
    case fr::kJobOk: return FR_OK;
    case fr::kJobEmpty: return fail(FR_E_EMPTY_MASK, "the mask holds no voxel");
    case fr::kJobCount:
      return fail(FR_E_ARG, "n_mask does not match the %lld mask voxels", (long long)d.count);
    case fr::kJobNgRange:
      return fail(FR_E_RANGE, "fixed bin width gives more than 255 gray levels (Xmax %g, lower %g)",
                  d.xmax, d.lo);
    default: return fail(FR_E_RANGE, "device error code %d", d.err);
  }
}

// Read the parameter block back (synchronises the stream).
fr_status read_params(Pool* p, hipStream_t st, fr::DiscParams* out) {
  HIP_TRY(hipMemcpyAsync(p->host_params, p->params, sizeof(fr::DiscParams), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  *out = *p->host_params;
  return FR_OK;
}

// Discretise and wait for the parameters (fr_discretise, fr_map_matrices).
fr_status run_discretise(const void* volume, int32_t dtype, int32_t nx, int32_t ny, int32_t nz,
                         const uint8_t* mask, int32_t mode, double value, double lower,
                         uint8_t* levels, Pool* p, hipStream_t st, fr::DiscParams* out) {
  fr_status e = enqueue_discretise(volume, dtype, nx, ny, nz, mask, mode, value, lower, levels, p, -1, st);
  if (e != FR_OK) return e;
  if ((e = read_params(p, st, out)) != FR_OK) return e;
  if (out->count == 0) return fail(FR_E_EMPTY_MASK, "the mask holds no voxel");
  return params_status(*out);
}

// Event pairs around map-kernel launches, for fr_profile_read.
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<std::pair<hipEvent_t, hipEvent_t>> g_prof_pending;
std::vector<std::pair<hipEvent_t, hipEvent_t>> g_prof_free;

fr_status prof_begin(hipStream_t st, std::pair<hipEvent_t, hipEvent_t>* ev) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  if (g_prof_free.empty()) {
    hipEvent_t a, b;
    HIP_TRY(hipEventCreate(&a));
    HIP_TRY(hipEventCreate(&b));
    g_prof_free.push_back({a, b});
  }
  *ev = g_prof_free.back();
  g_prof_free.pop_back();
  HIP_TRY(hipEventRecord(ev->first, st));
  return FR_OK;
}

fr_status prof_end(hipStream_t st, const std::pair<hipEvent_t, hipEvent_t>& ev) {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  HIP_TRY(hipEventRecord(ev.second, st));
  g_prof_pending.push_back(ev);
  return FR_OK;
}

// Upper bound of the present levels of one neighbourhood: min(Ng bound, cube).
int level_cap(int32_t disc_mode, double disc_value, int32_t radius) {
  const int S = 2 * radius + 1;
  const int C = S * S * S;
  const int ngb = disc_mode == FR_FBN ? (int)disc_value : 255;
  return ngb < C ? ngb : C;
}

bool default_options(const fr::MapOptions& o) {
  return o.glcm_dist == 1 && o.gldm_alpha == 0 && o.averaged == 0;
}

fr_status check_options(const fr::MapOptions& o) {
  if (o.glcm_dist < 1 || o.glcm_dist > 2 * FR_MAX_RADIUS)
    return fail(FR_E_RANGE, "glcm_distance %d outside 1..%d", o.glcm_dist, 2 * FR_MAX_RADIUS);
  if (o.gldm_alpha < 0 || o.gldm_alpha > 254)
    return fail(FR_E_RANGE, "gldm_alpha %d outside 0..254", o.gldm_alpha);
  if (o.averaged != 0 && o.averaged != 1) return fail(FR_E_ARG, "aggregation must be 0 or 1");
  if (o.reserved != 0) return fail(FR_E_ARG, "options.reserved must be 0");
  return FR_OK;
}

// Options of the public struct (NULL = defaults).
fr_status read_options(const fr_map_options* in, fr::MapOptions* o) {
  o->glcm_dist = in ? in->glcm_distance : 1;
  o->gldm_alpha = in ? in->gldm_alpha : 0;
  o->averaged = in ? in->aggregation : 0;
  o->reserved = in ? in->reserved : 0;
  return check_options(*o);
}

// Device buffers of the map passes of one call.
struct PassBuffers {
  fr::DiscParams* params;  // the call's parameter block (overflow counters inside)
  int2* over[2];           // overflow lists (n_items entries each)
  void* gscratch;          // generic-kernel scratch: generic_grid slices
  int generic_grid;
  unsigned char* mcc;      // MCC stash of n_items problems (NULL: MCC in the map kernel)
};

// The call needs the generic kernel: radius above 3, non-default options,
// or neighbourhoods that may hold more than 64 present levels.
bool needs_generic(int32_t radius, const fr::MapOptions& opt, int lcap) {
  return radius > 3 || !default_options(opt) || (radius >= 2 && lcap > 64);
}

// Enqueue the map passes for a.n_items items (a.params, a.list, a.out or
// a.stage set): the 32-level instance over every voxel, the 64-level one over
// the voxels it hands on, the generic kernel over the rest (only the passes
// the level bound can need); radii above 3 and non-default options run
// entirely on the generic kernel.
fr_status enqueue_map_passes(fr::MapArgs a, int32_t dtype, int32_t radius, int lcap, bool debug,
                             const PassBuffers& pb, hipStream_t stream) {
  const bool fast = radius <= 3 && default_options(a.opt);
  if (fast) {
    a.items = nullptr;
    a.items_count = nullptr;
    a.over = pb.over[0];
    a.over_count = &pb.params->n_over[0];
    a.over_job = 0;
    a.mcc = debug ? nullptr : pb.mcc;
    a.mcc_cap = a.n_items;
    a.mcc_count = pb.params->n_mcc;
    HIP_TRY(fr::launch_map(a, dtype, radius, 32, debug, stream));
    if (radius >= 2 && lcap > 32) {
      // the 64-level instance stashes its problems with <= 32 levels in the
      // same stash (a voxel reaches one pass only) and solves wider ones
      fr::MapArgs b = a;
      b.items = pb.over[0];
      b.items_count = &pb.params->n_over[0];
      b.over = pb.over[1];
      b.over_count = &pb.params->n_over[1];
      HIP_TRY(fr::launch_map(b, dtype, radius, 64, debug, stream));
      if (lcap > 64)
        HIP_TRY(fr::launch_map_generic(a, nullptr, nullptr, pb.over[1], &pb.params->n_over[1], 0,
                                       dtype, pb.gscratch, lcap, pb.generic_grid, stream));
    }
    if (a.mcc) HIP_TRY(fr::launch_mcc(pb.params->n_mcc, &pb.params->err, a.mcc, a.mcc_cap, stream));
  } else {
    HIP_TRY(fr::launch_map_generic(a, nullptr, nullptr, nullptr, nullptr, (int32_t)a.n_items, dtype,
                                   pb.gscratch, lcap, pb.generic_grid, stream));
  }
  return FR_OK;
}

fr_status map_common(const void* volume, int32_t dtype, int32_t nx, int32_t ny, int32_t nz,
                     const uint8_t* mask, const double* spacing_mm, int32_t disc_mode,
                     double disc_value, double disc_lower, int32_t kernel_radius,
                     uint32_t families, const fr::MapOptions& opt, int64_t n_mask,
                     const int64_t* sample, int64_t n_sample, int32_t ng_expected, int32_t* glcm,
                     int32_t* glrlm, int32_t* glszm, int32_t* gldm, int32_t* ngtdm_n,
                     int64_t* ngtdm_S, int32_t* hist, float* out_maps, int64_t out_capacity_floats,
                     void* hip_stream) {
  const bool debug = sample != nullptr;
  fr_status st = check_volume_args(volume, dtype, nx, ny, nz, mask, disc_mode, disc_value);
  if (st != FR_OK) return st;
  if (!spacing_mm) return fail(FR_E_ARG, "spacing_mm is NULL");
  for (int i = 0; i < 3; ++i)
    if (!(spacing_mm[i] > 0.0) || !isfinite(spacing_mm[i]))
      return fail(FR_E_ARG, "spacing_mm[%d] must be finite and > 0", i);
  if (kernel_radius < 1 || kernel_radius > FR_MAX_RADIUS)
    return fail(FR_E_RANGE, "kernel_radius %d outside 1..%d", kernel_radius, FR_MAX_RADIUS);
  if (families == 0 || (families & ~(uint32_t)FR_ALL))
    return fail(FR_E_RANGE, "families mask 0x%x invalid", families);
  if ((st = check_options(opt)) != FR_OK) return st;
  if (n_mask <= 0) return fail(FR_E_EMPTY_MASK, "n_mask must be positive");
  const int64_t nvox = (int64_t)nx * ny * nz;
  if (n_mask > nvox) return fail(FR_E_ARG, "n_mask %lld exceeds the volume", (long long)n_mask);
  const int32_t count = fr_map_count(families);
  const int64_t n_items = debug ? n_sample : n_mask;
  if (debug && n_sample <= 0) return fail(FR_E_ARG, "n_sample must be positive");
  if (!debug && out_capacity_floats < (int64_t)count * n_mask)
    return fail(FR_E_CAPACITY, "out_maps holds %lld floats, %lld needed",
                (long long)out_capacity_floats, (long long)count * n_mask);
  if ((st = check_device_ptr(out_maps, "out_maps")) != FR_OK) return st;
  if (debug) {
    const void* ptrs[] = {sample, glcm, glrlm, glszm, gldm, ngtdm_n, ngtdm_S, hist};
    const char* names[] = {"sample", "glcm", "glrlm", "glszm", "gldm", "ngtdm_n", "ngtdm_S", "hist"};
    for (int i = 0; i < 8; ++i)
      if ((st = check_device_ptr(ptrs[i], names[i])) != FR_OK) return st;
  }
  Pool* p = nullptr;
  if ((st = pool_get(nvox, &p)) != FR_OK) return st;
  if ((st = pool_over(p, n_items)) != FR_OK) return st;
  if (!debug && (st = pool_stage(p, n_items)) != FR_OK) return st;
  hipStream_t stream = (hipStream_t)hip_stream;
  const int S = 2 * kernel_radius + 1;
  const int C = S * S * S;
  if (debug) {
    // the dense tables are sized by the caller's Ng: check it before mapping
    fr::DiscParams dp;
    if ((st = run_discretise(volume, dtype, nx, ny, nz, mask, disc_mode, disc_value, disc_lower,
                             p->levels, p, stream, &dp)) != FR_OK)
      return st;
    if (dp.count != n_mask)
      return fail(FR_E_ARG, "n_mask %lld does not match the %lld mask voxels", (long long)n_mask,
                  (long long)dp.count);
    if (ng_expected != dp.ng)
      return fail(FR_E_ARG, "ng_expected %d but the VOI has Ng %d", ng_expected, dp.ng);
    const int64_t ng = dp.ng;
    HIP_TRY(hipMemsetAsync(glcm, 0, n_sample * ng * ng * sizeof(int32_t), stream));
    HIP_TRY(hipMemsetAsync(glrlm, 0, n_sample * ng * S * sizeof(int32_t), stream));
    HIP_TRY(hipMemsetAsync(glszm, 0, n_sample * ng * C * sizeof(int32_t), stream));
    HIP_TRY(hipMemsetAsync(gldm, 0, n_sample * ng * 27 * sizeof(int32_t), stream));
    HIP_TRY(hipMemsetAsync(ngtdm_n, 0, n_sample * ng * sizeof(int32_t), stream));
    HIP_TRY(hipMemsetAsync(ngtdm_S, 0, n_sample * ng * sizeof(int64_t), stream));
    HIP_TRY(hipMemsetAsync(hist, 0, n_sample * ng * sizeof(int32_t), stream));
  } else {
    // no host synchronisation: the mask count and Ng are checked on the
    // device, and every later kernel stops on an error (fr_map_status)
    if ((st = enqueue_discretise(volume, dtype, nx, ny, nz, mask, disc_mode, disc_value, disc_lower,
                                 p->levels, p, n_mask, stream)) != FR_OK)
      return st;
  }

  fr::MapArgs a;
  memset(&a, 0, sizeof a);
  a.params = p->params;
  a.vol = volume;
  a.levels = p->levels;
  a.list = p->list;
  a.sample = sample;
  a.out = out_maps;
  a.stage = debug ? nullptr : p->stage;
  a.n_out = n_items;
  a.n_items = n_items;
  a.n_list = n_mask;
  a.nx = nx;
  a.ny = ny;
  a.nz = nz;
  a.families = families;
  a.count = count;
  a.voxel_volume = spacing_mm[0] * spacing_mm[1] * spacing_mm[2];
  a.nblk = 0;  // chosen by the launcher from the instance's occupancy
  a.radius = kernel_radius;
  a.opt = opt;
  if (debug) {
    a.d_glcm = glcm;
    a.d_glrlm = glrlm;
    a.d_glszm = glszm;
    a.d_gldm = gldm;
    a.d_ngn = ngtdm_n;
    a.d_ngS = ngtdm_S;
    a.d_hist = hist;
  }
  bool prof;
  {
    std::lock_guard<std::mutex> lk(g_prof_mu);
    prof = g_prof_on && !debug;
  }
  const int lcap = level_cap(disc_mode, disc_value, kernel_radius);
  if (needs_generic(kernel_radius, opt, lcap) &&
      (st = pool_gscratch(p, (size_t)fr::kGenericGrid * fr::generic_scratch_bytes(lcap))) != FR_OK)
    return st;
  if (!debug && kernel_radius <= 3 && default_options(opt) && (st = pool_mcc(p, n_items)) != FR_OK)
    return st;
  const PassBuffers pb = {p->params, {p->over[0], p->over[1]}, p->gscratch, fr::kGenericGrid,
                          debug ? nullptr : p->mcc};
  std::pair<hipEvent_t, hipEvent_t> ev;
  if (prof && (st = prof_begin(stream, &ev)) != FR_OK) return st;
  if ((st = enqueue_map_passes(a, dtype, kernel_radius, lcap, debug, pb, stream)) != FR_OK) return st;
  if (prof && (st = prof_end(stream, ev)) != FR_OK) return st;
  if (!debug) HIP_TRY(fr::launch_transpose(p->stage, out_maps, n_items, count, p->params, stream));
  return FR_OK;
}

// ------------------------------------------------------------------------
// Allocation-free mapping (fr_map_noalloc): every buffer of the call lives
// in one fixed device array, resolved per device at the first call.
// ------------------------------------------------------------------------
constexpr size_t kNoAllocBytes = FR_NOALLOC_SCRATCH_BYTES;
constexpr int kNoAllocGenericGrid = 8;  // generic-kernel slices (rarely needed)
constexpr int kMaxDevices = 64;

std::mutex g_noalloc_mu;
void* g_noalloc_ptr[kMaxDevices] = {};

struct NoAllocLayout {
  size_t params, bcount, boff, bmin, bmax, levels, list, over0, over1, stage, gscratch, total;
  bool staged;  // staging rows + transpose (else direct map-major stores)
};

size_t na_align(size_t x) { return (x + 255) / 256 * 256; }

NoAllocLayout noalloc_layout(int64_t nvox, int64_t n_mask, bool staged, size_t gscratch) {
  NoAllocLayout L;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = na_align(o + bytes);
    return at;
  };
  const size_t nseg = (size_t)((nvox + fr::kDiscSeg - 1) / fr::kDiscSeg);
  L.params = take(sizeof(fr::DiscParams));
  L.bcount = take(nseg * sizeof(int32_t));
  L.boff = take(nseg * sizeof(int64_t));
  L.bmin = take(nseg * sizeof(double));
  L.bmax = take(nseg * sizeof(double));
  L.levels = take((size_t)nvox);
  L.list = take((size_t)n_mask * sizeof(int32_t));
  L.over0 = take((size_t)n_mask * sizeof(int2));
  L.over1 = take((size_t)n_mask * sizeof(int2));
  L.stage = take(staged ? (size_t)n_mask * fr::kStageStride * sizeof(float) : 0);
  L.gscratch = take(gscratch);
  L.total = o;
  L.staged = staged;
  return L;
}

}  // namespace

// The allocation-free entry point's scratch: one array per device that
// loads the library, held until the process ends.  Host code uses only the
// address hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {

fr_status noalloc_scratch(unsigned char** out) {
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(FR_E_DEVICE, "device ordinal %d out of range", dev);
  std::lock_guard<std::mutex> lk(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* ptr = nullptr;
    const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return fail(FR_E_DEVICE, "hipGetSymbolAddress of the scratch array failed: %s",
                  hipGetErrorString(e));
    g_noalloc_ptr[dev] = ptr;
  }
  *out = (unsigned char*)g_noalloc_ptr[dev];
  return FR_OK;
}

}  // namespace

namespace fr {
void set_error(const char* msg) { g_err = msg; }
void clear_error() { g_err.clear(); }
const char* last_error() { return g_err.c_str(); }
}  // namespace fr

extern "C" {

fr_status fr_discretise(const void* volume, int32_t dtype, int32_t nx, int32_t ny, int32_t nz,
                        const uint8_t* mask, int32_t disc_mode, double disc_value,
                        double disc_lower, uint8_t* levels, int32_t* ng, double* xmin,
                        double* xmax, int64_t* n_mask, void* hip_stream) {
  g_err.clear();
  fr_status st = check_volume_args(volume, dtype, nx, ny, nz, mask, disc_mode, disc_value);
  if (st != FR_OK) return st;
  if ((st = check_device_ptr(levels, "levels")) != FR_OK) return st;
  Pool* p = nullptr;
  if ((st = pool_get((int64_t)nx * ny * nz, &p)) != FR_OK) return st;
  fr::DiscParams dp;
  st = run_discretise(volume, dtype, nx, ny, nz, mask, disc_mode, disc_value, disc_lower, levels, p,
                      (hipStream_t)hip_stream, &dp);
  if (st != FR_OK) return st;
  if (ng) *ng = dp.ng;
  if (xmin) *xmin = dp.xmin;
  if (xmax) *xmax = dp.xmax;
  if (n_mask) *n_mask = dp.count;
  return FR_OK;
}

int32_t fr_map_count(uint32_t families) {
  if (families & ~(uint32_t)FR_ALL) return 0;
  int32_t n = 0;
  for (int q = 0; q < 6; ++q)
    if (families & (1u << q)) n += kCount[q];
  return n;
}

const char* fr_map_name(uint32_t families, int32_t k) {
  if (families == 0 || (families & ~(uint32_t)FR_ALL)) return nullptr;
  std::call_once(g_names_once, build_names);
  if (k < 0 || k >= (int32_t)g_names[families].size()) return nullptr;
  return g_names[families][k].c_str();
}

fr_status fr_map_ex(const void* volume, int32_t dtype, int32_t nx, int32_t ny, int32_t nz,
                    const uint8_t* mask, const double* spacing_mm, int32_t disc_mode,
                    double disc_value, double disc_lower, int32_t kernel_radius,
                    uint32_t families, const fr_map_options* options, int64_t n_mask,
                    float* out_maps, int64_t out_capacity_floats, void* hip_stream) {
  g_err.clear();
  fr::MapOptions opt;
  fr_status st = read_options(options, &opt);
  if (st != FR_OK) return st;
  return map_common(volume, dtype, nx, ny, nz, mask, spacing_mm, disc_mode, disc_value,
                    disc_lower, kernel_radius, families, opt, n_mask, nullptr, 0, 0, nullptr,
                    nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, out_maps,
                    out_capacity_floats, hip_stream);
}

fr_status fr_map(const void* volume, int32_t dtype, int32_t nx, int32_t ny, int32_t nz,
                 const uint8_t* mask, const double* spacing_mm, int32_t disc_mode,
                 double disc_value, double disc_lower, int32_t kernel_radius, uint32_t families,
                 int64_t n_mask, float* out_maps, int64_t out_capacity_floats, void* hip_stream) {
  return fr_map_ex(volume, dtype, nx, ny, nz, mask, spacing_mm, disc_mode, disc_value, disc_lower,
                   kernel_radius, families, nullptr, n_mask, out_maps, out_capacity_floats,
                   hip_stream);
}

fr_status fr_map_status(void* hip_stream, int32_t* ng) {
  g_err.clear();
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  fr::DiscParams* dp = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_last_mu);
    if (dev < (int)g_last_params.size()) dp = g_last_params[dev];
  }
  if (!dp) return fail(FR_E_ARG, "no map was enqueued on device %d", dev);
  fr::DiscParams d;
  hipStream_t st = (hipStream_t)hip_stream;
  HIP_TRY(hipMemcpyAsync(&d, dp, sizeof d, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  if (ng) *ng = d.ng;
  return params_status(d);
}

fr_status fr_map_matrices(const void* volume, int32_t dtype, int32_t nx, int32_t ny, int32_t nz,
                          const uint8_t* mask, const double* spacing_mm, int32_t disc_mode,
                          double disc_value, double disc_lower, int32_t kernel_radius,
                          uint32_t families, const fr_map_options* options, int64_t n_mask,
                          const int64_t* sample, int64_t n_sample, int32_t ng_expected,
                          int32_t* glcm, int32_t* glrlm, int32_t* glszm, int32_t* gldm,
                          int32_t* ngtdm_n, int64_t* ngtdm_S, int32_t* hist, float* out_maps,
                          void* hip_stream) {
  g_err.clear();
  if (!sample) return fail(FR_E_ARG, "sample is NULL");
  fr::MapOptions opt;
  fr_status st = read_options(options, &opt);
  if (st != FR_OK) return st;
  return map_common(volume, dtype, nx, ny, nz, mask, spacing_mm, disc_mode, disc_value,
                    disc_lower, kernel_radius, families, opt, n_mask, sample, n_sample, ng_expected,
                    glcm, glrlm, glszm, gldm, ngtdm_n, ngtdm_S, hist, out_maps,
                    (int64_t)fr_map_count(families) * n_sample, hip_stream);
}

fr_status fr_map_noalloc(const void* volume, int32_t dtype, int32_t nx, int32_t ny, int32_t nz,
                         const uint8_t* mask, const double* spacing_mm, int32_t disc_mode,
                         double disc_value, double disc_lower, int32_t kernel_radius,
                         uint32_t families, int64_t n_mask, float* out_maps,
                         int64_t out_capacity_floats, void* hip_stream) {
  g_err.clear();
  fr_status st = check_volume_args(volume, dtype, nx, ny, nz, mask, disc_mode, disc_value);
  if (st != FR_OK) return st;
  if (!spacing_mm) return fail(FR_E_ARG, "spacing_mm is NULL");
  for (int i = 0; i < 3; ++i)
    if (!(spacing_mm[i] > 0.0) || !isfinite(spacing_mm[i]))
      return fail(FR_E_ARG, "spacing_mm[%d] must be finite and > 0", i);
  if (kernel_radius < 1 || kernel_radius > FR_MAX_RADIUS)
    return fail(FR_E_RANGE, "kernel_radius %d outside 1..%d", kernel_radius, FR_MAX_RADIUS);
  if (families == 0 || (families & ~(uint32_t)FR_ALL))
    return fail(FR_E_RANGE, "families mask 0x%x invalid", families);
  if (n_mask <= 0) return fail(FR_E_EMPTY_MASK, "n_mask must be positive");
  const int64_t nvox = (int64_t)nx * ny * nz;
  if (n_mask > nvox) return fail(FR_E_ARG, "n_mask %lld exceeds the volume", (long long)n_mask);
  const int32_t count = fr_map_count(families);
  if (out_capacity_floats < (int64_t)count * n_mask)
    return fail(FR_E_CAPACITY, "out_maps holds %lld floats, %lld needed",
                (long long)out_capacity_floats, (long long)count * n_mask);
  if ((st = check_device_ptr(out_maps, "out_maps")) != FR_OK) return st;
  fr::MapOptions opt = {1, 0, 0, 0};
  const int lcap = level_cap(disc_mode, disc_value, kernel_radius);
  const size_t gbytes = needs_generic(kernel_radius, opt, lcap)
                            ? (size_t)kNoAllocGenericGrid * fr::generic_scratch_bytes(lcap)
                            : 0;
  // staging rows (coalesced output) when they fit, else direct stores
  NoAllocLayout L = noalloc_layout(nvox, n_mask, true, gbytes);
  if (L.total > kNoAllocBytes) L = noalloc_layout(nvox, n_mask, false, gbytes);
  if (L.total > kNoAllocBytes)
    return fail(FR_E_CAPACITY,
                "the job needs %zu bytes of scratch, more than the %zu of the allocation-free entry "
                "point (fr_map handles it)",
                L.total, kNoAllocBytes);
  unsigned char* base = nullptr;
  if ((st = noalloc_scratch(&base)) != FR_OK) return st;
  hipStream_t stream = (hipStream_t)hip_stream;
  fr::DiscScratch ds;
  ds.nblocks = (nvox + fr::kDiscSeg - 1) / fr::kDiscSeg;
  ds.block_count = (int32_t*)(base + L.bcount);
  ds.block_offset = (int64_t*)(base + L.boff);
  ds.block_min = (double*)(base + L.bmin);
  ds.block_max = (double*)(base + L.bmax);
  ds.params = (fr::DiscParams*)(base + L.params);
  // the scan kernel writes the whole parameter block (error state, counters
  // and queues at zero) before any later kernel reads it: nothing else of
  // the previous call's contents is read
  uint8_t* levels = base + L.levels;
  int32_t* list = (int32_t*)(base + L.list);
  if ((st = enqueue_discretise_into(volume, dtype, nx, ny, nz, mask, disc_mode, disc_value,
                                    disc_lower, levels, list, ds, n_mask, stream)) != FR_OK)
    return st;
  fr::MapArgs a;
  memset(&a, 0, sizeof a);
  a.params = ds.params;
  a.vol = volume;
  a.levels = levels;
  a.list = list;
  a.out = out_maps;
  a.stage = L.staged ? (float*)(base + L.stage) : nullptr;
  a.n_out = n_mask;
  a.n_items = n_mask;
  a.n_list = n_mask;
  a.nx = nx;
  a.ny = ny;
  a.nz = nz;
  a.families = families;
  a.count = count;
  a.voxel_volume = spacing_mm[0] * spacing_mm[1] * spacing_mm[2];
  a.radius = kernel_radius;
  a.opt = opt;
  const PassBuffers pb = {ds.params, {(int2*)(base + L.over0), (int2*)(base + L.over1)},
                          gbytes ? (void*)(base + L.gscratch) : nullptr, kNoAllocGenericGrid,
                          nullptr};
  if ((st = enqueue_map_passes(a, dtype, kernel_radius, lcap, false, pb, stream)) != FR_OK) return st;
  if (L.staged) HIP_TRY(fr::launch_transpose(a.stage, out_maps, n_mask, count, ds.params, stream));
  return FR_OK;
}

fr_status fr_profile_enable(int32_t enable) {
  g_err.clear();
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_on = enable != 0;
  return FR_OK;
}

fr_status fr_profile_read(double* map_kernel_ms, int64_t* launches) {
  g_err.clear();
  std::lock_guard<std::mutex> lk(g_prof_mu);
  double tot = 0.0;
  int64_t n = 0;
  for (auto& ev : g_prof_pending) {
    HIP_TRY(hipEventSynchronize(ev.second));
    float ms = 0.f;
    HIP_TRY(hipEventElapsedTime(&ms, ev.first, ev.second));
    tot += ms;
    n++;
    g_prof_free.push_back(ev);
  }
  g_prof_pending.clear();
  if (map_kernel_ms) *map_kernel_ms = tot;
  if (launches) *launches = n;
  return FR_OK;
}

const char* fr_last_error(void) { return g_err.c_str(); }

const char* fr_version(void) { return "flashrad-mi355x 0.1 (gfx950)"; }

// Set by the build from the sources it compiles (see build.py).
#ifndef FR_SOURCE_HASH
#define FR_SOURCE_HASH "unknown"
#endif
const char* fr_source_hash(void) { return FR_SOURCE_HASH; }

}  // extern "C"
