// Internal declarations shared by the HIP translation units of libflashrad.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/fr.h"

namespace fr {

// Small parameter block written by the discretisation kernels and read by
// the map kernel and (once per call) by the host.
struct DiscParams {
  double xmin;      // VOI minimum
  double xmax;      // VOI maximum
  double lo;        // FBW lower bound actually used
  int64_t count;    // number of mask voxels
  int32_t ng;       // VOI gray-level count
  int32_t err;      // kJob* code: nonzero stops every later kernel of the job
  // entries appended to the two overflow lists of a single-job map (voxels
  // with more present levels than the 32- and 64-level instances hold) and
  // two work-queue heads; all zeroed by the discretisation scan
  int32_t n_over[2];
  int32_t queue[2];
  // MCC problems stashed by a single-job map for the MCC kernel: those with
  // at most 16 and with 17..32 present levels
  int32_t n_mcc[2];
};

// Segment of the volume handled by one discretisation block.
constexpr int kDiscThreads = 256;
constexpr int kDiscPerThread = 16;
constexpr int kDiscSeg = kDiscThreads * kDiscPerThread;  // 4096 voxels

struct DiscScratch {
  int64_t nblocks;
  int32_t* block_count;   // [nblocks]
  int64_t* block_offset;  // [nblocks]
  double* block_min;      // [nblocks]
  double* block_max;      // [nblocks]
  DiscParams* params;     // [1]
};

// Enqueue the three discretisation kernels: block statistics, block scan +
// parameters, level map + compaction of the mask voxel list.  With
// expect_count >= 0 the scan also checks the mask-voxel count (kJobCount).
// The list (nvox entries) never overflows: a segment writes its own voxels.
hipError_t launch_discretise(const void* vol, int dtype, int64_t nvox, const uint8_t* mask,
                             int mode, double value, double lower, uint8_t* levels,
                             int32_t* list, const DiscScratch& s, int64_t expect_count,
                             hipStream_t st);

// Settings of the IBSI extraction variants (defaults: distance 1, alpha 0,
// merged); only the generic kernel implements the non-default ones.
struct MapOptions {
  int32_t glcm_dist;   // GLCM neighbour offset: distance x each of the 13 directions
  int32_t gldm_alpha;  // GLDM: a neighbour depends on v when |g_u - g_v| <= alpha
  int32_t averaged;    // GLCM and GLRLM features averaged over the 13 directions
  int32_t reserved;
};

struct MapArgs {
  const DiscParams* params; // device parameter block of the job (Ng, error state)
  const void* vol;          // raw volume (int16 or float)
  const uint8_t* levels;    // discretised volume, 0 outside mask
  const int32_t* list;      // compact index -> linear voxel index
  const int64_t* sample;    // optional: restrict to these compact indices
  float* out;               // [count][n_out]
  float* stage;             // optional voxel-major staging [n_items][kStageStride]
  int64_t n_out;            // row stride of out (n_mask or n_sample)
  int64_t n_items;          // voxels to process (n_mask or n_sample)
  int64_t n_list;           // entries of list (n_mask); sample values are checked against it
  int32_t nx, ny, nz;
  int32_t ng;               // VOI Ng
  uint32_t families;
  int32_t count;            // maps per voxel (fr_map_count(families))
  double voxel_volume;
  int64_t nblk;             // workgroups; b takes [b n / nblk, (b + 1) n / nblk)
  // optional item list (a previous pass's overflow): item k is position
  // items[k].y, with *items_count entries (read on the device)
  const int2* items;
  const int32_t* items_count;
  // where a voxel with more present levels than the instance holds goes:
  // (over_job, position) appended at over[atomicAdd(over_count, 1)]
  int2* over;
  int32_t* over_count;
  int32_t over_job;
  int32_t radius;           // kernel radius (the generic kernel reads it)
  MapOptions opt;
  // optional MCC stash (the 32- and 64-level instances write each
  // neighbourhood's MCC problem of <= 32 levels there for the MCC kernel
  // instead of solving it in LDS):
  // room for mcc_cap problems of kMccProblemBytes, counted in *mcc_count
  unsigned char* mcc;
  int64_t mcc_cap;
  int32_t* mcc_count;
  // debug matrix dump (all null in production)
  int32_t* d_glcm;
  int32_t* d_glrlm;
  int32_t* d_glszm;
  int32_t* d_gldm;
  int32_t* d_ngn;
  int64_t* d_ngS;
  int32_t* d_hist;
};

// Bytes of one stashed MCC problem (its present-level count, its output
// address and the upper triangle of its co-occurrence counts, up to 32
// levels); a stash holds one problem per mapped voxel at most.
constexpr int64_t kMccProblemBytes = 1072;

// Row stride (floats) of the voxel-major staging buffer: every voxel's maps
// are one contiguous 384-byte row, written with full cache lines.
constexpr int kStageStride = 96;

// One job of a batched map: device pointers and settings, plus the job's
// range in the batch-wide discretisation segment table.
struct BatchJob {
  const void* vol;
  const uint8_t* mask;
  uint8_t* levels;     // job's slice of the batch level buffer
  int32_t* list;       // job's slice of the batch mask-voxel lists
  float* stage;        // job's slice of the batch staging rows
  float* out;          // caller's out_maps [count][n_mask]
  int64_t nvox, n_mask;
  int32_t nx, ny, nz, dtype;
  int32_t mode, radius, lcap, count;  // lcap: bound of the present levels, min(Ng, cube)
  double value, lower, voxel_volume;
  uint32_t families;
  int32_t seg_base, nseg;
  MapOptions opt;
  int32_t vpw;         // voxels per work item of the job (fused batch pass)
  int32_t reserved;
};

// Error codes a job can raise on the device (DiscParams::err).
enum { kJobOk = 0, kJobNgRange = 1, kJobEmpty = 2, kJobCount = 3 };

// Batched discretisation: seg_job[b] names the job of global segment b
// (seg_job NULL: a single job, jobs[0], with seg_base 0).
hipError_t launch_discretise_batch(const BatchJob* jobs, int32_t n_jobs, const int32_t* seg_job,
                                   int64_t n_seg, const DiscScratch& s, hipStream_t st);

// Persistent batched map kernel for one (dtype, radius) variant on the
// instance with lmax (32 or 64) local levels: items[w] = (job, first
// compact index), vpw voxels each (items NULL: a single job, jobs[0], item
// w starting at voxel w * vpw); with n_items_dev set, the item count is
// read on the device.  A voxel with more than lmax present levels is
// appended as (job, voxel) to over[*over_count] (radius >= 2).  With queue
// set (a zeroed counter), workgroups take items dynamically from it, so
// kernels running side by side balance; otherwise item w goes to
// workgroup w mod grid.  With mcc set (lmax 32), the MCC problems go to
// that stash of mcc_cap problems (counts in mcc_count[0..1]) and
// launch_mcc must follow.
hipError_t launch_map_batch(const BatchJob* jobs, const DiscParams* params, const int2* items,
                            int32_t n_items, const int32_t* n_items_dev, int32_t vpw, int dtype,
                            int radius, int lmax, int grid, int2* over, int32_t* over_count,
                            int32_t* queue, unsigned char* mcc, int64_t mcc_cap, int32_t* mcc_count,
                            hipStream_t st);

// Fused batched pass over the jobs of every fixed radius (1..3) of one raw
// type: one persistent kernel whose work items name their job (and thereby
// the radius), taken from a work queue.  lmax 32: items[w] = (job, first
// compact index), jobs[job].vpw voxels each; the MCC problems go to the
// stash (launch_mcc must follow); a neighbourhood with more than 32 present
// levels is appended as (job, voxel) to over[*over_count].  lmax 64:
// items are (job, voxel) pairs (an earlier pass's overflow, count read on
// the device), radius 2 or 3, MCC problems with <= 32 levels stashed as
// well, wider ones solved in the kernel; more than 64 levels go to over.  grid: resident workgroups (map_fused_blocks_per_cu).
hipError_t launch_map_fused(const BatchJob* jobs, const DiscParams* params, const int2* items,
                            int32_t n_items, const int32_t* n_items_dev, int dtype, int lmax,
                            int grid, int2* over, int32_t* over_count, int32_t* queue,
                            unsigned char* mcc, int64_t mcc_cap, int32_t* mcc_count, hipStream_t st);
int map_fused_blocks_per_cu(int dtype, int lmax);

// Generic map kernel: any radius 1..kGenericMaxRadius, up to 255 present
// levels, every MapOptions setting.  One workgroup of kGenericThreads per
// voxel, persistent over the items; per-workgroup tables in global scratch.
constexpr int kGenericMaxRadius = 5;
constexpr int kGenericThreads = 256;
// Bytes of global scratch one workgroup of the generic kernel needs for
// neighbourhoods of at most lcap (1..255) present levels.
size_t generic_scratch_bytes(int lcap);
// Workgroups of a generic launch (each takes one scratch slice).
constexpr int kGenericGrid = 256;
// Single job (a, its params and list; a.opt, a.radius and a.count set) or
// batch (jobs != NULL: item (job, voxel)); items / n_items_dev as
// launch_map_batch (items NULL with jobs NULL: every voxel 0 .. n_items-1
// of the single job).  scratch holds grid slices of
// generic_scratch_bytes(lcap); every neighbourhood mapped has at most lcap
// present levels (lcap >= min(Ng, (2r+1)^3)).
hipError_t launch_map_generic(const MapArgs& a, const BatchJob* jobs, const DiscParams* params,
                              const int2* items, const int32_t* n_items_dev, int32_t n_items,
                              int dtype, void* scratch, int lcap, int grid, hipStream_t st);
// Resident workgroups per CU of a batched map variant (occupancy; stash:
// the instance that stashes its MCC problems).
int map_batch_blocks_per_cu(int dtype, int radius, int lmax, bool stash);
// Batched transpose: items[w] = (job, first compact index of a 64-voxel tile)
// (items NULL: a single job, tile w starting at voxel 64 w).
hipError_t launch_transpose_batch(const BatchJob* jobs, const DiscParams* params, const int2* items,
                                  int32_t n_items, hipStream_t st);

// Enqueue the fused map kernel; lmax is the compact-level capacity (32 or 64).
// With a.stage set, maps go to the staging rows and launch_transpose must
// follow on the same stream.  a.params must be set; a.items / a.over as in
// MapArgs.  With a.mcc set (not debug) the MCC problems with <= 32 levels
// go to the stash and launch_mcc must follow before the maps are read.
hipError_t launch_map(const MapArgs& a, int dtype, int radius, int lmax, bool debug,
                      hipStream_t st);
// Resident workgroups of a plain map instance on the current device.
int map_resident(int dtype, int radius, int lmax);

// The MCC of every problem in a stash of cap problems (device counts
// n_mcc[0..1]: problems with <= 16 levels from the stash's start, wider
// ones from its end), written to each problem's output address; nothing
// when *err (if err is set) holds a job error.
hipError_t launch_mcc(const int32_t* n_mcc, const int32_t* err, const unsigned char* stash,
                      int64_t cap, hipStream_t st);
// out[k * n + m] = stage[m * kStageStride + k] for k < count, m < n (nothing
// when params->err is set).
hipError_t launch_transpose(const float* stage, float* out, int64_t n, int count,
                            const DiscParams* params, hipStream_t st);

// Host validation of one job shared by the batch and the server: fills
// *bj (device pointers left as given), *lcap (bound of the present levels
// of one neighbourhood, min(Ng bound, cube)) and returns FR_OK or an
// fr_status with a message in msg.
int32_t validate_job(const ::fr_job& J, int j, BatchJob* bj, int* lcap, char* msg,
                     size_t msg_len, bool need_out);

// Tuned launch settings of a (dtype, radius, level bound) variant (defaults
// when the autotuner has not seen it): voxels per work item, grid multiple,
// the first pass's instance (32 or 64 local levels).
void tuned_settings(int dtype, int radius, int lcap, int* vpw, int* grid_mult, int* kernel_lmax);

// dst[0 .. n) = 0 by a kernel (so the clear can be captured in a graph).
hipError_t launch_zero_i32(int32_t* dst, int n, hipStream_t st);

}  // namespace fr
