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
  int32_t err;      // nonzero: Ng out of range
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
// parameters, level map + compaction of the mask voxel list.
hipError_t launch_discretise(const void* vol, int dtype, int64_t nvox, const uint8_t* mask,
                             int mode, double value, double lower, uint8_t* levels,
                             int32_t* list, const DiscScratch& s, hipStream_t st);

struct MapArgs {
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
  double voxel_volume;
  int64_t nblk;             // workgroups; b takes [b n / nblk, (b + 1) n / nblk)
  // debug matrix dump (all null in production)
  int32_t* d_glcm;
  int32_t* d_glrlm;
  int32_t* d_glszm;
  int32_t* d_gldm;
  int32_t* d_ngn;
  int64_t* d_ngS;
  int32_t* d_hist;
};

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
  int32_t mode, radius, lmax, count;
  double value, lower, voxel_volume;
  uint32_t families;
  int32_t seg_base, nseg;
};

// Error codes a batched job can raise on the device (DiscParams::err).
enum { kJobOk = 0, kJobNgRange = 1, kJobEmpty = 2, kJobCount = 3, kJobLocalLevels = 4 };

// Batched discretisation: seg_job[b] names the job of global segment b
// (seg_job NULL: a single job, jobs[0], with seg_base 0).
hipError_t launch_discretise_batch(const BatchJob* jobs, int32_t n_jobs, const int32_t* seg_job,
                                   int64_t n_seg, const DiscScratch& s, hipStream_t st);

// Persistent batched map kernel for one (dtype, radius, lmax) variant:
// items[w] = (job, first compact index), vpw voxels each (items NULL: a
// single job, jobs[0], item w starting at voxel w * vpw).
hipError_t launch_map_batch(const BatchJob* jobs, const DiscParams* params, const int2* items,
                            int32_t n_items, int32_t vpw, int dtype,
                            int radius, int lmax, int grid, hipStream_t st);
// Resident workgroups per CU of a batched map variant (occupancy).
int map_batch_blocks_per_cu(int dtype, int radius, int lmax);
// Batched transpose: items[w] = (job, first compact index of a 64-voxel tile)
// (items NULL: a single job, tile w starting at voxel 64 w).
hipError_t launch_transpose_batch(const BatchJob* jobs, const DiscParams* params, const int2* items,
                                  int32_t n_items, hipStream_t st);

// Enqueue the fused map kernel; lmax is the compact-level capacity (32 or 64).
// With a.stage set, maps go to the staging rows and launch_transpose must
// follow on the same stream.
hipError_t launch_map(const MapArgs& a, int dtype, int radius, int lmax, bool debug,
                      hipStream_t st);

// out[k * n + m] = stage[m * kStageStride + k] for k < count, m < n.
hipError_t launch_transpose(const float* stage, float* out, int64_t n, int count, hipStream_t st);

// Host validation of one job shared by the batch and the server: fills
// *bj (device pointers left as given), *lmax (local-level class 32/64) and
// returns FR_OK or an fr_status with a message in msg.
int32_t validate_job(const ::fr_job& J, int j, BatchJob* bj, int* lmax, char* msg,
                     size_t msg_len, bool need_out);

// Tuned launch settings of a variant (defaults when the autotuner has not
// seen it): voxels per work item, grid multiple, kernel LDS capacity.
void tuned_settings(int dtype, int radius, int lmax, int* vpw, int* grid_mult, int* kernel_lmax);

}  // namespace fr
