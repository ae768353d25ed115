// Intensity discretisation and mask compaction for gfx950.
//
// IBSI fixed bin number / fixed bin width (the paper keeps discretisation
// on the CPU in its hybrid backend; here it is three small HBM-bound
// kernels on the map's stream):
//   k_disc_stats   per 4096-voxel segment: mask count, min, max (one pass)
//   k_disc_scan    one block: exclusive scan of the segment counts, global
//                  min/max, Ng, written to a small parameter block
//   k_disc_levels  level of every voxel (0 outside the mask) and the
//                  raster-ordered list of mask voxels (compact index ->
//                  linear index), each segment writing at its scanned offset
// Loads are lane-interleaved inside a segment (element j*256 + t), so every
// wavefront load and store is contiguous.
#include <math.h>

#include "fr_internal.h"

namespace fr {
namespace {

// Mask count, min and max of one 4096-voxel segment, written at `slot`.
template <typename T>
__device__ inline void disc_stats_seg(const T* __restrict__ vol, const uint8_t* __restrict__ mask,
                                      int64_t n, int64_t seg, int64_t slot, int32_t* bcount,
                                      double* bmin, double* bmax) {
  const int64_t base = seg * kDiscSeg;
  int cnt = 0;
  double mn = INFINITY, mx = -INFINITY;
#pragma unroll
  for (int j = 0; j < kDiscPerThread; ++j) {
    const int64_t i = base + j * kDiscThreads + threadIdx.x;
    if (i < n && mask[i]) {
      const double x = (double)vol[i];
      cnt++;
      mn = fmin(mn, x);
      mx = fmax(mx, x);
    }
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    cnt += __shfl_xor(cnt, o);
    mn = fmin(mn, __shfl_xor(mn, o));
    mx = fmax(mx, __shfl_xor(mx, o));
  }
  __shared__ int sc[kDiscThreads / 64];
  __shared__ double smn[kDiscThreads / 64], smx[kDiscThreads / 64];
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  if (lane == 0) {
    sc[w] = cnt;
    smn[w] = mn;
    smx[w] = mx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < kDiscThreads / 64; ++q) {
      cnt += sc[q];
      mn = fmin(mn, smn[q]);
      mx = fmax(mx, smx[q]);
    }
    bcount[slot] = cnt;
    bmin[slot] = mn;
    bmax[slot] = mx;
  }
}

template <typename T>
__global__ __launch_bounds__(kDiscThreads) void k_disc_stats(const T* __restrict__ vol,
                                                             const uint8_t* __restrict__ mask,
                                                             int64_t n, int32_t* bcount,
                                                             double* bmin, double* bmax) {
  disc_stats_seg(vol, mask, n, blockIdx.x, blockIdx.x, bcount, bmin, bmax);
}

constexpr int kScanThreads = 1024;

// Exclusive scan of the counts of segments [s0, s0 + nb), the VOI min/max
// and the gray-level count, written to *P (one block of kScanThreads).
// expect_count >= 0 adds the check of the mask-voxel count.
__device__ inline void disc_scan_range(int64_t s0, int64_t nb, const int32_t* bcount_all,
                                       const double* bmin_all, const double* bmax_all,
                                       int64_t* boff_all, DiscParams* P, int mode, double value,
                                       double lower, int64_t expect_count) {
  const int32_t* bcount = bcount_all + s0;
  const double* bmin = bmin_all + s0;
  const double* bmax = bmax_all + s0;
  int64_t* boff = boff_all + s0;
  __shared__ long long wsum[kScanThreads / 64];
  __shared__ double wmn[kScanThreads / 64], wmx[kScanThreads / 64];
  __shared__ long long chunk_total;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  long long carry = 0;
  double mn = INFINITY, mx = -INFINITY;
  for (int64_t c0 = 0; c0 < nb; c0 += kScanThreads) {
    const int64_t i = c0 + threadIdx.x;
    long long v = 0;
    if (i < nb) {
      v = bcount[i];
      mn = fmin(mn, bmin[i]);
      mx = fmax(mx, bmax[i]);
    }
    long long x = v;  // inclusive scan inside the wavefront
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      const long long y = __shfl_up(x, o);
      if (lane >= o) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    if (threadIdx.x == 0) {
      long long run = 0;
      for (int q = 0; q < kScanThreads / 64; ++q) {
        const long long t = wsum[q];
        wsum[q] = run;
        run += t;
      }
      chunk_total = run;
    }
    __syncthreads();
    if (i < nb) boff[i] = carry + wsum[w] + x - v;
    carry += chunk_total;
    __syncthreads();
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    mn = fmin(mn, __shfl_xor(mn, o));
    mx = fmax(mx, __shfl_xor(mx, o));
  }
  if (lane == 0) {
    wmn[w] = mn;
    wmx[w] = mx;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int q = 1; q < kScanThreads / 64; ++q) {
      mn = fmin(mn, wmn[q]);
      mx = fmax(mx, wmx[q]);
    }
    DiscParams p;
    p.xmin = mn;
    p.xmax = mx;
    p.count = carry;
    p.err = 0;
    p.n_over[0] = 0;
    p.n_over[1] = 0;
    p.queue[0] = 0;
    p.queue[1] = 0;
    p.n_mcc[0] = 0;
    p.n_mcc[1] = 0;
    if (mode == 2) {  // fixed bin number: Ng given
      p.lo = mn;
      p.ng = (int32_t)value;
    } else {  // fixed bin width: Ng = level of the VOI maximum
#pragma clang fp contract(off)
      p.lo = isfinite(lower) ? lower : mn;
      const double qmax = floor((mx - p.lo) / value) + 1.0;
      if (!(qmax <= 255.0)) p.err = kJobNgRange;
      p.ng = qmax < 1.0 ? 1 : (qmax > 255.0 ? 255 : (int32_t)qmax);
    }
    if (carry == 0) p.err = kJobEmpty;
    if (p.err == 0 && expect_count >= 0 && carry != expect_count) p.err = kJobCount;
    *P = p;
  }
}


__global__ __launch_bounds__(kScanThreads) void k_disc_scan(int64_t nb, const int32_t* bcount,
                                                            const double* bmin,
                                                            const double* bmax, int64_t* boff,
                                                            DiscParams* P, int mode, double value,
                                                            double lower, int64_t expect_count) {
  disc_scan_range(0, nb, bcount, bmin, bmax, boff, P, mode, value, lower, expect_count);
}

// Levels of one segment (0 outside the mask) and its mask voxels appended
// to `list` at the segment's scanned offset.
template <typename T>
__device__ inline void disc_levels_seg(const T* __restrict__ vol, const uint8_t* __restrict__ mask,
                                       int64_t n, int64_t seg, int64_t off,
                                       const DiscParams* P, int mode, double value,
                                       uint8_t* levels, int32_t* list) {
#pragma clang fp contract(off)
  __shared__ int wcnt[kDiscThreads / 64];
  const double xmin = P->xmin, lo = P->lo;
  const double range = P->xmax - P->xmin;
  const int ng = P->ng;
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t base = seg * kDiscSeg;
  int64_t pos = off;
  for (int j = 0; j < kDiscPerThread; ++j) {
    const int64_t i = base + j * kDiscThreads + threadIdx.x;
    const bool in = i < n && mask[i] != 0;
    int g = 0;
    if (in) {
      const double x = (double)vol[i];
      if (mode == 2) {
        g = 1;
        if (range > 0.0) {
          const double t = x - xmin;
          const double q = ((double)ng * t) / range;
          g = (int)floor(q) + 1;
          if (g > ng) g = ng;
        }
      } else {
        const double t = x - lo;
        double gg = floor(t / value) + 1.0;
        if (gg < 1.0) gg = 1.0;
        if (gg > 255.0) gg = 255.0;
        g = (int)gg;
      }
    }
    if (i < n) levels[i] = (uint8_t)g;
    const uint64_t b = __ballot(in);
    if (lane == 0) wcnt[w] = __popcll(b);
    __syncthreads();
    int before = 0, total = 0;
#pragma unroll
    for (int q = 0; q < kDiscThreads / 64; ++q) {
      const int c = wcnt[q];
      before += (q < w) ? c : 0;
      total += c;
    }
    if (in) list[pos + before + __popcll(b & below)] = (int32_t)i;
    pos += total;
    __syncthreads();
  }
}


template <typename T>
__global__ __launch_bounds__(kDiscThreads) void k_disc_levels(const T* __restrict__ vol,
                                                              const uint8_t* __restrict__ mask,
                                                              int64_t n, const int64_t* boff,
                                                              const DiscParams* P, int mode,
                                                              double value, uint8_t* levels,
                                                              int32_t* list) {
  disc_levels_seg(vol, mask, n, blockIdx.x, boff[blockIdx.x], P, mode, value, levels, list);
}

// ---- batched: global segment b belongs to job seg_job[b] ------------------
__global__ __launch_bounds__(kDiscThreads) void k_bdisc_stats(const BatchJob* __restrict__ jobs,
                                                              const int32_t* __restrict__ seg_job,
                                                              int32_t* bcount, double* bmin,
                                                              double* bmax) {
  const BatchJob& J = jobs[seg_job ? seg_job[blockIdx.x] : 0];  // no table: one job
  const int64_t seg = (int64_t)blockIdx.x - J.seg_base;
  if (J.dtype == 1)
    disc_stats_seg((const int16_t*)J.vol, J.mask, J.nvox, seg, blockIdx.x, bcount, bmin, bmax);
  else
    disc_stats_seg((const float*)J.vol, J.mask, J.nvox, seg, blockIdx.x, bcount, bmin, bmax);
}

__global__ __launch_bounds__(kScanThreads) void k_bdisc_scan(const BatchJob* __restrict__ jobs,
                                                             const int32_t* bcount,
                                                             const double* bmin, const double* bmax,
                                                             int64_t* boff, DiscParams* params) {
  const BatchJob& J = jobs[blockIdx.x];
  disc_scan_range(J.seg_base, J.nseg, bcount, bmin, bmax, boff, &params[blockIdx.x], J.mode,
                  J.value, J.lower, J.n_mask);
}

__global__ __launch_bounds__(kDiscThreads) void k_bdisc_levels(const BatchJob* __restrict__ jobs,
                                                               const int32_t* __restrict__ seg_job,
                                                               const int64_t* boff,
                                                               const DiscParams* params) {
  const int j = seg_job ? seg_job[blockIdx.x] : 0;
  const BatchJob& J = jobs[j];
  const int64_t seg = (int64_t)blockIdx.x - J.seg_base;
  // a job whose mask count disagrees with n_mask must not write past its list
  if (params[j].err == kJobCount || params[j].err == kJobEmpty) return;
  if (J.dtype == 1)
    disc_levels_seg((const int16_t*)J.vol, J.mask, J.nvox, seg, boff[blockIdx.x], &params[j], J.mode,
                    J.value, J.levels, J.list);
  else
    disc_levels_seg((const float*)J.vol, J.mask, J.nvox, seg, boff[blockIdx.x], &params[j], J.mode,
                    J.value, J.levels, J.list);
}

}  // namespace

__global__ __launch_bounds__(256) void k_zero_i32(int32_t* dst, int n) {
  for (int i = blockIdx.x * 256 + threadIdx.x; i < n; i += gridDim.x * 256) dst[i] = 0;
}

hipError_t launch_discretise_batch(const BatchJob* jobs, int32_t n_jobs, const int32_t* seg_job,
                                   int64_t n_seg, const DiscScratch& s, hipStream_t st) {
  hipLaunchKernelGGL(k_bdisc_stats, dim3((unsigned)n_seg), dim3(kDiscThreads), 0, st, jobs, seg_job,
                     s.block_count, s.block_min, s.block_max);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_bdisc_scan, dim3((unsigned)n_jobs), dim3(kScanThreads), 0, st, jobs,
                     s.block_count, s.block_min, s.block_max, s.block_offset, s.params);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_bdisc_levels, dim3((unsigned)n_seg), dim3(kDiscThreads), 0, st, jobs, seg_job,
                     s.block_offset, s.params);
  return hipGetLastError();
}

hipError_t launch_discretise(const void* vol, int dtype, int64_t nvox, const uint8_t* mask,
                             int mode, double value, double lower, uint8_t* levels,
                             int32_t* list, const DiscScratch& s, int64_t expect_count,
                             hipStream_t st) {
  const dim3 grid((unsigned)s.nblocks), block(kDiscThreads);
  if (dtype == 1) {
    hipLaunchKernelGGL(k_disc_stats<int16_t>, grid, block, 0, st, (const int16_t*)vol, mask,
                       nvox, s.block_count, s.block_min, s.block_max);
  } else {
    hipLaunchKernelGGL(k_disc_stats<float>, grid, block, 0, st, (const float*)vol, mask, nvox,
                       s.block_count, s.block_min, s.block_max);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_disc_scan, dim3(1), dim3(kScanThreads), 0, st, (int64_t)s.nblocks,
                     s.block_count, s.block_min, s.block_max, s.block_offset, s.params, mode,
                     value, lower, expect_count);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (dtype == 1) {
    hipLaunchKernelGGL(k_disc_levels<int16_t>, grid, block, 0, st, (const int16_t*)vol, mask,
                       nvox, s.block_offset, s.params, mode, value, levels, list);
  } else {
    hipLaunchKernelGGL(k_disc_levels<float>, grid, block, 0, st, (const float*)vol, mask, nvox,
                       s.block_offset, s.params, mode, value, levels, list);
  }
  return hipGetLastError();
}

hipError_t launch_zero_i32(int32_t* dst, int n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_zero_i32, dim3((unsigned)((n + 255) / 256 < 64 ? (n + 255) / 256 : 64)), dim3(256), 0,
                     st, dst, n);
  return hipGetLastError();
}

}  // namespace fr
