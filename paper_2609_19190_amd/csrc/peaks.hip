// On-device peak measurements for the roofline of the map kernel (gfx950).
//
// A separate small library (libfrpeaks.so), not part of the product ABI:
// the benchmark calls frp_measure() to re-measure, on the GPU it runs on,
// the three resources the spatial-mapping kernel is priced against:
//   HBM   stream copy of a large buffer (bytes read + bytes written)
//   LDS   ds_read_b32 and ds_add_u32 throughput over whole workgroups,
//         lane-consecutive addresses (no bank conflicts)
//   FP64  fused multiply-add throughput (8 independent chains per lane)
// Each figure is the best of a few timed launches (HIP events).
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

typedef float v4f __attribute__((ext_vector_type(4)));

// Four 16-byte loads in flight per lane; n4 is a multiple of 4 * grid * 256.
__global__ __launch_bounds__(256) void k_copy(const v4f* __restrict__ src,
                                              v4f* __restrict__ dst, int64_t n4) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += 4 * stride) {
    const v4f a = __builtin_nontemporal_load(&src[i]);
    const v4f b = __builtin_nontemporal_load(&src[i + stride]);
    const v4f c = __builtin_nontemporal_load(&src[i + 2 * stride]);
    const v4f d = __builtin_nontemporal_load(&src[i + 3 * stride]);
    __builtin_nontemporal_store(a, &dst[i]);
    __builtin_nontemporal_store(b, &dst[i + stride]);
    __builtin_nontemporal_store(c, &dst[i + 2 * stride]);
    __builtin_nontemporal_store(d, &dst[i + 3 * stride]);
  }
}

constexpr int kLdsWords = 8192;  // 32 KiB per workgroup

// Every lane reads ITER words at lane-consecutive addresses that move by a
// runtime stride (256 words) per step, so the compiler cannot find the
// period of the addresses and hoist the loads; the sum is written out.
template <int ITER>
__global__ __launch_bounds__(256) void k_lds_read(uint32_t* out, uint32_t seed, int stride) {
  __shared__ uint32_t buf[kLdsWords];
  for (int i = threadIdx.x; i < kLdsWords; i += 256) buf[i] = (uint32_t)i * seed;
  __syncthreads();
  uint32_t acc0 = 0, acc1 = 0, acc2 = 0, acc3 = 0;
  const int t = threadIdx.x;
#pragma unroll 8
  for (int i = 0; i < ITER; i += 4) {
    acc0 += buf[(t + (i + 0) * stride) & (kLdsWords - 1)];
    acc1 += buf[(t + (i + 1) * stride + 64) & (kLdsWords - 1)];
    acc2 += buf[(t + (i + 2) * stride + 128) & (kLdsWords - 1)];
    acc3 += buf[(t + (i + 3) * stride + 192) & (kLdsWords - 1)];
  }
  out[(int64_t)blockIdx.x * 256 + t] = acc0 + acc1 + acc2 + acc3;
}

template <int ITER>
__global__ __launch_bounds__(256) void k_lds_add(uint32_t* out, uint32_t seed) {
  __shared__ uint32_t buf[kLdsWords];
  for (int i = threadIdx.x; i < kLdsWords; i += 256) buf[i] = 0u;
  __syncthreads();
  const int t = threadIdx.x;
#pragma unroll 16
  for (int i = 0; i < ITER; ++i) atomicAdd(&buf[(t + i * 256) & (kLdsWords - 1)], seed + (uint32_t)i);
  __syncthreads();
  out[(int64_t)blockIdx.x * 256 + t] = buf[t] + buf[t + 4096];
}

template <int ITER>
__global__ __launch_bounds__(256) void k_fma64(double* out, double x, double y) {
  double a[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) a[k] = (double)(threadIdx.x + k);
  for (int i = 0; i < ITER; ++i) {
#pragma unroll
    for (int k = 0; k < 8; ++k) a[k] = fma(a[k], x, y);
  }
  double s = 0.0;
#pragma unroll
  for (int k = 0; k < 8; ++k) s += a[k];
  out[(int64_t)blockIdx.x * 256 + threadIdx.x] = s;
}

template <typename F>
float best_ms(F&& launch, int reps, hipStream_t st) {
  hipEvent_t a, b;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return -1.f;
  float best = 1e30f;
  launch();  // warm-up
  for (int r = 0; r < reps; ++r) {
    (void)hipEventRecord(a, st);
    launch();
    (void)hipEventRecord(b, st);
    (void)hipEventSynchronize(b);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, a, b);
    if (ms < best) best = ms;
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  return best;
}

}  // namespace

extern "C" {

// out[0] HBM copy GB/s (read + write bytes), out[1] LDS ds_read_b32 GB/s,
// out[2] LDS ds_add_u32 GB/s (4 bytes per lane-operation), out[3] FP64
// FMA TFLOP/s (2 flops per FMA), out[4] compute units.  copy_mib sizes
// the copied buffer.  Returns 0, or -1 on a HIP error.
int frp_measure(double* out, int n_out, int copy_mib) {
  if (!out || n_out < 5 || copy_mib < 16) return -1;
  int dev = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return -1;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return -1;
  hipStream_t st = nullptr;
  const int blocks = cus * 16;
  const int copy_grid = cus * 16;
  const int64_t quantum = 4LL * copy_grid * 256;  // float4 elements per full sweep
  const int64_t n4 = (int64_t)copy_mib * (1 << 20) / 16 / quantum * quantum;
  v4f *src = nullptr, *dst = nullptr;
  uint32_t* ou = nullptr;
  double* od = nullptr;
  if (hipMalloc((void**)&src, n4 * 16) != hipSuccess || hipMalloc((void**)&dst, n4 * 16) != hipSuccess ||
      hipMalloc((void**)&ou, (size_t)blocks * 256 * 4) != hipSuccess ||
      hipMalloc((void**)&od, (size_t)blocks * 256 * 8) != hipSuccess) {
    (void)hipFree(src);
    (void)hipFree(dst);
    (void)hipFree(ou);
    (void)hipFree(od);
    return -1;
  }
  (void)hipMemset(src, 1, n4 * 16);
  const float t_copy = best_ms([&] { hipLaunchKernelGGL(k_copy, dim3(copy_grid), dim3(256), 0, st, src, dst, n4); }, 5, st);
  constexpr int IT = 4096;
  const float t_rd = best_ms([&] { hipLaunchKernelGGL(k_lds_read<IT>, dim3(blocks), dim3(256), 0, st, ou, 3u, 256); }, 5, st);
  const float t_add = best_ms([&] { hipLaunchKernelGGL(k_lds_add<IT>, dim3(blocks), dim3(256), 0, st, ou, 5u); }, 5, st);
  constexpr int IF = 2048;
  const float t_fma = best_ms([&] { hipLaunchKernelGGL(k_fma64<IF>, dim3(blocks), dim3(256), 0, st, od, 0.999999, 1e-9); }, 5, st);
  const hipError_t e = hipDeviceSynchronize();
  (void)hipFree(src);
  (void)hipFree(dst);
  (void)hipFree(ou);
  (void)hipFree(od);
  if (e != hipSuccess || t_copy <= 0.f || t_rd <= 0.f || t_add <= 0.f || t_fma <= 0.f) return -1;
  const double lanes = (double)blocks * 256;
  out[0] = 2.0 * (double)n4 * 16 / (t_copy * 1e-3) / 1e9;
  out[1] = lanes * IT * 4.0 / (t_rd * 1e-3) / 1e9;
  out[2] = lanes * IT * 4.0 / (t_add * 1e-3) / 1e9;
  out[3] = lanes * IF * 8 * 2.0 / (t_fma * 1e-3) / 1e12;
  out[4] = (double)cus;
  return 0;
}

}  // extern "C"
