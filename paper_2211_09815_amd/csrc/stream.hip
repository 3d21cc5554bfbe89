// STREAM-like bandwidth kernels (measurement support): the achievable HBM
// rate of a pure read, a copy and a pure write of 16-byte vectors, the
// ceilings against which the path's kernels are read.  Grid-stride loops
// over 2048 workgroups of 256 threads (8 per CU on 256 CUs).
#include "pm_internal.h"

namespace pmx {
namespace {

constexpr int kStreamBlocks = 2048;

__global__ __launch_bounds__(kThreads) void k_stream_read(const float4* __restrict__ a, int64_t n, float* sink) {
  const int64_t stride = int64_t(gridDim.x) * kThreads;
  float acc = 0.f;
  for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < n; i += stride) {
    const float4 v = a[i];
    acc += (v.x + v.y) + (v.z + v.w);
  }
  // a store that never happens for finite data keeps the loads alive
  if (acc == -3.0e38f) sink[0] = acc;
}

__global__ __launch_bounds__(kThreads) void k_stream_copy(const float4* __restrict__ a, float4* __restrict__ b,
                                                          int64_t n) {
  const int64_t stride = int64_t(gridDim.x) * kThreads;
  for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < n; i += stride) b[i] = a[i];
}

__global__ __launch_bounds__(kThreads) void k_stream_write(float4* __restrict__ b, int64_t n) {
  const int64_t stride = int64_t(gridDim.x) * kThreads;
  const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
  for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < n; i += stride) b[i] = z;
}

}  // namespace
}  // namespace pmx

using namespace pmx;

extern "C" int pm_stream(pm_plan h, int mode, const void* src, void* dst, int64_t nbytes, hipStream_t stream) {
  Plan* p = reinterpret_cast<Plan*>(h);
  if (!p) return set_error(nullptr, PM_EINVAL, "plan is NULL");
  if (nbytes <= 0 || nbytes % 16) return set_error(p, PM_EINVAL, "nbytes must be a positive multiple of 16");
  if ((mode == PM_STREAM_READ || mode == PM_STREAM_COPY) && (!src || reinterpret_cast<uintptr_t>(src) % 16))
    return set_error(p, PM_EINVAL, "src must be a 16-byte aligned device pointer");
  if ((mode == PM_STREAM_COPY || mode == PM_STREAM_WRITE) && (!dst || reinterpret_cast<uintptr_t>(dst) % 16))
    return set_error(p, PM_EINVAL, "dst must be a 16-byte aligned device pointer");
  const int64_t n = nbytes / 16;
  int cur = -1;
  PM_HIP_CHECK(p, hipGetDevice(&cur));
  if (cur != p->device) PM_HIP_CHECK(p, hipSetDevice(p->device));
  switch (mode) {
    case PM_STREAM_READ:
      hipLaunchKernelGGL(k_stream_read, dim3(kStreamBlocks), dim3(kThreads), 0, stream,
                         static_cast<const float4*>(src), n, reinterpret_cast<float*>(p->partials));
      break;
    case PM_STREAM_COPY:
      hipLaunchKernelGGL(k_stream_copy, dim3(kStreamBlocks), dim3(kThreads), 0, stream,
                         static_cast<const float4*>(src), static_cast<float4*>(dst), n);
      break;
    case PM_STREAM_WRITE:
      hipLaunchKernelGGL(k_stream_write, dim3(kStreamBlocks), dim3(kThreads), 0, stream, static_cast<float4*>(dst), n);
      break;
    default:
      return set_error(p, PM_EINVAL, "unknown stream mode %d", mode);
  }
  PM_HIP_CHECK(p, hipGetLastError());
  return PM_OK;
}
