// Shell-averaged power spectrum of a real field, from its half spectrum.
//
// The paper defines the power spectrum through <delta(k) delta(k')> = V P(k)
// (Sec. 2.1, eq. Plin).  The estimator here averages |delta(k) V / N_c|^2 / V
// over the modes of each spherical shell of the integer wavevector m
// (k = 2 pi m / L): shell b holds the modes with round(|m|) = b, which for an
// integer |m|^2 = m2 is exactly b (b - 1) < m2 <= b (b + 1), so the shell of
// every mode is decided in integer arithmetic.  Half-spectrum modes with
// 0 < mz < n/2 stand for themselves and their conjugates (weight 2); the
// mz = 0 and mz = n/2 planes hold both members of each pair (weight 1).
//
// The reduction is deterministic: workgroup (x plane, shell) sums the modes
// of its shell in that plane in a fixed order and writes one partial; a
// second kernel sums the partials of each shell over the planes in a fixed
// order.  No atomics, so repeated calls give bitwise equal results.
//
// Two entry points share the kernels: pm_power_spectrum keeps its partials
// in the plan's spectrum scratch, pm_power_spectrum_noalloc in the file-scope
// device array `scratch` below, for callers that cannot allocate.
#include <cmath>
#include <mutex>

#include "pm_internal.h"

namespace pmx {
namespace {

constexpr int kSpecThreads = 256;
constexpr int kMaxMesh = 1024;                                      // largest mesh side of the library
constexpr int64_t kPartialDoubles = int64_t(kMaxMesh / 2) * kMaxMesh * 3;   // [shells][planes][3]

// floor(sqrt(v)) for 0 <= v < 2^52, exact
__device__ __forceinline__ int64_t isqrt_floor(int64_t v) {
  int64_t r = int64_t(sqrt(double(v)));
  while (r * r > v) --r;
  while ((r + 1) * (r + 1) <= v) ++r;
  return r;
}

// three sums over the workgroup in a fixed order; valid in thread 0
__device__ __forceinline__ void block_sum3(double& a, double& b, double& c) {
  __shared__ double ws[3][kSpecThreads / 64];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    a += __shfl_down(a, off, 64);
    b += __shfl_down(b, off, 64);
    c += __shfl_down(c, off, 64);
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) {
    ws[0][wid] = a;
    ws[1][wid] = b;
    ws[2][wid] = c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    a = b = c = 0.0;
    for (int w = 0; w < kSpecThreads / 64; ++w) {
      a += ws[0][w];
      b += ws[1][w];
      c += ws[2][w];
    }
  }
}

// part[((b - 1) n + ix) 3 + {0, 1, 2}] = sum over the modes of plane ix in
// shell b of w |delta_k|^2, w |m| and w.  Every slot is written, zero when
// the plane does not reach the shell, so the buffer needs no clearing.
template <typename T>
__global__ __launch_bounds__(kSpecThreads) void k_pk_partials(const Cx<T>* __restrict__ dk, int n,
                                                             double* __restrict__ part) {
  const int ix = blockIdx.x;
  const int b = blockIdx.y + 1;
  const int half = n / 2, nh = half + 1;
  const int64_t mx = ix < half ? ix : ix - n;
  const int64_t lo2 = int64_t(b) * (b - 1), hi2 = int64_t(b) * (b + 1);   // lo2 < m2 <= hi2
  double sp = 0.0, sk = 0.0, sw = 0.0;
  if (mx * mx <= hi2) {
    for (int iy = threadIdx.x; iy < n; iy += kSpecThreads) {
      const int64_t my = iy < half ? iy : iy - n;
      const int64_t r2 = mx * mx + my * my;
      if (r2 > hi2) continue;
      // mz in [z0, z1]: mz^2 > lo2 - r2, mz^2 <= hi2 - r2, 0 <= mz <= n/2
      const int64_t z0 = lo2 < r2 ? 0 : isqrt_floor(lo2 - r2) + 1;
      int64_t z1 = isqrt_floor(hi2 - r2);
      if (z1 > half) z1 = half;
      const Cx<T>* row = dk + (int64_t(ix) * n + iy) * nh;
      for (int64_t mz = z0; mz <= z1; ++mz) {
        const Cx<T> v = row[mz];
        const double w = (mz == 0 || mz == half) ? 1.0 : 2.0;
        const double re = double(v.x), im = double(v.y);
        sp += w * (re * re + im * im);
        sk += w * sqrt(double(r2 + mz * mz));
        sw += w;
      }
    }
  }
  block_sum3(sp, sk, sw);
  if (threadIdx.x == 0) {
    double* o = part + ((int64_t(b) - 1) * n + ix) * 3;
    o[0] = sp;
    o[1] = sk;
    o[2] = sw;
  }
}

// one workgroup per shell: the plane partials summed in a fixed order, then
// P = (V / N_c^2) sum w |delta_k|^2 / sum w, k = k_f sum w |m| / sum w
__global__ __launch_bounds__(kSpecThreads) void k_pk_shells(const double* __restrict__ part, int n, double pscale,
                                                           double kf, double* __restrict__ k, double* __restrict__ P,
                                                           double* __restrict__ count) {
  const int b = blockIdx.x;   // shell b + 1
  double sp = 0.0, sk = 0.0, sw = 0.0;
  for (int ix = threadIdx.x; ix < n; ix += kSpecThreads) {
    const double* o = part + (int64_t(b) * n + ix) * 3;
    sp += o[0];
    sk += o[1];
    sw += o[2];
  }
  block_sum3(sp, sk, sw);
  if (threadIdx.x == 0) {
    P[b] = pscale * sp / sw;
    k[b] = kf * sk / sw;
    count[b] = sw;
  }
}

// launches both kernels; part holds at least (n/2) n 3 doubles
hipError_t pk_launch(int n, double box, int dtype, const void* dk, double* part, double* k, double* P,
                     double* count, hipStream_t st) {
  const dim3 grid(unsigned(n), unsigned(n / 2));
  if (dtype == PM_F64)
    hipLaunchKernelGGL(k_pk_partials<double>, grid, dim3(kSpecThreads), 0, st,
                       static_cast<const Cx<double>*>(dk), n, part);
  else
    hipLaunchKernelGGL(k_pk_partials<float>, grid, dim3(kSpecThreads), 0, st, static_cast<const Cx<float>*>(dk),
                       n, part);
  const double ncell = double(n) * double(n) * double(n);
  const double V = box * box * box;
  hipLaunchKernelGGL(k_pk_shells, dim3(unsigned(n / 2)), dim3(kSpecThreads), 0, st, part, n, V / (ncell * ncell),
                     2.0 * M_PI / box, k, P, count);
  return hipGetLastError();
}

bool pow2_side(int n) { return n >= 4 && n <= kMaxMesh && (n & (n - 1)) == 0; }

// ---------------------------------------------------------------------------
// allocation-free variant: the partials live in this file-scope device array
// (one copy per GPU, held until the process ends).  Its address on a device
// comes from hipGetSymbolAddress, taken once per device with that device
// current; host code never uses the name itself as a device address.
// ---------------------------------------------------------------------------
__device__ __align__(256) double scratch[kPartialDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double* g_scratch_ptr[kMaxDevices] = {};

// address of `scratch` on the current device (looked up on the first call)
int scratch_on_current_device(double** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return set_error(nullptr, PM_EDEVICE, "hipGetDevice: %s", hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices)
    return set_error(nullptr, PM_EDEVICE, "device %d is beyond the %d devices the scratch table covers", dev,
                     kMaxDevices);
  std::lock_guard<std::mutex> lock(g_scratch_mutex);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !ptr)
      return set_error(nullptr, PM_EDEVICE, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
    g_scratch_ptr[dev] = static_cast<double*>(ptr);
  }
  *out = g_scratch_ptr[dev];
  return PM_OK;
}

}  // namespace
}  // namespace pmx

using namespace pmx;

extern "C" int pm_power_spectrum(pm_plan h, const void* delta_k, double* k, double* P, double* count,
                                 hipStream_t stream) {
  Plan* p = reinterpret_cast<Plan*>(h);
  if (!p) return set_error(nullptr, PM_EINVAL, "plan is NULL");
  if (!delta_k || !k || !P || !count) return set_error(p, PM_EINVAL, "delta_k, k, P and count must not be NULL");
  const int n = p->n[0];
  if (p->n[1] != n || p->n[2] != n) return set_error(p, PM_EUNSUPPORTED, "the power spectrum needs a cubic mesh");
  const double box = p->cfg.box[0];
  if (!(std::isfinite(box) && box > 0.0) || p->cfg.box[1] != box || p->cfg.box[2] != box)
    return set_error(p, PM_EUNSUPPORTED, "the power spectrum needs a cubic box of finite positive side");
  // the partials ((n/2) n 3 doubles) fit in one half spectrum of the plan
  if (size_t(n / 2) * n * 3 * sizeof(double) > size_t(p->nspec) * 2 * p->real_bytes)
    return set_error(p, PM_ESHAPE, "mesh too small for the spectrum partials");
  int cur = -1;
  PM_HIP_CHECK(p, hipGetDevice(&cur));
  if (cur != p->device) PM_HIP_CHECK(p, hipSetDevice(p->device));
  PM_HIP_CHECK(p, pk_launch(n, box, p->cfg.mesh_dtype, delta_k, static_cast<double*>(p->spec[3]), k, P, count,
                            stream));
  return PM_OK;
}

extern "C" int pm_power_spectrum_noalloc(int n, double box, int mesh_dtype, const void* delta_k, double* k,
                                         double* P, double* count, hipStream_t stream) {
  if (!delta_k || !k || !P || !count)
    return set_error(nullptr, PM_EINVAL, "delta_k, k, P and count must not be NULL");
  if (n > kMaxMesh)
    return set_error(nullptr, PM_ESHAPE, "mesh side %d exceeds the %d that the static scratch (%lld bytes) holds",
                     n, kMaxMesh, static_cast<long long>(kPartialDoubles * sizeof(double)));
  if (!pow2_side(n)) return set_error(nullptr, PM_ESHAPE, "mesh side must be a power of two in [4, %d]", kMaxMesh);
  if (!(std::isfinite(box) && box > 0.0)) return set_error(nullptr, PM_EINVAL, "box must be finite and > 0");
  if (mesh_dtype != PM_F32 && mesh_dtype != PM_F64) return set_error(nullptr, PM_EINVAL, "dtype must be PM_F32 or PM_F64");
  double* part = nullptr;
  if (int rc = scratch_on_current_device(&part)) return rc;
  const hipError_t e = pk_launch(n, box, mesh_dtype, delta_k, part, k, P, count, stream);
  if (e != hipSuccess) return set_error(nullptr, PM_EDEVICE, "power spectrum launch: %s", hipGetErrorString(e));
  return PM_OK;
}
