// Particle kernels: CIC paint with optional fused drift (Sec. 2.2 eq. cic and
// Sec. 2.3 eq. KDFK), CIC gather with fused kick, force VJP gather
// (Sec. 4.2, eq. KDFKO_adj) and the density-MSE mesh kernel (Sec. 5.2).
//
// Particles are processed in lattice order, so consecutive lanes paint to
// and gather from neighbouring cells; the paint accumulates with hardware
// floating-point atomics at L2 (no return value).  Positions are formed in
// FP64 from the exact lattice coordinate and the stored displacement, then the
// in-cell fraction is rounded to the mesh type.  Reductions that feed
// gradients (xi.p, pi.a, (delta - target)^2) are written as per-workgroup
// FP64 partial sums and combined by one workgroup in a fixed order, so they
// are deterministic.
#include "pm_internal.h"

namespace pmx {

namespace {

struct Geo {
  int64_t N;          // particles
  int np1, np2;       // lattice dims 1 and 2
  double r0, r1, r2;  // lattice spacing (cells)
  double off;         // lattice offset (cells)
  int n0, n1, n2;     // mesh dims (powers of two)
  int64_t ncell;
};

__device__ __forceinline__ void lattice_of(const Geo& g, int64_t n, double q[3]) {
  const int64_t row = n / g.np2;
  const int k = int(n - row * g.np2);
  const int64_t i = row / g.np1;
  const int j = int(row - i * g.np1);
  q[0] = double(i) * g.r0 + g.off;
  q[1] = double(j) * g.r1 + g.off;
  q[2] = double(k) * g.r2 + g.off;
}

// base node (wrapped) and fraction in [0, 1] for one axis
template <typename T>
__device__ __forceinline__ void cic_axis(double u, int nmask, int& i0, int& i1, T& f) {
  const double fl = floor(u);
  f = T(u - fl);
  const int64_t b = int64_t(fl);
  i0 = int(b & nmask);
  i1 = int((b + 1) & nmask);
}

template <typename T>
struct Cic {
  int ix[2], iy[2], iz[2];
  T wx[2], wy[2], wz[2];
  __device__ __forceinline__ void init(const Geo& g, const double x[3]) {
    T f;
    cic_axis<T>(x[0], g.n0 - 1, ix[0], ix[1], f); wx[0] = T(1) - f; wx[1] = f;
    cic_axis<T>(x[1], g.n1 - 1, iy[0], iy[1], f); wy[0] = T(1) - f; wy[1] = f;
    cic_axis<T>(x[2], g.n2 - 1, iz[0], iz[1], f); wz[0] = T(1) - f; wz[1] = f;
  }
  __device__ __forceinline__ int64_t idx(int a, int b, int c, const Geo& g) const {
    return (int64_t(ix[a]) * g.n1 + iy[b]) * g.n2 + iz[c];
  }
};

__device__ __forceinline__ void atomic_add(float* p, float v) { unsafeAtomicAdd(p, v); }
__device__ __forceinline__ void atomic_add(double* p, double v) { unsafeAtomicAdd(p, v); }

__device__ __forceinline__ double block_sum(double v) {
  __shared__ double ws[kThreads / 64];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) ws[wid] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < kThreads / 64; ++w) t += ws[w];
  return t;
}

// ---------------------------------------------------------------------------
// paint (+ drift)
// ---------------------------------------------------------------------------
template <typename S, typename T>
struct PaintP {
  Geo g;
  S* s;
  const S* p;
  const T* xi;
  T* pi;
  const T* w;
  T* mesh;
  S D;
  double* partials;  // slot 0: sum xi.p (adjoint drift)
};

template <typename S, typename T, int MODE, int NCH, bool UNIT>
__global__ __launch_bounds__(kThreads) void k_paint(PaintP<S, T> a) {
  const Geo& g = a.g;
  const int64_t stride = int64_t(gridDim.x) * kThreads;
  double xp = 0.0;
  for (int64_t n = int64_t(blockIdx.x) * kThreads + threadIdx.x; n < g.N; n += stride) {
    S s[3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) s[ax] = a.s[ax * g.N + n];
    T wch[4];
    if (MODE == DRIFT_FWD) {
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) {
        s[ax] += a.p[ax * g.N + n] * a.D;
        a.s[ax * g.N + n] = s[ax];
      }
    } else if (MODE == DRIFT_ADJ) {
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) {
        const S pv = a.p[ax * g.N + n];
        const T xv = a.xi[ax * g.N + n];
        xp += double(xv) * double(pv);
        s[ax] -= pv * a.D;
        a.s[ax * g.N + n] = s[ax];
        const T pin = a.pi[ax * g.N + n] + T(xv * T(a.D));
        a.pi[ax * g.N + n] = pin;
        wch[1 + ax] = pin;
      }
    }
    if (UNIT) wch[0] = T(1);
    if (MODE != DRIFT_ADJ) {
#pragma unroll
      for (int c = UNIT ? 1 : 0; c < NCH; ++c) wch[c] = a.w[int64_t(c - (UNIT ? 1 : 0)) * g.N + n];
    }
    double q[3];
    lattice_of(g, n, q);
    const double x[3] = {q[0] + double(s[0]), q[1] + double(s[1]), q[2] + double(s[2])};
    Cic<T> cic;
    cic.init(g, x);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          const T w = cic.wx[i] * cic.wy[j] * cic.wz[k];
          const int64_t idx = cic.idx(i, j, k, g);
#pragma unroll
          for (int c = 0; c < NCH; ++c) atomic_add(a.mesh + c * g.ncell + idx, w * wch[c]);
        }
  }
  if (MODE == DRIFT_ADJ) {
    const double t = block_sum(xp);
    if (threadIdx.x == 0) a.partials[blockIdx.x * 4 + 0] = t;
  }
}

// ---------------------------------------------------------------------------
// gather (+ kick / VJP)
// ---------------------------------------------------------------------------
template <typename S, typename T>
struct GatherP {
  Geo g;
  const S* s;
  const T* mesh;   // [nf][ncell]
  T* out;          // plain: [nf][N]; VJP/MSE: xbar [3][N]
  T* acc;          // optional acceleration output
  S* p;            // kick target
  T* xi;           // adjoint kick target
  const T* cot;    // cotangent [3][N]
  const T* acc_in; // if set, the kick and cot.a use these accelerations
  S K;             // kick coefficient
  double* partials;  // slot 1: sum cot.a
};

template <typename S, typename T, int MODE, int NF>
__global__ __launch_bounds__(kThreads) void k_gather(GatherP<S, T> a) {
  const Geo& g = a.g;
  const int64_t stride = int64_t(gridDim.x) * kThreads;
  double ca = 0.0;
  for (int64_t n = int64_t(blockIdx.x) * kThreads + threadIdx.x; n < g.N; n += stride) {
    double q[3];
    lattice_of(g, n, q);
    double x[3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) x[ax] = q[ax] + double(a.s[ax * g.N + n]);
    Cic<T> cic;
    cic.init(g, x);
    T v[NF];
#pragma unroll
    for (int c = 0; c < NF; ++c) v[c] = T(0);
    T cot[3] = {T(0), T(0), T(0)};
    if (MODE == GATHER_VJP || MODE == GATHER_KICK_ADJ) {
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) cot[ax] = a.cot[ax * g.N + n];
    }
    T dv[3] = {T(0), T(0), T(0)};  // sum_corner dW_k * h(corner)
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          const int64_t idx = cic.idx(i, j, k, g);
          const T w = cic.wx[i] * cic.wy[j] * cic.wz[k];
          T m[NF];
#pragma unroll
          for (int c = 0; c < NF; ++c) m[c] = a.mesh[c * g.ncell + idx];
          if (MODE == GATHER_PLAIN || MODE == GATHER_KICK_FWD || MODE == GATHER_VJP ||
              MODE == GATHER_KICK_ADJ) {
#pragma unroll
            for (int c = 0; c < (MODE == GATHER_PLAIN || MODE == GATHER_KICK_FWD ? NF : 3); ++c) v[c] += w * m[c];
          }
          if (MODE == GATHER_VJP || MODE == GATHER_KICK_ADJ || MODE == GATHER_MSE) {
            // h = sum_j cot_j g_j + rhobar   (VJP)   or   h = mbar   (MSE)
            T h;
            if (MODE == GATHER_MSE) h = m[0];
            else h = cot[0] * m[0] + cot[1] * m[1] + cot[2] * m[2] + m[3];
            const T sx = i ? T(1) : T(-1), sy = j ? T(1) : T(-1), sz = k ? T(1) : T(-1);
            dv[0] += sx * cic.wy[j] * cic.wz[k] * h;
            dv[1] += sy * cic.wx[i] * cic.wz[k] * h;
            dv[2] += sz * cic.wx[i] * cic.wy[j] * h;
          }
        }
    if (MODE == GATHER_PLAIN) {
#pragma unroll
      for (int c = 0; c < NF; ++c) a.out[c * g.N + n] = v[c];
    } else if (MODE == GATHER_KICK_FWD) {
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) {
        a.p[ax * g.N + n] += S(v[ax]) * a.K;
        if (a.acc) a.acc[ax * g.N + n] = v[ax];
      }
    } else if (MODE == GATHER_VJP) {
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) {
        a.out[ax * g.N + n] = dv[ax];
        if (a.acc) a.acc[ax * g.N + n] = v[ax];
        ca += double(cot[ax]) * double(v[ax]);
      }
    } else if (MODE == GATHER_KICK_ADJ) {
      if (a.acc_in) {
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) v[ax] = a.acc_in[ax * g.N + n];
      }
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) {
        ca += double(cot[ax]) * double(v[ax]);
        a.p[ax * g.N + n] -= S(v[ax]) * a.K;
        a.xi[ax * g.N + n] += dv[ax] * T(a.K);
        if (a.acc) a.acc[ax * g.N + n] = v[ax];
      }
    } else if (MODE == GATHER_MSE) {
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) a.out[ax * g.N + n] = dv[ax];
    }
  }
  if (MODE == GATHER_VJP || MODE == GATHER_KICK_ADJ) {
    const double t = block_sum(ca);
    if (threadIdx.x == 0) a.partials[blockIdx.x * 4 + 1] = t;
  }
}

// (delta - target) on the mesh: mesh <- 2 (rho Nc/Np - 1 - target) / Np,
// partial sums of (delta - target)^2 in slot 2
template <typename T>
__global__ __launch_bounds__(kThreads) void k_mse_mesh(T* mesh, const T* target, int64_t ncell, double ratio,
                                                       double inv_np, double* partials) {
  const int64_t stride = int64_t(gridDim.x) * kThreads;
  double acc = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < ncell; i += stride) {
    const double d = double(mesh[i]) * ratio - 1.0 - double(target[i]);
    acc += d * d;
    mesh[i] = T(2.0 * d * inv_np);
  }
  const double t = block_sum(acc);
  if (threadIdx.x == 0) partials[blockIdx.x * 4 + 2] = t;
}

// density contrast in place: mesh <- mesh * ratio - 1
template <typename T>
__global__ __launch_bounds__(kThreads) void k_contrast(T* mesh, int64_t ncell, double ratio) {
  const int64_t stride = int64_t(gridDim.x) * kThreads;
  for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < ncell; i += stride)
    mesh[i] = T(double(mesh[i]) * ratio - 1.0);
}

// out[0] (+)= sum_k f[k] * sum_b part[b*4 + k]; summed in a fixed order
// (slots whose factor is zero are skipped, so stale slots never contribute)
__global__ __launch_bounds__(kThreads) void k_reduce(const double* part, int nblocks, double f0, double f1,
                                                     double f2, double f3, double* out, int accumulate) {
  const double f[4] = {f0, f1, f2, f3};
  double v = 0.0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (f[k] == 0.0) continue;
    double s = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += kThreads) s += part[b * 4 + k];
    v += f[k] * s;
  }
  const double t = block_sum(v);
  if (threadIdx.x == 0) out[0] = accumulate ? out[0] + t : t;
}

template <typename S, typename T>
Geo make_geo(const Plan* p) {
  Geo g;
  g.N = p->nptcl;
  g.np1 = p->np[1];
  g.np2 = p->np[2];
  g.r0 = p->r[0];
  g.r1 = p->r[1];
  g.r2 = p->r[2];
  g.off = p->cfg.lattice_offset;
  g.n0 = p->n[0];
  g.n1 = p->n[1];
  g.n2 = p->n[2];
  g.ncell = p->ncell;
  return g;
}

template <typename S, typename T>
int paint_typed(Plan* p, DriftMode mode, const PaintArgs& in, hipStream_t st) {
  PaintP<S, T> a;
  a.g = make_geo<S, T>(p);
  a.s = static_cast<S*>(const_cast<void*>(in.s));
  a.p = static_cast<const S*>(in.p);
  a.xi = static_cast<const T*>(in.xi);
  a.pi = static_cast<T*>(in.pi);
  a.w = static_cast<const T*>(in.w);
  a.mesh = static_cast<T*>(in.mesh);
  a.D = S(in.D);
  a.partials = in.partials;
  const int nch = in.unit + in.nw;
  const dim3 grid(blocks_for_particles(p)), block(kThreads);
  timing_begin(p, PM_K_PAINT, st);
#define PM_PAINT(MODE, NCH, UNIT) hipLaunchKernelGGL((k_paint<S, T, MODE, NCH, UNIT>), grid, block, 0, st, a)
  if (mode == DRIFT_FWD) {
    PM_PAINT(DRIFT_FWD, 1, true);
  } else if (mode == DRIFT_ADJ) {
    PM_PAINT(DRIFT_ADJ, 4, true);
  } else if (in.unit) {
    switch (nch) {
      case 1: PM_PAINT(DRIFT_NONE, 1, true); break;
      case 2: PM_PAINT(DRIFT_NONE, 2, true); break;
      case 3: PM_PAINT(DRIFT_NONE, 3, true); break;
      default: PM_PAINT(DRIFT_NONE, 4, true); break;
    }
  } else {
    switch (nch) {
      case 1: PM_PAINT(DRIFT_NONE, 1, false); break;
      case 2: PM_PAINT(DRIFT_NONE, 2, false); break;
      case 3: PM_PAINT(DRIFT_NONE, 3, false); break;
      default: PM_PAINT(DRIFT_NONE, 4, false); break;
    }
  }
#undef PM_PAINT
  timing_end(p, PM_K_PAINT, st);
  PM_HIP_CHECK(p, hipGetLastError());
  return PM_OK;
}

template <typename S, typename T>
int gather_typed(Plan* p, GatherMode mode, const GatherArgs& in, hipStream_t st) {
  GatherP<S, T> a;
  a.g = make_geo<S, T>(p);
  a.s = static_cast<const S*>(in.s);
  a.mesh = static_cast<const T*>(in.mesh);
  a.out = static_cast<T*>(in.out);
  a.acc = static_cast<T*>(in.acc);
  a.p = static_cast<S*>(in.p);
  a.xi = static_cast<T*>(in.xi);
  a.cot = static_cast<const T*>(in.cot);
  a.acc_in = static_cast<const T*>(in.acc_in);
  a.K = S(in.K);
  a.partials = in.partials;
  const dim3 grid(blocks_for_particles(p)), block(kThreads);
  timing_begin(p, PM_K_GATHER, st);
#define PM_GATHER(MODE, NF) hipLaunchKernelGGL((k_gather<S, T, MODE, NF>), grid, block, 0, st, a)
  switch (mode) {
    case GATHER_PLAIN:
      switch (in.nf) {
        case 1: PM_GATHER(GATHER_PLAIN, 1); break;
        case 2: PM_GATHER(GATHER_PLAIN, 2); break;
        case 3: PM_GATHER(GATHER_PLAIN, 3); break;
        default: PM_GATHER(GATHER_PLAIN, 4); break;
      }
      break;
    case GATHER_KICK_FWD: PM_GATHER(GATHER_KICK_FWD, 3); break;
    case GATHER_VJP: PM_GATHER(GATHER_VJP, 4); break;
    case GATHER_KICK_ADJ: PM_GATHER(GATHER_KICK_ADJ, 4); break;
    case GATHER_MSE: PM_GATHER(GATHER_MSE, 1); break;
  }
#undef PM_GATHER
  timing_end(p, PM_K_GATHER, st);
  PM_HIP_CHECK(p, hipGetLastError());
  return PM_OK;
}

}  // namespace

int blocks_for_particles(const Plan* p) {
  const int64_t need = (p->nptcl + kThreads - 1) / kThreads;
  const int64_t cap = 2048;  // 8 workgroups per CU on 256 CUs; <= kMaxPartials
  return int(need < cap ? (need < 1 ? 1 : need) : cap);
}

int paint_launch(Plan* p, DriftMode mode, const PaintArgs& a, hipStream_t st) {
  const int nch = a.unit + a.nw;
  PM_HIP_CHECK(p, hipMemsetAsync(a.mesh, 0, size_t(nch) * p->ncell * p->real_bytes, st));
  const bool s64 = p->cfg.state_dtype == PM_F64, m64 = p->cfg.mesh_dtype == PM_F64;
  if (m64) return paint_typed<double, double>(p, mode, a, st);
  if (s64) return paint_typed<double, float>(p, mode, a, st);
  return paint_typed<float, float>(p, mode, a, st);
}

int gather_launch(Plan* p, GatherMode mode, const GatherArgs& a, hipStream_t st) {
  const bool s64 = p->cfg.state_dtype == PM_F64, m64 = p->cfg.mesh_dtype == PM_F64;
  if (m64) return gather_typed<double, double>(p, mode, a, st);
  if (s64) return gather_typed<double, float>(p, mode, a, st);
  return gather_typed<float, float>(p, mode, a, st);
}

int mse_mesh_launch(Plan* p, void* mesh, const void* target, double* partials, hipStream_t st) {
  const double ratio = double(p->ncell) / double(p->nptcl);
  const double inv_np = 1.0 / double(p->nptcl);
  const int64_t need = (p->ncell + kThreads - 1) / kThreads;
  const int blocks = int(need < 2048 ? need : 2048);
  if (p->cfg.mesh_dtype == PM_F64)
    hipLaunchKernelGGL((k_mse_mesh<double>), dim3(blocks), dim3(kThreads), 0, st, static_cast<double*>(mesh),
                       static_cast<const double*>(target), p->ncell, ratio, inv_np, partials);
  else
    hipLaunchKernelGGL((k_mse_mesh<float>), dim3(blocks), dim3(kThreads), 0, st, static_cast<float*>(mesh),
                       static_cast<const float*>(target), p->ncell, ratio, inv_np, partials);
  PM_HIP_CHECK(p, hipGetLastError());
  return blocks;
}

int contrast_launch(Plan* p, void* mesh, hipStream_t st) {
  const double ratio = double(p->ncell) / double(p->nptcl);
  const int64_t need = (p->ncell + kThreads - 1) / kThreads;
  const int blocks = int(need < 2048 ? need : 2048);
  if (p->cfg.mesh_dtype == PM_F64)
    hipLaunchKernelGGL((k_contrast<double>), dim3(blocks), dim3(kThreads), 0, st, static_cast<double*>(mesh), p->ncell,
                       ratio);
  else
    hipLaunchKernelGGL((k_contrast<float>), dim3(blocks), dim3(kThreads), 0, st, static_cast<float*>(mesh), p->ncell,
                       ratio);
  PM_HIP_CHECK(p, hipGetLastError());
  return PM_OK;
}

int reduce_partials(Plan* p, int nblocks, const double* f, double* out, bool accumulate, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kThreads), 0, st, p->partials, nblocks, f[0], f[1], f[2], f[3], out,
                     accumulate ? 1 : 0);
  PM_HIP_CHECK(p, hipGetLastError());
  return PM_OK;
}

}  // namespace pmx
