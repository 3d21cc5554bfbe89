// Light-cone observation (Sec. 2.4) and its VJP (Sec. 3.4; eq. explicit_adj
// for the discrete chain rule), the adjoint's bump at an integer time, and
// the kick and drift operators of eq. KDFK as standalone calls.
//
// Per particle and in FP64 whatever the state dtype:
//   x(u) = h00 x0 + h10 v0 + h01 x1 + h11 v1,  v = da w p,  w = 1/(a^3 E(a)),
//   chi(u) = h00 c0 + h10 t0 + h01 c1 + h11 t1,  t = da dchi/da,
//   f(u) = |x(u) - X| - chi(u),
// with the cubic Hermite basis h of u = (a - a0)/da.  Observed in the step
// when f(0) < 0 <= f(1); the root is found by Newton steps kept inside a
// sign-change bracket (bisection when a step leaves it).  The VJP solves the
// root again and differentiates through it: du*/dz = -(df/dz)/(df/du).
//
// The observation test reads only the two positions of a particle; the
// momenta, the root and the seven outputs are touched for observed particles
// only, so a step costs about one read of the two displacement arrays.
#include "pm_internal.h"
#include "tiles.h"

namespace pmx {
namespace {

struct LcGeo {
  TileGeo g;
  double a0, da, om;
  double X[3];
  double c0, t0, c1, t1;                 // chi and da dchi/da at both ends
  double w0, w1;                         // 1/(a^3 E) at both ends
  double c0o, t0o, c1o, t1o, w0o, w1o;   // their Omega_m derivatives
  int step;
};

struct Traj {
  double x0[3], v0[3], x1[3], v1[3];
};

__device__ __forceinline__ void hermite(double u, double h[4], double d[4], double dd[4]) {
  const double u2 = u * u, u3 = u2 * u;
  h[0] = 2.0 * u3 - 3.0 * u2 + 1.0;
  h[1] = u3 - 2.0 * u2 + u;
  h[2] = -2.0 * u3 + 3.0 * u2;
  h[3] = u3 - u2;
  d[0] = 6.0 * u2 - 6.0 * u;
  d[1] = 3.0 * u2 - 4.0 * u + 1.0;
  d[2] = -6.0 * u2 + 6.0 * u;
  d[3] = 3.0 * u2 - 2.0 * u;
  dd[0] = 12.0 * u - 6.0;
  dd[1] = 6.0 * u - 4.0;
  dd[2] = -12.0 * u + 6.0;
  dd[3] = 6.0 * u - 2.0;
}

__device__ __forceinline__ double comb(const double b[4], double y0, double t0, double y1, double t1) {
  return b[0] * y0 + b[1] * t0 + b[2] * y1 + b[3] * t1;
}

// f(u) and df/du
__device__ __forceinline__ void front_eval(const LcGeo& L, const Traj& T, double u, double& f, double& fu) {
  double h[4], d[4], dd[4];
  hermite(u, h, d, dd);
  double r2 = 0.0, rv = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double pos = comb(h, T.x0[k], T.v0[k], T.x1[k], T.v1[k]) - L.X[k];
    const double vel = comb(d, T.x0[k], T.v0[k], T.x1[k], T.v1[k]);
    r2 += pos * pos;
    rv += pos * vel;
  }
  const double r = sqrt(r2);
  f = r - comb(h, L.c0, L.t0, L.c1, L.t1);
  fu = rv / r - comb(d, L.c0, L.t0, L.c1, L.t1);
}

// root of f in [0, 1], given f(0) = f0 < 0 <= f1 = f(1) (for states that
// only approximately satisfy that, the root is kept in [0, 1])
__device__ double solve_root(const LcGeo& L, const Traj& T, double f0, double f1) {
  double lo = 0.0, hi = 1.0;
  double u = f0 / (f0 - f1);
  if (!(u >= 0.0 && u <= 1.0)) u = 0.5;
  for (int it = 0; it < 64; ++it) {
    double f, fu;
    front_eval(L, T, u, f, fu);
    if (f == 0.0) return u;
    if (f < 0.0) lo = u;
    else hi = u;
    double un = u - f / fu;
    if (!(un > lo && un < hi)) un = 0.5 * (lo + hi);
    const double du = un - u;
    u = un;
    if (fabs(du) <= 1e-15) break;
  }
  return u;
}

template <typename S>
__device__ __forceinline__ void load_ends(const LcGeo& L, int64_t n, const S* s0, const S* s1, Traj& T, double& f0,
                                          double& f1) {
  const int64_t N = L.g.N;
  double q[3];
  lattice_pos(L.g, n, q);
  double r0 = 0.0, r1 = 0.0;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    T.x0[k] = q[k] + double(s0[k * N + n]);
    T.x1[k] = q[k] + double(s1[k * N + n]);
    const double d0 = T.x0[k] - L.X[k], d1 = T.x1[k] - L.X[k];
    r0 += d0 * d0;
    r1 += d1 * d1;
  }
  f0 = sqrt(r0) - L.c0;
  f1 = sqrt(r1) - L.c1;
}

template <typename S>
__global__ __launch_bounds__(kThreads) void k_lightcone(const LcGeo L, const S* __restrict__ s0,
                                                        const S* __restrict__ p0, const S* __restrict__ s1,
                                                        const S* __restrict__ p1, S* __restrict__ obs,
                                                        int* __restrict__ ostep, double* __restrict__ partials) {
  const int64_t N = L.g.N;
  int64_t start, end;
  chunk_of(N, start, end);
  double cnt = 0.0;
  for (int64_t n = start + threadIdx.x; n < end; n += kThreads) {
    Traj T;
    double f0, f1;
    load_ends(L, n, s0, s1, T, f0, f1);
    if (!(f0 < 0.0 && f1 >= 0.0)) continue;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      T.v0[k] = L.da * L.w0 * double(p0[k * N + n]);
      T.v1[k] = L.da * L.w1 * double(p1[k * N + n]);
    }
    const double u = solve_root(L, T, f0, f1);
    double h[4], d[4], dd[4];
    hermite(u, h, d, dd);
    const double ah = L.a0 + u * L.da;
    const double sf = ah * ah * ah * sqrt(L.om / (ah * ah * ah) + (1.0 - L.om)) / L.da;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      obs[k * N + n] = S(comb(h, T.x0[k], T.v0[k], T.x1[k], T.v1[k]));
      obs[(3 + k) * N + n] = S(sf * comb(d, T.x0[k], T.v0[k], T.x1[k], T.v1[k]));
    }
    obs[6 * N + n] = S(ah);
    ostep[n] = L.step;
    cnt += 1.0;
  }
  const double t = block_sum_d(cnt);
  if (threadIdx.x == 0) {
    double* pp = partials + 4 * blockIdx.x;
    pp[0] = t;
    pp[1] = pp[2] = pp[3] = 0.0;
  }
}

template <typename S, typename T>
__global__ __launch_bounds__(kThreads) void k_lightcone_vjp(const LcGeo L, const S* __restrict__ s0,
                                                            const S* __restrict__ p0, const S* __restrict__ s1,
                                                            const S* __restrict__ p1, const int* __restrict__ ostep,
                                                            const T* __restrict__ obar, T* __restrict__ x0b,
                                                            T* __restrict__ p0b, T* __restrict__ x1b,
                                                            T* __restrict__ p1b, double* __restrict__ partials) {
  const int64_t N = L.g.N;
  int64_t start, end;
  chunk_of(N, start, end);
  double om_acc = 0.0;
  for (int64_t n = start + threadIdx.x; n < end; n += kThreads) {
    if (ostep[n] != L.step) continue;
    Traj Tr;
    double f0, f1, pa[3], pb[3];
    load_ends(L, n, s0, s1, Tr, f0, f1);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      pa[k] = double(p0[k * N + n]);
      pb[k] = double(p1[k * N + n]);
      Tr.v0[k] = L.da * L.w0 * pa[k];
      Tr.v1[k] = L.da * L.w1 * pb[k];
    }
    const double u = solve_root(L, Tr, f0, f1);
    double h[4], d[4], dd[4];
    hermite(u, h, d, dd);
    double pos[3], vel[3], acc[3], r2 = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      pos[k] = comb(h, Tr.x0[k], Tr.v0[k], Tr.x1[k], Tr.v1[k]) - L.X[k];
      vel[k] = comb(d, Tr.x0[k], Tr.v0[k], Tr.x1[k], Tr.v1[k]);
      acc[k] = comb(dd, Tr.x0[k], Tr.v0[k], Tr.x1[k], Tr.v1[k]);
      r2 += pos[k] * pos[k];
    }
    // |x - X| has no gradient at the observer itself; take it as zero there
    const double rinv = r2 > 0.0 ? 1.0 / sqrt(r2) : 0.0;
    const double ah = L.a0 + u * L.da;
    const double a3 = ah * ah * ah;
    const double E = sqrt(L.om / a3 + (1.0 - L.om));
    const double Sf = a3 * E;
    const double dS_da = 3.0 * ah * ah * E + a3 * (-1.5 * L.om / (a3 * ah * E));
    const double dS_dom = a3 * (1.0 / a3 - 1.0) / (2.0 * E);
    double gx[3], gp[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      gx[k] = double(obar[k * N + n]);
      gp[k] = double(obar[(3 + k) * N + n]);
    }
    const double ga = double(obar[6 * N + n]);
    double Gu = ga * L.da, fu = -comb(d, L.c0, L.t0, L.c1, L.t1), gpv = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      Gu += gx[k] * vel[k] + gp[k] * (dS_da * vel[k] + Sf * acc[k] / L.da);
      fu += pos[k] * rinv * vel[k];
      gpv += gp[k] * vel[k];
    }
    const double lam = -Gu / fu;
    const double spd = Sf / L.da;
    double pv0 = 0.0, pv1 = 0.0;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double cx = gx[k] + lam * pos[k] * rinv;
      const double cp = gp[k] * spd;
      const double v0b = h[1] * cx + d[1] * cp;
      const double v1b = h[3] * cx + d[3] * cp;
      if (x0b) x0b[k * N + n] += T(h[0] * cx + d[0] * cp);
      if (x1b) x1b[k * N + n] += T(h[2] * cx + d[2] * cp);
      if (p0b) p0b[k * N + n] += T(L.da * L.w0 * v0b);
      if (p1b) p1b[k * N + n] += T(L.da * L.w1 * v1b);
      pv0 += pa[k] * v0b;
      pv1 += pb[k] * v1b;
    }
    om_acc += gpv / L.da * dS_dom - lam * comb(h, L.c0o, L.t0o, L.c1o, L.t1o) + L.da * (pv0 * L.w0o + pv1 * L.w1o);
  }
  const double t = block_sum_d(om_acc);
  if (threadIdx.x == 0) {
    double* pp = partials + 4 * blockIdx.x;
    pp[0] = t;
    pp[1] = pp[2] = pp[3] = 0.0;
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_adj_bump(T* __restrict__ xi, T* __restrict__ pi,
                                                       const T* __restrict__ xb, const T* __restrict__ pb,
                                                       const T* __restrict__ c, T Kb, const T* __restrict__ a,
                                                       const double* __restrict__ cb, int64_t n3,
                                                       double* __restrict__ partials) {
  const int64_t stride = int64_t(gridDim.x) * kThreads;
  double dot = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < n3; i += stride) {
    xi[i] = xi[i] + (c ? fma(Kb, c[i], xb[i]) : xb[i]);
    if (pb) {
      const T pbi = pb[i];
      pi[i] = pi[i] + pbi;
      if (a) dot += double(pbi) * double(a[i]);
    }
  }
  const double t = block_sum_d(dot);
  if (threadIdx.x == 0) {
    double* pp = partials + 4 * blockIdx.x;
    pp[0] = t;
    pp[1] = (blockIdx.x == 0 && cb) ? cb[0] : 0.0;
    pp[2] = pp[3] = 0.0;
  }
}

template <typename S, typename T>
__global__ __launch_bounds__(kThreads) void k_kick(const S* __restrict__ p, const T* __restrict__ a, S K,
                                                   S* __restrict__ out, int64_t n3) {
  const int64_t stride = int64_t(gridDim.x) * kThreads;
  for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < n3; i += stride) out[i] = fma(S(a[i]), K, p[i]);
}

template <typename S>
__global__ __launch_bounds__(kThreads) void k_drift(const S* __restrict__ s, const S* __restrict__ p, S D,
                                                    S* __restrict__ out, int64_t n3) {
  const int64_t stride = int64_t(gridDim.x) * kThreads;
  for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < n3; i += stride) out[i] = fma(p[i], D, s[i]);
}

#define LC_PLAN(h)                              \
  Plan* p = reinterpret_cast<Plan*>(h);         \
  if (!p) return set_error(nullptr, PM_EINVAL, "plan is NULL")

int lc_ptr(Plan* p, const void* ptr, const char* name) {
  if (!ptr) return set_error(p, PM_EINVAL, "%s is NULL", name);
  return PM_OK;
}

int lc_device(Plan* p) {
  int cur = -1;
  PM_HIP_CHECK(p, hipGetDevice(&cur));
  if (cur != p->device) PM_HIP_CHECK(p, hipSetDevice(p->device));
  return PM_OK;
}

int elementwise_blocks(int64_t n3) {
  const int64_t need = (n3 + kThreads - 1) / kThreads;
  return int(need < 2048 ? (need < 1 ? 1 : need) : 2048);   // <= kMaxPartials
}

int check_lc_step(Plan* p, const pm_lc_step* st) {
  if (!st) return set_error(p, PM_EINVAL, "light-cone step is NULL");
  if (st->step < 1) return set_error(p, PM_EINVAL, "light-cone step index must be >= 1");
  if (!(st->c0.a > 0.0 && st->c0.a < st->c1.a && st->c1.a <= 1.0))
    return set_error(p, PM_EINVAL, "light-cone step needs 0 < c0.a < c1.a <= 1");
  if (!(st->omega_m > 0.0 && st->omega_m <= 1.0)) return set_error(p, PM_EINVAL, "Omega_m out of range");
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(st->observer[k])) return set_error(p, PM_EINVAL, "observer position is not finite");
  return PM_OK;
}

// x[c][n] = 0 for the particles observed in steps 1..last (the frozen
// sources of the truncated adjoint)
template <typename T>
__global__ __launch_bounds__(kThreads) void k_truncate(T* __restrict__ x, const int32_t* __restrict__ obs_step,
                                                       int32_t last, int64_t N) {
  const int64_t stride = int64_t(gridDim.x) * kThreads;
  for (int64_t n = int64_t(blockIdx.x) * kThreads + threadIdx.x; n < N; n += stride) {
    const int32_t k = obs_step[n];
    if (k > 0 && k <= last) {
#pragma unroll
      for (int c = 0; c < 3; ++c) x[c * N + n] = T(0);
    }
  }
}

// largest |q + s - X| over the particles: per-block maxima in part[b * 4],
// then one workgroup folds them (NaN if any distance is NaN)
template <typename S>
__global__ __launch_bounds__(kThreads) void k_reach(TileGeo g, const S* __restrict__ s, double X0, double X1,
                                                    double X2, double* part) {
  auto fold = [](double m, double a) { return (a > m || a != a) ? a : m; };
  double m = 0.0;
  const int64_t stride = int64_t(gridDim.x) * kThreads;
  for (int64_t n = int64_t(blockIdx.x) * kThreads + threadIdx.x; n < g.N; n += stride) {
    double q[3];
    lattice_pos(g, n, q);
    const double d0 = q[0] + double(s[n]) - X0, d1 = q[1] + double(s[g.N + n]) - X1,
                 d2 = q[2] + double(s[2 * g.N + n]) - X2;
    m = fold(m, sqrt(fma(d0, d0, fma(d1, d1, d2 * d2))));
  }
  const double t = block_max_d(m);
  if (threadIdx.x == 0) part[blockIdx.x * 4] = t;
}

__global__ __launch_bounds__(kThreads) void k_reach_fold(const double* part, int nblocks, double* out) {
  auto fold = [](double m, double a) { return (a > m || a != a) ? a : m; };
  double m = 0.0;
  for (int b = threadIdx.x; b < nblocks; b += kThreads) m = fold(m, part[b * 4]);
  const double t = block_max_d(m);
  if (threadIdx.x == 0) out[0] = t;
}

LcGeo lc_geo(const Plan* p, const pm_lc_step* st) {
  LcGeo L;
  L.g = tile_geo(p);
  L.a0 = st->c0.a;
  L.da = st->c1.a - st->c0.a;
  L.om = st->omega_m;
  for (int k = 0; k < 3; ++k) L.X[k] = st->observer[k];
  L.c0 = st->c0.chi;
  L.t0 = L.da * st->c0.dchi;
  L.c1 = st->c1.chi;
  L.t1 = L.da * st->c1.dchi;
  L.w0 = st->c0.w;
  L.w1 = st->c1.w;
  L.c0o = st->c0.chi_om;
  L.t0o = L.da * st->c0.dchi_om;
  L.c1o = st->c1.chi_om;
  L.t1o = L.da * st->c1.dchi_om;
  L.w0o = st->c0.w_om;
  L.w1o = st->c1.w_om;
  L.step = st->step;
  return L;
}

}  // namespace
}  // namespace pmx

using namespace pmx;

extern "C" int pm_lightcone(pm_plan h, const pm_lc_step* st, const void* s0, const void* p0, const void* s1,
                            const void* p1, void* obs, int32_t* obs_step, double* count, hipStream_t stream) {
  LC_PLAN(h);
  if (int rc = check_lc_step(p, st)) return rc;
  const void* ptrs[] = {s0, p0, s1, p1, obs, obs_step, count};
  const char* names[] = {"s0", "p0", "s1", "p1", "obs", "obs_step", "count"};
  for (int k = 0; k < 7; ++k)
    if (int rc = lc_ptr(p, ptrs[k], names[k])) return rc;
  if (int rc = lc_device(p)) return rc;
  const LcGeo L = lc_geo(p, st);
  const int blocks = blocks_for_particles(p);
  const double sb = p->cfg.state_dtype == PM_F64 ? 8.0 : 4.0;
  timing_begin(p, PM_K_LIGHTCONE, stream);
  if (p->cfg.state_dtype == PM_F64)
    hipLaunchKernelGGL(k_lightcone<double>, dim3(blocks), dim3(kThreads), 0, stream, L,
                       static_cast<const double*>(s0), static_cast<const double*>(p0), static_cast<const double*>(s1),
                       static_cast<const double*>(p1), static_cast<double*>(obs), obs_step, p->partials);
  else
    hipLaunchKernelGGL(k_lightcone<float>, dim3(blocks), dim3(kThreads), 0, stream, L,
                       static_cast<const float*>(s0), static_cast<const float*>(p0), static_cast<const float*>(s1),
                       static_cast<const float*>(p1), static_cast<float*>(obs), obs_step, p->partials);
  PM_HIP_CHECK(p, hipGetLastError());
  timing_end(p, PM_K_LIGHTCONE, stream, 6.0 * double(p->nptcl) * sb, 6.0 * double(p->nptcl) * sb);
  const double f[4] = {1.0, 0.0, 0.0, 0.0};
  return reduce_partials(p, blocks, f, count, true, stream);
}

extern "C" int pm_lightcone_reach(pm_plan h, const void* disp, const double* observer, double* r_max,
                                  hipStream_t stream) {
  LC_PLAN(h);
  if (int rc = lc_ptr(p, disp, "disp")) return rc;
  if (int rc = lc_ptr(p, r_max, "r_max")) return rc;
  if (!observer) return set_error(p, PM_EINVAL, "observer is NULL");
  for (int k = 0; k < 3; ++k)
    if (!std::isfinite(observer[k])) return set_error(p, PM_EINVAL, "observer position is not finite");
  if (int rc = lc_device(p)) return rc;
  const TileGeo g = tile_geo(p);
  const int blocks = elementwise_blocks(p->nptcl);
  if (p->cfg.state_dtype == PM_F64)
    hipLaunchKernelGGL(k_reach<double>, dim3(blocks), dim3(kThreads), 0, stream, g, static_cast<const double*>(disp),
                       observer[0], observer[1], observer[2], p->partials);
  else
    hipLaunchKernelGGL(k_reach<float>, dim3(blocks), dim3(kThreads), 0, stream, g, static_cast<const float*>(disp),
                       observer[0], observer[1], observer[2], p->partials);
  hipLaunchKernelGGL(k_reach_fold, dim3(1), dim3(kThreads), 0, stream, p->partials, blocks, r_max);
  PM_HIP_CHECK(p, hipGetLastError());
  return PM_OK;
}

extern "C" int pm_lightcone_truncate(pm_plan h, void* x, const int32_t* obs_step, int32_t last,
                                     hipStream_t stream) {
  LC_PLAN(h);
  if (int rc = lc_ptr(p, x, "x")) return rc;
  if (int rc = lc_ptr(p, obs_step, "obs_step")) return rc;
  if (int rc = lc_device(p)) return rc;
  if (last < 1) return PM_OK;
  const int blocks = elementwise_blocks(p->nptcl);
  if (p->cfg.mesh_dtype == PM_F64)
    hipLaunchKernelGGL(k_truncate<double>, dim3(blocks), dim3(kThreads), 0, stream, static_cast<double*>(x), obs_step,
                       last, p->nptcl);
  else
    hipLaunchKernelGGL(k_truncate<float>, dim3(blocks), dim3(kThreads), 0, stream, static_cast<float*>(x), obs_step,
                       last, p->nptcl);
  PM_HIP_CHECK(p, hipGetLastError());
  return PM_OK;
}

extern "C" int pm_lightcone_vjp(pm_plan h, const pm_lc_step* st, const void* s0, const void* p0, const void* s1,
                                const void* p1, const int32_t* obs_step, const void* obs_bar, void* x0_bar,
                                void* p0_bar, void* x1_bar, void* p1_bar, double* theta_bar, hipStream_t stream) {
  LC_PLAN(h);
  if (int rc = check_lc_step(p, st)) return rc;
  const void* ptrs[] = {s0, p0, s1, p1, obs_step, obs_bar, theta_bar};
  const char* names[] = {"s0", "p0", "s1", "p1", "obs_step", "obs_bar", "theta_bar"};
  for (int k = 0; k < 7; ++k)
    if (int rc = lc_ptr(p, ptrs[k], names[k])) return rc;
  if (int rc = lc_device(p)) return rc;
  const LcGeo L = lc_geo(p, st);
  const int blocks = blocks_for_particles(p);
  timing_begin(p, PM_K_LIGHTCONE, stream);
#define PM_LC_VJP(S, T)                                                                                      \
  hipLaunchKernelGGL((k_lightcone_vjp<S, T>), dim3(blocks), dim3(kThreads), 0, stream, L,                   \
                     static_cast<const S*>(s0), static_cast<const S*>(p0), static_cast<const S*>(s1),        \
                     static_cast<const S*>(p1), obs_step, static_cast<const T*>(obs_bar),                   \
                     static_cast<T*>(x0_bar), static_cast<T*>(p0_bar), static_cast<T*>(x1_bar),             \
                     static_cast<T*>(p1_bar), p->partials)
  if (p->cfg.mesh_dtype == PM_F64) PM_LC_VJP(double, double);
  else if (p->cfg.state_dtype == PM_F64) PM_LC_VJP(double, float);
  else PM_LC_VJP(float, float);
#undef PM_LC_VJP
  PM_HIP_CHECK(p, hipGetLastError());
  timing_end(p, PM_K_LIGHTCONE, stream, 4.0 * double(p->nptcl), 4.0 * double(p->nptcl));
  const double f[4] = {1.0, 0.0, 0.0, 0.0};
  return reduce_partials(p, blocks, f, theta_bar, true, stream);
}

extern "C" int pm_adj_bump(pm_plan h, void* xi, void* pi, const void* x_bar, const void* p_bar, const void* c,
                           double Kb, double dKb, const void* acc, const double* omega_m_bar, double* theta_bar,
                           hipStream_t stream) {
  LC_PLAN(h);
  const void* ptrs[] = {xi, x_bar, theta_bar};
  const char* names[] = {"xi", "x_bar", "theta_bar"};
  for (int k = 0; k < 3; ++k)
    if (int rc = lc_ptr(p, ptrs[k], names[k])) return rc;
  if (p_bar && !pi) return set_error(p, PM_EINVAL, "pi is NULL");
  if (!p_bar && acc) return set_error(p, PM_EINVAL, "acc needs p_bar");
  if (!std::isfinite(Kb) || !std::isfinite(dKb)) return set_error(p, PM_EINVAL, "Kb and dKb must be finite");
  if (int rc = lc_device(p)) return rc;
  const int64_t n3 = 3 * p->nptcl;
  const int blocks = elementwise_blocks(n3);
  const double mb = p->cfg.mesh_dtype == PM_F64 ? 8.0 : 4.0;
  timing_begin(p, PM_K_LIGHTCONE, stream);
  if (p->cfg.mesh_dtype == PM_F64)
    hipLaunchKernelGGL(k_adj_bump<double>, dim3(blocks), dim3(kThreads), 0, stream, static_cast<double*>(xi),
                       static_cast<double*>(pi), static_cast<const double*>(x_bar), static_cast<const double*>(p_bar),
                       static_cast<const double*>(c), Kb, static_cast<const double*>(acc), omega_m_bar, n3, p->partials);
  else
    hipLaunchKernelGGL(k_adj_bump<float>, dim3(blocks), dim3(kThreads), 0, stream, static_cast<float*>(xi),
                       static_cast<float*>(pi), static_cast<const float*>(x_bar), static_cast<const float*>(p_bar),
                       static_cast<const float*>(c), float(Kb), static_cast<const float*>(acc), omega_m_bar, n3,
                       p->partials);
  PM_HIP_CHECK(p, hipGetLastError());
  const double bump_bytes = double(n3) * mb * ((p_bar ? 6.0 : 3.0) + (c ? 1.0 : 0.0) + (acc ? 1.0 : 0.0));
  timing_end(p, PM_K_LIGHTCONE, stream, bump_bytes, bump_bytes);
  const double f[4] = {acc ? dKb : 0.0, omega_m_bar ? Kb : 0.0, 0.0, 0.0};
  if (f[0] == 0.0 && f[1] == 0.0) return PM_OK;
  return reduce_partials(p, blocks, f, theta_bar, true, stream);
}

extern "C" int pm_kick(pm_plan h, const void* pv, const void* acc, double K, void* p_out, hipStream_t stream) {
  LC_PLAN(h);
  if (int rc = lc_ptr(p, pv, "p")) return rc;
  if (int rc = lc_ptr(p, acc, "acc")) return rc;
  if (int rc = lc_ptr(p, p_out, "p_out")) return rc;
  if (!std::isfinite(K)) return set_error(p, PM_EINVAL, "K must be finite");
  if (int rc = lc_device(p)) return rc;
  const int64_t n3 = 3 * p->nptcl;
  const int blocks = elementwise_blocks(n3);
  if (p->cfg.mesh_dtype == PM_F64)
    hipLaunchKernelGGL((k_kick<double, double>), dim3(blocks), dim3(kThreads), 0, stream,
                       static_cast<const double*>(pv), static_cast<const double*>(acc), K,
                       static_cast<double*>(p_out), n3);
  else if (p->cfg.state_dtype == PM_F64)
    hipLaunchKernelGGL((k_kick<double, float>), dim3(blocks), dim3(kThreads), 0, stream,
                       static_cast<const double*>(pv), static_cast<const float*>(acc), K,
                       static_cast<double*>(p_out), n3);
  else
    hipLaunchKernelGGL((k_kick<float, float>), dim3(blocks), dim3(kThreads), 0, stream,
                       static_cast<const float*>(pv), static_cast<const float*>(acc), float(K),
                       static_cast<float*>(p_out), n3);
  PM_HIP_CHECK(p, hipGetLastError());
  return PM_OK;
}

extern "C" int pm_drift(pm_plan h, const void* s, const void* pv, double D, void* s_out, hipStream_t stream) {
  LC_PLAN(h);
  if (int rc = lc_ptr(p, s, "s")) return rc;
  if (int rc = lc_ptr(p, pv, "p")) return rc;
  if (int rc = lc_ptr(p, s_out, "s_out")) return rc;
  if (!std::isfinite(D)) return set_error(p, PM_EINVAL, "D must be finite");
  if (int rc = lc_device(p)) return rc;
  const int64_t n3 = 3 * p->nptcl;
  const int blocks = elementwise_blocks(n3);
  if (p->cfg.state_dtype == PM_F64)
    hipLaunchKernelGGL(k_drift<double>, dim3(blocks), dim3(kThreads), 0, stream, static_cast<const double*>(s),
                       static_cast<const double*>(pv), D, static_cast<double*>(s_out), n3);
  else
    hipLaunchKernelGGL(k_drift<float>, dim3(blocks), dim3(kThreads), 0, stream, static_cast<const float*>(s),
                       static_cast<const float*>(pv), float(D), static_cast<float*>(s_out), n3);
  PM_HIP_CHECK(p, hipGetLastError());
  return PM_OK;
}
