// 2LPT initial conditions (Sec. 2.1, eq. lpt) and their VJP, on the
// particle lattice, for pm_lpt / pm_lpt_vjp.
//
//   delta1(k) = A(k) W(k),  W = rfft(omega),  A = sqrt(P(k) / V_cell)
//   s1_j  = irfft( M1_j delta1 ),        M1_j = i k_j / k^2  (Nyquist of j -> 0)
//   H_ij  = irfft( M_ij delta1 ),        M_ij = k_i k_j / k^2 (i != j: Nyquist of i or j -> 0)
//   S     = sum_{i<j} (H_ii H_jj - H_ij^2)
//   s2_j  = irfft( M1_j rfft(S) )
//   s = r (D1 s1 + D2 s2),  p = r (P1 s1 + P2 s2)
// (s1 = -grad phi1 with laplacian phi1 = delta1, i.e. phi1 = -delta1/k^2; the
// same for s2 with phi2 sourced by S.)  k is in radians per lattice spacing;
// P(k) uses k_phys = |k| N / L in h/Mpc and V_cell = (L/N)^3.
//
// The VJP runs the same operators transposed: every step is irfft(M rfft(.))
// with a Hermitian multiplier, whose transpose is irfft(conj(M) rfft(.)).
// The Omega_m derivative through A(k) is the half-spectrum sum
//   (1/N) sum_k w_k Re[ dA/dOmega_m(k) W(k) conj(G(k)) ],  G = rfft(delta1bar),
// with w_k = 1 on the kz = 0 and kz = N/2 planes and 2 elsewhere.
#include <cmath>
#include <cstring>

#include "cosmo_eh.h"
#include "tiles.h"

namespace pmx {

namespace {

struct AmpP {
  double om, ob, h, ns, tcmb;
  double A, dA;      // P = A k^ns T^2 and dA/dOmega_m
  double box;        // Mpc/h
  int n;
  const double* tab; // A(k), dA/dOmega_m per m = |f|^2 (k_amp_table)
};

enum MulKind {
  MUL_ONE = 0,
  MUL_D1 = 1,   // + j (0..2): i k_j / k^2
  MUL_D2 = 4,   // + pair index (0..5): k_i k_j / k^2
};

__constant__ int kPairI[6] = {0, 1, 2, 0, 0, 1};
__constant__ int kPairJ[6] = {0, 1, 2, 1, 2, 2};

// (x, y, z) of half-spectrum index idx < 2^31 on an n^3 lattice (n a power of two)
__device__ __forceinline__ void decode(int idx, int logn, int nh, double inv_nh, int& x, int& y, int& z) {
  const int row = divmod_small(idx, nh, inv_nh, z);
  y = row & ((1 << logn) - 1);
  x = row >> logn;
}

// A(k) depends on |k| only, and |k|^2 = (2 pi / n)^2 m with the integer
// m = fx^2 + fy^2 + fz^2 of the lattice mode (m <= 3 (n/2)^2).  The transfer
// function and its Omega_m derivative are evaluated once per m, not once per
// mode: one thread per table entry.
__global__ __launch_bounds__(kThreads) void k_amp_table(AmpP ap, double* __restrict__ tab, int mmax) {
  const int m = int(blockIdx.x) * kThreads + int(threadIdx.x);
  if (m > mmax) return;
  double A = 0.0, dA = 0.0;
  if (m > 0) {
    const int n = ap.n;
    const double dk = 6.283185307179586476925286766559 / n;
    const double kph = ::sqrt(double(m)) * dk * n / ap.box;
    const Dual T = eh_nowiggle<Dual>(kph, Dual{ap.om, 1.0}, ap.ob, ap.h, ap.tcmb);
    const double cell = ap.box / n;
    const double base = ::sqrt(ap.A * ::pow(kph, ap.ns) / (cell * cell * cell));
    A = T.v * base;
    dA = A * (0.5 * ap.dA / ap.A + T.d / T.v);
  }
  tab[2 * m] = A;
  tab[2 * m + 1] = dA;
}

// amplitude A(k) and its Omega_m derivative at lattice mode (x, y, z)
__device__ __forceinline__ void amp_at(const AmpP& ap, int x, int y, int z, double& A, double& dA) {
  const int n = ap.n;
  const int fx = x < n / 2 ? x : x - n;
  const int fy = y < n / 2 ? y : y - n;
  const int m = fx * fx + fy * fy + z * z;
  A = ap.tab[2 * m];
  dA = ap.tab[2 * m + 1];
}

// out = [out +] M(k) [A(k)] in, M conj'ed if CONJ; one thread per mode of
// the half spectrum, in index order
template <typename T>
__global__ __launch_bounds__(kThreads) void k_mul(const Cx<T>* __restrict__ in, Cx<T>* __restrict__ out, int n,
                                                  int logn, int kind, int use_amp, int conj, int accumulate, AmpP ap) {
  const int nh = n / 2 + 1;
  const double dk = 6.283185307179586476925286766559 / n;
  const int64_t nmodes = int64_t(n) * n * nh;   // < 2^31 for n <= 1024
  const int64_t idx = int64_t(blockIdx.x) * kThreads + threadIdx.x;
  if (idx < nmodes) {
    const unsigned ui = unsigned(idx), row = ui / unsigned(nh);
    const int z = int(ui - row * unsigned(nh));
    const int y = int(row) & (n - 1), x = int(row) >> logn;
    const int f[3] = {x < n / 2 ? x : x - n, y < n / 2 ? y : y - n, z};
    const bool nyq[3] = {2 * x == n, 2 * y == n, 2 * z == n};
    double k[3];
    for (int a = 0; a < 3; ++a) k[a] = f[a] * dk;   // dk = 2 pi / n exactly (n a power of two)
    const double k2 = k[0] * k[0] + k[1] * k[1] + k[2] * k[2];
    const double inv = k2 > 0 ? 1.0 / k2 : 0.0;
    double re = 0.0, im = 0.0;  // multiplier re + i im
    if (kind == MUL_ONE) {
      re = 1.0;
    } else if (kind < MUL_D2) {
      const int j = kind - MUL_D1;
      im = nyq[j] ? 0.0 : k[j] * inv;
    } else {
      const int p = kind - MUL_D2;
      const int i = kPairI[p], j = kPairJ[p];
      re = (i != j && (nyq[i] || nyq[j])) ? 0.0 : k[i] * k[j] * inv;
    }
    if (conj) im = -im;
    if (use_amp) {
      double A, dA;
      amp_at(ap, x, y, z, A, dA);
      re *= A;
      im *= A;
    }
    const Cx<T> v = in[idx];
    T ore = T(re * double(v.x) - im * double(v.y));
    T oim = T(re * double(v.y) + im * double(v.x));
    if (accumulate) {
      ore += out[idx].x;
      oim += out[idx].y;
    }
    out[idx] = cmk<Cx<T>>(ore, oim);
  }
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_second_order(const T* __restrict__ H, T* __restrict__ S,
                                                           int64_t N) {
  const int64_t stride = int64_t(gridDim.x) * kThreads;
  for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < N; i += stride) {
    const T h00 = H[i], h11 = H[N + i], h22 = H[2 * N + i];
    const T h01 = H[3 * N + i], h02 = H[4 * N + i], h12 = H[5 * N + i];
    S[i] = h00 * h11 + h00 * h22 + h11 * h22 - h01 * h01 - h02 * h02 - h12 * h12;
  }
}

template <typename S, typename T>
__global__ __launch_bounds__(kThreads) void k_combine(const T* __restrict__ s1, const T* __restrict__ s2,
                                                      S* __restrict__ s, S* __restrict__ p, int64_t N, double r,
                                                      double D1, double D2, double P1, double P2) {
  const int64_t stride = int64_t(gridDim.x) * kThreads;
  for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < 3 * N; i += stride) {
    const double a = double(s1[i]), b = double(s2[i]);
    s[i] = S(r * (D1 * a + D2 * b));
    p[i] = S(r * (P1 * a + P2 * b));
  }
}

__device__ __forceinline__ double block_sum_l(double v) {
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

// s1bar = r (D1 xi + P1 pi), s2bar = r (D2 xi + P2 pi); partial sums
// slot 0: xi.s1, 1: pi.s1, 2: xi.s2, 3: pi.s2.  s2bar may overwrite s2 (each
// element is read before it is written, by the same thread).
template <typename T>
__global__ __launch_bounds__(kThreads) void k_bars(const T* xi, const T* pi, const T* s1, const T* s2, T* s1b,
                                                   T* s2b, int64_t N, double r,
                                                   double D1, double D2, double P1, double P2, double* partials) {
  const int64_t stride = int64_t(gridDim.x) * kThreads;
  double d[4] = {0, 0, 0, 0};
  for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < 3 * N; i += stride) {
    const double x = double(xi[i]), q = double(pi[i]);
    const double a = double(s1[i]), b = double(s2[i]);
    d[0] += x * a;
    d[1] += q * a;
    d[2] += x * b;
    d[3] += q * b;
    s1b[i] = T(r * (D1 * x + P1 * q));
    s2b[i] = T(r * (D2 * x + P2 * q));
  }
  for (int k = 0; k < 4; ++k) {
    const double t = block_sum_l(d[k]);
    if (threadIdx.x == 0) partials[blockIdx.x * 4 + k] = t;
  }
}

// Hbar_ii = Sbar sum_{j != i} H_jj, Hbar_ij = -2 Sbar H_ij (in place over H)
template <typename T>
__global__ __launch_bounds__(kThreads) void k_hbar(const T* __restrict__ Sb, T* __restrict__ H, int64_t N) {
  const int64_t stride = int64_t(gridDim.x) * kThreads;
  for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < N; i += stride) {
    const T s = Sb[i];
    const T h00 = H[i], h11 = H[N + i], h22 = H[2 * N + i];
    H[i] = s * (h11 + h22);
    H[N + i] = s * (h00 + h22);
    H[2 * N + i] = s * (h00 + h11);
    H[3 * N + i] = T(-2) * s * H[3 * N + i];
    H[4 * N + i] = T(-2) * s * H[4 * N + i];
    H[5 * N + i] = T(-2) * s * H[5 * N + i];
  }
}

// partial sums (slot 0) of w_k Re[dA W conj(G)] over the half spectrum
template <typename T>
__global__ __launch_bounds__(kThreads) void k_theta_amp(const Cx<T>* __restrict__ W, const Cx<T>* __restrict__ G,
                                                        int n, int logn, AmpP ap, double* partials) {
  const int nh = n / 2 + 1;
  const int total = n * n * nh;
  const int stride = gridDim.x * kThreads;
  const double inv_nh = 1.0 / double(nh);
  double acc = 0.0;
  for (int idx = blockIdx.x * kThreads + threadIdx.x; idx < total; idx += stride) {
    int x, y, z;
    decode(idx, logn, nh, inv_nh, x, y, z);
    double A, dA;
    amp_at(ap, x, y, z, A, dA);
    const double w = (z == 0 || 2 * z == n) ? 1.0 : 2.0;
    const Cx<T> a = W[idx], g = G[idx];
    acc += w * dA * (double(a.x) * double(g.x) + double(a.y) * double(g.y));
  }
  const double t = block_sum_l(acc);
  if (threadIdx.x == 0) partials[blockIdx.x * 4 + 0] = t;
}

// largest |f|^2 of a mode of the n^3 lattice's half spectrum
int amp_mmax(int n) { return 3 * (n / 2) * (n / 2); }

int grid_for(int64_t work) {
  const int64_t need = (work + kThreads - 1) / kThreads;
  return int(need < 2048 ? (need < 1 ? 1 : need) : 2048);
}

}  // namespace

int check_lattice(Plan* p) {
  const int n = p->np[0];
  if (p->np[1] != n || p->np[2] != n || n < 4 || n > 1024 || (n & (n - 1)))
    return set_error(p, PM_ESHAPE, "2LPT needs a cubic power-of-two particle lattice in [4, 1024]");
  if (!(p->cfg.box[0] > 0.0) || p->cfg.box[1] != p->cfg.box[0] || p->cfg.box[2] != p->cfg.box[0])
    return set_error(p, PM_EINVAL, "2LPT needs a cubic box of positive size");
  return PM_OK;
}

// lattice scratch: 16 real fields and 3 half spectra.  Kernels take the
// groups s1 (fields 0..2), H (3..8), s2 (10..12) and s1bar (13..15) as one
// base pointer each, so every group must be contiguous.  When the lattice has
// the mesh's shape, the plan's 4 meshes and first 3 spectra (idle outside the
// steps; nothing of the 2LPT calls outlives them) hold s1 and S (field 9) and
// the spectra, and only 12 real fields (H, s2, s1bar) are allocated.
bool lattice_is_mesh(const Plan* p) { return p->np[0] == p->n[0] && p->np[1] == p->n[1] && p->np[2] == p->n[2]; }

int ensure_lattice(Plan* p) {
  if (p->lpt_ready) return PM_OK;
  const int64_t n = p->np[0];
  const int64_t N = n * n * n;
  const int64_t ns = n * n * (n / 2 + 1);
  const size_t rb = p->real_bytes;
  const bool shared = lattice_is_mesh(p);
  if (hipMalloc(&p->lreal[0], size_t(shared ? 12 : 16) * N * rb) != hipSuccess) {
    (void)hipGetLastError();
    return set_error(p, PM_ENOMEM, "could not allocate 2LPT lattice fields");
  }
  if (!shared && hipMalloc(&p->lspec[0], size_t(3) * ns * 2 * rb) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipFree(p->lreal[0]);
    p->lreal[0] = nullptr;
    return set_error(p, PM_ENOMEM, "could not allocate 2LPT lattice spectra");
  }
  if (hipMalloc(&p->amp_tab, size_t(amp_mmax(int(n)) + 1) * 2 * sizeof(double)) != hipSuccess) {
    (void)hipGetLastError();
    (void)hipFree(p->lreal[0]);
    (void)hipFree(p->lspec[0]);
    p->lreal[0] = p->lspec[0] = nullptr;
    p->amp_tab = nullptr;
    return set_error(p, PM_ENOMEM, "could not allocate the 2LPT amplitude table");
  }
  p->lpt_ready = true;
  return PM_OK;
}

namespace {

template <typename T>
struct Lat {
  int n;
  int64_t N, ns;
  T* real(Plan* p, int i) const {
    if (lattice_is_mesh(p)) {
      if (i < 3) return static_cast<T*>(p->mesh[i]);
      if (i == 9) return static_cast<T*>(p->mesh[3]);
      return static_cast<T*>(p->lreal[0]) + int64_t(i < 9 ? i - 3 : i - 4) * N;
    }
    return static_cast<T*>(p->lreal[0]) + int64_t(i) * N;
  }
  Cx<T>* spec(Plan* p, int i) const {
    if (lattice_is_mesh(p)) return static_cast<Cx<T>*>(p->spec[i]);
    return static_cast<Cx<T>*>(p->lspec[0]) + int64_t(i) * ns;
  }
};

// the amplitude parameters of this call, and its table of A(k) and
// dA/dOmega_m formed on the stream
int amp_params(Plan* p, const pm_cosmo* c, const pm_ic_coef* ic, hipStream_t st, AmpP& ap) {
  ap.om = c->omega_m;
  ap.ob = c->omega_b;
  ap.h = c->h;
  ap.ns = c->n_s;
  ap.tcmb = c->t_cmb;
  ap.A = ic->A;
  ap.dA = ic->dA;
  ap.box = p->cfg.box[0];
  ap.n = p->np[0];
  ap.tab = p->amp_tab;
  const int mmax = amp_mmax(ap.n);
  hipLaunchKernelGGL(k_amp_table, dim3(unsigned(mmax / kThreads + 1)), dim3(kThreads), 0, st, ap, p->amp_tab, mmax);
  PM_HIP_CHECK(p, hipGetLastError());
  return PM_OK;
}

template <typename T>
int mul(Plan* p, const Lat<T>& L, const Cx<T>* in, Cx<T>* out, int kind, bool amp, bool conj, bool acc,
        const AmpP& ap, hipStream_t st) {
  const int64_t nmodes = int64_t(L.n) * L.n * (L.n / 2 + 1);
  hipLaunchKernelGGL((k_mul<T>), dim3(unsigned((nmodes + kThreads - 1) / kThreads)), dim3(kThreads), 0, st, in, out, L.n,
                     ilog2(L.n), kind, amp ? 1 : 0, conj ? 1 : 0, acc ? 1 : 0, ap);
  PM_HIP_CHECK(p, hipGetLastError());
  return PM_OK;
}

// forward fields: s1 -> real 0..2, H -> real 3..8, s2 -> real 10..12;
// W = rfft(omega) stays in spec 0, delta1(k) = A(k) W(k) is formed once in
// spec 2 (overwritten by the second-order step).  The first-order part (W,
// s1) alone when second_order is false.
template <typename T>
int forward_fields(Plan* p, const Lat<T>& L, const T* omega, const AmpP& ap, hipStream_t st,
                   bool second_order = true) {
  const FftShape fs{L.n, L.n, L.n};
  const T scale = T(2.0 / double(L.N));
  int rc = fft_r2c_3d<T>(p, fs, omega, L.spec(p, 0), 1, L.N, L.ns, st);
  if (rc) return rc;
  if ((rc = mul<T>(p, L, L.spec(p, 0), L.spec(p, 2), MUL_ONE, true, false, false, ap, st))) return rc;
  for (int j = 0; j < 3; ++j) {
    if ((rc = mul<T>(p, L, L.spec(p, 2), L.spec(p, 1), MUL_D1 + j, false, false, false, ap, st))) return rc;
    if ((rc = fft_c2r_3d<T>(p, fs, L.spec(p, 1), L.real(p, j), 1, L.ns, L.N, scale, st))) return rc;
  }
  if (!second_order) return PM_OK;
  for (int q = 0; q < 6; ++q) {
    if ((rc = mul<T>(p, L, L.spec(p, 2), L.spec(p, 1), MUL_D2 + q, false, false, false, ap, st))) return rc;
    if ((rc = fft_c2r_3d<T>(p, fs, L.spec(p, 1), L.real(p, 3 + q), 1, L.ns, L.N, scale, st))) return rc;
  }
  hipLaunchKernelGGL((k_second_order<T>), dim3(grid_for(L.N)), dim3(kThreads), 0, st, L.real(p, 3), L.real(p, 9),
                     L.N);
  PM_HIP_CHECK(p, hipGetLastError());
  if ((rc = fft_r2c_3d<T>(p, fs, L.real(p, 9), L.spec(p, 1), 1, L.N, L.ns, st))) return rc;
  for (int j = 0; j < 3; ++j) {
    if ((rc = mul<T>(p, L, L.spec(p, 1), L.spec(p, 2), MUL_D1 + j, false, false, false, ap, st))) return rc;
    if ((rc = fft_c2r_3d<T>(p, fs, L.spec(p, 2), L.real(p, 10 + j), 1, L.ns, L.N, scale, st))) return rc;
  }
  return PM_OK;
}

template <typename S, typename T>
int lpt_fwd_typed(Plan* p, const void* omega, const pm_cosmo* c, const pm_ic_coef* ic, pm_state* stt,
                  hipStream_t st) {
  Lat<T> L{p->np[0], int64_t(p->np[0]) * p->np[0] * p->np[0], int64_t(p->np[0]) * p->np[0] * (p->np[0] / 2 + 1)};
  AmpP ap;
  int rc = amp_params(p, c, ic, st, ap);
  if (rc) return rc;
  if ((rc = forward_fields<T>(p, L, static_cast<const T*>(omega), ap, st))) return rc;
  const double r = p->r[0];
  hipLaunchKernelGGL((k_combine<S, T>), dim3(grid_for(3 * L.N)), dim3(kThreads), 0, st, L.real(p, 0),
                     L.real(p, 10), static_cast<S*>(stt->s), static_cast<S*>(stt->p), L.N, r, ic->D1, ic->D2, ic->P1,
                     ic->P2);
  PM_HIP_CHECK(p, hipGetLastError());
  return PM_OK;
}

// kept: H and s2 of the same omega and cosmology are still in the lattice
// scratch (cfg.lpt_keep); only W and s1, which share the plan's meshes and
// spectra, are formed again
template <typename T>
int lpt_bwd_typed(Plan* p, const void* omega, const pm_cosmo* c, const pm_ic_coef* ic, const pm_adj* adj,
                  void* omega_bar, double* theta_bar, bool kept, hipStream_t st) {
  Lat<T> L{p->np[0], int64_t(p->np[0]) * p->np[0] * p->np[0], int64_t(p->np[0]) * p->np[0] * (p->np[0] / 2 + 1)};
  AmpP ap;
  int rc = amp_params(p, c, ic, st, ap);
  if (rc) return rc;
  const FftShape fs{L.n, L.n, L.n};
  const T scale = T(2.0 / double(L.N));
  const double r = p->r[0];
  if ((rc = forward_fields<T>(p, L, static_cast<const T*>(omega), ap, st, !kept))) return rc;
  // lattice fields: s1 0..2, H 3..8, S 9, s2 10..12; after k_bars s1bar is
  // in 13..15 and s2bar replaces s2 in 10..12.
  {
    const int nb = grid_for(3 * L.N);
    hipLaunchKernelGGL((k_bars<T>), dim3(nb), dim3(kThreads), 0, st, static_cast<const T*>(adj->xi),
                       static_cast<const T*>(adj->pi), L.real(p, 0), L.real(p, 10), L.real(p, 13), L.real(p, 10), L.N,
                       r, ic->D1, ic->D2, ic->P1, ic->P2, p->partials);
    PM_HIP_CHECK(p, hipGetLastError());
    // theta_bar[0] += r (dD1 xi.s1 + dP1 pi.s1 + dD2 xi.s2 + dP2 pi.s2)
    const double f0[4] = {r * ic->dD1, r * ic->dP1, r * ic->dD2, r * ic->dP2};
    if ((rc = reduce_partials(p, nb, f0, theta_bar, true, st))) return rc;
    // theta_bar[1] += r (D1 xi.s1 + P1 pi.s1 + 2 D2 xi.s2 + 2 P2 pi.s2) / sigma8
    const double is8 = 1.0 / c->sigma8;
    const double f1[4] = {r * ic->D1 * is8, r * ic->P1 * is8, 2 * r * ic->D2 * is8, 2 * r * ic->P2 * is8};
    if ((rc = reduce_partials(p, nb, f1, theta_bar + 1, true, st))) return rc;
  }
  // Sbar = irfft( sum_j conj(M1_j) rfft(s2bar_j) )  -> real 9
  for (int j = 0; j < 3; ++j) {
    if ((rc = fft_r2c_3d<T>(p, fs, L.real(p, 10 + j), L.spec(p, 1), 1, L.N, L.ns, st))) return rc;
    if ((rc = mul<T>(p, L, L.spec(p, 1), L.spec(p, 2), MUL_D1 + j, false, true, j > 0, ap, st))) return rc;
  }
  if ((rc = fft_c2r_3d<T>(p, fs, L.spec(p, 2), L.real(p, 9), 1, L.ns, L.N, scale, st))) return rc;
  // Hbar in place over H (real 3..8)
  hipLaunchKernelGGL((k_hbar<T>), dim3(grid_for(L.N)), dim3(kThreads), 0, st, L.real(p, 9), L.real(p, 3), L.N);
  PM_HIP_CHECK(p, hipGetLastError());
  // G = sum_j conj(M1_j) rfft(s1bar_j) + sum_pairs conj(M_ij) rfft(Hbar_ij)  -> spec 2
  for (int j = 0; j < 3; ++j) {
    if ((rc = fft_r2c_3d<T>(p, fs, L.real(p, 13 + j), L.spec(p, 1), 1, L.N, L.ns, st))) return rc;
    if ((rc = mul<T>(p, L, L.spec(p, 1), L.spec(p, 2), MUL_D1 + j, false, true, j > 0, ap, st))) return rc;
  }
  for (int q = 0; q < 6; ++q) {
    if ((rc = fft_r2c_3d<T>(p, fs, L.real(p, 3 + q), L.spec(p, 1), 1, L.N, L.ns, st))) return rc;
    if ((rc = mul<T>(p, L, L.spec(p, 1), L.spec(p, 2), MUL_D2 + q, false, true, true, ap, st))) return rc;
  }
  // theta_bar[0] += (1/N) sum w Re[dA W conj(G)]
  {
    const int nb = grid_for(L.ns);
    hipLaunchKernelGGL((k_theta_amp<T>), dim3(nb), dim3(kThreads), 0, st, L.spec(p, 0), L.spec(p, 2), L.n,
                       ilog2(L.n), ap, p->partials);
    PM_HIP_CHECK(p, hipGetLastError());
    const double f[4] = {1.0 / double(L.N), 0.0, 0.0, 0.0};
    if ((rc = reduce_partials(p, nb, f, theta_bar, true, st))) return rc;
  }
  // omega_bar = irfft( A G )
  if ((rc = mul<T>(p, L, L.spec(p, 2), L.spec(p, 1), MUL_ONE, true, false, false, ap, st))) return rc;
  return fft_c2r_3d<T>(p, fs, L.spec(p, 1), static_cast<T*>(omega_bar), 1, L.ns, L.N, scale, st);
}

}  // namespace

int lpt_forward(Plan* p, const void* omega, const pm_cosmo* c, const pm_ic_coef* ic, pm_state* st, hipStream_t s) {
  p->lpt_kept = false;
  int rc = check_lattice(p);
  if (rc) return rc;
  if ((rc = ensure_lattice(p))) return rc;
  if (p->cfg.mesh_dtype == PM_F64) rc = lpt_fwd_typed<double, double>(p, omega, c, ic, st, s);
  else if (p->cfg.state_dtype == PM_F64) rc = lpt_fwd_typed<double, float>(p, omega, c, ic, st, s);
  else rc = lpt_fwd_typed<float, float>(p, omega, c, ic, st, s);
  if (rc == PM_OK && p->cfg.lpt_keep) {
    p->lpt_kept = true;
    p->lpt_omega = omega;
    p->lpt_cosmo = *c;
    p->lpt_ic = *ic;
  }
  return rc;
}

int lpt_backward(Plan* p, const void* omega, const pm_cosmo* c, const pm_ic_coef* ic, const pm_adj* adj,
                 void* omega_bar, double* theta_bar, hipStream_t s) {
  // the fields pm_lpt kept serve this omega and cosmology only, and this
  // call overwrites them either way
  const bool kept = p->lpt_kept && omega == p->lpt_omega && std::memcmp(c, &p->lpt_cosmo, sizeof(pm_cosmo)) == 0 &&
                    std::memcmp(ic, &p->lpt_ic, sizeof(pm_ic_coef)) == 0;
  p->lpt_kept = false;
  int rc = check_lattice(p);
  if (rc) return rc;
  if ((rc = ensure_lattice(p))) return rc;
  if (p->cfg.mesh_dtype == PM_F64) return lpt_bwd_typed<double>(p, omega, c, ic, adj, omega_bar, theta_bar, kept, s);
  return lpt_bwd_typed<float>(p, omega, c, ic, adj, omega_bar, theta_bar, kept, s);
}

}  // namespace pmx

using namespace pmx;

extern "C" int pm_lpt(pm_plan h, const void* omega, const pm_cosmo* cosmo, const pm_ic_coef* ic, pm_state* st,
                      hipStream_t stream) {
  Plan* p = reinterpret_cast<Plan*>(h);
  if (!p) return set_error(nullptr, PM_EINVAL, "plan is NULL");
  if (!omega || !cosmo || !ic || !st || !st->s || !st->p) return set_error(p, PM_EINVAL, "pm_lpt: NULL argument");
  if (!(ic->A > 0.0)) return set_error(p, PM_EINVAL, "pm_lpt: ic->A must be > 0 (use pm_tables)");
  return lpt_forward(p, omega, cosmo, ic, st, stream);
}

extern "C" int pm_lpt_vjp(pm_plan h, const void* omega, const pm_cosmo* cosmo, const pm_ic_coef* ic,
                          const pm_adj* adj, void* omega_bar, double* theta_bar, hipStream_t stream) {
  Plan* p = reinterpret_cast<Plan*>(h);
  if (!p) return set_error(nullptr, PM_EINVAL, "plan is NULL");
  if (!omega || !cosmo || !ic || !adj || !adj->xi || !adj->pi || !omega_bar || !theta_bar)
    return set_error(p, PM_EINVAL, "pm_lpt_vjp: NULL argument");
  if (!(ic->A > 0.0)) return set_error(p, PM_EINVAL, "pm_lpt_vjp: ic->A must be > 0 (use pm_tables)");
  if (!(cosmo->sigma8 > 0.0)) return set_error(p, PM_EINVAL, "pm_lpt_vjp: sigma8 must be > 0");
  return lpt_backward(p, omega, cosmo, ic, adj, omega_bar, theta_bar, stream);
}
