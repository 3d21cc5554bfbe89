// Internal declarations shared by the HIP sources of libpm (not installed).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <string>

#include "pm.h"

namespace pmx {

constexpr int kThreads = 256;        // threads per workgroup for all kernels
constexpr int kTwiddleLog2 = 12;     // twiddle table exp(-2 pi i m / 4096)
constexpr int kTwiddleSize = 1 << kTwiddleLog2;
constexpr int kMaxPartials = 4096;   // per-block partial sums for reductions
constexpr int kReduceBlocks = 128;   // first level of the two-level reductions
constexpr int kScalars = 16 + kReduceBlocks;   // device scalars: [0, 16) named, then reduction staging

// ---------------------------------------------------------------------------
// complex helpers
// ---------------------------------------------------------------------------
template <typename T> struct alignas(2 * sizeof(T)) Cx {
  using value_type = T;
  T x, y;
};
template <typename T> using cplx = Cx<T>;

template <typename C> __host__ __device__ __forceinline__ C cmk(typename C::value_type re, typename C::value_type im) {
  C c; c.x = re; c.y = im; return c;
}
template <typename C> __device__ __forceinline__ C cadd(C a, C b) { return cmk<C>(a.x + b.x, a.y + b.y); }
template <typename C> __device__ __forceinline__ C csub(C a, C b) { return cmk<C>(a.x - b.x, a.y - b.y); }
template <typename C> __device__ __forceinline__ C cmul(C a, C b) {
  return cmk<C>(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename C> __device__ __forceinline__ C cconj(C a) { return cmk<C>(a.x, -a.y); }
template <typename C> __device__ __forceinline__ C cscale(C a, typename C::value_type s) { return cmk<C>(a.x * s, a.y * s); }
// multiply by -i (forward) or +i (inverse)
template <bool INV, typename C> __device__ __forceinline__ C cmul_mi(C a) {
  return INV ? cmk<C>(-a.y, a.x) : cmk<C>(a.y, -a.x);
}

// ---------------------------------------------------------------------------
// plan
// ---------------------------------------------------------------------------
constexpr int kTimingFamilies = 11;    // PM_K_* ids are 1..10
constexpr int kTimingSlots = 1024;     // launches recorded per family between reads
struct TimingFamily {
  hipEvent_t ev[2 * kTimingSlots] = {};   // created by pm_timing_enable (families 1..9)
  double bytes[kTimingSlots];
  double method_bytes[kTimingSlots];
  int nev = 0;
  double total_ms = 0.0;
  double total_bytes = 0.0;
  double total_method_bytes = 0.0;
  int64_t launches = 0;
  int64_t dropped = 0;
};
struct Timing {
  unsigned mask = 0;                   // bit k set: family k is timed
  bool created = false;
  TimingFamily fam[kTimingFamilies];
};

struct Plan {
  pm_config cfg;
  int device = 0;
  int n[3];            // mesh shape
  int nh;              // n[2]/2 + 1
  int64_t ncell;       // n0 n1 n2
  int64_t nspec;       // n0 n1 nh
  int np[3];           // lattice shape
  int64_t nptcl;
  double r[3];         // lattice spacing in cells per axis
  size_t real_bytes;   // bytes of one mesh-dtype scalar
  // scratch owned by the plan
  void* mesh[4] = {nullptr, nullptr, nullptr, nullptr};   // real meshes [ncell]
  void* spec[4] = {nullptr, nullptr, nullptr, nullptr};   // half spectra [nspec]
  void* tw = nullptr;                                      // twiddles (mesh dtype complex)
  double* partials = nullptr;                              // [kMaxPartials * 4]
  double* scalars = nullptr;                               // [kScalars] device scalars
  void* kick_al = nullptr;                                 // 3 N mesh dtype: the pending a or alpha of a native loop
  // paint binning (paint.hip): tiles of tile[0] x tile[1] x tile[2] cells
  int tile[3] = {8, 8, 32};
  int64_t ntiles = 0;
  int halo_cells = 0;
  unsigned* bin_counts = nullptr;   // [ntiles]
  unsigned* bin_offs = nullptr;     // [ntiles + 1]
  unsigned* bin_bsum = nullptr;     // [4 * kThreads]
  void* bin_keys = nullptr;         // [N] (tile, rank)
  void* bin_rec = nullptr;          // [N] float4 CIC records (FP32 meshes), else null
  unsigned* bin_list = nullptr;     // [N]
  void* bin_halo = nullptr;         // [4][ntiles][halo_cells] mesh dtype
  double* tile_partials = nullptr;  // [ntiles][4] per-tile reduction slots
  // lattice scratch for pm_lpt / pm_lpt_vjp (allocated lazily on first use)
  void* lreal[10] = {};
  void* lspec[2] = {};
  double* amp_tab = nullptr;   // [3 (np/2)^2 + 1][2] A(k), dA/dOmega_m per integer |f|^2
  bool lpt_ready = false;
  // the second-order fields of the last pm_lpt, kept for the next pm_lpt_vjp
  // of the same omega and cosmology (cfg.lpt_keep)
  bool lpt_kept = false;
  const void* lpt_omega = nullptr;
  pm_cosmo lpt_cosmo{};
  pm_ic_coef lpt_ic{};
  Timing timing;
  std::string err;
};

extern thread_local std::string g_create_error;

int set_error(Plan* p, int code, const char* fmt, ...);

#define PM_HIP_CHECK(plan, call)                                                   \
  do {                                                                             \
    hipError_t e_ = (call);                                                        \
    if (e_ != hipSuccess)                                                          \
      return pmx::set_error((plan), PM_EDEVICE, "%s: %s", #call, hipGetErrorString(e_)); \
  } while (0)

// kernel-launch bracketing for the timing facility.  `bytes` is the launch's
// algorithmic HBM traffic: every array it touches read or written once,
// including the implementation's own intermediate data (sort keys, CIC
// records, particle lists, halo faces).  `method_bytes` is the part the
// method itself needs: the particle state and mesh fields of the operation
// read or written once, with each 3-D FFT charged as one read and one write
// of its input and output (to its first and last pass), and nothing for the
// intermediates.
void timing_begin(Plan* p, int kernel, hipStream_t s);
void timing_end(Plan* p, int kernel, hipStream_t s, double bytes, double method_bytes);

inline int ilog2(int64_t v) { int l = 0; while ((int64_t(1) << l) < v) ++l; return l; }
__host__ __device__ constexpr int ilog2c(int v) { return v <= 1 ? 0 : 1 + ilog2c(v >> 1); }

// Map a linear workgroup id so that consecutive tiles land on the same XCD:
// the hardware hands workgroup b to XCD b % 8, so tile (b % 8) * per + b / 8
// gives each XCD a contiguous run of tiles (shared L2 for neighbours).
__device__ __forceinline__ int64_t xcd_tile(int64_t b, int64_t nblocks) {
  const int64_t nx = 8;
  int64_t per = nblocks / nx;
  int64_t rem = nblocks % nx;
  int64_t x = b % nx, i = b / nx;
  // XCDs x < rem own per + 1 tiles, the others per
  return x * per + (x < rem ? x : rem) + i;
}

// ---------------------------------------------------------------------------
// FFT launchers (fft.hip).  Shapes are explicit so that both the mesh and the
// particle lattice can be transformed.  All arrays use the layouts of pm.h.
// ---------------------------------------------------------------------------
struct FftShape {
  int n0, n1, n2;     // real shape, each a power of two in [4, 1024]
};

// Spectral multipliers of the force path, applied between the forward and
// inverse transforms along axis 0 (T_j = i k_j coef / k^2).
enum SpecOp {
  SPEC_NONE = 0,
  SPEC_GRAD3 = 1,     // out_j = T_j * in0, j = 0..2 (Poisson gradient)
  SPEC_ADJ4 = 2,      // out_0..2 = T_j * in0, out_3 = -sum_j T_j in_{1+j}
};

// The z faces of the tiled paint's halo (the cells above a tile's top plane,
// which belong to the bottom plane of the tile above) can be left out of the
// halo fold and added instead by the first z pass of the R2C that reads the
// painted mesh: there every such cell is one value of a line already in
// registers, while the fold would read and write a whole cache line for it.
struct ZFold {
  const void* halo;     // [nch][ntiles][hc] mesh dtype (channel = batch index); null: no fold
  int64_t ntiles;
  int hc, face;         // halo cells per tile; index of the z face within them
  int ln1;              // log2 of the mesh's y size
  int ltx, lty, ltz;    // log2 of the tile dims
  int nty, ntz;         // tiles along y and z
};

template <typename T>
int fft_r2c_3d(Plan* p, const FftShape& s, const T* in, cplx<T>* out, int batch,
               int64_t in_stride, int64_t out_stride, hipStream_t st);
// out may alias nothing; in is destroyed (used in place for the two c2c passes)
template <typename T>
int fft_c2r_3d(Plan* p, const FftShape& s, cplx<T>* in, T* out, int batch,
               int64_t in_stride, int64_t out_stride, T scale, hipStream_t st);
// real fields -> spectral multipliers -> real fields, in place:
//   GRAD3: reals[0] -> reals[0..2] = g_0..2;
//   ADJ4:  reals[0..3] = [rho, gbar_0..2] -> [g_0..2, rhobar].
// specs[0..3] are half-spectrum scratch buffers (clobbered).  zf (may be
// null): z faces of the paint that produced reals, still to be added.
template <typename T>
int fft_spectral_op(Plan* p, const FftShape& s, SpecOp op, T* const* reals, cplx<T>* const* specs,
                    T coef, const ZFold* zf, hipStream_t st);
// elementwise spectral multiplies used by the standalone Poisson call
template <typename T>
int poisson_grad_spec(Plan* p, const FftShape& s, const cplx<T>* in, cplx<T>* out, T coef,
                      hipStream_t st);

// ---------------------------------------------------------------------------
// particle kernels (particles.hip)
// ---------------------------------------------------------------------------
// DRIFT_SET: the adjoint drift with the new positions taken from s_set (a
// forward checkpoint) instead of s - p D
enum DriftMode { DRIFT_NONE = 0, DRIFT_FWD = 1, DRIFT_ADJ = 2, DRIFT_SET = 3 };

struct PaintArgs {
  const void* s;        // [3][N] state
  void* s_out;          // drift writes here (same as s, in place)
  const void* p;        // momentum (drift)
  const void* xi;       // adjoint drift
  void* pi;             // adjoint drift (in/out)
  const void* w;        // [nw][N] mesh-dtype weights or null
  int nw;               // number of weighted channels
  int unit;             // 1 if channel 0 is unit mass
  void* mesh;           // [nch][ncell]
  double D;             // drift coefficient
  double* partials;     // per-block partial sum of xi.p (adjoint drift)
  const void* s_set;    // DRIFT_SET: [3][N] state dtype, positions to land on
  bool defer_z;         // leave the z faces of the halo to the next R2C (paint_zfold)
  // kick left pending by the previous gather, applied by the drift before it
  // moves the particles: p += a Kp (forward), p -= a Kp and xi += alpha Kx
  // (adjoint); kick_a null: none
  const void* kick_a;   // 3 N mesh dtype a ([3][N], or [pos][3] with kick_sorted)
  const void* kick_al;  // 3 N mesh dtype alpha (adjoint), same layout
  double Kp, Kx;
  // the pending a (and alpha) are in the tile order of the previous binning
  // (the gather wrote them at each particle's list position), particle-major:
  // particle n's three values are at 3 (offs[key.x] + key.y) + 0..2 of its
  // previous (tile, rank) key
  bool kick_sorted;
  // pi (adjoint drift, and the weights of its four-channel paint) is
  // particle-major, [N][3], instead of [3][N]: the layout a native adjoint
  // loop keeps it in, so that the paint reads one 12-byte run per particle
  // through the lists instead of three scattered components
  bool pi_pm;
};
// pi (mesh dtype) between [3][N] and particle-major [N][3] in place (to_pm:
// to [N][3]), through the plan's mesh workspace of 4 ncell values, which
// must hold 3 N of them (pi_layout_fits)
bool pi_layout_fits(const Plan* p);
int pi_layout(Plan* p, void* pi, bool to_pm, hipStream_t st);
// apply a pending kick without a drift (the end of a native loop); a and al
// are particle-major in the tile order of the last binning (see
// PaintArgs::kick_sorted);
// acc_out (optional): a in lattice order
int kick_flush(Plan* p, void* pstate, const void* a, double Kp, bool adjoint, void* xi, const void* al, double Kx,
               void* acc_out, hipStream_t st);
int paint_launch(Plan* p, DriftMode mode, const PaintArgs& a, hipStream_t st);
// tile binning only (drift + bins + per-tile lists), as done by paint_launch
int bin_launch(Plan* p, DriftMode mode, const PaintArgs& a, hipStream_t st);
// tile shape of the binned paint for a mesh
void tile_dims(const int n[3], int tile[3], int64_t& ntiles, int& halo_cells);
// the z faces a paint with defer_z left in the plan's halo buffer
ZFold paint_zfold(const Plan* p);

enum GatherMode {
  GATHER_PLAIN = 0,     // out[c] = readout(mesh[c])
  GATHER_KICK_FWD = 1,  // a = readout(g), p += a K, optional store a
  GATHER_VJP = 2,       // a, alpha from (g0..2, rhobar), cotangent abar; partial abar.a
  GATHER_KICK_ADJ = 3,  // as VJP with cotangent pi, then p -= a K, xi += alpha K
  GATHER_MSE = 4,       // xbar = sum dW (mesh0), mesh0 = 2 (delta - target)/Np
};
struct GatherArgs {
  const void* s;        // [3][N] state
  const void* mesh;     // [nf][ncell]
  int nf;
  void* out;            // plain: [nf][N]; VJP/MSE: xbar [3][N]; sorted_out: [pos][3]
  void* acc;            // acceleration out (optional)
  void* p;              // kick target
  void* xi;             // adjoint kick target
  const void* cot;      // cotangent [3][N] (abar or pi)
  const void* acc_in;   // cached accelerations for the adjoint kick (optional)
  bool binned;          // the plan's tile bins already match s (set after a paint of s)
  // PLAIN (nf = 3) and VJP: write out (and acc) at each particle's position
  // in the tile lists instead of its lattice index, particle-major ([pos][3],
  // contiguous per tile), for a consumer that looks them up through the bins
  // (PaintArgs::kick_sorted)
  bool sorted_out;
  // cot is particle-major, [N][3] (PaintArgs::pi_pm)
  bool cot_pm;
  double K;
  double* partials;     // per-block partial of cot . a
};
int gather_launch(Plan* p, GatherMode mode, const GatherArgs& a, hipStream_t st);

// density-contrast difference for the MSE: m = 2 (rho Nc/Np - 1 - target)/Np,
// with the per-block partial sums of (delta - target)^2
int mse_mesh_launch(Plan* p, void* mesh, const void* target, double* partials, hipStream_t st);

// mesh <- mesh N_c/N_p - 1 (density contrast of a unit-mass paint)
int contrast_launch(Plan* p, void* mesh, hipStream_t st);

// deterministic reduction of per-block partials: out[k] (+)= sum_b part[b*4+k]
// scaled: out[o] (+)= sum_k f[k] * sum_b part[b*4+k] for up to 4 outputs
int reduce_partials(Plan* p, int nblocks, const double* coef /*host [4]*/, double* out,
                    bool accumulate, hipStream_t st);
int reduce_buffer(Plan* p, const double* buf, int64_t nblocks, const double* coef, double* out,
                  bool accumulate, hipStream_t st);

int blocks_for_particles(const Plan* p);

// ---------------------------------------------------------------------------
// initial conditions (lpt.hip)
// ---------------------------------------------------------------------------
// 2LPT lattice: shape check, and the scratch allocated once (pm_plan_create
// with lpt_scratch, else the first 2LPT call)
int check_lattice(Plan* p);
int ensure_lattice(Plan* p);
int lpt_forward(Plan* p, const void* omega, const pm_cosmo* c, const pm_ic_coef* ic, pm_state* st,
                hipStream_t s);
int lpt_backward(Plan* p, const void* omega, const pm_cosmo* c, const pm_ic_coef* ic,
                 const pm_adj* adj, void* omega_bar, double* theta_bar, hipStream_t s);

}  // namespace pmx
