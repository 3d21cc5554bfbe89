// C-ABI entry points of libpm: plan management and the hot-path calls
// (paint, FFT, Poisson gradient, readout, force, force VJP, KDK forward and
// adjoint steps, density objective).  Every call validates its arguments
// before launching and reports errors through pm_last_error.
#include <cmath>
#include <cstdarg>
#include <cstring>
#include <new>

#include "pm_internal.h"

using namespace pmx;

namespace pmx {

thread_local std::string g_create_error;

int set_error(Plan* p, int code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  if (p) p->err = buf;
  else g_create_error = buf;
  return code;
}

void timing_begin(Plan* p, int kernel, hipStream_t s) {
  Timing& t = p->timing;
  if (!t.created || kernel <= 0 || kernel >= kTimingFamilies || !(t.mask & (1u << kernel))) return;
  TimingFamily& f = t.fam[kernel];
  if (f.nev + 2 > 2 * kTimingSlots) return;
  (void)hipEventRecord(f.ev[f.nev], s);
}

void timing_end(Plan* p, int kernel, hipStream_t s, double bytes, double method_bytes) {
  Timing& t = p->timing;
  if (!t.created || kernel <= 0 || kernel >= kTimingFamilies || !(t.mask & (1u << kernel))) return;
  TimingFamily& f = t.fam[kernel];
  if (f.nev + 2 > 2 * kTimingSlots) {
    ++f.dropped;
    return;
  }
  (void)hipEventRecord(f.ev[f.nev + 1], s);
  f.bytes[f.nev / 2] = bytes;
  f.method_bytes[f.nev / 2] = method_bytes;
  f.nev += 2;
}

}  // namespace pmx

namespace {

bool pow2_in(int v, int lo, int hi) { return v >= lo && v <= hi && (v & (v - 1)) == 0; }

int validate_cfg(const pm_config* c, std::string& why) {
  if (!c) { why = "config is NULL"; return PM_EINVAL; }
  for (int a = 0; a < 3; ++a) {
    if (!pow2_in(c->mesh[a], 4, 1024)) { why = "mesh sizes must be powers of two in [4, 1024]"; return PM_ESHAPE; }
    if (c->ptcl[a] < 1 || c->ptcl[a] > 65536) { why = "particle lattice sizes must be in [1, 65536]"; return PM_ESHAPE; }
  }
  if ((c->mesh_dtype != PM_F32 && c->mesh_dtype != PM_F64) || (c->state_dtype != PM_F32 && c->state_dtype != PM_F64)) {
    why = "dtype must be PM_F32 or PM_F64";
    return PM_EINVAL;
  }
  if (c->mesh_dtype == PM_F64 && c->state_dtype == PM_F32) {
    why = "FP64 mesh with FP32 state is not supported";
    return PM_EUNSUPPORTED;
  }
  if (c->deterministic != 0 && c->deterministic != 1) { why = "deterministic must be 0 or 1"; return PM_EINVAL; }
  if (c->lpt_scratch != 0 && c->lpt_scratch != 1) { why = "lpt_scratch must be 0 or 1"; return PM_EINVAL; }
  if (c->lpt_keep != 0 && c->lpt_keep != 1) { why = "lpt_keep must be 0 or 1"; return PM_EINVAL; }
  if (c->lpt_scratch) {
    const int n = c->ptcl[0];
    if (c->ptcl[1] != n || c->ptcl[2] != n || !pow2_in(n, 4, 1024)) {
      why = "lpt_scratch needs a cubic power-of-two particle lattice in [4, 1024]";
      return PM_ESHAPE;
    }
    if (!(c->box[0] > 0.0) || c->box[1] != c->box[0] || c->box[2] != c->box[0]) {
      why = "lpt_scratch needs a cubic box of positive size";
      return PM_EINVAL;
    }
  }
  const int64_t np = int64_t(c->ptcl[0]) * c->ptcl[1] * c->ptcl[2];
  if (np > (int64_t(1) << 31)) { why = "at most 2^31 particles"; return PM_ESHAPE; }
  if (!std::isfinite(c->lattice_offset)) { why = "lattice_offset must be finite"; return PM_EINVAL; }
  return PM_OK;
}

struct Sizes {
  int64_t ncell, nspec, nptcl, ntiles;
  int halo_cells;
  size_t rb;
  size_t mesh_bytes, spec_bytes, tw_bytes, part_bytes, scal_bytes, bin_bytes, kick_bytes;
  size_t total() const {
    return mesh_bytes + spec_bytes + tw_bytes + part_bytes + scal_bytes + bin_bytes + kick_bytes;
  }
};

Sizes sizes_of(const pm_config* c) {
  Sizes s;
  s.ncell = int64_t(c->mesh[0]) * c->mesh[1] * c->mesh[2];
  s.nspec = int64_t(c->mesh[0]) * c->mesh[1] * (c->mesh[2] / 2 + 1);
  s.rb = c->mesh_dtype == PM_F64 ? 8 : 4;
  s.mesh_bytes = size_t(4) * s.ncell * s.rb;
  s.spec_bytes = size_t(4) * s.nspec * 2 * s.rb;
  s.tw_bytes = size_t(kTwiddleSize) * 2 * s.rb;
  s.part_bytes = size_t(kMaxPartials) * 4 * sizeof(double);
  s.scal_bytes = size_t(kScalars) * sizeof(double);
  // a or alpha of the kick a native loop leaves pending: 3 N mesh-dtype values
  // (particle-major in tile order)
  s.kick_bytes = size_t(3) * size_t(int64_t(c->ptcl[0]) * c->ptcl[1] * c->ptcl[2]) * s.rb;
  int tile[3];
  tile_dims(c->mesh, tile, s.ntiles, s.halo_cells);
  s.nptcl = int64_t(c->ptcl[0]) * c->ptcl[1] * c->ptcl[2];
  // CIC records (FP32 meshes), keys, per-tile partials, halo faces, list, counts, offsets, block sums
  s.bin_bytes = (s.rb == 4 ? size_t(s.nptcl) * 16 : 0) + size_t(s.nptcl) * 8 + size_t(s.ntiles) * 4 * sizeof(double) +
                size_t(4) * s.ntiles * s.halo_cells * s.rb + size_t(s.nptcl) * 4 + size_t(s.ntiles) * 4 +
                size_t(s.ntiles + 1) * 4 + size_t(4 * kThreads) * 4;
  return s;
}

Plan* P(pm_plan h) { return reinterpret_cast<Plan*>(h); }

template <typename T>
__global__ void k_finite(const T* x, int64_t n, int* bad) {
  const int64_t stride = int64_t(gridDim.x) * blockDim.x;
  bool ok = true;
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) ok = ok && isfinite(x[i]);
  if (!ok) *bad = 1;
}

#define CHECK_PLAN(h)                                   \
  Plan* p = P(h);                                       \
  if (!p) return set_error(nullptr, PM_EINVAL, "plan is NULL")

int check_ptr(Plan* p, const void* ptr, const char* name) {
  if (!ptr) return set_error(p, PM_EINVAL, "%s is NULL", name);
  return PM_OK;
}

int set_device(Plan* p) {
  int cur = -1;
  PM_HIP_CHECK(p, hipGetDevice(&cur));
  if (cur != p->device) PM_HIP_CHECK(p, hipSetDevice(p->device));
  return PM_OK;
}

FftShape mesh_shape(const Plan* p) { return FftShape{p->n[0], p->n[1], p->n[2]}; }

template <typename T>
T* mesh_ptr(Plan* p, int i) { return static_cast<T*>(p->mesh[i]); }
template <typename T>
cplx<T>* spec_ptr(Plan* p, int i) { return static_cast<cplx<T>*>(p->spec[i]); }

// The Poisson equation for phi~ = a phi in units H0 = 1 has the source
// 1.5 Omega_m delta (Sec. 2.2); every entry point takes Omega_m and forms the
// coefficient here, so callers never repeat the 1.5.
double poisson_coef(double omega_m) { return 1.5 * omega_m; }

// coefficient of the fused Poisson multiplier: 1.5 Omega_m N_c / N_p (delta = rho N_c/N_p - 1)
double mass_coef(const Plan* p, double omega_m) {
  return poisson_coef(omega_m) * double(p->ncell) / double(p->nptcl);
}

// Both follow a paint made with defer_z: the R2C adds the paint's z faces.
template <typename T>
int force_fields(Plan* p, double omega_m, hipStream_t st) {
  // mesh0 holds the painted mass; leaves g_0..2 in mesh0..2
  T* reals[3] = {mesh_ptr<T>(p, 0), mesh_ptr<T>(p, 1), mesh_ptr<T>(p, 2)};
  cplx<T>* specs[3] = {spec_ptr<T>(p, 0), spec_ptr<T>(p, 1), spec_ptr<T>(p, 2)};
  const ZFold zf = paint_zfold(p);
  return fft_spectral_op<T>(p, mesh_shape(p), SPEC_GRAD3, reals, specs, T(mass_coef(p, omega_m)), &zf, st);
}

template <typename T>
int vjp_fields(Plan* p, double omega_m, hipStream_t st) {
  // mesh0..3 hold [rho, gbar_x, gbar_y, gbar_z]; leaves [g_x, g_y, g_z, rhobar]
  T* reals[4] = {mesh_ptr<T>(p, 0), mesh_ptr<T>(p, 1), mesh_ptr<T>(p, 2), mesh_ptr<T>(p, 3)};
  cplx<T>* specs[4] = {spec_ptr<T>(p, 0), spec_ptr<T>(p, 1), spec_ptr<T>(p, 2), spec_ptr<T>(p, 3)};
  const ZFold zf = paint_zfold(p);
  return fft_spectral_op<T>(p, mesh_shape(p), SPEC_ADJ4, reals, specs, T(mass_coef(p, omega_m)), &zf, st);
}

// paint (with the z faces deferred) and the force or VJP fields
int paint_force_fields(Plan* p, DriftMode mode, PaintArgs pa, double omega_m, hipStream_t st) {
  pa.defer_z = true;
  if (int rc = paint_launch(p, mode, pa, st)) return rc;
  return p->cfg.mesh_dtype == PM_F64 ? force_fields<double>(p, omega_m, st) : force_fields<float>(p, omega_m, st);
}
int paint_vjp_fields(Plan* p, DriftMode mode, PaintArgs pa, double omega_m, hipStream_t st) {
  pa.defer_z = true;
  if (int rc = paint_launch(p, mode, pa, st)) return rc;
  return p->cfg.mesh_dtype == PM_F64 ? vjp_fields<double>(p, omega_m, st) : vjp_fields<float>(p, omega_m, st);
}

int check_omega_m(Plan* p, double omega_m) {
  if (!std::isfinite(omega_m) || omega_m <= 0) return set_error(p, PM_EINVAL, "omega_m must be finite and > 0");
  return PM_OK;
}

int check_step(Plan* p, const pm_step_coef* c, const char* name) {
  if (!c) return set_error(p, PM_EINVAL, "%s is NULL", name);
  const double v[6] = {c->Ka, c->D, c->Kb, c->dKa, c->dD, c->dKb};
  for (double x : v)
    if (!std::isfinite(x)) return set_error(p, PM_EINVAL, "%s has a non-finite entry", name);
  return PM_OK;
}

size_t state_bytes(const Plan* p);

int check_adj_args(Plan* p, const pm_state* stt, const pm_adj* adj, const pm_step_coef* cur,
                   const pm_step_coef* prev, double omega_m, const double* theta_bar) {
  if (!stt || !adj) return set_error(p, PM_EINVAL, "state or adjoint is NULL");
  if (int rc = check_ptr(p, stt->s, "state.s")) return rc;
  if (int rc = check_ptr(p, stt->p, "state.p")) return rc;
  if (int rc = check_ptr(p, adj->xi, "adj.xi")) return rc;
  if (int rc = check_ptr(p, adj->pi, "adj.pi")) return rc;
  if (int rc = check_ptr(p, theta_bar, "theta_bar")) return rc;
  if (int rc = check_step(p, cur, "cur")) return rc;
  if (prev)
    if (int rc = check_step(p, prev, "prev")) return rc;
  return check_omega_m(p, omega_m);
}

// Reverse step i (eq. KDFKO_adj with merged kicks).  With s_set, the drift
// lands on the stored positions s_{i-1} instead of s_i - p_{i-1/2} D_i; with
// p_set, p_{i-3/2} is replaced by the stored momentum after the kick.
int step_adj(Plan* p, pm_state* stt, pm_adj* adj, const pm_step_coef* cur, const pm_step_coef* prev, double omega_m,
             double* theta_bar, const void* s_set, const void* p_set, hipStream_t st) {
  PaintArgs pa{};
  pa.s = stt->s;
  pa.p = stt->p;
  pa.xi = adj->xi;
  pa.pi = adj->pi;
  pa.unit = 1;
  pa.nw = 3;
  pa.mesh = p->mesh[0];
  pa.D = cur->D;
  pa.partials = p->partials;
  pa.s_set = s_set;
  if (int rc = paint_vjp_fields(p, s_set ? DRIFT_SET : DRIFT_ADJ, pa, omega_m, st)) return rc;
  const double K = cur->Ka + (prev ? prev->Kb : 0.0);
  const double dK = cur->dKa + (prev ? prev->dKb : 0.0);
  GatherArgs ga{};
  ga.s = stt->s;
  ga.mesh = p->mesh[0];
  ga.nf = 4;
  ga.p = stt->p;
  ga.xi = adj->xi;
  ga.cot = adj->pi;
  ga.K = K;
  ga.binned = true;
  if (int rc = gather_launch(p, GATHER_KICK_ADJ, ga, st)) return rc;
  // theta_bar[0] += (xi.p) dD  (drift partials)  +  (pi.a)(dK + K/Omega_m)  (tile partials; a is
  // proportional to Omega_m, so zeta = (pi.a)/Omega_m)
  const double fd[4] = {cur->dD, 0.0, 0.0, 0.0};
  if (int rc = reduce_partials(p, blocks_for_particles(p), fd, theta_bar, true, st)) return rc;
  const double fk[4] = {0.0, dK + K / omega_m, 0.0, 0.0};
  if (int rc = reduce_buffer(p, p->tile_partials, p->ntiles, fk, theta_bar, true, st)) return rc;
  if (p_set) PM_HIP_CHECK(p, hipMemcpyAsync(stt->p, p_set, state_bytes(p), hipMemcpyDeviceToDevice, st));
  return PM_OK;
}

size_t state_bytes(const Plan* p) {
  return size_t(3) * size_t(p->nptcl) * (p->cfg.state_dtype == PM_F64 ? 8 : 4);
}

// checkpoint steps strictly increasing in [1, n], every buffer given
int check_checkpoints(Plan* p, const pm_checkpoints* ck, int n) {
  if (!ck) return PM_OK;
  if (ck->count < 0) return set_error(p, PM_EINVAL, "checkpoint count must be >= 0");
  if (ck->count == 0) return PM_OK;
  if (!ck->step || !ck->s || !ck->p) return set_error(p, PM_EINVAL, "checkpoint arrays are NULL");
  for (int k = 0; k < ck->count; ++k) {
    const int j = ck->step[k];
    if (j < 1 || j > n) return set_error(p, PM_EINVAL, "checkpoint step %d outside [1, %d]", j, n);
    if (k > 0 && j <= ck->step[k - 1]) return set_error(p, PM_EINVAL, "checkpoint steps must increase");
    if (!ck->s[k] || !ck->p[k]) return set_error(p, PM_EINVAL, "checkpoint %d has a NULL buffer", j);
  }
  return PM_OK;
}

// index of step j among the checkpoints, or -1
int checkpoint_index(const pm_checkpoints* ck, int j) {
  if (!ck) return -1;
  for (int k = 0; k < ck->count; ++k)
    if (ck->step[k] == j) return k;
  return -1;
}

}  // namespace

extern "C" {

const char* pm_strerror(int code) {
  switch (code) {
    case PM_OK: return "ok";
    case PM_EINVAL: return "invalid argument";
    case PM_ESHAPE: return "unsupported shape";
    case PM_ENOMEM: return "device allocation failed";
    case PM_EDEVICE: return "HIP error";
    case PM_EUNSUPPORTED: return "unsupported configuration";
    case PM_ENONFINITE: return "non-finite value";
    default: return "unknown error";
  }
}

const char* pm_last_error(pm_plan h) {
  if (!h) return g_create_error.c_str();
  return P(h)->err.c_str();
}

size_t pm_workspace_bytes(const pm_config* cfg) {
  std::string why;
  if (validate_cfg(cfg, why) != PM_OK) return 0;
  size_t total = sizes_of(cfg).total();
  // 2LPT lattice scratch (16 real fields, 3 half spectra; 12 real fields when
  // the lattice has the mesh's shape and shares the plan's meshes and
  // spectra) and the amplitude table (two doubles per |f|^2 <= 3 (n/2)^2),
  // allocated by the first pm_lpt / pm_lpt_vjp call on a cubic lattice
  const int64_t n = cfg->ptcl[0];
  if (cfg->ptcl[1] == n && cfg->ptcl[2] == n) {
    const size_t rb = cfg->mesh_dtype == PM_F64 ? 8 : 4;
    const bool shared = cfg->mesh[0] == n && cfg->mesh[1] == n && cfg->mesh[2] == n;
    total += shared ? size_t(12) * n * n * n * rb
                    : size_t(16) * n * n * n * rb + size_t(3) * n * n * (n / 2 + 1) * 2 * rb;
    total += size_t(3 * (n / 2) * (n / 2) + 1) * 2 * sizeof(double);
  }
  return total;
}

int pm_plan_create(const pm_config* cfg, pm_plan* out) {
  if (!out) return set_error(nullptr, PM_EINVAL, "out is NULL");
  *out = nullptr;
  std::string why;
  int rc = validate_cfg(cfg, why);
  if (rc) return set_error(nullptr, rc, "%s", why.c_str());
  Plan* p = new (std::nothrow) Plan();
  if (!p) return set_error(nullptr, PM_ENOMEM, "host allocation failed");
  p->cfg = *cfg;
  if (hipGetDevice(&p->device) != hipSuccess) {
    delete p;
    return set_error(nullptr, PM_EDEVICE, "no HIP device");
  }
  for (int a = 0; a < 3; ++a) {
    p->n[a] = cfg->mesh[a];
    p->np[a] = cfg->ptcl[a];
    p->r[a] = double(cfg->mesh[a]) / double(cfg->ptcl[a]);
  }
  p->nh = p->n[2] / 2 + 1;
  const Sizes s = sizes_of(cfg);
  p->ncell = s.ncell;
  p->nspec = s.nspec;
  p->nptcl = int64_t(p->np[0]) * p->np[1] * p->np[2];
  p->real_bytes = s.rb;
  tile_dims(p->n, p->tile, p->ntiles, p->halo_cells);
  // The tile offsets are scanned in blocks of 4 kThreads tiles whose sums one
  // workgroup scans again, so at most (4 kThreads)^2 tiles; and the CIC
  // record packs each base-node coordinate in 10 bits (tiles.h).  Both hold
  // for every mesh validate_cfg admits (sides <= 1024, tiles >= 8x8x16 cells
  // when the mesh is that large); refuse anything else before allocating.
  if ((p->ntiles + 4 * kThreads - 1) / (4 * kThreads) > 4 * kThreads || p->n[0] > 1024 || p->n[1] > 1024 ||
      p->n[2] > 1024) {
    delete p;
    return set_error(nullptr, PM_EUNSUPPORTED, "tile count or mesh side beyond the binning's limits");
  }
  void* mb = nullptr;
  void* sb = nullptr;
  void* bb = nullptr;
  if (hipMalloc(&mb, s.mesh_bytes) != hipSuccess || hipMalloc(&sb, s.spec_bytes) != hipSuccess ||
      hipMalloc(&bb, s.bin_bytes) != hipSuccess ||
      hipMalloc(&p->tw, s.tw_bytes) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&p->partials), s.part_bytes) != hipSuccess ||
      hipMalloc(reinterpret_cast<void**>(&p->scalars), s.scal_bytes) != hipSuccess ||
      hipMalloc(&p->kick_al, s.kick_bytes) != hipSuccess) {
    if (mb) (void)hipFree(mb);
    if (sb) (void)hipFree(sb);
    if (bb) (void)hipFree(bb);
    if (p->tw) (void)hipFree(p->tw);
    if (p->partials) (void)hipFree(p->partials);
    if (p->scalars) (void)hipFree(p->scalars);
    if (p->kick_al) (void)hipFree(p->kick_al);
    (void)hipGetLastError();
    delete p;
    return set_error(nullptr, PM_ENOMEM, "could not allocate %zu bytes of plan scratch", s.total());
  }
  for (int i = 0; i < 4; ++i) {
    p->mesh[i] = static_cast<char*>(mb) + size_t(i) * s.ncell * s.rb;
    p->spec[i] = static_cast<char*>(sb) + size_t(i) * s.nspec * 2 * s.rb;
  }
  {
    char* q = static_cast<char*>(bb);
    if (s.rb == 4) {
      p->bin_rec = q;  // 16-byte aligned first
      q += size_t(s.nptcl) * 16;
    }
    p->bin_keys = q;  // 8-byte aligned
    q += size_t(s.nptcl) * 8;
    p->tile_partials = reinterpret_cast<double*>(q);
    q += size_t(s.ntiles) * 4 * sizeof(double);
    p->bin_halo = q;
    q += size_t(4) * s.ntiles * s.halo_cells * s.rb;
    p->bin_list = reinterpret_cast<unsigned*>(q);
    q += size_t(s.nptcl) * 4;
    p->bin_counts = reinterpret_cast<unsigned*>(q);
    q += size_t(s.ntiles) * 4;
    p->bin_offs = reinterpret_cast<unsigned*>(q);
    q += size_t(s.ntiles + 1) * 4;
    p->bin_bsum = reinterpret_cast<unsigned*>(q);
  }
  // twiddles exp(-2 pi i m / 4096), computed in double precision
  if (s.rb == 8) {
    Cx<double>* h = new Cx<double>[kTwiddleSize];
    for (int m = 0; m < kTwiddleSize; ++m) {
      const double a = -2.0 * M_PI * double(m) / double(kTwiddleSize);
      h[m].x = std::cos(a);
      h[m].y = std::sin(a);
    }
    (void)hipMemcpy(p->tw, h, s.tw_bytes, hipMemcpyHostToDevice);
    delete[] h;
  } else {
    Cx<float>* h = new Cx<float>[kTwiddleSize];
    for (int m = 0; m < kTwiddleSize; ++m) {
      const double a = -2.0 * M_PI * double(m) / double(kTwiddleSize);
      h[m].x = float(std::cos(a));
      h[m].y = float(std::sin(a));
    }
    (void)hipMemcpy(p->tw, h, s.tw_bytes, hipMemcpyHostToDevice);
    delete[] h;
  }
  (void)hipMemset(p->partials, 0, s.part_bytes);
  (void)hipMemset(p->scalars, 0, s.scal_bytes);
  if (hipDeviceSynchronize() != hipSuccess) {
    (void)hipFree(mb);
    (void)hipFree(sb);
    (void)hipFree(bb);
    (void)hipFree(p->tw);
    (void)hipFree(p->partials);
    (void)hipFree(p->scalars);
    (void)hipFree(p->kick_al);
    delete p;
    return set_error(nullptr, PM_EDEVICE, "plan initialisation failed");
  }
  if (p->cfg.lpt_scratch) {
    // the 2LPT lattice scratch now (validate_cfg checked the lattice), so
    // that pm_lpt / pm_lpt_vjp allocate nothing
    if (int rc = ensure_lattice(p)) {
      const std::string why = p->err;
      (void)pm_plan_destroy(reinterpret_cast<pm_plan>(p));
      return set_error(nullptr, rc, "%s", why.c_str());
    }
  }
  *out = reinterpret_cast<pm_plan>(p);
  return PM_OK;
}

int pm_plan_destroy(pm_plan h) {
  CHECK_PLAN(h);
  (void)set_device(p);
  (void)hipDeviceSynchronize();
  (void)hipFree(p->mesh[0]);
  (void)hipFree(p->spec[0]);
  (void)hipFree(p->bin_rec ? p->bin_rec : p->bin_keys);   // the start of the binning buffer
  (void)hipFree(p->tw);
  (void)hipFree(p->partials);
  (void)hipFree(p->scalars);
  (void)hipFree(p->kick_al);
  for (void* q : p->lreal) if (q) (void)hipFree(q);
  for (void* q : p->lspec) if (q) (void)hipFree(q);
  (void)hipFree(p->amp_tab);
  for (auto& f : p->timing.fam)
    for (auto& e : f.ev)
      if (e) (void)hipEventDestroy(e);
  // nothing above may leave a sticky error for the caller's next HIP call
  (void)hipGetLastError();
  delete p;
  return PM_OK;
}

int pm_paint(pm_plan h, const void* disp, const void* weights, int nch, void* mesh, hipStream_t st) {
  CHECK_PLAN(h);
  if (int rc = check_ptr(p, disp, "disp")) return rc;
  if (int rc = check_ptr(p, mesh, "mesh")) return rc;
  if (nch < 1 || nch > 4) return set_error(p, PM_EINVAL, "nch must be in 1..4");
  if (!weights && nch != 1) return set_error(p, PM_EINVAL, "unit-mass paint needs nch = 1");
  if (int rc = set_device(p)) return rc;
  PaintArgs a{};
  a.s = disp;
  a.w = weights;
  a.nw = weights ? nch : 0;
  a.unit = weights ? 0 : 1;
  a.mesh = mesh;
  return paint_launch(p, DRIFT_NONE, a, st);
}

int pm_fft(pm_plan h, int dir, void* in, void* out, int batch, hipStream_t st) {
  CHECK_PLAN(h);
  if (int rc = check_ptr(p, in, "in")) return rc;
  if (int rc = check_ptr(p, out, "out")) return rc;
  if (dir != 1 && dir != -1) return set_error(p, PM_EINVAL, "dir must be +1 or -1");
  if (batch < 1 || batch > 4) return set_error(p, PM_EINVAL, "batch must be in 1..4");
  if (in == out) return set_error(p, PM_EINVAL, "in and out must not overlap");
  if (int rc = set_device(p)) return rc;
  const FftShape s = mesh_shape(p);
  if (p->cfg.mesh_dtype == PM_F64) {
    if (dir == 1)
      return fft_r2c_3d<double>(p, s, static_cast<const double*>(in), static_cast<cplx<double>*>(out), batch,
                                p->ncell, p->nspec, st);
    return fft_c2r_3d<double>(p, s, static_cast<cplx<double>*>(in), static_cast<double*>(out), batch, p->nspec,
                              p->ncell, 2.0 / double(p->ncell), st);
  }
  if (dir == 1)
    return fft_r2c_3d<float>(p, s, static_cast<const float*>(in), static_cast<cplx<float>*>(out), batch, p->ncell,
                             p->nspec, st);
  return fft_c2r_3d<float>(p, s, static_cast<cplx<float>*>(in), static_cast<float*>(out), batch, p->nspec,
                           p->ncell, float(2.0 / double(p->ncell)), st);
}

int pm_poisson_grad(pm_plan h, const void* delta_k, void* grad_k, double omega_m, hipStream_t st) {
  CHECK_PLAN(h);
  if (int rc = check_ptr(p, delta_k, "delta_k")) return rc;
  if (int rc = check_ptr(p, grad_k, "grad_k")) return rc;
  if (int rc = check_omega_m(p, omega_m)) return rc;
  if (int rc = set_device(p)) return rc;
  const FftShape s = mesh_shape(p);
  const double coef = poisson_coef(omega_m);
  if (p->cfg.mesh_dtype == PM_F64)
    return poisson_grad_spec<double>(p, s, static_cast<const cplx<double>*>(delta_k),
                                     static_cast<cplx<double>*>(grad_k), coef, st);
  return poisson_grad_spec<float>(p, s, static_cast<const cplx<float>*>(delta_k), static_cast<cplx<float>*>(grad_k),
                                  float(coef), st);
}

int pm_readout(pm_plan h, const void* disp, const void* mesh, int nch, void* out, hipStream_t st) {
  CHECK_PLAN(h);
  if (int rc = check_ptr(p, disp, "disp")) return rc;
  if (int rc = check_ptr(p, mesh, "mesh")) return rc;
  if (int rc = check_ptr(p, out, "out")) return rc;
  if (nch < 1 || nch > 4) return set_error(p, PM_EINVAL, "nch must be in 1..4");
  if (int rc = set_device(p)) return rc;
  GatherArgs a{};
  a.s = disp;
  a.mesh = mesh;
  a.nf = nch;
  a.out = out;
  return gather_launch(p, GATHER_PLAIN, a, st);
}

int pm_force(pm_plan h, const void* disp, double omega_m, void* acc, hipStream_t st) {
  CHECK_PLAN(h);
  if (int rc = check_ptr(p, disp, "disp")) return rc;
  if (int rc = check_ptr(p, acc, "acc")) return rc;
  if (int rc = check_omega_m(p, omega_m)) return rc;
  if (int rc = set_device(p)) return rc;
  PaintArgs pa{};
  pa.s = disp;
  pa.unit = 1;
  pa.mesh = p->mesh[0];
  if (int rc = paint_force_fields(p, DRIFT_NONE, pa, omega_m, st)) return rc;
  GatherArgs ga{};
  ga.s = disp;
  ga.mesh = p->mesh[0];
  ga.nf = 3;
  ga.out = acc;
  ga.binned = true;
  return gather_launch(p, GATHER_PLAIN, ga, st);
}

int pm_force_vjp(pm_plan h, const void* disp, const void* acc_bar, double omega_m, void* disp_bar,
                 double* omega_m_bar, void* acc_out, hipStream_t st) {
  CHECK_PLAN(h);
  if (int rc = check_ptr(p, disp, "disp")) return rc;
  if (int rc = check_ptr(p, acc_bar, "acc_bar")) return rc;
  if (int rc = check_ptr(p, disp_bar, "disp_bar")) return rc;
  if (int rc = check_ptr(p, omega_m_bar, "omega_m_bar")) return rc;
  if (int rc = check_omega_m(p, omega_m)) return rc;
  if (int rc = set_device(p)) return rc;
  PaintArgs pa{};
  pa.s = disp;
  pa.unit = 1;
  pa.w = acc_bar;
  pa.nw = 3;
  pa.mesh = p->mesh[0];
  if (int rc = paint_vjp_fields(p, DRIFT_NONE, pa, omega_m, st)) return rc;
  GatherArgs ga{};
  ga.s = disp;
  ga.mesh = p->mesh[0];
  ga.nf = 4;
  ga.out = disp_bar;
  ga.acc = acc_out;
  ga.cot = acc_bar;
  ga.binned = true;
  if (int rc = gather_launch(p, GATHER_VJP, ga, st)) return rc;
  // a is proportional to Omega_m: d(abar.a)/dOmega_m = (abar.a)/Omega_m
  const double f[4] = {0.0, 1.0 / omega_m, 0.0, 0.0};
  return reduce_buffer(p, p->tile_partials, p->ntiles, f, omega_m_bar, true, st);
}

int pm_fwd_init(pm_plan h, pm_state* stt, const pm_step_coef* first, double omega_m, hipStream_t st) {
  CHECK_PLAN(h);
  if (!stt) return set_error(p, PM_EINVAL, "state is NULL");
  if (int rc = check_ptr(p, stt->s, "state.s")) return rc;
  if (int rc = check_ptr(p, stt->p, "state.p")) return rc;
  if (int rc = check_step(p, first, "first")) return rc;
  if (int rc = check_omega_m(p, omega_m)) return rc;
  if (int rc = set_device(p)) return rc;
  PaintArgs pa{};
  pa.s = stt->s;
  pa.unit = 1;
  pa.mesh = p->mesh[0];
  if (int rc = paint_force_fields(p, DRIFT_NONE, pa, omega_m, st)) return rc;
  GatherArgs ga{};
  ga.s = stt->s;
  ga.mesh = p->mesh[0];
  ga.nf = 3;
  ga.p = stt->p;
  ga.K = first->Ka;
  ga.binned = true;
  return gather_launch(p, GATHER_KICK_FWD, ga, st);
}

int pm_step_fwd(pm_plan h, pm_state* stt, const pm_step_coef* cur, const pm_step_coef* next, double omega_m,
                hipStream_t st) {
  CHECK_PLAN(h);
  if (!stt) return set_error(p, PM_EINVAL, "state is NULL");
  if (int rc = check_ptr(p, stt->s, "state.s")) return rc;
  if (int rc = check_ptr(p, stt->p, "state.p")) return rc;
  if (int rc = check_step(p, cur, "cur")) return rc;
  if (next)
    if (int rc = check_step(p, next, "next")) return rc;
  if (int rc = check_omega_m(p, omega_m)) return rc;
  if (int rc = set_device(p)) return rc;
  PaintArgs pa{};
  pa.s = stt->s;
  pa.p = stt->p;
  pa.unit = 1;
  pa.mesh = p->mesh[0];
  pa.D = cur->D;
  if (int rc = paint_force_fields(p, DRIFT_FWD, pa, omega_m, st)) return rc;
  GatherArgs ga{};
  ga.s = stt->s;
  ga.mesh = p->mesh[0];
  ga.nf = 3;
  ga.p = stt->p;
  ga.K = cur->Kb + (next ? next->Ka : 0.0);
  ga.acc = next ? nullptr : stt->acc;
  ga.binned = true;
  return gather_launch(p, GATHER_KICK_FWD, ga, st);
}

int pm_adj_init(pm_plan h, pm_state* stt, pm_adj* adj, const pm_step_coef* last, double omega_m,
                double* theta_bar, hipStream_t st) {
  CHECK_PLAN(h);
  if (!stt || !adj) return set_error(p, PM_EINVAL, "state or adjoint is NULL");
  if (int rc = check_ptr(p, stt->s, "state.s")) return rc;
  if (int rc = check_ptr(p, stt->p, "state.p")) return rc;
  if (int rc = check_ptr(p, adj->xi, "adj.xi")) return rc;
  if (int rc = check_ptr(p, adj->pi, "adj.pi")) return rc;
  if (int rc = check_ptr(p, theta_bar, "theta_bar")) return rc;
  if (int rc = check_step(p, last, "last")) return rc;
  if (int rc = check_omega_m(p, omega_m)) return rc;
  if (int rc = set_device(p)) return rc;
  PaintArgs pa{};
  pa.s = stt->s;
  pa.unit = 1;
  pa.w = adj->pi;
  pa.nw = 3;
  pa.mesh = p->mesh[0];
  if (int rc = paint_vjp_fields(p, DRIFT_NONE, pa, omega_m, st)) return rc;
  GatherArgs ga{};
  ga.s = stt->s;
  ga.mesh = p->mesh[0];
  ga.nf = 4;
  ga.p = stt->p;
  ga.xi = adj->xi;
  ga.cot = adj->pi;
  ga.acc_in = stt->acc;
  ga.K = last->Kb;
  ga.binned = true;
  if (int rc = gather_launch(p, GATHER_KICK_ADJ, ga, st)) return rc;
  // theta_bar[0] += (pi.a) dKb + zeta Kb,  zeta = (pi.a) / Omega_m
  const double f[4] = {0.0, last->dKb + last->Kb / omega_m, 0.0, 0.0};
  return reduce_buffer(p, p->tile_partials, p->ntiles, f, theta_bar, true, st);
}

int pm_step_adj(pm_plan h, pm_state* stt, pm_adj* adj, const pm_step_coef* cur, const pm_step_coef* prev,
                double omega_m, double* theta_bar, hipStream_t st) {
  CHECK_PLAN(h);
  if (int rc = check_adj_args(p, stt, adj, cur, prev, omega_m, theta_bar)) return rc;
  if (int rc = set_device(p)) return rc;
  return step_adj(p, stt, adj, cur, prev, omega_m, theta_bar, nullptr, nullptr, st);
}

int pm_run_fwd(pm_plan h, pm_state* stt, const pm_step_coef* coefs, int n, double omega_m, hipStream_t st) {
  return pm_run_fwd_ckpt(h, stt, coefs, n, omega_m, nullptr, st);
}

int pm_run_adj(pm_plan h, pm_state* stt, pm_adj* adj, const pm_step_coef* coefs, int n, double omega_m,
               double* theta_bar, hipStream_t st) {
  return pm_run_adj_ckpt(h, stt, adj, coefs, n, omega_m, nullptr, theta_bar, st);
}

// The native loops.  With st->acc given, every kick is left pending: the
// gather only stores a (and alpha) in lattice order, and the next step's
// drift, which reads and writes p (and xi) in lattice order anyway, applies
// the kick before it moves the particles; the last one is applied at the end.
// Kicks and drifts use the same fused multiply-adds in both places, so the
// result is bitwise that of the step calls.  Without st->acc the loops are the
// step calls.
int pm_run_fwd_ckpt(pm_plan h, pm_state* stt, const pm_step_coef* coefs, int n, double omega_m,
                    const pm_checkpoints* ck, hipStream_t st) {
  CHECK_PLAN(h);
  if (!coefs || n < 1) return set_error(p, PM_EINVAL, "need n >= 1 step coefficients");
  if (int rc = check_checkpoints(p, ck, n)) return rc;
  const size_t bytes = state_bytes(p);
  if (!stt || !stt->acc) {
    if (int rc = pm_fwd_init(h, stt, &coefs[0], omega_m, st)) return rc;
    for (int i = 0; i < n; ++i) {
      const int k = checkpoint_index(ck, i + 1);
      if (k >= 0) PM_HIP_CHECK(p, hipMemcpyAsync(ck->p[k], stt->p, bytes, hipMemcpyDeviceToDevice, st));
      if (int rc = pm_step_fwd(h, stt, &coefs[i], i + 1 < n ? &coefs[i + 1] : nullptr, omega_m, st)) return rc;
      if (k >= 0) PM_HIP_CHECK(p, hipMemcpyAsync(ck->s[k], stt->s, bytes, hipMemcpyDeviceToDevice, st));
    }
    return PM_OK;
  }
  if (int rc = check_ptr(p, stt->s, "state.s")) return rc;
  if (int rc = check_ptr(p, stt->p, "state.p")) return rc;
  for (int i = 0; i < n; ++i)
    if (int rc = check_step(p, &coefs[i], "coefs[i]")) return rc;
  if (int rc = check_omega_m(p, omega_m)) return rc;
  if (int rc = set_device(p)) return rc;
  // a_0 = F(x_0); the kick p_0 + a_0 Ka_1 is left pending.  Each gather
  // writes a in the tile order of its bins (contiguous per tile) into the
  // plan's spare 3 N buffer (particle-major), and the next drift reads it back through the
  // bins; the last kick writes a_n to st->acc in lattice order.
  PaintArgs pa{};
  pa.s = stt->s;
  pa.unit = 1;
  pa.mesh = p->mesh[0];
  if (int rc = paint_force_fields(p, DRIFT_NONE, pa, omega_m, st)) return rc;
  GatherArgs ga{};
  ga.s = stt->s;
  ga.mesh = p->mesh[0];
  ga.nf = 3;
  ga.out = p->kick_al;
  ga.sorted_out = true;
  ga.binned = true;
  if (int rc = gather_launch(p, GATHER_PLAIN, ga, st)) return rc;
  double Kp = coefs[0].Ka;
  for (int i = 0; i < n; ++i) {
    PaintArgs pb{};
    pb.s = stt->s;
    pb.p = stt->p;
    pb.unit = 1;
    pb.mesh = p->mesh[0];
    pb.D = coefs[i].D;
    pb.kick_a = p->kick_al;
    pb.kick_sorted = true;
    pb.Kp = Kp;
    if (int rc = paint_force_fields(p, DRIFT_FWD, pb, omega_m, st)) return rc;
    // the drift has applied the kick and moved the particles: (s_{i+1}, p_{i+1/2})
    const int k = checkpoint_index(ck, i + 1);
    if (k >= 0) {
      PM_HIP_CHECK(p, hipMemcpyAsync(ck->p[k], stt->p, bytes, hipMemcpyDeviceToDevice, st));
      PM_HIP_CHECK(p, hipMemcpyAsync(ck->s[k], stt->s, bytes, hipMemcpyDeviceToDevice, st));
    }
    if (int rc = gather_launch(p, GATHER_PLAIN, ga, st)) return rc;   // a_{i+1}
    Kp = coefs[i].Kb + (i + 1 < n ? coefs[i + 1].Ka : 0.0);
  }
  return kick_flush(p, stt->p, p->kick_al, Kp, false, nullptr, nullptr, 0.0, stt->acc, st);
}

namespace {

// reverse steps n..1 of the native loop from (s_n, p_{n-1/2}), (xi_{n-1/2},
// pi_n): what pm_run_adj_ckpt runs after pm_adj_init, and pm_run_adj_from
// from wherever the step calls left off
int run_adj_steps(Plan* p, pm_state* stt, pm_adj* adj, const pm_step_coef* coefs, int n, double omega_m,
                  const pm_checkpoints* ck, double* theta_bar, hipStream_t st) {
  const bool defer = stt->acc != nullptr;
  // the native loop keeps pi particle-major while it runs (the four-channel
  // paint and the VJP gather read it through the tile lists), and gives it
  // back as [3][N]
  const bool pm = defer && pi_layout_fits(p);
  if (pm)
    if (int rc = pi_layout(p, adj->pi, true, st)) return rc;
  bool pending = false;
  double Kp = 0.0, Kx = 0.0;
  for (int i = n - 1; i >= 0; --i) {
    // reverse step i + 1 ends at t_i: resume from checkpoint i if there is one
    const int k = i >= 1 ? checkpoint_index(ck, i) : -1;
    const void* s_set = k >= 0 ? ck->s[k] : nullptr;
    const void* p_set = k >= 0 ? ck->p[k] : nullptr;
    const pm_step_coef* cur = &coefs[i];
    const pm_step_coef* prev = i > 0 ? &coefs[i - 1] : nullptr;
    if (!defer) {
      if (int rc = step_adj(p, stt, adj, cur, prev, omega_m, theta_bar, s_set, p_set, st)) return rc;
      continue;
    }
    PaintArgs pa{};
    pa.s = stt->s;
    pa.p = stt->p;
    pa.xi = adj->xi;
    pa.pi = adj->pi;
    pa.unit = 1;
    pa.nw = 3;
    pa.mesh = p->mesh[0];
    pa.D = cur->D;
    pa.partials = p->partials;
    pa.s_set = s_set;
    pa.pi_pm = pm;
    if (pending) {
      pa.kick_a = stt->acc;
      pa.kick_al = p->kick_al;
      pa.kick_sorted = true;
      pa.Kp = Kp;
      pa.Kx = Kx;
    }
    if (int rc = paint_vjp_fields(p, s_set ? DRIFT_SET : DRIFT_ADJ, pa, omega_m, st)) return rc;
    const double K = cur->Ka + (prev ? prev->Kb : 0.0);
    const double dK = cur->dKa + (prev ? prev->dKb : 0.0);
    // a and alpha at x_i, pi.a partials; the kick p -= a K, xi += alpha K is
    // left pending, with a and alpha in the tile order of the bins
    GatherArgs ga{};
    ga.s = stt->s;
    ga.mesh = p->mesh[0];
    ga.nf = 4;
    ga.out = p->kick_al;
    ga.acc = stt->acc;
    ga.cot = adj->pi;
    ga.cot_pm = pm;
    ga.sorted_out = true;
    ga.binned = true;
    if (int rc = gather_launch(p, GATHER_VJP, ga, st)) return rc;
    const double fd[4] = {cur->dD, 0.0, 0.0, 0.0};
    if (int rc = reduce_partials(p, blocks_for_particles(p), fd, theta_bar, true, st)) return rc;
    const double fk[4] = {0.0, dK + K / omega_m, 0.0, 0.0};
    if (int rc = reduce_buffer(p, p->tile_partials, p->ntiles, fk, theta_bar, true, st)) return rc;
    pending = true;
    Kp = K;
    Kx = K;
    if (p_set) {
      // the stored momentum already holds this kick
      PM_HIP_CHECK(p, hipMemcpyAsync(stt->p, p_set, state_bytes(p), hipMemcpyDeviceToDevice, st));
      Kp = 0.0;
    }
  }
  if (defer && pending)
    if (int rc = kick_flush(p, stt->p, stt->acc, Kp, true, adj->xi, p->kick_al, Kx, nullptr, st)) return rc;
  return pm ? pi_layout(p, adj->pi, false, st) : PM_OK;
}

}  // namespace

int pm_run_adj_ckpt(pm_plan h, pm_state* stt, pm_adj* adj, const pm_step_coef* coefs, int n, double omega_m,
                    const pm_checkpoints* ck, double* theta_bar, hipStream_t st) {
  CHECK_PLAN(h);
  if (!coefs || n < 1) return set_error(p, PM_EINVAL, "need n >= 1 step coefficients");
  if (int rc = check_checkpoints(p, ck, n)) return rc;
  for (int i = 0; i < n; ++i)
    if (int rc = check_step(p, &coefs[i], "coefs[i]")) return rc;
  if (int rc = pm_adj_init(h, stt, adj, &coefs[n - 1], omega_m, theta_bar, st)) return rc;
  const int kn = checkpoint_index(ck, n);
  if (kn >= 0) PM_HIP_CHECK(p, hipMemcpyAsync(stt->p, ck->p[kn], state_bytes(p), hipMemcpyDeviceToDevice, st));
  return run_adj_steps(p, stt, adj, coefs, n, omega_m, ck, theta_bar, st);
}

int pm_run_adj_from(pm_plan h, pm_state* stt, pm_adj* adj, const pm_step_coef* coefs, int n, double omega_m,
                    double* theta_bar, hipStream_t st) {
  CHECK_PLAN(h);
  if (!coefs || n < 1) return set_error(p, PM_EINVAL, "need n >= 1 step coefficients");
  for (int i = 0; i < n; ++i)
    if (int rc = check_step(p, &coefs[i], "coefs[i]")) return rc;
  if (int rc = check_adj_args(p, stt, adj, &coefs[n - 1], nullptr, omega_m, theta_bar)) return rc;
  if (int rc = set_device(p)) return rc;
  return run_adj_steps(p, stt, adj, coefs, n, omega_m, nullptr, theta_bar, st);
}

int pm_density_mse(pm_plan h, const void* disp, const void* target, double* J, void* disp_bar, hipStream_t st) {
  CHECK_PLAN(h);
  if (int rc = check_ptr(p, disp, "disp")) return rc;
  if (int rc = check_ptr(p, target, "target")) return rc;
  if (int rc = check_ptr(p, J, "J")) return rc;
  if (int rc = set_device(p)) return rc;
  PaintArgs pa{};
  pa.s = disp;
  pa.unit = 1;
  pa.mesh = p->mesh[0];
  if (int rc = paint_launch(p, DRIFT_NONE, pa, st)) return rc;
  const int nb = mse_mesh_launch(p, p->mesh[0], target, p->partials, st);
  if (nb < 0) return nb;
  const double f[4] = {0.0, 0.0, 1.0 / double(p->ncell), 0.0};
  if (int rc = reduce_partials(p, nb, f, J, false, st)) return rc;
  if (!disp_bar) return PM_OK;
  GatherArgs ga{};
  ga.s = disp;
  ga.mesh = p->mesh[0];
  ga.nf = 1;
  ga.out = disp_bar;
  ga.binned = true;
  return gather_launch(p, GATHER_MSE, ga, st);
}

int pm_density(pm_plan h, const void* disp, void* delta, hipStream_t st) {
  CHECK_PLAN(h);
  if (int rc = check_ptr(p, disp, "disp")) return rc;
  if (int rc = check_ptr(p, delta, "delta")) return rc;
  if (int rc = set_device(p)) return rc;
  PaintArgs pa{};
  pa.s = disp;
  pa.unit = 1;
  pa.mesh = delta;
  if (int rc = paint_launch(p, DRIFT_NONE, pa, st)) return rc;
  return contrast_launch(p, delta, st);
}

int pm_check_finite(pm_plan h, const void* x, int64_t n, int dtype, int* bad, hipStream_t st) {
  CHECK_PLAN(h);
  if (int rc = check_ptr(p, x, "x")) return rc;
  if (int rc = check_ptr(p, bad, "bad")) return rc;
  if (n < 0 || (dtype != PM_F32 && dtype != PM_F64)) return set_error(p, PM_EINVAL, "bad n or dtype");
  if (n == 0) return PM_OK;
  if (int rc = set_device(p)) return rc;
  const int64_t need = (n + kThreads - 1) / kThreads;
  const int blocks = int(need < 2048 ? need : 2048);
  if (dtype == PM_F64)
    hipLaunchKernelGGL((k_finite<double>), dim3(blocks), dim3(kThreads), 0, st, static_cast<const double*>(x), n, bad);
  else
    hipLaunchKernelGGL((k_finite<float>), dim3(blocks), dim3(kThreads), 0, st, static_cast<const float*>(x), n, bad);
  PM_HIP_CHECK(p, hipGetLastError());
  return PM_OK;
}

int pm_timing_enable(pm_plan h, unsigned mask) {
  CHECK_PLAN(h);
  Timing& t = p->timing;
  if (mask && !t.created) {
    for (int k = 1; k < kTimingFamilies; ++k)
      for (auto& e : t.fam[k].ev)
        if (hipEventCreate(&e) != hipSuccess) return set_error(p, PM_EDEVICE, "hipEventCreate failed");
    t.created = true;
  }
  t.mask = mask;
  for (auto& f : t.fam) {
    f.nev = 0;
    f.total_ms = 0.0;
    f.total_bytes = 0.0;
    f.total_method_bytes = 0.0;
    f.launches = 0;
    f.dropped = 0;
  }
  return PM_OK;
}

int pm_timing_read(pm_plan h, int kernel, double* total_ms, int64_t* launches, double* total_bytes,
                   double* total_method_bytes) {
  CHECK_PLAN(h);
  if (kernel <= 0 || kernel >= kTimingFamilies) return set_error(p, PM_EINVAL, "unknown kernel family %d", kernel);
  TimingFamily& f = p->timing.fam[kernel];
  for (int i = 0; i + 1 < f.nev; i += 2) {
    float ms = 0.f;
    PM_HIP_CHECK(p, hipEventSynchronize(f.ev[i + 1]));
    PM_HIP_CHECK(p, hipEventElapsedTime(&ms, f.ev[i], f.ev[i + 1]));
    f.total_ms += ms;
    f.total_bytes += f.bytes[i / 2];
    f.total_method_bytes += f.method_bytes[i / 2];
    f.launches += 1;
  }
  f.nev = 0;
  if (total_ms) *total_ms = f.total_ms;
  if (launches) *launches = f.launches;
  if (total_bytes) *total_bytes = f.total_bytes;
  if (total_method_bytes) *total_method_bytes = f.total_method_bytes;
  if (f.dropped) return set_error(p, PM_EINVAL, "%lld launches were not recorded (read more often)",
                                  static_cast<long long>(f.dropped));
  return PM_OK;
}

}  // extern "C"
