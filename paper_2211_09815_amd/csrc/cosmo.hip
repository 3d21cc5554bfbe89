// Host FP64 cosmology tables (pm_tables): growth functions, FastPM factors,
// KDK step coefficients and the initial-condition factors, each with its
// derivative with respect to Omega_m carried by forward-mode dual numbers.
//
// Paper passages: Appendix A (growth ODEs in the suppression factors
// G_m = D_m / a^m with growing-mode initial values at a_ic), eq. G_eval
// (G_D = a^2 H D_1', G_K = a^3 H^2 [D_1'' + (2 + H'/H) D_1'], with
// D_m' = a^m (m G_m + G_m') and D_m'' = a^m (m^2 G_m + 2 m G_m' + G_m'')),
// Sec. 2.3 (drift factor D = (D_1(t_b) - D_1(t_a))/G_D(t_c), kick factor
// K = (G_D(t_b) - G_D(t_a))/G_K(t_c)), eq. lpt (p = a^2 H (D_1' s1 + D_2' s2))
// and eq. Plin (P(k) proportional to k^n_s T^2(k), normalised here to sigma8).
//
// Flat LambdaCDM without radiation, H0 = 1, a_ic = 1e-4.  The ODEs are
// integrated with classical fourth-order Runge-Kutta in ln a (step <= 1e-3,
// landing exactly on every requested a); sigma8 uses composite Simpson in
// ln k over [1e-5, 1e2] h/Mpc with 2^15 intervals.
#include <algorithm>
#include <cmath>
#include <vector>

#include "cosmo_eh.h"
#include "pm_internal.h"

using namespace pmx;

namespace {

constexpr double kAic = 1e-4;
constexpr double kMaxDlna = 1e-3;

template <typename R>
R hubble_E(double a, R om) {
  return dsqrt(om / (a * a * a) + (1.0 - om));
}

// y = (G1, G1', G2, G2') with ' = d/d ln a
template <typename R>
void growth_rhs(double lna, const R y[4], R out[4], R om) {
  const double a = std::exp(lna);
  const R e = hubble_E(a, om);
  const R oma = om / (a * a * a * e * e);   // Omega_m(a)
  const R hh = -1.5 * oma;                   // H'/H for flat LambdaCDM
  out[0] = y[1];
  out[1] = -(4.0 + hh) * y[1] - (3.0 + hh - 1.5 * oma) * y[0];
  out[2] = y[3];
  out[3] = -(6.0 + hh) * y[3] - (8.0 + 2.0 * hh - 1.5 * oma) * y[2] + 1.5 * oma * y[0] * y[0];
}

template <typename R>
void rk4_step(double lna, double h, R y[4], R om) {
  R k1[4], k2[4], k3[4], k4[4], t[4];
  growth_rhs(lna, y, k1, om);
  for (int i = 0; i < 4; ++i) t[i] = y[i] + (0.5 * h) * k1[i];
  growth_rhs(lna + 0.5 * h, t, k2, om);
  for (int i = 0; i < 4; ++i) t[i] = y[i] + (0.5 * h) * k2[i];
  growth_rhs(lna + 0.5 * h, t, k3, om);
  for (int i = 0; i < 4; ++i) t[i] = y[i] + h * k3[i];
  growth_rhs(lna + h, t, k4, om);
  for (int i = 0; i < 4; ++i) y[i] = y[i] + (h / 6.0) * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
}

template <typename R>
struct GrowthAt {
  R D1, dD1, ddD1, D2, dD2, GD, GK;
};

// growth functions at every a in `as` (any order, all >= a_ic)
template <typename R>
std::vector<GrowthAt<R>> growth_at(const std::vector<double>& as, R om) {
  std::vector<size_t> order(as.size());
  for (size_t i = 0; i < order.size(); ++i) order[i] = i;
  std::sort(order.begin(), order.end(), [&](size_t x, size_t y) { return as[x] < as[y]; });
  std::vector<GrowthAt<R>> out(as.size());
  R y[4] = {cst<R>(1.0), cst<R>(0.0), cst<R>(3.0 / 7.0), cst<R>(0.0)};
  double lna = std::log(kAic);
  for (size_t oi : order) {
    const double target = std::log(as[oi]);
    const double span = target - lna;
    if (span > 0) {
      const int nsteps = std::max(1, int(std::ceil(span / kMaxDlna)));
      const double h = span / nsteps;
      for (int s = 0; s < nsteps; ++s) rk4_step(lna + s * h, h, y, om);
      lna = target;
    }
    R d[4];
    growth_rhs(lna, y, d, om);
    const double a = as[oi];
    GrowthAt<R> g;
    g.D1 = a * y[0];
    g.dD1 = a * (y[0] + y[1]);
    g.ddD1 = a * (y[0] + 2.0 * y[1] + d[1]);
    g.D2 = (a * a) * y[2];
    g.dD2 = (a * a) * (2.0 * y[2] + y[3]);
    const R e = hubble_E(a, om);
    const R hh = -1.5 * om / (a * a * a * e * e);
    g.GD = (a * a) * e * g.dD1;
    g.GK = (a * a * a) * e * e * (g.ddD1 + (2.0 + hh) * g.dD1);
    out[oi] = g;
  }
  return out;
}

template <typename R>
R tophat2(double x) {
  double w;
  if (x < 1e-3) w = 1.0 - x * x / 10.0 + x * x * x * x / 280.0;
  else w = 3.0 * (std::sin(x) - x * std::cos(x)) / (x * x * x);
  return cst<R>(w * w);
}

// I = int d ln k k^3 k^n_s T^2 W^2(8k) / (2 pi^2), Simpson in ln k
template <typename R>
R sigma8_shape_integral(R om, double ob, double h, double ns, double tcmb) {
  const int n = 1 << 15;
  const double lo = std::log(1e-5), hi = std::log(1e2);
  const double dx = (hi - lo) / n;
  R acc = cst<R>(0.0);
  for (int i = 0; i <= n; ++i) {
    const double k = std::exp(lo + i * dx);
    const R T = eh_nowiggle<R>(k, om, ob, h, tcmb);
    const R f = (std::pow(k, 3.0 + ns) / (2.0 * M_PI * M_PI)) * T * T * tophat2<R>(8.0 * k);
    const double wgt = (i == 0 || i == n) ? 1.0 : (i % 2 ? 4.0 : 2.0);
    acc = acc + wgt * f;
  }
  return acc * (dx / 3.0);
}

}  // namespace

extern "C" int pm_tables(const pm_cosmo* c, const double* a_grid, int n, pm_step_coef* coefs, pm_ic_coef* ic) {
  if (!c || !a_grid || n < 0) return set_error(nullptr, PM_EINVAL, "pm_tables: bad arguments");
  if (!(c->omega_m > 0.0 && c->omega_m <= 1.0) || !(c->omega_b >= 0.0 && c->omega_b < c->omega_m) ||
      !(c->h > 0.0) || !(c->sigma8 > 0.0) || !(c->t_cmb > 0.0) || !std::isfinite(c->n_s))
    return set_error(nullptr, PM_EINVAL, "pm_tables: cosmological parameters out of range");
  for (int i = 0; i <= n; ++i) {
    if (!(a_grid[i] >= kAic && a_grid[i] <= 10.0)) return set_error(nullptr, PM_EINVAL, "pm_tables: a out of range");
    if (i > 0 && !(a_grid[i] > a_grid[i - 1])) return set_error(nullptr, PM_EINVAL, "pm_tables: a_grid must increase");
  }
  const Dual om{c->omega_m, 1.0};
  std::vector<double> as;
  for (int i = 0; i < n; ++i) {
    as.push_back(a_grid[i]);
    as.push_back(0.5 * (a_grid[i] + a_grid[i + 1]));
    as.push_back(a_grid[i + 1]);
  }
  as.push_back(a_grid[0]);
  as.push_back(1.0);
  const auto g = growth_at<Dual>(as, om);
  if (coefs) {
    for (int i = 0; i < n; ++i) {
      const auto& g0 = g[3 * i];
      const auto& gh = g[3 * i + 1];
      const auto& g1 = g[3 * i + 2];
      const Dual Ka = (gh.GD - g0.GD) / g0.GK;
      const Dual D = (g1.D1 - g0.D1) / gh.GD;
      const Dual Kb = (g1.GD - gh.GD) / g1.GK;
      coefs[i] = pm_step_coef{Ka.v, D.v, Kb.v, Ka.d, D.d, Kb.d};
    }
  }
  if (ic) {
    const auto& g0 = g[3 * n];
    const auto& g1 = g[3 * n + 1];
    const double a0 = a_grid[0];
    const Dual e0 = hubble_E(a0, om);
    const Dual P1 = (a0 * a0) * e0 * g0.dD1;
    const Dual P2 = (a0 * a0) * e0 * g0.dD2;
    const Dual I = sigma8_shape_integral<Dual>(om, c->omega_b, c->h, c->n_s, c->t_cmb);
    const Dual A = (c->sigma8 * c->sigma8) / (g1.D1 * g1.D1 * I);
    *ic = pm_ic_coef{g0.D1.v, g0.D2.v, P1.v, P2.v, A.v, g0.D1.d, g0.D2.d, P1.d, P2.d, A.d};
  }
  return PM_OK;
}

// ---------------------------------------------------------------------------
// Light-cone factors (Sec. 2.4): comoving distance to the light front
// chi(a) = (c/H0) int_a^1 da' / (a'^2 E(a')), its a-derivative and the
// velocity factor w = 1/(a^3 E) of dx/da = p w, with d/dOmega_m by dual
// numbers.  With a' = y^2 the integrand becomes 2 / (y^3 E(y^2)), which is
// smooth down to a' -> 0; it is integrated with 8-point Gauss-Legendre on
// kLcPanels equal panels in y.
// ---------------------------------------------------------------------------
namespace {

constexpr double kCOverH0 = 2997.92458;   // Mpc/h
constexpr int kGlOrder = 8;
constexpr int kLcPanels = 256;

// nodes and weights of m-point Gauss-Legendre on [-1, 1]: Newton iteration on
// the three-term Legendre recurrence from the usual cosine first guesses
void gauss_legendre(int m, double* x, double* w) {
  for (int i = 0; i < m; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (m + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p1 = 1.0, p0 = 0.0;
      for (int j = 1; j <= m; ++j) {
        const double pm1 = p0;
        p0 = p1;
        p1 = ((2.0 * j - 1.0) * z * p0 - (j - 1.0) * pm1) / j;
      }
      dp = m * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

Dual light_front_integral(double a, Dual om) {
  double gx[kGlOrder], gw[kGlOrder];
  gauss_legendre(kGlOrder, gx, gw);
  const double y0 = std::sqrt(a);
  const double h = (1.0 - y0) / kLcPanels;
  Dual acc = cst<Dual>(0.0);
  for (int k = 0; k < kLcPanels; ++k) {
    const double mid = y0 + (k + 0.5) * h;
    for (int j = 0; j < kGlOrder; ++j) {
      const double y = mid + 0.5 * h * gx[j];
      acc = acc + (gw[j] * 0.5 * h) * (2.0 / (y * y * y * hubble_E(y * y, om)));
    }
  }
  return acc;
}

}  // namespace

extern "C" int pm_lightcone_tables(const pm_cosmo* c, const double* a_grid, int n, double cell, pm_lc_coef* out) {
  if (!c || !a_grid || !out || n < 0 || !(cell > 0.0))
    return set_error(nullptr, PM_EINVAL, "pm_lightcone_tables: bad arguments");
  if (!(c->omega_m > 0.0 && c->omega_m <= 1.0))
    return set_error(nullptr, PM_EINVAL, "pm_lightcone_tables: Omega_m out of range");
  for (int k = 0; k <= n; ++k)
    if (!(a_grid[k] > 0.0 && a_grid[k] <= 1.0))
      return set_error(nullptr, PM_EINVAL, "pm_lightcone_tables: a must be in (0, 1]");
  const Dual om{c->omega_m, 1.0};
  const double kc = kCOverH0 / cell;
  for (int k = 0; k <= n; ++k) {
    const double a = a_grid[k];
    const Dual chi = kc * light_front_integral(a, om);
    const Dual e = hubble_E(a, om);
    const Dual dchi = -kc / ((a * a) * e);
    const Dual w = 1.0 / ((a * a * a) * e);
    out[k] = pm_lc_coef{a, chi.v, dchi.v, w.v, chi.d, dchi.d, w.d};
  }
  return PM_OK;
}
