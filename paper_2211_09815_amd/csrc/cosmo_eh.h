// Forward-mode dual numbers and the Eisenstein & Hu (1998) no-wiggle
// transfer function, usable from host (pm_tables) and device (pm_lpt).
//
// The paper's initial conditions (Sec. 2.1, eq. Plin) use the EH98 fitting
// formula for T(k); its no-wiggle form (EH98 Sec. 4.2) is:
//   s        = 44.5 ln(9.83 / (Om h^2)) / sqrt(1 + 10 (Ob h^2)^(3/4))   [Mpc]
//   alpha    = 1 - 0.328 ln(431 Om h^2) fb + 0.38 ln(22.3 Om h^2) fb^2
//   Gamma    = Om h (alpha + (1 - alpha) / (1 + (0.43 k s)^4))          [k in 1/Mpc]
//   q        = k Theta^2 / Gamma                                       [k in h/Mpc]
//   T        = L0 / (L0 + C0 q^2),  L0 = ln(2e + 1.8 q),  C0 = 14.2 + 731/(1 + 62.5 q)
// with fb = Ob/Om and Theta = T_cmb / 2.7.  Dual numbers carry d/dOmega_m.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

namespace pmx {

struct Dual {
  double v, d;
};

__host__ __device__ inline Dual dual(double v, double d = 0.0) { return Dual{v, d}; }
__host__ __device__ inline Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
__host__ __device__ inline Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
__host__ __device__ inline Dual operator-(Dual a) { return {-a.v, -a.d}; }
__host__ __device__ inline Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
__host__ __device__ inline Dual operator/(Dual a, Dual b) {
  return {a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)};
}
__host__ __device__ inline Dual operator+(Dual a, double b) { return {a.v + b, a.d}; }
__host__ __device__ inline Dual operator+(double a, Dual b) { return {a + b.v, b.d}; }
__host__ __device__ inline Dual operator-(Dual a, double b) { return {a.v - b, a.d}; }
__host__ __device__ inline Dual operator-(double a, Dual b) { return {a - b.v, -b.d}; }
__host__ __device__ inline Dual operator*(Dual a, double b) { return {a.v * b, a.d * b}; }
__host__ __device__ inline Dual operator*(double a, Dual b) { return {a * b.v, a * b.d}; }
__host__ __device__ inline Dual operator/(Dual a, double b) { return {a.v / b, a.d / b}; }
__host__ __device__ inline Dual operator/(double a, Dual b) { return {a / b.v, -a * b.d / (b.v * b.v)}; }
__host__ __device__ inline Dual dsqrt(Dual a) {
  const double s = ::sqrt(a.v);
  return {s, a.d / (2.0 * s)};
}
__host__ __device__ inline Dual dlog(Dual a) { return {::log(a.v), a.d / a.v}; }
__host__ __device__ inline Dual dpow(Dual a, double e) {
  const double p = ::pow(a.v, e);
  return {p, e * ::pow(a.v, e - 1.0) * a.d};
}
__host__ __device__ inline double dsqrt(double a) { return ::sqrt(a); }
__host__ __device__ inline double dlog(double a) { return ::log(a); }
__host__ __device__ inline double dpow(double a, double e) { return ::pow(a, e); }
template <typename R> __host__ __device__ inline R cst(double v);
template <> __host__ __device__ inline double cst<double>(double v) { return v; }
template <> __host__ __device__ inline Dual cst<Dual>(double v) { return Dual{v, 0.0}; }
__host__ __device__ inline double val(double a) { return a; }
__host__ __device__ inline double val(Dual a) { return a.v; }

// T(k) for k in h/Mpc; R = double or Dual (derivative with respect to om)
template <typename R>
__host__ __device__ inline R eh_nowiggle(double k, R om, double ob, double h, double t_cmb) {
  const double theta2 = (t_cmb / 2.7) * (t_cmb / 2.7);
  const R omh2 = om * (h * h);
  const double obh2 = ob * h * h;
  const R fb = ob / om;
  const R s = 44.5 * dlog(9.83 / omh2) / ::sqrt(1.0 + 10.0 * ::pow(obh2, 0.75));
  const R alpha = 1.0 - 0.328 * dlog(431.0 * omh2) * fb + 0.38 * dlog(22.3 * omh2) * fb * fb;
  const R ks = s * (k * h);
  const R t = 0.43 * ks;
  const R t2 = t * t;
  const R gamma = om * h * (alpha + (1.0 - alpha) / (1.0 + t2 * t2));
  const R q = k * theta2 / gamma;
  const R L0 = dlog(2.0 * 2.718281828459045235360287 + 1.8 * q);
  const R C0 = 14.2 + 731.0 / (1.0 + 62.5 * q);
  return L0 / (L0 + C0 * q * q);
}

}  // namespace pmx
