// 3-D real FFTs for the particle-mesh force (Sec. 2.2 of the paper: one
// forward and three inverse transforms per force evaluation), composed from
// the LDS pass kernels of fft_lines.hip, fft_z.hip and fft_fused.hip.
//
// Passes over HBM:
//   z: real lines -> half-length complex FFT + split into N/2+1 bins,
//   y: strided columns (W adjacent kz per tile),
//   x: strided columns over the flattened (y, kz) plane (no ragged tiles).
// The force path (fft_spectral_op) runs z and y forward, then one fused pass
// along x (forward FFT, multipliers, inverse FFT of every output), then y and
// z inverse; every pass over the 3 or 4 fields is one launch.
#include "fft_core.h"

namespace pmx {

using fftk::Ptrs4;

namespace {

// y pass: lines of n1 with stride nh, columns kz (nh), outer x (stride n1*nh);
// array dual (>= 0) also to dual_out, then times ky in place
template <typename T>
int y_pass(Plan* p, const FftShape& s, const Ptrs4& a, int batch, bool inv, hipStream_t st, int dual = -1,
           void* dual_out = nullptr) {
  const int nh = s.n2 / 2 + 1;
  return fftk::lines_pass<T>(p, a, batch, inv, s.n1, nh, nh, int64_t(s.n1) * nh, s.n0, st, dual, dual_out);
}

// x pass: lines of n0 with stride n1*nh over the flattened (y, kz) plane
template <typename T>
int x_pass(Plan* p, const FftShape& s, const Ptrs4& a, int batch, bool inv, hipStream_t st) {
  const int64_t plane = int64_t(s.n1) * (s.n2 / 2 + 1);
  return fftk::lines_pass<T>(p, a, batch, inv, s.n0, plane, plane, 0, 1, st);
}

template <typename T>
Ptrs4 strided(const void* base, int64_t stride, int batch) {
  Ptrs4 r{};
  for (int i = 0; i < batch; ++i)
    r.p[i] = const_cast<char*>(static_cast<const char*>(base)) + size_t(i) * size_t(stride) * sizeof(T);
  return r;
}

}  // namespace

template <typename T>
int fft_r2c_3d(Plan* p, const FftShape& s, const T* in, cplx<T>* out, int batch, int64_t in_stride,
               int64_t out_stride, hipStream_t st) {
  const Ptrs4 i4 = strided<T>(in, in_stride, batch);
  const Ptrs4 o4 = strided<cplx<T>>(out, out_stride, batch);
  int rc = fftk::r2c_z_pass<T>(p, s, i4, o4, batch, nullptr, st);
  if (!rc) rc = y_pass<T>(p, s, o4, batch, false, st);
  if (!rc) rc = x_pass<T>(p, s, o4, batch, false, st);
  return rc;
}

template <typename T>
int fft_c2r_3d(Plan* p, const FftShape& s, cplx<T>* in, T* out, int batch, int64_t in_stride,
               int64_t out_stride, T scale, hipStream_t st) {
  const Ptrs4 i4 = strided<cplx<T>>(in, in_stride, batch);
  const Ptrs4 o4 = strided<T>(out, out_stride, batch);
  int rc = x_pass<T>(p, s, i4, batch, true, st);
  if (!rc) rc = y_pass<T>(p, s, i4, batch, true, st);
  if (!rc) rc = fftk::c2r_z_pass<T>(p, s, i4, o4, batch, scale, st);
  return rc;
}

template <typename T>
int fft_spectral_op(Plan* p, const FftShape& s, SpecOp op, T* const* reals, cplx<T>* const* specs, T coef,
                    const ZFold* zf, hipStream_t st) {
  const int nin = op == SPEC_GRAD3 ? 1 : 4;
  const int nout = op == SPEC_GRAD3 ? 3 : 4;
  const Ptrs4 rin = fftk::ptrs(reals, nin);
  const Ptrs4 spec_in = fftk::ptrs(specs, nin);
  int rc = fftk::r2c_z_pass<T>(p, s, rin, spec_in, nin, zf, st);
  if (!rc) rc = y_pass<T>(p, s, spec_in, nin, false, st);
  if (rc) return rc;
  // outputs in place: GRAD3 g_j -> specs[j]; ADJ4 g_0 -> specs[0],
  // g_1 -> specs[2], g_2 -> specs[3], rhobar -> specs[1] (safe under the
  // kernel's read-before-write order).  The x pass writes g_0, the common
  // factor h of g_1 and g_2 (into g_1's array) and rhobar; the y pass turns
  // h into ky h (g_1) and, as a second transform, h into g_2's array, whose
  // kz the z pass applies.
  Ptrs4 so{};
  if (op == SPEC_GRAD3) {
    so = fftk::ptrs(specs, 3);
  } else {
    so.p[0] = specs[0];
    so.p[1] = specs[2];
    so.p[2] = specs[3];
    so.p[3] = specs[1];
  }
  if ((rc = fftk::x_fused_pass<T>(p, s, op, spec_in, so, coef, st))) return rc;
  const int64_t ncell = int64_t(s.n0) * s.n1 * s.n2;
  // the y pass over g_0, h (two transforms) and rhobar
  Ptrs4 sy{};
  sy.p[0] = so.p[0];
  sy.p[1] = so.p[1];
  sy.p[2] = so.p[3];
  rc = y_pass<T>(p, s, sy, nout - 1, true, st, 1, so.p[2]);
  if (!rc) rc = fftk::c2r_z_pass<T>(p, s, so, fftk::ptrs(reals, nout), nout, T(2.0) / T(ncell), st, 2);
  return rc;
}

template int fft_r2c_3d<float>(Plan*, const FftShape&, const float*, Cx<float>*, int, int64_t, int64_t, hipStream_t);
template int fft_r2c_3d<double>(Plan*, const FftShape&, const double*, Cx<double>*, int, int64_t, int64_t, hipStream_t);
template int fft_c2r_3d<float>(Plan*, const FftShape&, Cx<float>*, float*, int, int64_t, int64_t, float, hipStream_t);
template int fft_c2r_3d<double>(Plan*, const FftShape&, Cx<double>*, double*, int, int64_t, int64_t, double,
                                hipStream_t);
template int fft_spectral_op<float>(Plan*, const FftShape&, SpecOp, float* const*, Cx<float>* const*, float,
                                    const ZFold*, hipStream_t);
template int fft_spectral_op<double>(Plan*, const FftShape&, SpecOp, double* const*, Cx<double>* const*, double,
                                     const ZFold*, hipStream_t);

}  // namespace pmx
