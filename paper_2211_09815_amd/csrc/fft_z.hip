// z passes of the 3-D real transforms: real lines of N = 2M values <-> half
// spectra of M + 1 bins, through one complex FFT of length M per line.
#include "fft_core.h"

namespace pmx {
namespace fftk {

namespace {

// real -> complex.  z[n] = x[2n] + i x[2n+1];  Z = FFT_M(z);  with
// Zc = conj(Z[M-k]):  X[k] = (Z + Zc)/2 - i exp(-2 pi i k/N) (Z - Zc)/2,
// k = 0..M.  FOLD: x[z] += the paint's z-face halo value of the tile below,
// for every z on a tile boundary (z = 2n is even there).
template <typename T, int LOGM, bool FOLD>
__global__ __launch_bounds__(kFT, 4) void k_fft_r2c_z(Ptrs4 ins, Ptrs4 outs, int64_t nlines,
                                                      const cplx<T>* __restrict__ tw, ZFold zf) {
  using C = cplx<T>;
  using R = T;
  constexpr int EPT = Cfg<T>::EPT;
  constexpr int M = 1 << LOGM;
  constexpr int LOGL = LOGM + 1;
  constexpr int LOGW = tile_log2<T>() - LOGM;
  constexpr int W = 1 << LOGW;
  constexpr int PITCH = W + 1;
  C* tws = reinterpret_cast<C*>(fft_smem);
  C* lds = tws + 2 * M;
  const int64_t l0 = xcd_tile(blockIdx.x, int64_t(gridDim.x)) << LOGW;
  const C* src = reinterpret_cast<const C*>(static_cast<const T*>(ins.p[blockIdx.y])) + l0 * M;
  C* dst = static_cast<C*>(outs.p[blockIdx.y]) + l0 * (M + 1);
  const int lines_here = int(nlines - l0 < W ? nlines - l0 : W);
  const int tid = threadIdx.x;
  {
    C v[EPT];
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int f = tid + i * kFT;
      v[i] = ((f >> LOGM) < lines_here) ? src[f] : cmk<C>(0, 0);
    }
    if constexpr (FOLD) {
      // the z faces these lines need, entry t * W + l for line l and tile
      // boundary z = t tz, staged in LDS after the data with reads that run
      // along y (the fastest index of a face)
      T* zb = reinterpret_cast<T*>(lds + M * PITCH);
      const T* halo = static_cast<const T*>(zf.halo) + int64_t(blockIdx.y) * zf.ntiles * zf.hc;
      const int nt = (2 * M) >> zf.ltz;
      for (int j = tid; j < nt * W; j += kFT) {
        const int l = j & (W - 1), t = j >> LOGW;
        T h = T(0);
        if (l < lines_here) {
          const int64_t line = l0 + l;
          const int x = int(line >> zf.ln1), y = int(line & ((int64_t(1) << zf.ln1) - 1));
          const int tb = (t - 1) & (zf.ntz - 1);
          const int64_t below = (int64_t(x >> zf.ltx) * zf.nty + (y >> zf.lty)) * zf.ntz + tb;
          h = halo[below * zf.hc + zf.face + ((x & ((1 << zf.ltx) - 1)) << zf.lty) + (y & ((1 << zf.lty) - 1))];
        }
        zb[j] = h;
      }
      __syncthreads();
#pragma unroll
      for (int i = 0; i < EPT; ++i) {
        const int f = tid + i * kFT;
        const int z = 2 * (f & (M - 1));
        if ((z & ((1 << zf.ltz) - 1)) == 0) v[i].x += zb[((z >> zf.ltz) << LOGW) + (f >> LOGM)];
      }
    }
    load_twiddles<LOGL>(tws, tw);
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int f = tid + i * kFT;
      lds[(f & (M - 1)) * PITCH + (f >> LOGM)] = v[i];
    }
  }
  fft_lds<EPT, false, LOGM, LOGW, LOGL>(lds, tws);
  auto bin = [&](int l, int k) {
    const C z = lds[(k & (M - 1)) * PITCH + l];
    const C zc = cconj(lds[((M - k) & (M - 1)) * PITCH + l]);
    const C e = cscale(cadd(z, zc), R(0.5));
    const C d = cscale(csub(z, zc), R(0.5));
    const C od = cmk<C>(d.y, -d.x);  // -i d
    return cadd(e, cmul(tws[k], od));
  };
#pragma unroll 4
  for (int i = 0; i < EPT; ++i) {
    const int f = tid + i * kFT;
    const int l = f >> LOGM, k = f & (M - 1);
    if (l < lines_here) dst[int64_t(l) * (M + 1) + k] = bin(l, k);
  }
  for (int l = tid; l < lines_here; l += kFT) dst[int64_t(l) * (M + 1) + M] = bin(l, M);
}

// complex -> real.  From X[0..M] (imaginary parts of X[0] and X[M] ignored):
// E = (X[k] + conj X[M-k])/2,  O = (X[k] - conj X[M-k]) conj(w^k)/2,
// Z = E + i O,  z = IFFT_M(Z) (unnormalised),  x[2n] + i x[2n+1] = scale z[n].
// Array kz_arr first takes X[k] times kz = 2 pi k / (2M), zero at k = M.
template <typename T, int LOGM>
__global__ __launch_bounds__(kFT, 4) void k_fft_c2r_z(Ptrs4 ins, Ptrs4 outs, int64_t nlines, T scale,
                                                      const cplx<T>* __restrict__ tw, int kz_arr) {
  using C = cplx<T>;
  using R = T;
  constexpr int EPT = Cfg<T>::EPT;
  constexpr int M = 1 << LOGM;
  constexpr int LOGL = LOGM + 1;
  constexpr int LOGW = tile_log2<T>() - LOGM;
  constexpr int W = 1 << LOGW;
  constexpr int PITCH = W + 1;
  C* tws = reinterpret_cast<C*>(fft_smem);
  C* lds = tws + 2 * M;
  const int64_t l0 = xcd_tile(blockIdx.x, int64_t(gridDim.x)) << LOGW;
  const C* src = static_cast<const C*>(ins.p[blockIdx.y]) + l0 * (M + 1);
  C* dst = reinterpret_cast<C*>(static_cast<T*>(outs.p[blockIdx.y])) + l0 * M;
  const int lines_here = int(nlines - l0 < W ? nlines - l0 : W);
  const int tid = threadIdx.x;
  {
    C a[EPT], b[EPT];
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int f = tid + i * kFT;
      const int l = f >> LOGM, k = f & (M - 1);
      a[i] = cmk<C>(0, 0);
      b[i] = cmk<C>(0, 0);
      if (l < lines_here) {
        const C* line = src + int64_t(l) * (M + 1);
        a[i] = line[k];
        b[i] = line[M - k];
      }
    }
    if (int(blockIdx.y) == kz_arr) {
      // the z factor of the gradient (the Nyquist bin M, and k = 0, get zero)
      const T two_pi = T(6.283185307179586476925286766559);
#pragma unroll
      for (int i = 0; i < EPT; ++i) {
        const int k = (tid + i * kFT) & (M - 1);
        const T ka = two_pi * T(k) / T(2 * M);
        const T kb = k == 0 ? T(0) : two_pi * T(M - k) / T(2 * M);
        a[i] = cmk<C>(ka * a[i].x, ka * a[i].y);
        b[i] = cmk<C>(kb * b[i].x, kb * b[i].y);
      }
    }
    load_twiddles<LOGL>(tws, tw);
    __syncthreads();
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int f = tid + i * kFT;
      const int l = f >> LOGM, k = f & (M - 1);
      if (k == 0) { a[i].y = 0; b[i].y = 0; }
      const C bc = cconj(b[i]);
      const C e = cscale(cadd(a[i], bc), R(0.5));
      const C o = cmul(cscale(csub(a[i], bc), R(0.5)), cconj(tws[k]));
      lds[k * PITCH + l] = cmk<C>(e.x - o.y, e.y + o.x);  // e + i o
    }
  }
  fft_lds<EPT, true, LOGM, LOGW, LOGL>(lds, tws);
#pragma unroll 4
  for (int i = 0; i < EPT; ++i) {
    const int f = tid + i * kFT;
    const int l = f >> LOGM, n = f & (M - 1);
    if (l < lines_here) dst[f] = cscale(lds[n * PITCH + l], scale);
  }
}

template <typename T>
int64_t z_tiles(const FftShape& s, int logM) {
  const int64_t nlines = int64_t(s.n0) * s.n1;
  const int logW = tile_log2<T>() - logM;
  return (nlines + (int64_t(1) << logW) - 1) >> logW;
}

}  // namespace

template <typename T>
int r2c_z_pass(Plan* p, const FftShape& s, const Ptrs4& in, const Ptrs4& out, int batch, const ZFold* zf,
               hipStream_t st) {
  const int nh = s.n2 / 2 + 1;
  const int logM = ilog2(s.n2 / 2);
  const int64_t nlines = int64_t(s.n0) * s.n1;
  const dim3 grid(unsigned(z_tiles<T>(s, logM)), unsigned(batch));
  const size_t lds = lds_bytes<T>(logM, logM + 1);
  const cplx<T>* tw = static_cast<const cplx<T>*>(p->tw);
  if (logM < 1 || logM > 9) return set_error(p, PM_EUNSUPPORTED, "FFT length %d is not supported", s.n2);
  const bool fold = zf && zf->halo;
  const ZFold zfv = fold ? *zf : ZFold{};
  // the fold stages one value per line and tile boundary after the data
  const size_t lds_fold = fold ? lds + (size_t(1) << (tile_log2<T>() - logM)) * (s.n2 >> zfv.ltz) * sizeof(T) : lds;
  timing_begin(p, PM_K_FFT_R2C_Z, st);
  (void)with_log2<1, 9>(logM, [&](auto L) {
    constexpr int LOGM = decltype(L)::value;
    if (fold) {
      allow_lds(p, k_fft_r2c_z<T, LOGM, true>, lds_fold);
      hipLaunchKernelGGL((k_fft_r2c_z<T, LOGM, true>), grid, dim3(kFT), lds_fold, st, in, out, nlines, tw, zfv);
    } else {
      allow_lds(p, k_fft_r2c_z<T, LOGM, false>, lds);
      hipLaunchKernelGGL((k_fft_r2c_z<T, LOGM, false>), grid, dim3(kFT), lds, st, in, out, nlines, tw, zfv);
    }
    return PM_OK;
  });
  // lines read and half spectra written (+ one halo value per tile boundary)
  // method bytes: the 3-D R2C's real input read and half spectrum written
  const double fold_bytes = fold ? double(s.n2 >> zf->ltz) * sizeof(T) : 0.0;
  const double io = double(s.n2) * sizeof(T) + double(nh) * sizeof(cplx<T>);
  timing_end(p, PM_K_FFT_R2C_Z, st, double(batch) * double(nlines) * (io + fold_bytes),
             double(batch) * double(nlines) * io);
  PM_HIP_CHECK(p, hipGetLastError());
  return PM_OK;
}

template <typename T>
int c2r_z_pass(Plan* p, const FftShape& s, const Ptrs4& in, const Ptrs4& out, int batch, T scale, hipStream_t st,
               int kz_arr) {
  const int nh = s.n2 / 2 + 1;
  const int logM = ilog2(s.n2 / 2);
  const int64_t nlines = int64_t(s.n0) * s.n1;
  const dim3 grid(unsigned(z_tiles<T>(s, logM)), unsigned(batch));
  const size_t lds = lds_bytes<T>(logM, logM + 1);
  const cplx<T>* tw = static_cast<const cplx<T>*>(p->tw);
  if (logM < 1 || logM > 9) return set_error(p, PM_EUNSUPPORTED, "FFT length %d is not supported", s.n2);
  timing_begin(p, PM_K_FFT_C2R_Z, st);
  (void)with_log2<1, 9>(logM, [&](auto L) {
    constexpr int LOGM = decltype(L)::value;
    allow_lds(p, k_fft_c2r_z<T, LOGM>, lds);
    hipLaunchKernelGGL((k_fft_c2r_z<T, LOGM>), grid, dim3(kFT), lds, st, in, out, nlines, scale, tw, kz_arr);
    return PM_OK;
  });
  // method bytes: the 3-D C2R's half spectrum read and real output written
  const double io = double(batch) * double(nlines) * (double(s.n2) * sizeof(T) + double(nh) * sizeof(cplx<T>));
  timing_end(p, PM_K_FFT_C2R_Z, st, io, io);
  PM_HIP_CHECK(p, hipGetLastError());
  return PM_OK;
}

template int r2c_z_pass<float>(Plan*, const FftShape&, const Ptrs4&, const Ptrs4&, int, const ZFold*, hipStream_t);
template int r2c_z_pass<double>(Plan*, const FftShape&, const Ptrs4&, const Ptrs4&, int, const ZFold*, hipStream_t);
template int c2r_z_pass<float>(Plan*, const FftShape&, const Ptrs4&, const Ptrs4&, int, float, hipStream_t, int);
template int c2r_z_pass<double>(Plan*, const FftShape&, const Ptrs4&, const Ptrs4&, int, double, hipStream_t, int);

}  // namespace fftk
}  // namespace pmx
