// Pass along x of the force path: forward FFT along x, the Poisson-gradient
// multipliers of Sec. 2.2 (and the transposed multipliers of the force VJP),
// and the inverse FFTs along x of every output, in one kernel.  The spectrum
// along x and the gradient spectra along x are never written to HBM.
#include "fft_core.h"

namespace pmx {
namespace fftk {

namespace {

// wavenumbers of a column of the flattened (y, kz) plane
template <typename T>
struct KCol {
  T ky, kz;
  bool ny, nz;   // on the Nyquist plane of y / z
};

// The thread index passed through an empty asm statement: values derived from
// it inside one phase of the kernel (addresses, wavenumbers) cannot be hoisted
// or shared across phases, which bounds their register lifetime to the phase.
__device__ __forceinline__ int fresh_tid() {
  int t = int(threadIdx.x);
  asm volatile("" : "+v"(t));
  return t;
}

template <typename T>
__device__ __forceinline__ KCol<T> kcol(int64_t col, int n1, int n2, int nh) {
  const T two_pi = T(6.283185307179586476925286766559);
  const int y = int(col / nh);
  const int z = int(col - int64_t(y) * nh);
  const int fy = y < (n1 >> 1) ? y : y - n1;
  KCol<T> r;
  r.ky = two_pi * T(fy) / T(n1);
  r.kz = two_pi * T(z) / T(n2);
  r.ny = (2 * y == n1);
  r.nz = (2 * z == n2);
  return r;
}

// T_j = i k_j coef / k^2, zero at k = 0 and on the Nyquist plane of j.
// GRAD3:  out_j = T_j in_0,                                j = 0..2
// ADJ4:   out_3 = -sum_j T_j in_{1+j},  out_j = T_j in_0,  j = 0..2
// The tile columns run over the flattened (y, kz) plane of the half
// spectrum.  ADJ4 first consumes in_1..3 and writes out_3, then consumes
// in_0 and writes out_0..2, so out_3 may alias in_1..3 and out_0..2 may
// alias any input.
template <typename T, int LOGM, int OP>
__global__ __launch_bounds__(kFT, 4) void k_fft_x_fused(Ptrs4 ins, Ptrs4 outs, int n1, int n2, int nh, T coef,
                                                        const cplx<T>* __restrict__ tw) {
  using C = cplx<T>;
  constexpr int EPT = Cfg<T>::EPT;
  constexpr int M = 1 << LOGM;  // = n0
  constexpr int LOGW = tile_log2<T>() - LOGM;
  constexpr int W = 1 << LOGW;
  constexpr int PITCH = W + 1;
  // when W <= kFT all elements of a thread lie in one column
  constexpr bool ONE_COL = W <= kFT;
  C* tws = reinterpret_cast<C*>(fft_smem);
  C* lds = tws + M;
  const int64_t ncols = int64_t(n1) * nh;
  const int64_t ls = ncols;
  const int64_t c0 = xcd_tile(blockIdx.x, int64_t(gridDim.x)) << LOGW;
  const T two_pi = T(6.283185307179586476925286766559);
  const KCol<T> k0 = kcol<T>(c0 + (int(threadIdx.x) & (W - 1)), n1, n2, nh);
  auto kc = [&](int c) { return ONE_COL ? k0 : kcol<T>(c0 + c, n1, n2, nh); };
  auto kxj = [&](int j, T& kx, bool& nx) {
    const int fx = j < (M >> 1) ? j : j - M;
    kx = two_pi * T(fx) / T(M);
    nx = (2 * j == M);
  };
  auto load_forward = [&](const void* src_v) {
    const C* src = static_cast<const C*>(src_v) + c0;
    // ADJ4 carries EPT accumulators through this phase: load in two halves
    constexpr int NH = OP == SPEC_ADJ4 ? 2 : 1;
    constexpr int EH = EPT / NH;
#pragma unroll
    for (int h = 0; h < NH; ++h) {
      const int tid = fresh_tid();
      C v[EH];
#pragma unroll
      for (int i = 0; i < EH; ++i) {
        const int f = tid + (h * EH + i) * kFT;
        const int c = f & (W - 1), j = f >> LOGW;
        v[i] = (c0 + c < ncols) ? src[int64_t(j) * ls + c] : cmk<C>(0, 0);
      }
      if (h == 0) __syncthreads();  // earlier readers of lds are done
#pragma unroll
      for (int i = 0; i < EH; ++i) {
        const int f = tid + (h * EH + i) * kFT;
        lds[(f >> LOGW) * PITCH + (f & (W - 1))] = v[i];
      }
    }
    fft_lds<EPT, false, LOGM, LOGW, LOGM>(lds, tws);
  };
  auto inverse_store = [&](void* dst_v) {
    fft_lds<EPT, true, LOGM, LOGW, LOGM>(lds, tws);
    C* dst = static_cast<C*>(dst_v) + c0;
    const int tid = fresh_tid();
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int f = tid + i * kFT;
      const int c = f & (W - 1), j = f >> LOGW;
      if (c0 + c < ncols) dst[int64_t(j) * ls + c] = lds[j * PITCH + c];
    }
  };

  load_twiddles<LOGM>(tws, tw);
  if constexpr (OP == SPEC_ADJ4) {
    C acc[EPT];
#pragma unroll
    for (int i = 0; i < EPT; ++i) acc[i] = cmk<C>(0, 0);
#pragma unroll 1
    for (int q = 0; q < 3; ++q) {
      load_forward(ins.p[1 + q]);
      const int tid = fresh_tid();
#pragma unroll
      for (int i = 0; i < EPT; ++i) {
        const int f = tid + i * kFT;
        const int c = f & (W - 1), j = f >> LOGW;
        const KCol<T> kk = kc(c);
        T kx;
        bool nx;
        kxj(j, kx, nx);
        const T kq = q == 0 ? (nx ? T(0) : kx) : q == 1 ? (kk.ny ? T(0) : kk.ky) : (kk.nz ? T(0) : kk.kz);
        const C x = lds[j * PITCH + c];
        acc[i] = cmk<C>(acc[i].x + kq * x.x, acc[i].y + kq * x.y);
      }
    }
    __syncthreads();
    const int tid = fresh_tid();
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int f = tid + i * kFT;
      const int c = f & (W - 1), j = f >> LOGW;
      const KCol<T> kk = kc(c);
      T kx;
      bool nx;
      kxj(j, kx, nx);
      const T k2 = kx * kx + kk.ky * kk.ky + kk.kz * kk.kz;
      const T g = k2 > T(0) ? coef / k2 : T(0);
      // -i g s, s = sum_j k_j in_{1+j}
      lds[j * PITCH + c] = cmk<C>(acc[i].y * g, -acc[i].x * g);
    }
    inverse_store(outs.p[3]);
  }
  C reg[EPT];
  load_forward(ins.p[0]);
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int f = int(threadIdx.x) + i * kFT;
    reg[i] = lds[(f >> LOGW) * PITCH + (f & (W - 1))];
  }
#pragma unroll 1
  for (int comp = 0; comp < 3; ++comp) {
    __syncthreads();
    const int tid = fresh_tid();
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int f = tid + i * kFT;
      const int c = f & (W - 1), j = f >> LOGW;
      const KCol<T> kk = kc(c);
      T kx;
      bool nx;
      kxj(j, kx, nx);
      const T k2 = kx * kx + kk.ky * kk.ky + kk.kz * kk.kz;
      const T kj = comp == 0 ? (nx ? T(0) : kx) : comp == 1 ? (kk.ny ? T(0) : kk.ky) : (kk.nz ? T(0) : kk.kz);
      const T g = k2 > T(0) ? kj * coef / k2 : T(0);
      // i g in
      lds[j * PITCH + c] = cmk<C>(-reg[i].y * g, reg[i].x * g);
    }
    inverse_store(outs.p[comp]);
  }
}

// standalone Poisson gradient on the half spectrum (pm_poisson_grad)
template <typename T>
__global__ __launch_bounds__(kThreads) void k_poisson_grad(const cplx<T>* __restrict__ in, cplx<T>* __restrict__ out,
                                                           int n0, int n1, int n2, int nh, int64_t nspec, T coef) {
  using C = cplx<T>;
  const int64_t idx = int64_t(blockIdx.x) * kThreads + threadIdx.x;
  if (idx >= nspec) return;
  const int z = int(idx % nh);
  const int64_t t = idx / nh;
  const int y = int(t % n1);
  const int x = int(t / n1);
  const T two_pi = T(6.283185307179586476925286766559);
  const int fx = x < (n0 >> 1) ? x : x - n0;
  const int fy = y < (n1 >> 1) ? y : y - n1;
  const T kx = two_pi * T(fx) / T(n0), ky = two_pi * T(fy) / T(n1), kz = two_pi * T(z) / T(n2);
  const T k2 = kx * kx + ky * ky + kz * kz;
  const T g = k2 > T(0) ? coef / k2 : T(0);
  const C v = in[idx];
  const T kk[3] = {2 * x == n0 ? T(0) : kx, 2 * y == n1 ? T(0) : ky, 2 * z == n2 ? T(0) : kz};
#pragma unroll
  for (int j = 0; j < 3; ++j) {
    const T s = kk[j] * g;
    out[j * nspec + idx] = cmk<C>(-v.y * s, v.x * s);
  }
}

}  // namespace

template <typename T>
int x_fused_pass(Plan* p, const FftShape& s, SpecOp op, const Ptrs4& in, const Ptrs4& out, T coef, hipStream_t st) {
  const int nh = s.n2 / 2 + 1;
  const int logM = ilog2(s.n0);
  if (logM < 2 || logM > 10) return set_error(p, PM_EUNSUPPORTED, "FFT length %d is not supported", s.n0);
  const int logW = tile_log2<T>() - logM;
  const int64_t ncols = int64_t(s.n1) * nh;
  const int64_t ntiles = (ncols + (int64_t(1) << logW) - 1) >> logW;
  const size_t lds = lds_bytes<T>(logM, logM);
  const cplx<T>* tw = static_cast<const cplx<T>*>(p->tw);
  const int nin = op == SPEC_GRAD3 ? 1 : 4;
  const int nout = op == SPEC_GRAD3 ? 3 : 4;
  timing_begin(p, PM_K_FFT_POISSON, st);
  (void)with_log2<2, 10>(logM, [&](auto L) {
    constexpr int LOGM = decltype(L)::value;
    auto kern = op == SPEC_GRAD3 ? k_fft_x_fused<T, LOGM, SPEC_GRAD3> : k_fft_x_fused<T, LOGM, SPEC_ADJ4>;
    allow_lds(p, kern, lds);
    hipLaunchKernelGGL(kern, dim3(unsigned(ntiles)), dim3(kFT), lds, st, in, out, s.n1, s.n2, nh, coef, tw);
    return PM_OK;
  });
  timing_end(p, PM_K_FFT_POISSON, st, double(nin + nout) * double(ncols) * double(s.n0) * sizeof(cplx<T>));
  PM_HIP_CHECK(p, hipGetLastError());
  return PM_OK;
}

template int x_fused_pass<float>(Plan*, const FftShape&, SpecOp, const Ptrs4&, const Ptrs4&, float, hipStream_t);
template int x_fused_pass<double>(Plan*, const FftShape&, SpecOp, const Ptrs4&, const Ptrs4&, double, hipStream_t);

}  // namespace fftk

template <typename T>
int poisson_grad_spec(Plan* p, const FftShape& s, const cplx<T>* in, cplx<T>* out, T coef, hipStream_t st) {
  const int nh = s.n2 / 2 + 1;
  const int64_t nspec = int64_t(s.n0) * s.n1 * nh;
  const unsigned blocks = unsigned((nspec + kThreads - 1) / kThreads);
  hipLaunchKernelGGL((fftk::k_poisson_grad<T>), dim3(blocks), dim3(kThreads), 0, st, in, out, s.n0, s.n1, s.n2, nh,
                     nspec, coef);
  PM_HIP_CHECK(p, hipGetLastError());
  return PM_OK;
}

template int poisson_grad_spec<float>(Plan*, const FftShape&, const Cx<float>*, Cx<float>*, float, hipStream_t);
template int poisson_grad_spec<double>(Plan*, const FftShape&, const Cx<double>*, Cx<double>*, double, hipStream_t);

}  // namespace pmx
