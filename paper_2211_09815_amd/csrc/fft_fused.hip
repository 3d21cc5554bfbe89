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

// Elements per thread of the fused pass.  FP32 up to 512-point columns takes
// 8 instead of the other passes' 16: the pass keeps the forward spectrum in
// registers through the first inverse transform, which at 16 elements per
// thread spills past the 128 VGPRs of two workgroups per CU; at 8 the tile
// holds 8 columns (64-byte row runs) and three workgroups fit.
constexpr int x_ept(bool f32, int logm) { return f32 && logm <= 9 ? 8 : (f32 ? 16 : 8); }

// T_j = i k_j coef / k^2, zero at k = 0 and on the Nyquist plane of j.
// GRAD3:  out_0 = T_0 in_0,  out_1 = h
// ADJ4:   out_3 = -sum_j T_j in_{1+j},  out_0 = T_0 in_0,  out_1 = h
// with h = i coef / k^2 in_0 (zero on the x Nyquist plane), the common factor
// of the y and z components: the y pass forms T_1 in_0 = ky h and h from it
// (lines_pass with a second transform), and the z pass multiplies by kz.
// Writing one array for both saves a spectrum write here and a read there.
// The tile columns run over the flattened (y, kz) plane of the half
// spectrum.  ADJ4 first consumes in_1..3 and writes out_3, then consumes
// in_0 and writes out_0 and out_1, so out_3 may alias in_1..3 and out_0..1
// may alias any input.
template <typename T, int LOGM, int OP>
__global__ __launch_bounds__(kFT, 4) void k_fft_x_fused(Ptrs4 ins, Ptrs4 outs, int n1, int n2, int nh, T coef,
                                                        const cplx<T>* __restrict__ tw) {
  using C = cplx<T>;
  constexpr int EPT = x_ept(sizeof(T) == 4, LOGM);
  constexpr int LRMAX = EPT >= 16 ? 4 : 3;
  constexpr int M = 1 << LOGM;  // = n0
  constexpr int LOGW = ilog2c(kFT * EPT) - LOGM;
  constexpr int W = 1 << LOGW;
  constexpr int S = RegPlan<LOGM, LRMAX, false>::S;
  // forward stages larger radix first, inverse stages in the reverse order,
  // so the forward's last stage and the inverse's first share one register
  // layout: the multipliers are applied in registers between them
  using FF = RegStage<C, EPT, LOGM, LRMAX, false, false>;
  using FL = RegStage<C, EPT, LOGM, LRMAX, false, true>;
  using IF = RegStage<C, EPT, LOGM, LRMAX, true, false>;
  using IL = RegStage<C, EPT, LOGM, LRMAX, true, true>;
  static_assert(FL::LR == IF::LR, "forward last and inverse first radix");
  // when W <= kFT all elements of a thread lie in one column
  constexpr bool ONE_COL = W <= kFT;
  C* tws = reinterpret_cast<C*>(fft_smem);
  C* lds = tws + M;
  const int64_t ncols = int64_t(n1) * nh;
  const int64_t ls = ncols;
  const int64_t c0 = xcd_tile(blockIdx.x, int64_t(gridDim.x)) << LOGW;
  const T two_pi = T(6.283185307179586476925286766559);
  const int col0 = int(threadIdx.x) & (W - 1);
  const KCol<T> kk0 = kcol<T>(c0 + col0, n1, n2, nh);
  auto colof = [&](int tid, int b) { return ONE_COL ? col0 : (tid + b * kFT) & (W - 1); };
  auto kkof = [&](int tid, int b) { return ONE_COL ? kk0 : kcol<T>(c0 + colof(tid, b), n1, n2, nh); };
  // kx and its Nyquist flag of output row reg_row(b, r) of the forward's last stage
  auto kxj = [&](int j, T& kx, bool& nx) {
    const int fx = j < (M >> 1) ? j : j - M;
    kx = two_pi * T(fx) / T(M);
    nx = (2 * j == M);
  };
  // ky, kz (zero on their Nyquist planes) of butterfly b's column
  auto kyz = [&](int tid, int b, T& ky, T& kz) {
    const KCol<T> kk = kkof(tid, b);
    ky = kk.ny ? T(0) : kk.ky;
    kz = kk.nz ? T(0) : kk.kz;
  };
  // g = coef / k^2 at the forward's last-stage element (b, r), and its kx
  // (zero on the Nyquist plane)
  auto gk = [&](int tid, int b, int r, T& g, T& kxn) {
    const KCol<T> kk = kkof(tid, b);
    T kx;
    bool nx;
    kxj(reg_row<FL::LR, LOGM, LOGW>(tid, b, r), kx, nx);
    // explicit fused multiply-adds: the force of the Poisson path and of the
    // VJP path must round identically (exact time reversal), whatever the
    // compiler would contract in either kernel
    const T k2 = fma(kx, kx, fma(kk.ky, kk.ky, kk.kz * kk.kz));
    g = k2 > T(0) ? coef / k2 : T(0);
    kxn = nx ? T(0) : kx;
  };

  // forward FFT along x of one input into X (frequency rows)
  auto forward = [&](const void* src_v, C (&X)[FL::B][FL::R], bool lds_busy) {
    const C* src = static_cast<const C*>(src_v) + c0;
    const int tid = fresh_tid();
    C v[FF::B][FF::R];
#pragma unroll
    for (int b = 0; b < FF::B; ++b) {
      const int col = colof(tid, b);
#pragma unroll
      for (int r = 0; r < FF::R; ++r)
        v[b][r] = c0 + col < ncols ? src[int64_t(reg_row<FF::LR, LOGM, LOGW>(tid, b, r)) * ls + col] : cmk<C>(0, 0);
    }
    if (lds_busy) __syncthreads();   // earlier readers of lds are done
    reg_first_stage<EPT, false, LOGM, LOGW, LRMAX, false>(v, lds);
    if constexpr (S == 1) {
#pragma unroll
      for (int b = 0; b < FL::B; ++b)
#pragma unroll
        for (int r = 0; r < FL::R; ++r) X[b][r] = v[b][r];
    } else {
      reg_middle_stages<EPT, false, LOGM, LOGW, LOGM, LRMAX, false, 1>(lds, tws);
      reg_last_stage<EPT, false, LOGM, LOGW, LOGM, LRMAX, false>(lds, tws, X);
    }
  };
  // inverse FFT along x of Y (frequency rows, the forward's last layout),
  // stored to dst
  auto store_rows = [&](int tid, const auto& u, int lr, void* dst) {
    constexpr int NB = sizeof(u) / sizeof(u[0]);
    constexpr int NR = sizeof(u[0]) / sizeof(C);
    C* d = static_cast<C*>(dst) + c0;
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      const int col = colof(tid, b);
      if (c0 + col >= ncols) continue;
#pragma unroll
      for (int r = 0; r < NR; ++r) d[int64_t(((tid + b * kFT) >> LOGW) + (r << (LOGM - lr))) * ls + col] = u[b][r];
    }
  };
  auto inverse_store = [&](C (&Y)[IF::B][IF::R], void* dst) {
    __syncthreads();   // earlier readers of lds are done
    reg_first_stage<EPT, true, LOGM, LOGW, LRMAX, true>(Y, lds);
    const int tid = fresh_tid();
    if constexpr (S == 1) {
      store_rows(tid, Y, IF::LR, dst);
    } else {
      reg_middle_stages<EPT, true, LOGM, LOGW, LOGM, LRMAX, true, 1>(lds, tws);
      C u[IL::B][IL::R];
      reg_last_stage<EPT, true, LOGM, LOGW, LOGM, LRMAX, true>(lds, tws, u);
      store_rows(tid, u, IL::LR, dst);
    }
  };
  // forward FFT along x of ky in_a + kz in_b (ky, kz of each column)
  auto forward_yz = [&](const void* src_a, const void* src_b, C (&X)[FL::B][FL::R]) {
    const C* sa = static_cast<const C*>(src_a) + c0;
    const C* sb = static_cast<const C*>(src_b) + c0;
    const int tid = fresh_tid();
    C v[FF::B][FF::R];
#pragma unroll
    for (int b = 0; b < FF::B; ++b) {
      const int col = colof(tid, b);
      T ky, kz;
      kyz(tid, b, ky, kz);
#pragma unroll
      for (int r = 0; r < FF::R; ++r) {
        const int64_t at = int64_t(reg_row<FF::LR, LOGM, LOGW>(tid, b, r)) * ls + col;
        v[b][r] = cmk<C>(0, 0);
        if (c0 + col < ncols) {
          const C a = sa[at], e = sb[at];
          v[b][r] = cmk<C>(ky * a.x + kz * e.x, ky * a.y + kz * e.y);
        }
      }
    }
    __syncthreads();   // earlier readers of lds are done
    reg_first_stage<EPT, false, LOGM, LOGW, LRMAX, false>(v, lds);
    if constexpr (S == 1) {
#pragma unroll
      for (int b = 0; b < FL::B; ++b)
#pragma unroll
        for (int r = 0; r < FL::R; ++r) X[b][r] = v[b][r];
    } else {
      reg_middle_stages<EPT, false, LOGM, LOGW, LOGM, LRMAX, false, 1>(lds, tws);
      reg_last_stage<EPT, false, LOGM, LOGW, LOGM, LRMAX, false>(lds, tws, X);
    }
  };

  load_twiddles<LOGM>(tws, tw);
  bool lds_busy = false;
  if constexpr (OP == SPEC_ADJ4) {
    // s = kx in_1 + ky in_2 + kz in_3: ky and kz are constant along x, so
    // in_2 and in_3 are combined before their one forward transform
    C acc[FL::B][FL::R];
    forward(ins.p[1], acc, false);
    lds_busy = true;
    {
      const int tid = fresh_tid();
#pragma unroll
      for (int b = 0; b < FL::B; ++b)
#pragma unroll
        for (int r = 0; r < FL::R; ++r) {
          T g, kxn;
          gk(tid, b, r, g, kxn);
          acc[b][r] = cmk<C>(kxn * acc[b][r].x, kxn * acc[b][r].y);
        }
    }
    {
      C X[FL::B][FL::R];
      forward_yz(ins.p[2], ins.p[3], X);
#pragma unroll
      for (int b = 0; b < FL::B; ++b)
#pragma unroll
        for (int r = 0; r < FL::R; ++r) acc[b][r] = cadd(acc[b][r], X[b][r]);
    }
    const int tid = fresh_tid();
#pragma unroll
    for (int b = 0; b < FL::B; ++b)
#pragma unroll
      for (int r = 0; r < FL::R; ++r) {
        T g, kxn;
        gk(tid, b, r, g, kxn);
        // -i g s
        acc[b][r] = cmk<C>(acc[b][r].y * g, -acc[b][r].x * g);
      }
    inverse_store(acc, outs.p[3]);
  }
  // out_0 = IFFT(i g kx X);  out_1 = IFFT(i g X) (h; ky and kz later)
  C X[FL::B][FL::R];
  forward(ins.p[0], X, lds_busy);
  {
    const int tid = fresh_tid();
    C Y[IF::B][IF::R];
#pragma unroll
    for (int b = 0; b < FL::B; ++b)
#pragma unroll
      for (int r = 0; r < FL::R; ++r) {
        T g, kxn;
        gk(tid, b, r, g, kxn);
        g *= kxn;
        Y[b][r] = cmk<C>(-X[b][r].y * g, X[b][r].x * g);
      }
    inverse_store(Y, outs.p[0]);
  }
  {
    const int tid = fresh_tid();
#pragma unroll
    for (int b = 0; b < FL::B; ++b)
#pragma unroll
      for (int r = 0; r < FL::R; ++r) {
        T g, kxn;
        gk(tid, b, r, g, kxn);
        X[b][r] = cmk<C>(-X[b][r].y * g, X[b][r].x * g);
      }
    inverse_store(X, outs.p[1]);
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
  const int logW = ilog2(kFT * x_ept(sizeof(T) == 4, logM)) - logM;
  const int64_t ncols = int64_t(s.n1) * nh;
  const int64_t ntiles = (ncols + (int64_t(1) << logW) - 1) >> logW;
  const size_t lds = size_t((1 << logM) + (1 << logM) * ((1 << logW) + 1)) * sizeof(cplx<T>);
  const cplx<T>* tw = static_cast<const cplx<T>*>(p->tw);
  const int nin = op == SPEC_GRAD3 ? 1 : 4;
  const int nout = op == SPEC_GRAD3 ? 2 : 3;
  timing_begin(p, PM_K_FFT_POISSON, st);
  (void)with_log2<2, 10>(logM, [&](auto L) {
    constexpr int LOGM = decltype(L)::value;
    auto kern = op == SPEC_GRAD3 ? k_fft_x_fused<T, LOGM, SPEC_GRAD3> : k_fft_x_fused<T, LOGM, SPEC_ADJ4>;
    allow_lds(p, kern, lds);
    hipLaunchKernelGGL(kern, dim3(unsigned(ntiles)), dim3(kFT), lds, st, in, out, s.n1, s.n2, nh, coef, tw);
    return PM_OK;
  });
  // method bytes: none (the spectra along x are intermediates of the 3-D transforms)
  timing_end(p, PM_K_FFT_POISSON, st, double(nin + nout) * double(ncols) * double(s.n0) * sizeof(cplx<T>), 0.0);
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
