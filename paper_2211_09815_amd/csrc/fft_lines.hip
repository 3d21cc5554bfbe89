// Strided complex FFT pass (the y and x passes of the 3-D transforms).
#include "fft_core.h"

namespace pmx {
namespace fftk {

namespace {

// Lines of length 2^LOGM with element stride ls; a tile is W adjacent columns
// (stride 1) out of ncols, repeated over outer blocks of stride ostride
// (gridDim.x = column tiles * outer blocks) and over the arrays of a batch
// (blockIdx.y).
template <typename T, int LOGM, bool INV>
__global__ __launch_bounds__(kFT, 4) void k_fft_lines(Ptrs4 arrs, int64_t ls, int64_t ncols, int64_t ostride,
                                                      const cplx<T>* __restrict__ tw) {
  using C = cplx<T>;
  constexpr int EPT = Cfg<T>::EPT;
  constexpr int LRMAX = EPT >= 16 ? 4 : 3;
  constexpr int LOGW = tile_log2<T>() - LOGM;
  constexpr int W = 1 << LOGW;
  using F = RegStage<C, EPT, LOGM, LRMAX, false, false>;
  using L = RegStage<C, EPT, LOGM, LRMAX, false, true>;
  C* tws = reinterpret_cast<C*>(fft_smem);
  C* lds = tws + (1 << LOGM);
  const int64_t ncb = (ncols + W - 1) >> LOGW;
  const int64_t tile = xcd_tile(blockIdx.x, int64_t(gridDim.x));
  const int64_t o = tile / ncb;
  const int64_t c0 = (tile - o * ncb) << LOGW;
  C* base = static_cast<C*>(arrs.p[blockIdx.y]) + o * ostride + c0;
  const int tid = threadIdx.x;
  {
    // the first stage's operands straight from HBM, all loads in flight
    C v[F::B][F::R];
#pragma unroll
    for (int b = 0; b < F::B; ++b) {
      const int c = reg_col<F::LR, LOGM, LOGW>(tid, b);
#pragma unroll
      for (int r = 0; r < F::R; ++r)
        v[b][r] = (c0 + c < ncols) ? base[reg_row<F::LR, LOGM, LOGW>(tid, b, r) * ls + c] : cmk<C>(0, 0);
    }
    load_twiddles<LOGM>(tws, tw);
    reg_first_stage<EPT, INV, LOGM, LOGW, LRMAX, false>(v, lds);
    if constexpr (RegPlan<LOGM, LRMAX, false>::S == 1) {
#pragma unroll
      for (int b = 0; b < F::B; ++b) {
        const int c = reg_col<F::LR, LOGM, LOGW>(tid, b);
        if (c0 + c < ncols)
#pragma unroll
          for (int r = 0; r < F::R; ++r) base[reg_row<F::LR, LOGM, LOGW>(tid, b, r) * ls + c] = v[b][r];
      }
      return;
    }
  }
  reg_middle_stages<EPT, INV, LOGM, LOGW, LOGM, LRMAX, false, 1>(lds, tws);
  C u[L::B][L::R];
  reg_last_stage<EPT, INV, LOGM, LOGW, LOGM, LRMAX, false>(lds, tws, u);
#pragma unroll
  for (int b = 0; b < L::B; ++b) {
    const int c = reg_col<L::LR, LOGM, LOGW>(tid, b);
    if (c0 + c < ncols)
#pragma unroll
      for (int r = 0; r < L::R; ++r) base[reg_row<L::LR, LOGM, LOGW>(tid, b, r) * ls + c] = u[b][r];
  }
}

}  // namespace

template <typename T>
int lines_pass(Plan* p, const Ptrs4& arrs, int batch, bool inv, int M, int64_t ls, int64_t ncols, int64_t ostride,
               int64_t nouter, hipStream_t st) {
  const int logM = ilog2(M);
  const int logW = tile_log2<T>() - logM;
  const int64_t ncb = (ncols + (int64_t(1) << logW) - 1) >> logW;
  const dim3 grid(unsigned(ncb * nouter), unsigned(batch));
  const size_t lds = lds_bytes<T>(logM, logM);
  const cplx<T>* tw = static_cast<const cplx<T>*>(p->tw);
  if (logM < 2 || logM > 10) return set_error(p, PM_EUNSUPPORTED, "FFT length %d is not supported", M);
  timing_begin(p, PM_K_FFT_LINES, st);
  (void)with_log2<2, 10>(logM, [&](auto L) {
    constexpr int LOGM = decltype(L)::value;
    auto kern = inv ? k_fft_lines<T, LOGM, true> : k_fft_lines<T, LOGM, false>;
    allow_lds(p, kern, lds);
    hipLaunchKernelGGL(kern, grid, dim3(kFT), lds, st, arrs, ls, ncols, ostride, tw);
    return PM_OK;
  });
  timing_end(p, PM_K_FFT_LINES, st, 2.0 * double(batch) * double(ncols) * double(nouter) * M * sizeof(cplx<T>),
             0.0);   // method bytes: an inner pass moves only intermediates
  PM_HIP_CHECK(p, hipGetLastError());
  return PM_OK;
}

template int lines_pass<float>(Plan*, const Ptrs4&, int, bool, int, int64_t, int64_t, int64_t, int64_t, hipStream_t);
template int lines_pass<double>(Plan*, const Ptrs4&, int, bool, int, int64_t, int64_t, int64_t, int64_t, hipStream_t);

}  // namespace fftk
}  // namespace pmx
