// Strided complex FFT pass (the y and x passes of the 3-D transforms).
#include "fft_core.h"

namespace pmx {
namespace fftk {

namespace {

// Lines of length 2^LOGM with element stride ls; a tile is W adjacent columns
// (stride 1) out of ncols, repeated over outer blocks of stride ostride
// (gridDim.x = column tiles * outer blocks) and over the arrays of a batch
// (blockIdx.y).  Array `dual` (-1: none) is transformed twice: as it is, into
// dual_out, then times the line's wavenumber 2 pi f / 2^LOGM (f the signed
// frequency index along the line, zero on the Nyquist row), in place; the
// second transform reads the tile again (from L2: the first has just read it).
template <typename T, int LOGM, bool INV>
__global__ __launch_bounds__(kFT, 4) void k_fft_lines(Ptrs4 arrs, int64_t ls, int64_t ncols, int64_t ostride,
                                                      const cplx<T>* __restrict__ tw, int dual, void* dual_out) {
  using C = cplx<T>;
  constexpr int EPT = Cfg<T>::EPT;
  constexpr int LRMAX = EPT >= 16 ? 4 : 3;
  constexpr int M = 1 << LOGM;
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
  const int64_t at0 = o * ostride + c0;
  C* base = static_cast<C*>(arrs.p[blockIdx.y]) + at0;
  const bool twice = int(blockIdx.y) == dual;
  const int tid = threadIdx.x;
  // one transform of the tile of src into dst; with wk each element first
  // times its row's wavenumber (the multiply of the fused x pass's outputs);
  // the first one also loads the twiddles
  auto transform = [&](const C* src, C* dst, bool wk, bool first) {
    {
      // the first stage's operands straight from HBM, all loads in flight
      C v[F::B][F::R];
#pragma unroll
      for (int b = 0; b < F::B; ++b) {
        const int c = reg_col<F::LR, LOGM, LOGW>(tid, b);
#pragma unroll
        for (int r = 0; r < F::R; ++r)
          v[b][r] = (c0 + c < ncols) ? src[reg_row<F::LR, LOGM, LOGW>(tid, b, r) * ls + c] : cmk<C>(0, 0);
      }
      if (wk) {
        const T two_pi = T(6.283185307179586476925286766559);
#pragma unroll
        for (int b = 0; b < F::B; ++b)
#pragma unroll
          for (int r = 0; r < F::R; ++r) {
            const int j = reg_row<F::LR, LOGM, LOGW>(tid, b, r);
            const int fj = j < (M >> 1) ? j : j - M;
            const T k = 2 * j == M ? T(0) : two_pi * T(fj) / T(M);
            v[b][r] = cmk<C>(k * v[b][r].x, k * v[b][r].y);
          }
      }
      if (first) load_twiddles<LOGM>(tws, tw);
      else __syncthreads();   // earlier readers of lds are done
      reg_first_stage<EPT, INV, LOGM, LOGW, LRMAX, false>(v, lds);
      if constexpr (RegPlan<LOGM, LRMAX, false>::S == 1) {
#pragma unroll
        for (int b = 0; b < F::B; ++b) {
          const int c = reg_col<F::LR, LOGM, LOGW>(tid, b);
          if (c0 + c < ncols)
#pragma unroll
            for (int r = 0; r < F::R; ++r) dst[reg_row<F::LR, LOGM, LOGW>(tid, b, r) * ls + c] = v[b][r];
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
        for (int r = 0; r < L::R; ++r) dst[reg_row<L::LR, LOGM, LOGW>(tid, b, r) * ls + c] = u[b][r];
    }
  };
  if (!twice) {
    transform(base, base, false, true);
    return;
  }
  transform(base, static_cast<C*>(dual_out) + at0, false, true);
  transform(base, base, true, false);
}

}  // namespace

template <typename T>
int lines_pass(Plan* p, const Ptrs4& arrs, int batch, bool inv, int M, int64_t ls, int64_t ncols, int64_t ostride,
               int64_t nouter, hipStream_t st, int dual, void* dual_out) {
  const int logM = ilog2(M);
  const int logW = tile_log2<T>() - logM;
  const int64_t ncb = (ncols + (int64_t(1) << logW) - 1) >> logW;
  const dim3 grid(unsigned(ncb * nouter), unsigned(batch));
  const size_t lds = lds_bytes<T>(logM, logM);
  const cplx<T>* tw = static_cast<const cplx<T>*>(p->tw);
  if (logM < 2 || logM > 10) return set_error(p, PM_EUNSUPPORTED, "FFT length %d is not supported", M);
  if (dual >= batch || (dual >= 0 && !dual_out)) return set_error(p, PM_EINVAL, "bad second transform of a line pass");
  timing_begin(p, PM_K_FFT_LINES, st);
  (void)with_log2<2, 10>(logM, [&](auto L) {
    constexpr int LOGM = decltype(L)::value;
    auto kern = inv ? k_fft_lines<T, LOGM, true> : k_fft_lines<T, LOGM, false>;
    allow_lds(p, kern, lds);
    hipLaunchKernelGGL(kern, grid, dim3(kFT), lds, st, arrs, ls, ncols, ostride, tw, dual, dual_out);
    return PM_OK;
  });
  // each array read and written once, the dual array's second output written
  // (its second read comes from L2)
  const double nb = 2.0 * batch + (dual >= 0 ? 1.0 : 0.0);
  timing_end(p, PM_K_FFT_LINES, st, nb * double(ncols) * double(nouter) * M * sizeof(cplx<T>),
             0.0);   // method bytes: an inner pass moves only intermediates
  PM_HIP_CHECK(p, hipGetLastError());
  return PM_OK;
}

template int lines_pass<float>(Plan*, const Ptrs4&, int, bool, int, int64_t, int64_t, int64_t, int64_t, hipStream_t, int,
                               void*);
template int lines_pass<double>(Plan*, const Ptrs4&, int, bool, int, int64_t, int64_t, int64_t, int64_t, hipStream_t,
                                int, void*);

}  // namespace fftk
}  // namespace pmx
