// Building blocks of the LDS FFT kernels (fft_lines.hip, fft_z.hip,
// fft_fused.hip) and the launchers they export to fft.hip.
//
// Every 1-D transform of length M = 2^LOGM <= 1024 is done by one workgroup of
// 512 threads inside LDS.  A workgroup holds a tile of W = TILE / M lines
// (TILE = 8192 complex values in FP32, 4096 in FP64, i.e. 64 KiB); lines are
// stored point-major (element j of line c at j*(W+1) + c), so consecutive
// lanes touch consecutive LDS addresses in every Stockham stage.  The
// twiddles exp(-2 pi i m / L) of the tile's transform are copied into LDS once
// per workgroup from a table of exp(-2 pi i m / 4096) computed in double
// precision on the host.  Stages use radix 16 (FP32) or 8 (FP64) at most,
// with the log2(M) bits split as evenly as possible over the fewest stages.
// The transform length is a template parameter, so every LDS offset of a
// stage is a compile-time constant.
#pragma once

#include <map>
#include <mutex>
#include <type_traits>
#include <utility>

#include "pm_internal.h"

namespace pmx {
namespace fftk {

constexpr int kFT = 512;  // threads per FFT workgroup

template <typename T> struct Cfg;
template <> struct Cfg<float> { static constexpr int EPT = 16; };
template <> struct Cfg<double> { static constexpr int EPT = 8; };
template <typename T> constexpr int tile_log2() { return ilog2c(kFT * Cfg<T>::EPT); }

// up to four arrays of one batched pass (index = blockIdx.y)
struct Ptrs4 {
  void* p[4];
};

template <typename P>
inline Ptrs4 ptrs(P* const* a, int n) {
  Ptrs4 r{};
  for (int i = 0; i < n; ++i) r.p[i] = const_cast<void*>(static_cast<const void*>(a[i]));
  return r;
}

// dynamic LDS: [twiddles: L entries][data: M * (W + 1) entries]
extern __shared__ double2 fft_smem[];

template <typename T>
inline size_t lds_bytes(int logM, int logL) {
  const int M = 1 << logM;
  const int W = 1 << (tile_log2<T>() - logM);
  return size_t((1 << logL) + M * (W + 1)) * sizeof(cplx<T>);
}

// The kernels take their LDS size at launch; allow more than the default
// limit once per (device, kernel).  A runtime that needs no opt-in may reject
// the call: its error is cleared so that it cannot surface at the launch check.
template <typename K>
inline void allow_lds(const Plan* p, K kernel, size_t bytes) {
  static std::mutex mu;
  static std::map<std::pair<int, const void*>, size_t> done;
  const void* k = reinterpret_cast<const void*>(kernel);
  std::lock_guard<std::mutex> g(mu);
  size_t& have = done[{p->device, k}];
  if (have >= bytes) return;
  if (hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, int(bytes)) != hipSuccess)
    (void)hipGetLastError();
  have = bytes;
}

// call f(std::integral_constant<int, v>) for LO <= v <= HI
template <int LO, int HI, typename F>
inline int with_log2(int v, F&& f) {
  if constexpr (LO > HI) {
    (void)v;
    return PM_EUNSUPPORTED;
  } else {
    if (v == LO) return f(std::integral_constant<int, LO>{});
    return with_log2<LO + 1, HI>(v, f);
  }
}

// ---------------------------------------------------------------------------
// in-register DFTs of size 2, 4, 8, 16 (forward: exp(-2 pi i r k / R))
// ---------------------------------------------------------------------------
template <bool INV, typename C>
__device__ __forceinline__ void dft2(C& a, C& b) {
  C t = a;
  a = cadd(t, b);
  b = csub(t, b);
}

template <bool INV, typename C>
__device__ __forceinline__ void dft4(C& x0, C& x1, C& x2, C& x3) {
  C t0 = cadd(x0, x2), t1 = csub(x0, x2);
  C t2 = cadd(x1, x3), t3 = cmul_mi<INV>(csub(x1, x3));
  x0 = cadd(t0, t2);
  x2 = csub(t0, t2);
  x1 = cadd(t1, t3);
  x3 = csub(t1, t3);
}

// multiply by exp(-+ 2 pi i k / 16) for the constant k (k < 8)
template <int K, bool INV, typename C>
__device__ __forceinline__ C tw16(C x) {
  using R = typename C::value_type;
  constexpr double c[8] = {1.0, 0.92387953251128673848, 0.70710678118654752440, 0.38268343236508977173,
                           0.0, -0.38268343236508977173, -0.70710678118654752440, -0.92387953251128673848};
  constexpr double s[8] = {0.0, 0.38268343236508977173, 0.70710678118654752440, 0.92387953251128673848,
                           1.0, 0.92387953251128673848, 0.70710678118654752440, 0.38268343236508977173};
  if constexpr (K == 0) {
    return x;
  } else if constexpr (K == 4) {
    return cmul_mi<INV>(x);
  } else {
    const R cr = R(c[K]);
    const R si = INV ? R(s[K]) : R(-s[K]);
    return cmk<C>(x.x * cr - x.y * si, x.x * si + x.y * cr);
  }
}

template <bool INV, typename C>
__device__ __forceinline__ void dft8(C* v) {
  C e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
  C o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
  dft4<INV>(e0, e1, e2, e3);
  dft4<INV>(o0, o1, o2, o3);
  o1 = tw16<2, INV>(o1);
  o2 = tw16<4, INV>(o2);
  o3 = tw16<6, INV>(o3);
  v[0] = cadd(e0, o0); v[4] = csub(e0, o0);
  v[1] = cadd(e1, o1); v[5] = csub(e1, o1);
  v[2] = cadd(e2, o2); v[6] = csub(e2, o2);
  v[3] = cadd(e3, o3); v[7] = csub(e3, o3);
}

template <bool INV, typename C>
__device__ __forceinline__ void dft16(C* v) {
  C e[8], o[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) { e[i] = v[2 * i]; o[i] = v[2 * i + 1]; }
  dft8<INV>(e);
  dft8<INV>(o);
  o[1] = tw16<1, INV>(o[1]);
  o[2] = tw16<2, INV>(o[2]);
  o[3] = tw16<3, INV>(o[3]);
  o[4] = tw16<4, INV>(o[4]);
  o[5] = tw16<5, INV>(o[5]);
  o[6] = tw16<6, INV>(o[6]);
  o[7] = tw16<7, INV>(o[7]);
#pragma unroll
  for (int i = 0; i < 8; ++i) { v[i] = cadd(e[i], o[i]); v[i + 8] = csub(e[i], o[i]); }
}

template <int R, bool INV, typename C>
__device__ __forceinline__ void dft(C* v) {
  if constexpr (R == 2) dft2<INV>(v[0], v[1]);
  else if constexpr (R == 4) dft4<INV>(v[0], v[1], v[2], v[3]);
  else if constexpr (R == 8) dft8<INV>(v);
  else dft16<INV>(v);
}

// ---------------------------------------------------------------------------
// one Stockham stage of radix 2^LR on W = 2^LOGW lines of length 2^LOGM in
// LDS.  Input sub-transforms have length Ns = 2^LOGNS.  Every thread owns
// EPT / R butterflies.  tws holds exp(-2 pi i m / 2^LOGL).
// ---------------------------------------------------------------------------
template <int LR, int EPT, bool INV, int LOGM, int LOGW, int LOGNS, int LOGL, typename C>
__device__ __forceinline__ void fft_stage(C* buf, const C* tws) {
  constexpr int R = 1 << LR;
  constexpr int B = EPT / R;
  constexpr int NBF = (1 << LOGM) >> LR;     // butterflies per line
  constexpr int PITCH = (1 << LOGW) + 1;
  constexpr int TWSH = LOGL - LOGNS - LR;
  const int tid = threadIdx.x;
  C v[B][R];
  int dst[B];
#pragma unroll
  for (int b = 0; b < B; ++b) {
    const int g = tid + b * kFT;
    const int c = g & ((1 << LOGW) - 1);
    const int j = g >> LOGW;
    const int k = j & ((1 << LOGNS) - 1);
    const C* src = buf + j * PITCH + c;
#pragma unroll
    for (int r = 0; r < R; ++r) v[b][r] = src[r * NBF * PITCH];
    if constexpr (LOGNS > 0) {
      const int kt = k << TWSH;
#pragma unroll
      for (int r = 1; r < R; ++r) {
        C w = tws[kt * r];
        if (INV) w.y = -w.y;
        v[b][r] = cmul(v[b][r], w);
      }
    }
    dst[b] = (((j - k) << LR) + k) * PITCH + c;
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < B; ++b) {
    dft<R, INV>(v[b]);
#pragma unroll
    for (int r = 0; r < R; ++r) buf[dst[b] + r * ((1 << LOGNS) * PITCH)] = v[b][r];
  }
  __syncthreads();
}

template <int EPT, bool INV, int LOGM, int LOGW, int LOGL, int LOGNS, typename C>
__device__ __forceinline__ void fft_stages(C* buf, const C* tws) {
  if constexpr (LOGNS < LOGM) {
    constexpr int LRMAX = EPT >= 16 ? 4 : 3;
    constexpr int left = (LOGM - LOGNS + LRMAX - 1) / LRMAX;   // stages still to do
    constexpr int bits = (LOGM - LOGNS + left - 1) / left;
    fft_stage<bits, EPT, INV, LOGM, LOGW, LOGNS, LOGL>(buf, tws);
    fft_stages<EPT, INV, LOGM, LOGW, LOGL, LOGNS + bits>(buf, tws);
  }
}

// full transform of all W lines held in LDS (starts with a barrier so that
// the caller's LDS writes are visible; ends with one)
template <int EPT, bool INV, int LOGM, int LOGW, int LOGL, typename C>
__device__ __forceinline__ void fft_lds(C* buf, const C* tws) {
  __syncthreads();
  fft_stages<EPT, INV, LOGM, LOGW, LOGL, 0>(buf, tws);
}

// ---------------------------------------------------------------------------
// Transforms whose first stage starts from registers and whose last stage
// ends in registers.  With S stages, stage s of radix 2^bits(s) (larger
// radices first; REV reverses the order) takes thread t's butterflies
// b < EPT / R at g = t + b kFT: column c = g mod W, butterfly j = g / W, rows
// j + r M/R (r < R) in and, for the last stage, rows j + r M/R out (output
// index = frequency).  So a load into the first stage's registers and a store
// from the last stage's are row runs of W adjacent columns, and the last
// stage of a transform hands its registers straight to the first stage of a
// transform whose first radix equals that last radix (REV).  Only the S - 1
// exchanges between stages go through LDS.
// ---------------------------------------------------------------------------
template <int LOGM, int LRMAX, bool REV>
struct RegPlan {
  static constexpr int S = (LOGM + LRMAX - 1) / LRMAX;
  static constexpr int fwd_bits(int s) {
    int done = 0;
    for (int i = 0;; ++i) {
      const int left = S - i;
      const int b = (LOGM - done + left - 1) / left;
      if (i == s) return b;
      done += b;
    }
  }
  static constexpr int bits(int s) { return REV ? fwd_bits(S - 1 - s) : fwd_bits(s); }
  static constexpr int ns_log2(int s) {   // log2 of the sub-transform length entering stage s
    int n = 0;
    for (int i = 0; i < s; ++i) n += bits(i);
    return n;
  }
};

template <typename C, int EPT, int LOGM, int LRMAX, bool REV, bool LAST>
struct RegStage {
  using P = RegPlan<LOGM, LRMAX, REV>;
  static constexpr int LR = P::bits(LAST ? P::S - 1 : 0);
  static constexpr int R = 1 << LR;
  static constexpr int B = EPT / R;
};

// rows of the thread's registers for the first (or last) stage: v[b][r] is
// element (row_of(b, r), col_of(b)) of the tile
template <int LR, int LOGM, int LOGW>
__device__ __forceinline__ int reg_col(int tid, int b) {
  return (tid + b * kFT) & ((1 << LOGW) - 1);
}
template <int LR, int LOGM, int LOGW>
__device__ __forceinline__ int reg_row(int tid, int b, int r) {
  return ((tid + b * kFT) >> LOGW) + (r << (LOGM - LR));
}

// first stage from registers: DFT of each butterfly, results to LDS in the
// Stockham order of the next stage (the caller makes sure no thread still
// reads buf).  Ends with a barrier.  With a single stage nothing is written.
template <int EPT, bool INV, int LOGM, int LOGW, int LRMAX, bool REV, typename C, int B, int R>
__device__ __forceinline__ void reg_first_stage(C (&v)[B][R], C* buf) {
  using P = RegPlan<LOGM, LRMAX, REV>;
  constexpr int LR = P::bits(0);
  static_assert((1 << LR) == R && B * R == EPT, "register shape");
  constexpr int PITCH = (1 << LOGW) + 1;
#pragma unroll
  for (int b = 0; b < B; ++b) dft<R, INV>(v[b]);
  if constexpr (P::S > 1) {
    const int tid = threadIdx.x;
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const int g = tid + b * kFT;
      const int c = g & ((1 << LOGW) - 1), j = g >> LOGW;
#pragma unroll
      for (int r = 0; r < R; ++r) buf[((j << LR) + r) * PITCH + c] = v[b][r];
    }
    __syncthreads();
  }
}

// stages 1 .. S-2 through LDS (each ends with a barrier)
template <int EPT, bool INV, int LOGM, int LOGW, int LOGL, int LRMAX, bool REV, int s, typename C>
__device__ __forceinline__ void reg_middle_stages(C* buf, const C* tws) {
  using P = RegPlan<LOGM, LRMAX, REV>;
  if constexpr (s < P::S - 1) {
    fft_stage<P::bits(s), EPT, INV, LOGM, LOGW, P::ns_log2(s), LOGL>(buf, tws);
    reg_middle_stages<EPT, INV, LOGM, LOGW, LOGL, LRMAX, REV, s + 1>(buf, tws);
  }
}

// last stage into registers: v[b][r] = output row reg_row(b, r) of column
// reg_col(b).  Reads buf (no barrier at the end: the caller adds one before
// buf is written again).  With a single stage v already holds the result.
template <int EPT, bool INV, int LOGM, int LOGW, int LOGL, int LRMAX, bool REV, typename C, int B, int R>
__device__ __forceinline__ void reg_last_stage(const C* buf, const C* tws, C (&v)[B][R]) {
  using P = RegPlan<LOGM, LRMAX, REV>;
  if constexpr (P::S > 1) {
    constexpr int LR = P::bits(P::S - 1);
    static_assert((1 << LR) == R && B * R == EPT, "register shape");
    constexpr int PITCH = (1 << LOGW) + 1;
    constexpr int NBF = (1 << LOGM) >> LR;           // = the sub-transform length Ns here
    constexpr int TWSH = LOGL - LOGM;
    const int tid = threadIdx.x;
#pragma unroll
    for (int b = 0; b < B; ++b) {
      const int g = tid + b * kFT;
      const int c = g & ((1 << LOGW) - 1), j = g >> LOGW;
      const C* src = buf + j * PITCH + c;
#pragma unroll
      for (int r = 0; r < R; ++r) v[b][r] = src[r * NBF * PITCH];
      const int kt = j << TWSH;
#pragma unroll
      for (int r = 1; r < R; ++r) {
        C w = tws[kt * r];
        if (INV) w.y = -w.y;
        v[b][r] = cmul(v[b][r], w);
      }
      dft<R, INV>(v[b]);
    }
  }
}

// copy exp(-2 pi i m / 2^LOGL), m < 2^LOGL, from the 4096-entry table to LDS
template <int LOGL, typename C>
__device__ __forceinline__ void load_twiddles(C* tws, const C* __restrict__ tw) {
  for (int m = threadIdx.x; m < (1 << LOGL); m += kFT) tws[m] = tw[m << (kTwiddleLog2 - LOGL)];
}

// ---------------------------------------------------------------------------
// launchers (defined in fft_lines.hip, fft_z.hip, fft_fused.hip)
// ---------------------------------------------------------------------------
// strided complex pass over `batch` arrays: lines of length M (stride ls),
// W-wide tiles of adjacent columns out of ncols, repeated over nouter blocks
// of stride ostride.  Array `dual` (>= 0) is transformed twice: as it is into
// dual_out (same layout), and times the line's wavenumber in place.
template <typename T>
int lines_pass(Plan* p, const Ptrs4& arrs, int batch, bool inv, int M, int64_t ls, int64_t ncols,
               int64_t ostride, int64_t nouter, hipStream_t st, int dual = -1, void* dual_out = nullptr);
// z passes between real lines of n2 and half-spectrum lines of n2/2 + 1
template <typename T>
int r2c_z_pass(Plan* p, const FftShape& s, const Ptrs4& in, const Ptrs4& out, int batch, const ZFold* zf,
               hipStream_t st);
// kz_arr (>= 0): that array's spectrum is first multiplied by kz = 2 pi k / n2
// (zero on the Nyquist bin)
template <typename T>
int c2r_z_pass(Plan* p, const FftShape& s, const Ptrs4& in, const Ptrs4& out, int batch, T scale,
               hipStream_t st, int kz_arr = -1);
// fused forward x pass, spectral multipliers and inverse x passes
template <typename T>
int x_fused_pass(Plan* p, const FftShape& s, SpecOp op, const Ptrs4& in, const Ptrs4& out, T coef,
                 hipStream_t st);

}  // namespace fftk
}  // namespace pmx
