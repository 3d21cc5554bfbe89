// 3-D real FFTs for the particle-mesh force (Sec. 2.2 of the paper: one
// forward and three inverse transforms per force evaluation).
//
// Design (gfx950): every 1-D transform of length M <= 1024 is done by one
// workgroup inside LDS.  A workgroup holds a tile of W = 256*EPT/M lines;
// lines are stored point-major (element j of line c at j*(W+1) + c), so
// consecutive lanes touch consecutive LDS addresses in every Stockham stage.
// Stages use radix 16, then 8/4/2 for the remaining bits; the twiddles come
// from a table of exp(-2 pi i m / 4096) computed in double precision on the
// host.  The three axes are three passes over HBM:
//   z: real lines -> half-length complex FFT + split into N/2+1 bins,
//   y: strided columns (W adjacent kz per tile),
//   x: strided columns over the flattened (y, kz) plane (no ragged tiles).
// The first inverse pass along x can apply the Poisson-gradient multipliers
// on the fly (SpecOp), so the gradient spectra are never materialised.
#include "pm_internal.h"

namespace pmx {

namespace {

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

template <int R> constexpr int log2c() { return R == 2 ? 1 : R == 4 ? 2 : R == 8 ? 3 : 4; }

// ---------------------------------------------------------------------------
// one Stockham stage of radix R on W lines of length M = 2^logM in LDS.
// Input sub-transforms have length Ns = 2^logNs.  Every thread owns EPT/R
// butterflies; lines are indexed fastest across lanes (point-major layout).
// ---------------------------------------------------------------------------
template <int R, int EPT, bool INV, typename C>
__device__ __forceinline__ void fft_stage(C* buf, int logM, int logNs, int logW, int pitch,
                                          const C* __restrict__ tw) {
  constexpr int B = EPT / R;
  constexpr int LR = log2c<R>();
  const int tid = threadIdx.x;
  const int nbf = (1 << logM) >> LR;
  const int wmask = (1 << logW) - 1;
  const int nsmask = (1 << logNs) - 1;
  const int twsh = kTwiddleLog2 - logNs - LR;
  C v[B][R];
  int jj[B], cc[B];
#pragma unroll
  for (int b = 0; b < B; ++b) {
    const int g = tid + b * kThreads;
    const int c = g & wmask;
    const int j = g >> logW;
    const int k = j & nsmask;
    jj[b] = j;
    cc[b] = c;
#pragma unroll
    for (int r = 0; r < R; ++r) {
      C x = buf[(j + r * nbf) * pitch + c];
      if (r > 0) {
        C w = tw[(k * r) << twsh];
        if (INV) w.y = -w.y;
        x = cmul(x, w);
      }
      v[b][r] = x;
    }
  }
  __syncthreads();
#pragma unroll
  for (int b = 0; b < B; ++b) {
    dft<R, INV>(v[b]);
    const int j = jj[b];
    const int k = j & nsmask;
    const int d = ((j - k) << LR) + k;
#pragma unroll
    for (int r = 0; r < R; ++r) buf[(d + (r << logNs)) * pitch + cc[b]] = v[b][r];
  }
  __syncthreads();
}

// full transform of all W lines held in LDS (starts with a barrier so that
// the caller's LDS writes are visible; ends with one).
template <int EPT, bool INV, typename C>
__device__ __forceinline__ void fft_lds(C* buf, int logM, int logW, int pitch, const C* __restrict__ tw) {
  __syncthreads();
  int logNs = 0;
  while (logM - logNs >= 4) {
    fft_stage<16, EPT, INV>(buf, logM, logNs, logW, pitch, tw);
    logNs += 4;
  }
  switch (logM - logNs) {
    case 3: fft_stage<8, EPT, INV>(buf, logM, logNs, logW, pitch, tw); break;
    case 2: fft_stage<4, EPT, INV>(buf, logM, logNs, logW, pitch, tw); break;
    case 1: fft_stage<2, EPT, INV>(buf, logM, logNs, logW, pitch, tw); break;
    default: break;
  }
}

// elements per thread: the tile of a workgroup is 256 * EPT complex values
template <typename T> struct FftCfg;
template <> struct FftCfg<float> { static constexpr int EPT = 32, EPT_FUSED = 16; };
template <> struct FftCfg<double> { static constexpr int EPT = 16, EPT_FUSED = 16; };

template <typename T, int EPT> constexpr int lds_elems() { return kThreads * EPT + 1024; }

// ---------------------------------------------------------------------------
// strided complex pass: lines of length M with element stride ls; tiles of W
// adjacent columns (stride 1) out of ncols, repeated over nouter blocks of
// stride ostride and over batch (stride bstride).
// ---------------------------------------------------------------------------
template <typename T, bool INV>
__global__ __launch_bounds__(kThreads) void k_fft_lines(cplx<T>* __restrict__ data, int logM, int64_t ls,
                                                        int64_t ncols, int64_t ostride, int64_t nouter,
                                                        int64_t bstride, const cplx<T>* __restrict__ tw) {
  using C = cplx<T>;
  constexpr int EPT = FftCfg<T>::EPT;
  __shared__ C lds[lds_elems<T, EPT>()];
  const int logW = ilog2c(kThreads * EPT) - logM;
  const int W = 1 << logW;
  const int pitch = W + 1;
  const int64_t ncb = (ncols + W - 1) >> logW;
  const int64_t tile = xcd_tile(blockIdx.x, int64_t(gridDim.x));
  const int64_t o = tile / ncb;
  const int64_t c0 = (tile - o * ncb) << logW;
  C* base = data + int64_t(blockIdx.y) * bstride + o * ostride + c0;
  const int tid = threadIdx.x;
  const int wmask = W - 1;
  {
    // all loads in flight before the first LDS store
    C v[EPT];
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int f = tid + i * kThreads;
      const int c = f & wmask, j = f >> logW;
      v[i] = (c0 + c < ncols) ? base[j * ls + c] : cmk<C>(0, 0);
    }
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int f = tid + i * kThreads;
      lds[(f >> logW) * pitch + (f & wmask)] = v[i];
    }
  }
  fft_lds<EPT, INV>(lds, logM, logW, pitch, tw);
#pragma unroll 4
  for (int i = 0; i < EPT; ++i) {
    const int f = tid + i * kThreads;
    const int c = f & wmask, j = f >> logW;
    if (c0 + c < ncols) base[j * ls + c] = lds[j * pitch + c];
  }
}

// ---------------------------------------------------------------------------
// z pass, real -> complex.  Lines of N = 2M reals, output lines of M+1 bins.
// z[n] = x[2n] + i x[2n+1];  Z = FFT_M(z);  with Zc = conj(Z[M-k]):
//   X[k] = (Z + Zc)/2 - i exp(-2 pi i k/N) (Z - Zc)/2,   k = 0..M.
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kThreads) void k_fft_r2c_z(const T* __restrict__ in, cplx<T>* __restrict__ out,
                                                        int logM, int64_t nlines, int64_t in_bstride,
                                                        int64_t out_bstride, const cplx<T>* __restrict__ tw) {
  using C = cplx<T>;
  constexpr int EPT = FftCfg<T>::EPT;
  __shared__ C lds[lds_elems<T, EPT>()];
  const int M = 1 << logM;
  const int logW = ilog2c(kThreads * EPT) - logM;
  const int W = 1 << logW;
  const int pitch = W + 1;
  const int64_t l0 = xcd_tile(blockIdx.x, int64_t(gridDim.x)) << logW;
  const C* src = reinterpret_cast<const C*>(in + int64_t(blockIdx.y) * in_bstride) + l0 * M;
  C* dst = out + int64_t(blockIdx.y) * out_bstride + l0 * (M + 1);
  const int64_t lines_here = nlines - l0 < W ? nlines - l0 : W;
  const int tid = threadIdx.x;
  {
    C v[EPT];
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int f = tid + i * kThreads;
      v[i] = ((f >> logM) < lines_here) ? src[f] : cmk<C>(0, 0);
    }
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int f = tid + i * kThreads;
      lds[(f & (M - 1)) * pitch + (f >> logM)] = v[i];
    }
  }
  fft_lds<EPT, false>(lds, logM, logW, pitch, tw);
  const int total = int(lines_here) * (M + 1);
  const int twsh = kTwiddleLog2 - (logM + 1);
  using R = typename C::value_type;
  for (int f = tid; f < total; f += kThreads) {
    const int l = f / (M + 1);
    const int k = f - l * (M + 1);
    const C z = lds[(k & (M - 1)) * pitch + l];
    const C zc = cconj(lds[((M - k) & (M - 1)) * pitch + l]);
    const C e = cscale(cadd(z, zc), R(0.5));
    const C d = cscale(csub(z, zc), R(0.5));
    // o = -i d ; X = e + w o
    const C o = cmk<C>(d.y, -d.x);
    const C w = tw[k << twsh];
    dst[f] = cadd(e, cmul(w, o));
  }
}

// ---------------------------------------------------------------------------
// z pass, complex -> real.  From X[0..M] (imaginary parts of X[0] and X[M]
// ignored):  E = (X[k] + conj X[M-k])/2,  O = (X[k] - conj X[M-k]) conj(w^k)/2,
// Z = E + i O,  z = IFFT_M(Z) (unnormalised),  x[2n] + i x[2n+1] = scale z[n].
// ---------------------------------------------------------------------------
template <typename T>
__global__ __launch_bounds__(kThreads) void k_fft_c2r_z(const cplx<T>* __restrict__ in, T* __restrict__ out,
                                                        int logM, int64_t nlines, int64_t in_bstride,
                                                        int64_t out_bstride, T scale,
                                                        const cplx<T>* __restrict__ tw) {
  using C = cplx<T>;
  using R = T;
  constexpr int EPT = FftCfg<T>::EPT;
  __shared__ C lds[lds_elems<T, EPT>()];
  const int M = 1 << logM;
  const int logW = ilog2c(kThreads * EPT) - logM;
  const int W = 1 << logW;
  const int pitch = W + 1;
  const int64_t l0 = xcd_tile(blockIdx.x, int64_t(gridDim.x)) << logW;
  const C* src = in + int64_t(blockIdx.y) * in_bstride + l0 * (M + 1);
  C* dst = reinterpret_cast<C*>(out + int64_t(blockIdx.y) * out_bstride) + l0 * M;
  const int64_t lines_here = nlines - l0 < W ? nlines - l0 : W;
  const int tid = threadIdx.x;
  const int twsh = kTwiddleLog2 - (logM + 1);
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int f = tid + i * kThreads;
    const int l = f >> logM, k = f & (M - 1);
    C z = cmk<C>(0, 0);
    if (l < lines_here) {
      const C* line = src + int64_t(l) * (M + 1);
      C a = line[k];
      C b = line[M - k];
      if (k == 0) { a.y = 0; b.y = 0; }
      const C bc = cconj(b);
      const C e = cscale(cadd(a, bc), R(0.5));
      C w = tw[k << twsh];
      w.y = -w.y;  // conj(w^k)
      const C o = cmul(cscale(csub(a, bc), R(0.5)), w);
      z = cmk<C>(e.x - o.y, e.y + o.x);  // e + i o
    }
    lds[k * pitch + l] = z;
  }
  fft_lds<EPT, true>(lds, logM, logW, pitch, tw);
#pragma unroll 4
  for (int i = 0; i < EPT; ++i) {
    const int f = tid + i * kThreads;
    const int l = f >> logM, n = f & (M - 1);
    if (l < lines_here) dst[f] = cscale(lds[n * pitch + l], scale);
  }
}

// ---------------------------------------------------------------------------
// first inverse pass along x with the Poisson-gradient multipliers fused.
// The tile columns run over the flattened (y, kz) plane of the spectrum.
// T_j = i k_j coef / k^2, zero at k = 0 and on the Nyquist plane of j.
// GRAD3:  out_j = FFT_x^-1( T_j in_0 ),  j = 0..2
// ADJ4:   out_3 = FFT_x^-1( -sum_j T_j in_{1+j} ), then out_j as GRAD3.
// Every tile reads all of its inputs before writing, so outputs may alias
// inputs that the same tile has already consumed (see fft_c2r_fused).
// ---------------------------------------------------------------------------
struct Ptrs4 {
  void* p[4];
};

template <typename T, int OP>
__global__ __launch_bounds__(kThreads) void k_fft_x_fused(Ptrs4 ins, Ptrs4 outs, int logM, int n1,
                                                          int n2, int nh, T coef,
                                                          const cplx<T>* __restrict__ tw) {
  using C = cplx<T>;
  constexpr int EPT = FftCfg<T>::EPT_FUSED;
  __shared__ C lds[lds_elems<T, EPT>()];
  const int M = 1 << logM;  // = n0
  const int logW = ilog2c(kThreads * EPT) - logM;
  const int W = 1 << logW;
  const int pitch = W + 1;
  const int64_t ncols = int64_t(n1) * nh;
  const int64_t ls = ncols;
  const int64_t c0 = xcd_tile(blockIdx.x, int64_t(gridDim.x)) << logW;
  const int tid = threadIdx.x;
  const int wmask = W - 1;
  // all elements of a thread share one column when W <= kThreads
  const T two_pi = T(6.283185307179586476925286766559);
  auto kvec = [&](int j, int64_t col, T& kx, T& ky, T& kz, bool& nx, bool& ny, bool& nz) {
    const int y = int(col / nh);
    const int z = int(col - int64_t(y) * nh);
    const int fx = j < (M >> 1) ? j : j - M;
    const int fy = y < (n1 >> 1) ? y : y - n1;
    kx = two_pi * T(fx) / T(M);
    ky = two_pi * T(fy) / T(n1);
    kz = two_pi * T(z) / T(n2);
    nx = (2 * j == M);
    ny = (2 * y == n1);
    nz = (2 * z == n2);
  };
  C reg[EPT];
  const C* in0 = static_cast<const C*>(ins.p[0]);
  if (OP == SPEC_ADJ4) {
    const C* in1 = static_cast<const C*>(ins.p[1]);
    const C* in2 = static_cast<const C*>(ins.p[2]);
    const C* in3 = static_cast<const C*>(ins.p[3]);
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int f = tid + i * kThreads;
      const int c = f & wmask, j = f >> logW;
      const int64_t col = c0 + c;
      C acc = cmk<C>(0, 0);
      if (col < ncols) {
        T kx, ky, kz; bool nx, ny, nz;
        kvec(j, col, kx, ky, kz, nx, ny, nz);
        const T k2 = kx * kx + ky * ky + kz * kz;
        const T g = k2 > T(0) ? coef / k2 : T(0);
        const int64_t idx = int64_t(j) * ls + col;
        const C a = in1[idx], b = in2[idx], d = in3[idx];
        // s = sum_j k_j in_{1+j} (Nyquist of j removed); -i * s * g
        const T fx = nx ? T(0) : kx, fy = ny ? T(0) : ky, fz = nz ? T(0) : kz;
        const C s = cmk<C>(fx * a.x + fy * b.x + fz * d.x, fx * a.y + fy * b.y + fz * d.y);
        acc = cmk<C>(s.y * g, -s.x * g);
      }
      lds[j * pitch + c] = acc;
    }
    fft_lds<EPT, true>(lds, logM, logW, pitch, tw);
    C* o3 = static_cast<C*>(outs.p[3]);
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int f = tid + i * kThreads;
      const int c = f & wmask, j = f >> logW;
      if (c0 + c < ncols) o3[int64_t(j) * ls + c0 + c] = lds[j * pitch + c];
    }
  }
#pragma unroll
  for (int i = 0; i < EPT; ++i) {
    const int f = tid + i * kThreads;
    const int c = f & wmask, j = f >> logW;
    reg[i] = (c0 + c < ncols) ? in0[int64_t(j) * ls + c0 + c] : cmk<C>(0, 0);
  }
  for (int comp = 0; comp < 3; ++comp) {
    if (comp > 0 || OP == SPEC_ADJ4) __syncthreads();  // previous tile store done reading LDS
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int f = tid + i * kThreads;
      const int c = f & wmask, j = f >> logW;
      const int64_t col = c0 + c;
      C v = cmk<C>(0, 0);
      if (col < ncols) {
        T kx, ky, kz; bool nx, ny, nz;
        kvec(j, col, kx, ky, kz, nx, ny, nz);
        const T k2 = kx * kx + ky * ky + kz * kz;
        T kj = comp == 0 ? (nx ? T(0) : kx) : comp == 1 ? (ny ? T(0) : ky) : (nz ? T(0) : kz);
        const T g = k2 > T(0) ? kj * coef / k2 : T(0);
        // i * g * in
        v = cmk<C>(-reg[i].y * g, reg[i].x * g);
      }
      lds[j * pitch + c] = v;
    }
    fft_lds<EPT, true>(lds, logM, logW, pitch, tw);
    C* o = static_cast<C*>(outs.p[comp]);
#pragma unroll
    for (int i = 0; i < EPT; ++i) {
      const int f = tid + i * kThreads;
      const int c = f & wmask, j = f >> logW;
      if (c0 + c < ncols) o[int64_t(j) * ls + c0 + c] = lds[j * pitch + c];
    }
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

template <typename T>
int lines_pass(Plan* p, cplx<T>* data, bool inv, int M, int64_t ls, int64_t ncols, int64_t ostride,
               int64_t nouter, int batch, int64_t bstride, hipStream_t st) {
  constexpr int EPT = FftCfg<T>::EPT;
  const int logM = ilog2(M);
  const int logW = ilog2(kThreads * EPT) - logM;
  const int64_t ncb = (ncols + (int64_t(1) << logW) - 1) >> logW;
  dim3 grid(unsigned(ncb * nouter), unsigned(batch));
  const cplx<T>* tw = static_cast<const cplx<T>*>(p->tw);
  timing_begin(p, PM_K_FFT_LINES, st);
  if (inv)
    hipLaunchKernelGGL((k_fft_lines<T, true>), grid, dim3(kThreads), 0, st, data, logM, ls, ncols, ostride,
                       nouter, bstride, tw);
  else
    hipLaunchKernelGGL((k_fft_lines<T, false>), grid, dim3(kThreads), 0, st, data, logM, ls, ncols, ostride,
                       nouter, bstride, tw);
  timing_end(p, PM_K_FFT_LINES, st, 2.0 * double(batch) * double(ncols) * double(nouter) * M * sizeof(cplx<T>));
  PM_HIP_CHECK(p, hipGetLastError());
  return PM_OK;
}

}  // namespace

template <typename T>
int fft_r2c_3d(Plan* p, const FftShape& s, const T* in, cplx<T>* out, int batch, int64_t in_stride,
               int64_t out_stride, hipStream_t st) {
  constexpr int EPT = FftCfg<T>::EPT;
  const int nh = s.n2 / 2 + 1;
  const int logM = ilog2(s.n2 / 2);
  const int logW = ilog2(kThreads * EPT) - logM;
  const int64_t nlines = int64_t(s.n0) * s.n1;
  const int64_t ntiles = (nlines + (int64_t(1) << logW) - 1) >> logW;
  timing_begin(p, PM_K_FFT_R2C_Z, st);
  hipLaunchKernelGGL((k_fft_r2c_z<T>), dim3(unsigned(ntiles), unsigned(batch)), dim3(kThreads), 0, st, in, out,
                     logM, nlines, in_stride, out_stride, static_cast<const cplx<T>*>(p->tw));
  timing_end(p, PM_K_FFT_R2C_Z, st,
             double(batch) * double(nlines) * (double(s.n2) * sizeof(T) + double(nh) * sizeof(cplx<T>)));
  PM_HIP_CHECK(p, hipGetLastError());
  // y: lines of n1 with stride nh, columns kz (nh), outer x (stride n1*nh)
  int rc = lines_pass<T>(p, out, false, s.n1, nh, nh, int64_t(s.n1) * nh, s.n0, batch, out_stride, st);
  if (rc) return rc;
  // x: lines of n0 with stride n1*nh over the flattened (y, kz) plane
  return lines_pass<T>(p, out, false, s.n0, int64_t(s.n1) * nh, int64_t(s.n1) * nh, 0, 1, batch, out_stride, st);
}

template <typename T>
static int c2r_tail(Plan* p, const FftShape& s, cplx<T>* in, T* out, int batch, int64_t in_stride,
                    int64_t out_stride, T scale, hipStream_t st) {
  constexpr int EPT = FftCfg<T>::EPT;
  const int nh = s.n2 / 2 + 1;
  int rc = lines_pass<T>(p, in, true, s.n1, nh, nh, int64_t(s.n1) * nh, s.n0, batch, in_stride, st);
  if (rc) return rc;
  const int logM = ilog2(s.n2 / 2);
  const int logW = ilog2(kThreads * EPT) - logM;
  const int64_t nlines = int64_t(s.n0) * s.n1;
  const int64_t ntiles = (nlines + (int64_t(1) << logW) - 1) >> logW;
  timing_begin(p, PM_K_FFT_C2R_Z, st);
  hipLaunchKernelGGL((k_fft_c2r_z<T>), dim3(unsigned(ntiles), unsigned(batch)), dim3(kThreads), 0, st, in, out,
                     logM, nlines, in_stride, out_stride, scale, static_cast<const cplx<T>*>(p->tw));
  timing_end(p, PM_K_FFT_C2R_Z, st,
             double(batch) * double(nlines) * (double(s.n2) * sizeof(T) + double(nh) * sizeof(cplx<T>)));
  PM_HIP_CHECK(p, hipGetLastError());
  return PM_OK;
}

template <typename T>
int fft_c2r_3d(Plan* p, const FftShape& s, cplx<T>* in, T* out, int batch, int64_t in_stride,
               int64_t out_stride, T scale, hipStream_t st) {
  const int nh = s.n2 / 2 + 1;
  int rc = lines_pass<T>(p, in, true, s.n0, int64_t(s.n1) * nh, int64_t(s.n1) * nh, 0, 1, batch, in_stride, st);
  if (rc) return rc;
  return c2r_tail<T>(p, s, in, out, batch, in_stride, out_stride, scale, st);
}

template <typename T>
int fft_c2r_fused(Plan* p, const FftShape& s, SpecOp op, cplx<T>* const* specs, T* const* outs, T coef,
                  hipStream_t st) {
  constexpr int EPT = FftCfg<T>::EPT_FUSED;
  const int nh = s.n2 / 2 + 1;
  const int logM = ilog2(s.n0);
  const int logW = ilog2(kThreads * EPT) - logM;
  const int64_t ncols = int64_t(s.n1) * nh;
  const int64_t ntiles = (ncols + (int64_t(1) << logW) - 1) >> logW;
  Ptrs4 in{}, o{};
  int nout = 3;
  if (op == SPEC_GRAD3) {
    // specs[0] holds delta(k); results go to specs[0..2]
    in.p[0] = specs[0];
    o.p[0] = specs[0]; o.p[1] = specs[1]; o.p[2] = specs[2];
  } else {
    // specs[0] = rho(k), specs[1..3] = gbar_j(k); outputs g_0..2 and rhobar.
    // Tile-local order: out_3 is written after in_1..3 are read, so it may use
    // specs[1]; g_0 -> specs[0] (read first), g_1 -> specs[2], g_2 -> specs[3].
    for (int i = 0; i < 4; ++i) in.p[i] = specs[i];
    o.p[3] = specs[1]; o.p[0] = specs[0]; o.p[1] = specs[2]; o.p[2] = specs[3];
    nout = 4;
  }
  const cplx<T>* tw = static_cast<const cplx<T>*>(p->tw);
  timing_begin(p, PM_K_FFT_POISSON, st);
  if (op == SPEC_GRAD3)
    hipLaunchKernelGGL((k_fft_x_fused<T, SPEC_GRAD3>), dim3(unsigned(ntiles)), dim3(kThreads), 0, st, in, o, logM,
                       s.n1, s.n2, nh, coef, tw);
  else
    hipLaunchKernelGGL((k_fft_x_fused<T, SPEC_ADJ4>), dim3(unsigned(ntiles)), dim3(kThreads), 0, st, in, o, logM,
                       s.n1, s.n2, nh, coef, tw);
  timing_end(p, PM_K_FFT_POISSON, st,
             double(op == SPEC_GRAD3 ? 4 : 8) * double(ncols) * double(s.n0) * sizeof(cplx<T>));
  PM_HIP_CHECK(p, hipGetLastError());
  // remaining passes on each output spectrum (the spectra are p->spec-style
  // equal-stride blocks only by convention, so run them one at a time)
  const int64_t nspec = int64_t(s.n0) * s.n1 * nh;
  const int64_t ncell = int64_t(s.n0) * s.n1 * s.n2;
  const T scale = T(2.0) / T(ncell);
  for (int j = 0; j < nout; ++j) {
    cplx<T>* sp = static_cast<cplx<T>*>(o.p[j]);
    int rc = c2r_tail<T>(p, s, sp, outs[j], 1, nspec, ncell, scale, st);
    if (rc) return rc;
  }
  return PM_OK;
}

template <typename T>
int poisson_grad_spec(Plan* p, const FftShape& s, const cplx<T>* in, cplx<T>* out, T coef, hipStream_t st) {
  const int nh = s.n2 / 2 + 1;
  const int64_t nspec = int64_t(s.n0) * s.n1 * nh;
  const unsigned blocks = unsigned((nspec + kThreads - 1) / kThreads);
  hipLaunchKernelGGL((k_poisson_grad<T>), dim3(blocks), dim3(kThreads), 0, st, in, out, s.n0, s.n1, s.n2, nh, nspec,
                     coef);
  PM_HIP_CHECK(p, hipGetLastError());
  return PM_OK;
}

template int fft_r2c_3d<float>(Plan*, const FftShape&, const float*, Cx<float>*, int, int64_t, int64_t, hipStream_t);
template int fft_r2c_3d<double>(Plan*, const FftShape&, const double*, Cx<double>*, int, int64_t, int64_t, hipStream_t);
template int fft_c2r_3d<float>(Plan*, const FftShape&, Cx<float>*, float*, int, int64_t, int64_t, float, hipStream_t);
template int fft_c2r_3d<double>(Plan*, const FftShape&, Cx<double>*, double*, int, int64_t, int64_t, double,
                                hipStream_t);
template int fft_c2r_fused<float>(Plan*, const FftShape&, SpecOp, Cx<float>* const*, float* const*, float, hipStream_t);
template int fft_c2r_fused<double>(Plan*, const FftShape&, SpecOp, Cx<double>* const*, double* const*, double,
                                   hipStream_t);
template int poisson_grad_spec<float>(Plan*, const FftShape&, const Cx<float>*, Cx<float>*, float, hipStream_t);
template int poisson_grad_spec<double>(Plan*, const FftShape&, const Cx<double>*, Cx<double>*, double, hipStream_t);

}  // namespace pmx
