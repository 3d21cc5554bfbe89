// CIC paint (Sec. 2.2, eq. cic) with the optional fused drift of the KDK step
// (Sec. 2.3, eq. KDFK) or of the adjoint step (Sec. 3.6, eq. KDFKO_adj).
//
// Floating-point atomics to HBM are resolved far from the compute units on
// this multi-die GPU, so the paint never issues them on the mesh.  Instead
// particles are binned by the mesh tile that owns their base node, and each
// tile is accumulated in LDS by one workgroup:
//   bin:      drift (optional), base node, tile id; per-tile counts with one
//             atomic per distinct tile per wavefront; (tile, rank) per particle
//   scan:     exclusive prefix sum of the tile counts
//   scatter:  particle ids into per-tile lists
//   tiles:    one workgroup per tile sums the 8 CIC corners of its particles
//             in an LDS box of (TX+1)(TY+1)(TZ+1) cells, writes the TX*TY*TZ
//             core with plain stores and the upper faces to a halo buffer
//   halo:     every core cell on a lower face adds the halo faces of the
//             (up to 7) lower neighbour tiles
// Tiles are 8 x 8 x 16 cells (z contiguous), smaller when the mesh is.
//
// The LDS sums are 64-bit fixed point: integer LDS atomics are several times
// faster than floating-point ones here, and integer addition is associative,
// so the painted mesh is bitwise identical from run to run.  Each tile picks
// its own binary scale 2^e per channel so that the bound count * max|w| of
// any cell sum stays below 2^H, H = 61 for FP64 meshes and 51 for FP32
// meshes; the quantum 2^-e is far below the mesh type's rounding (about
// 1e-15 and 1e-12 relative for a tile of ~10^3 particles).  With H = 51 every
// contribution is below 2^51 in magnitude, so it is rounded to an integer by
// one FP64 fused multiply-add with 1.5 * 2^52 and read back from the bits,
// instead of a general double-to-int64 conversion.
#include "tiles.h"

namespace pmx {

namespace {

template <typename S, typename T>
struct BinP {
  TileGeo g;
  S* s;
  S* p;
  T* xi;
  T* pi;
  S D;
  unsigned* counts;   // [ntiles]
  uint2* keys;        // [N] (tile, rank)
  double* partials;   // slot 0: xi.p (adjoint drift)
  const S* s_set;     // DRIFT_SET: displacement after the drift
  // KICK: the kick the previous step's gather left pending, applied before
  // the drift: p += a Kp (forward) or p -= a Kp, xi += alpha Kx (adjoint)
  const T* ka;
  const T* kal;
  S Kp;
  T Kx;
  // ka / kal in the tile order of the previous binning, particle-major:
  // particle n's values at 3 (offs[key.x] + key.y) + ax of its previous key
  // (read before it is replaced); else [3][N] at ax N + n (selects k_bin's
  // KICK = 2 over 1)
  bool kick_sorted;
  const unsigned* offs;   // the previous binning's tile offsets
  float4* rec;        // FP32 meshes: per-particle CIC record (see tiles.h)
};

// Each thread takes U particles per round, all loads issued first.  Lanes of
// a wavefront that share a tile form a group; the group leaders then issue
// their count atomics together (one instruction, one round trip), and every
// lane takes its rank from its leader's result.
// KICK: 0 none; 1 a pending kick in lattice order ([3][N]); 2 in the tile
// order of the previous binning (BinP::kick_sorted), looked up through the
// previous keys: those loads go first, then the state's, and the dependent
// ones last, so that their round trips overlap the state's.
// PIPM: pi is particle-major, [N][3] (PaintArgs::pi_pm).
template <typename S, typename T, int MODE, int KICK, bool PIPM = false>
__global__ __launch_bounds__(kThreads) void k_bin(BinP<S, T> a) {
  static_assert(!KICK || MODE != DRIFT_NONE, "a pending kick comes with a drift");
  constexpr bool ADJ = MODE == DRIFT_ADJ || MODE == DRIFT_SET;
  static_assert(!PIPM || ADJ, "a particle-major pi comes with the adjoint drift");
  constexpr int U = 4;
  const TileGeo& g = a.g;
  int64_t start, end;
  chunk_of(g.N, start, end);
  const int lane = threadIdx.x & 63;
  double xp = 0.0;
  double pm[3] = {0.0, 0.0, 0.0};   // max |pi| after the adjoint drift
  auto fold = [](double m, double a) { return (a > m || a != a) ? a : m; };
  for (int64_t base = start; base < end; base += U * kThreads) {
    S sv[U][3], pv[U][3];
    T xv[U][3], piv[U][3], kav[U][KICK != 0 ? 3 : 1], kalv[U][KICK != 0 && ADJ ? 3 : 1];
    bool valid[U];
    int tile[U];
    uint2 kp[U];
    // the kick lookups are issued for every lane, past the end with the
    // chunk's last particle, so that no load sits under a branch (a branch
    // makes the compiler wait for all loads in flight at its join)
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t n = base + threadIdx.x + u * kThreads;
      valid[u] = n < end;
      if (KICK == 2) kp[u] = a.keys[valid[u] ? n : end - 1];
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t n = base + threadIdx.x + u * kThreads;
      if (!valid[u]) continue;
      if (KICK == 1) {
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
          kav[u][ax] = a.ka[ax * g.N + n];
          if (ADJ) kalv[u][ax] = a.kal[ax * g.N + n];
        }
      }
#pragma unroll
      for (int ax = 0; ax < 3; ++ax) {
        sv[u][ax] = (MODE == DRIFT_SET ? a.s_set : a.s)[ax * g.N + n];
        if (MODE != DRIFT_NONE) pv[u][ax] = a.p[ax * g.N + n];
        if (ADJ) {
          xv[u][ax] = a.xi[ax * g.N + n];
          piv[u][ax] = a.pi[PIPM ? 3 * n + ax : ax * g.N + n];
        }
      }
    }
    if constexpr (KICK == 2) {
      // the pending kick of particle n, particle-major at its previous
      // (tile, rank) position
      unsigned ob[U];
#pragma unroll
      for (int u = 0; u < U; ++u) ob[u] = a.offs[kp[u].x];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t kq = int64_t(ob[u]) + kp[u].y;
        const Comp3<T> k3 = reinterpret_cast<const Comp3<T>*>(a.ka)[kq];
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) kav[u][ax] = k3.c[ax];
        if (ADJ) {
          const Comp3<T> l3 = reinterpret_cast<const Comp3<T>*>(a.kal)[kq];
#pragma unroll
          for (int ax = 0; ax < 3; ++ax) kalv[u][ax] = l3.c[ax];
        }
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      tile[u] = 0;
      if (!valid[u]) continue;
      const int64_t n = base + threadIdx.x + u * kThreads;
      if constexpr (KICK != 0) {
        // the same fused multiply-adds as the gather's immediate kicks
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
          pv[u][ax] = fma(ADJ ? -S(kav[u][ax]) : S(kav[u][ax]), a.Kp, pv[u][ax]);
          a.p[ax * g.N + n] = pv[u][ax];
          if (ADJ) {
            xv[u][ax] = fma(kalv[u][ax], a.Kx, xv[u][ax]);
            a.xi[ax * g.N + n] = xv[u][ax];
          }
        }
      }
      if (MODE == DRIFT_FWD) {
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
          sv[u][ax] = fma(pv[u][ax], a.D, sv[u][ax]);
          a.s[ax * g.N + n] = sv[u][ax];
        }
      } else if (MODE == DRIFT_ADJ || MODE == DRIFT_SET) {
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
          xp += double(xv[u][ax]) * double(pv[u][ax]);
          if (MODE == DRIFT_ADJ) sv[u][ax] = fma(-pv[u][ax], a.D, sv[u][ax]);
          a.s[ax * g.N + n] = sv[u][ax];
          const T pn = fma(xv[u][ax], T(a.D), piv[u][ax]);
          a.pi[PIPM ? 3 * n + ax : ax * g.N + n] = pn;
          pm[ax] = fold(pm[ax], fabs(double(pn)));
        }
      }
      double q[3];
      lattice_pos(g, n, q);
      const double x0 = q[0] + double(sv[u][0]), x1 = q[1] + double(sv[u][1]), x2 = q[2] + double(sv[u][2]);
      const double f0 = floor(x0), f1 = floor(x1), f2 = floor(x2);
      const int b0 = int(int64_t(f0) & (g.n0 - 1));
      const int b1 = int(int64_t(f1) & (g.n1 - 1));
      const int b2 = int(int64_t(f2) & (g.n2 - 1));
      tile[u] = ((b0 >> g.ltx) * g.nty + (b1 >> g.lty)) * g.ntz + (b2 >> g.ltz);
      if constexpr (kUseRec<T>)
        a.rec[n] = make_float4(__uint_as_float(pack_cell(b0, b1, b2)), float(x0 - f0), float(x1 - f1),
                               float(x2 - f2));
    }
    int leader[U];
    unsigned within[U], gsize[U], baseidx[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      leader[u] = lane;
      within[u] = 0;
      gsize[u] = 0;
      unsigned long long pending = __ballot(valid[u]);
      while (pending) {
        const int ld = __ffsll(static_cast<long long>(pending)) - 1;
        const int lt = __shfl(tile[u], ld, 64);
        const unsigned long long same = __ballot(valid[u] && tile[u] == lt) & pending;
        if ((same >> lane) & 1ull) {
          leader[u] = ld;
          within[u] = unsigned(__popcll(same & ((1ull << lane) - 1ull)));
        }
        if (lane == ld) gsize[u] = unsigned(__popcll(same));
        pending &= ~same;
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      baseidx[u] = 0;
      if (valid[u] && leader[u] == lane) baseidx[u] = atomicAdd(a.counts + tile[u], gsize[u]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const unsigned b = __shfl(baseidx[u], leader[u], 64);
      const int64_t n = base + threadIdx.x + u * kThreads;
      if (valid[u]) a.keys[n] = make_uint2(unsigned(tile[u]), b + within[u]);
    }
  }
  if (MODE == DRIFT_ADJ || MODE == DRIFT_SET) {
    const double t = block_sum_d(xp);
    if (threadIdx.x == 0) a.partials[blockIdx.x * 4 + 0] = t;
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const double m = block_max_d(pm[ax]);
      if (threadIdx.x == 0) a.partials[blockIdx.x * 4 + 1 + ax] = m;
    }
  }
}

// exclusive scan of counts in blocks of 4 * kThreads: offs = local prefix,
// bsum[block] = block total
__global__ __launch_bounds__(kThreads) void k_scan_local(const unsigned* counts, unsigned* offs, unsigned* bsum,
                                                         int64_t n) {
  __shared__ unsigned sh[kThreads];
  const int64_t b0 = int64_t(blockIdx.x) * 4 * kThreads;
  unsigned v[4];
  unsigned tsum = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t idx = b0 + threadIdx.x * 4 + i;
    v[i] = idx < n ? counts[idx] : 0u;
    tsum += v[i];
  }
  sh[threadIdx.x] = tsum;
  __syncthreads();
  for (int off = 1; off < kThreads; off <<= 1) {
    const unsigned t = threadIdx.x >= off ? sh[threadIdx.x - off] : 0u;
    __syncthreads();
    sh[threadIdx.x] += t;
    __syncthreads();
  }
  unsigned run = sh[threadIdx.x] - tsum;  // exclusive prefix of this thread
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int64_t idx = b0 + threadIdx.x * 4 + i;
    if (idx < n) offs[idx] = run;
    run += v[i];
  }
  if (threadIdx.x == kThreads - 1) bsum[blockIdx.x] = sh[kThreads - 1];
}

// exclusive scan of the block sums (one workgroup, nb <= 4 * kThreads)
__global__ __launch_bounds__(kThreads) void k_scan_blocks(unsigned* bsum, int nb) {
  __shared__ unsigned sh[kThreads];
  unsigned v[4];
  unsigned tsum = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int idx = threadIdx.x * 4 + i;
    v[i] = idx < nb ? bsum[idx] : 0u;
    tsum += v[i];
  }
  sh[threadIdx.x] = tsum;
  __syncthreads();
  for (int off = 1; off < kThreads; off <<= 1) {
    const unsigned t = threadIdx.x >= off ? sh[threadIdx.x - off] : 0u;
    __syncthreads();
    sh[threadIdx.x] += t;
    __syncthreads();
  }
  unsigned run = sh[threadIdx.x] - tsum;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int idx = threadIdx.x * 4 + i;
    if (idx < nb) bsum[idx] = run;
    run += v[i];
  }
}

__global__ __launch_bounds__(kThreads) void k_scan_add(unsigned* offs, const unsigned* bsum, int64_t n,
                                                       unsigned total) {
  const int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x;
  if (i < n) offs[i] += bsum[i / (4 * kThreads)];
  if (i == n) offs[n] = total;
}

__global__ __launch_bounds__(kThreads) void k_scatter(const uint2* keys, const unsigned* offs, unsigned* list,
                                                      int64_t N) {
  constexpr int U = 4;   // keys per thread per round, all loads issued first
  int64_t start, end;
  chunk_of(N, start, end);
  for (int64_t base = start + threadIdx.x; base < end; base += U * kThreads) {
    uint2 k[U];
    unsigned o[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t n = base + u * kThreads;
      k[u] = n < end ? keys[n] : make_uint2(0u, 0u);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) o[u] = base + u * kThreads < end ? offs[k[u].x] : 0u;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t n = base + u * kThreads;
      if (n < end) list[o[u] + k[u].y] = unsigned(n);
    }
  }
}

// out[c] = max over blocks of part[b*4 + 1 + c], c < 3 (NaN if any is NaN):
// the largest |pi| of each channel after the adjoint drift
__global__ __launch_bounds__(kThreads) void k_wmax(const double* part, int nblocks, double* out) {
  auto fold = [](double m, double a) { return (a > m || a != a) ? a : m; };
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    double m = 0.0;
    for (int b = threadIdx.x; b < nblocks; b += kThreads) m = fold(m, part[b * 4 + 1 + c]);
    const double t = block_max_d(m);
    if (threadIdx.x == 0) out[c] = t;
  }
}

constexpr int kPaintThreads = 512;  // threads per tile workgroup of the paint

// One workgroup per tile; weights: channel 0 unit mass if UNIT, then w[c].
// Particles are taken in chunks of P per thread whose loads are all issued
// before any is used; the first chunk's are issued before the box is
// cleared.  A tile whose particles fit in one chunk takes the per-channel
// bound max|w| from the registers; larger tiles (the common case with three or
// more channels) take the weights' global maxima when the adjoint drift has
// formed them, else read their weights once more for it.
// FIXED: the 64-bit fixed-point sums described above (bitwise reproducible).
// Otherwise the box holds mesh-type sums updated with floating-point LDS
// atomics (ds_add_f32 / ds_add_f64), whose order, and so whose rounding,
// changes from run to run: the non-deterministic paint that plain GPU codes
// use, kept for comparison.
// WPM: the weights are particle-major, [N][NW] (PaintArgs::pi_pm).
template <typename S, typename T, int NCH, bool UNIT, bool FIXED, bool WPM = false>
__global__ __launch_bounds__(kPaintThreads) void k_paint_tiles(TileGeo g, const S* __restrict__ s,
                                                          const T* __restrict__ w, const unsigned* __restrict__ offs,
                                                          const unsigned* __restrict__ list, T* __restrict__ mesh,
                                                          T* __restrict__ halo, const double* __restrict__ wglob,
                                                          const float4* __restrict__ rec) {
  constexpr int NW = NCH - (UNIT ? 1 : 0);   // weighted channels
  constexpr int NWR = NW > 0 ? NW : 1;
  constexpr bool F32 = sizeof(T) == 4;
  constexpr int kHead = F32 ? 51 : 61;         // bits of headroom of the fixed point
  // particles per thread per chunk; one with three or more channels, which
  // brings the register use under the three workgroups per CU that LDS allows
  constexpr int P = (NCH >= 3 ? 512 : 2048) / kPaintThreads;
  constexpr unsigned CHUNK = P * kPaintThreads;
  constexpr unsigned NONE = 0xffffffffu;
  __shared__ unsigned long long box[NCH * kBoxMax];
  T* const fbox = reinterpret_cast<T*>(box);   // the box as mesh-type sums (!FIXED)
  __shared__ double wmax[kPaintThreads / 64][NCH];
  __shared__ double scale[NCH], inv_scale[NCH];
  const int64_t tile = tile_order(g, xcd_tile(blockIdx.x, int64_t(gridDim.x)));
  const int ey = g.ty + 1, ez = g.tz + 1;
  int o0, o1, o2;
  tile_origin(g, tile, o0, o1, o2);
  const unsigned beg = offs[tile], fin = offs[tile + 1];
  const int tid = threadIdx.x;

  constexpr bool REC = kUseRec<T>;
  unsigned nn[P];
  S xs[P][REC ? 1 : 3];
  float4 rs[P];
  T ws[P][NWR];
  auto load = [&](unsigned c0) {
#pragma unroll
    for (int k = 0; k < P; ++k) {
      const unsigned i = c0 + tid + k * kPaintThreads;
      nn[k] = i < fin ? list[i] : NONE;
    }
#pragma unroll
    for (int k = 0; k < P; ++k) {
      if (nn[k] == NONE) continue;
      if constexpr (REC) {
        rs[k] = rec[nn[k]];
      } else {
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) xs[k][ax] = s[ax * g.N + nn[k]];
      }
#pragma unroll
      for (int c = 0; c < NW; ++c) ws[k][c] = w[WPM ? int64_t(nn[k]) * NW + c : c * g.N + nn[k]];
    }
  };
  // Each lane visits the 8 CIC corners of its particles in the order
  // j XOR (lane mod 8): lanes whose particles share a cell then add to
  // different cells in the same LDS atomic instruction instead of
  // serialising on one address (the integer sums do not depend on the
  // order).  The flips and the box offsets of the 8 corners depend only on
  // the lane, so they are formed once.
  const int flx = (tid >> 2) & 1, fly = (tid >> 1) & 1, flz = tid & 1;
  int coff[8];
#pragma unroll
  for (int j = 0; j < 8; ++j)
    coff[j] = (((j >> 2) ^ flx) * ey + (((j >> 1) & 1) ^ fly)) * ez + ((j & 1) ^ flz);
  auto paint = [&]() {
    double sc[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) sc[c] = scale[c];
    // the scale folded into the geometric weights: channel 0's, or 1 when
    // that is 0 (an all-zero weighted channel 0); a power of two either
    // way, so the fold and the ratios below are exact.  A unit-mass channel
    // 0 of a painted tile always has a nonzero scale, so its contribution is
    // the folded weight itself.
    const double fs = sc[0] != 0.0 ? sc[0] : 1.0;
    const double inv_fs = 1.0 / fs;
#pragma unroll
    for (int k = 0; k < P; ++k) {
      if (nn[k] == NONE) continue;
      // local base node inside the tile (the particle was binned by it) and
      // the in-cell fractions
      int l0, l1, l2;
      T d0, d1, d2;
      if constexpr (REC) {
        unpack_rec(rs[k], o0, o1, o2, l0, l1, l2, d0, d1, d2);
      } else {
        double q[3];
        lattice_pos(g, nn[k], q);
        const double x0 = q[0] + double(xs[k][0]), x1 = q[1] + double(xs[k][1]), x2 = q[2] + double(xs[k][2]);
        const double f0 = floor(x0), f1 = floor(x1), f2 = floor(x2);
        l0 = int(int64_t(f0) & (g.n0 - 1)) - o0;
        l1 = int(int64_t(f1) & (g.n1 - 1)) - o1;
        l2 = int(int64_t(f2) & (g.n2 - 1)) - o2;
        d0 = T(x0 - f0);
        d1 = T(x1 - f1);
        d2 = T(x2 - f2);
      }
      // The corner weight is the readout's own product (wx wy) wz in the
      // mesh type, so that paint and readout share their weights exactly
      // (momentum conservation and adjointness hold to rounding).  The
      // folded binary scale fs rides on the x weights, which is exact; each
      // channel then takes its weight times its scale over fs.  Per axis, a
      // is the weight of the first corner the lane visits along that axis
      // and b of the second.
      const T s0 = FIXED ? T(fs) : T(1);
      const T xa = (flx ? d0 : T(1) - d0) * s0, xb = (flx ? T(1) - d0 : d0) * s0;
      const T ya = fly ? d1 : T(1) - d1, yb = fly ? T(1) - d1 : d1;
      const T za = flz ? d2 : T(1) - d2, zb = flz ? T(1) - d2 : d2;
      const T wxy[4] = {xa * ya, xa * yb, xb * ya, xb * yb};
      double wc[NCH];
#pragma unroll
      for (int c = 0; c < NCH; ++c)
        wc[c] = ((UNIT && c == 0) ? 1.0 : double(ws[k][c - (UNIT ? 1 : 0)])) * (sc[c] * inv_fs);
      const int r0 = (l0 * ey + l1) * ez + l2;
      if constexpr (!FIXED) {
        T wt[NCH];
#pragma unroll
        for (int c = 0; c < NCH; ++c) wt[c] = (UNIT && c == 0) ? T(1) : ws[k][c - (UNIT ? 1 : 0)];
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const T wg = wxy[j >> 1] * ((j & 1) ? zb : za);
          const int r = r0 + coff[j];
#pragma unroll
          for (int c = 0; c < NCH; ++c) atomicAdd(&fbox[c * kBoxMax + r], (UNIT && c == 0) ? wg : wg * wt[c]);
        }
        continue;
      }
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const double ww = double(wxy[j >> 1] * ((j & 1) ? zb : za));
        const int r = r0 + coff[j];
#pragma unroll
        for (int c = 0; c < NCH; ++c) {
          long long q;
          if constexpr (F32) {
            // |w| < 2^51: round to the nearest integer (ties to even) in the
            // low mantissa bits of 1.5 * 2^52 + w
            const double v = (UNIT && c == 0) ? ww + 6755399441055744.0 : fma(ww, wc[c], 6755399441055744.0);
            q = __double_as_longlong(v) - 0x4338000000000000ll;
          } else {
            q = __double2ll_rn((UNIT && c == 0) ? ww : ww * wc[c]);
          }
          atomicAdd(&box[c * kBoxMax + r], (unsigned long long)q);
        }
      }
    }
  };

  // the first chunk's loads are in flight while the box is cleared and the
  // scales are set
  const bool one_chunk = fin - beg <= CHUNK;
  load(beg);
  // clear every channel's whole box slot (no index arithmetic per cell)
  for (int i = tid; i < NCH * kBoxMax; i += kPaintThreads) box[i] = 0ull;
  // per-channel bound of any cell sum: count * max|w| (unit mass: count)
  if (FIXED && NW > 0) {
    double m[NCH];
#pragma unroll
    for (int c = 0; c < NCH; ++c) m[c] = 0.0;
    auto fold = [&](int c, double a) { m[c] = (a > m[c] || a != a) ? a : m[c]; };
    if (one_chunk) {
#pragma unroll
      for (int k = 0; k < P; ++k)
        if (nn[k] != NONE)
#pragma unroll
          for (int c = 0; c < NW; ++c) fold(c + (UNIT ? 1 : 0), fabs(double(ws[k][c])));
    } else if (wglob) {
      // a larger tile with the weights' global maxima at hand uses them
      // instead of reading its weights twice
#pragma unroll
      for (int c = 0; c < NW; ++c) fold(c + (UNIT ? 1 : 0), wglob[c]);
    } else {
      for (unsigned i = beg + tid; i < fin; i += kPaintThreads) {
        const unsigned n = list[i];
#pragma unroll
        for (int c = 0; c < NW; ++c) fold(c + (UNIT ? 1 : 0), fabs(double(w[WPM ? int64_t(n) * NW + c : c * g.N + n])));
      }
    }
#pragma unroll
    for (int c = 0; c < NCH; ++c)
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) fold(c, __shfl_down(m[c], off, 64));
    if ((tid & 63) == 0)
#pragma unroll
      for (int c = 0; c < NCH; ++c) wmax[tid >> 6][c] = m[c];
  }
  __syncthreads();
  if (FIXED && tid < NCH) {
    const int c = tid;
    double mx = 1.0;
    if (!(UNIT && c == 0)) {
      mx = 0.0;
      for (int wv = 0; wv < kPaintThreads / 64; ++wv) mx = (wmax[wv][c] > mx || wmax[wv][c] != wmax[wv][c]) ? wmax[wv][c] : mx;
    }
    const double bound = mx * double(fin - beg);
    int ebits = 0;
    if (bound > 0.0 && bound <= 1.0e300) {
      frexp(bound, &ebits);           // bound < 2^ebits
      scale[c] = ldexp(1.0, kHead - ebits);
      inv_scale[c] = ldexp(1.0, ebits - kHead);
    } else if (bound == 0.0) {
      scale[c] = 0.0;
      inv_scale[c] = 0.0;
    } else {                          // non-finite weights: poison the tile
      scale[c] = 0.0;
      inv_scale[c] = __longlong_as_double(0x7ff8000000000000ll);
    }
  }
  __syncthreads();
  for (unsigned c0 = beg;;) {
    paint();
    c0 += CHUNK;
    if (c0 >= fin) break;
    load(c0);
  }
  __syncthreads();
  // core: plain stores, rows of tz contiguous cells
  const int ncore = g.tx * g.ty * g.tz;
  for (int i = tid; i < NCH * ncore; i += kPaintThreads) {
    const int c = i >> (g.ltx + g.lty + g.ltz);
    const int r = i & (ncore - 1);
    const int lz = r & (g.tz - 1);
    const int ly = (r >> g.ltz) & (g.ty - 1);
    const int lx = r >> (g.ltz + g.lty);
    const int b = c * kBoxMax + (lx * ey + ly) * ez + lz;
    mesh[c * g.ncell + (int64_t(o0 + lx) * g.n1 + (o1 + ly)) * g.n2 + (o2 + lz)] =
        FIXED ? T(double(static_cast<long long>(box[b])) * inv_scale[c]) : fbox[b];
  }
  // halo faces: X (lx = tx, all ly, lz), Y (ly = ty, lx < tx), Z (lz = tz, lx < tx, ly < ty)
  const int fx = ey * ez, fy = g.tx * ez;
  const unsigned mez = 0xffffffffu / unsigned(ez) + 1u;
  for (int i = tid; i < NCH * g.hc; i += kPaintThreads) {
    const int c = i / g.hc;
    const int h = i - c * g.hc;
    int lx, ly, lz;
    if (h < fx) { lx = g.tx; ly = fdiv_small(h, mez); lz = h - ly * ez; }
    else if (h < fx + fy) { const int k = h - fx; lx = fdiv_small(k, mez); ly = g.ty; lz = k - lx * ez; }
    else { const int k = h - fx - fy; lx = k >> g.lty; ly = k & (g.ty - 1); lz = g.tz; }
    const int b = c * kBoxMax + (lx * ey + ly) * ez + lz;
    halo[(int64_t(c) * g.ntiles + tile) * g.hc + h] =
        FIXED ? T(double(static_cast<long long>(box[b])) * inv_scale[c]) : fbox[b];
  }
}

// core cells on the lower faces of each tile gather the halo faces of the
// lower neighbours d in {0,1}^3 \ {0} (wrapped), for every channel.  DEFER:
// the z face of the tile below (d = (0,0,1), the only contribution to the
// bottom-plane cells off the x and y faces) is left to the next R2C.  One
// workgroup takes 2^lpz tiles adjacent in z, so that the rows of their lower
// x and y faces, 16 cells each, join into whole 128-byte lines.
template <typename T, int NCH, bool DEFER>
__global__ __launch_bounds__(kThreads) void k_halo_add(TileGeo g, T* __restrict__ mesh, const T* __restrict__ halo,
                                                       int lpz) {
  const int64_t grp = xcd_tile(blockIdx.x, int64_t(gridDim.x));
  const int ngz = g.ntz >> lpz;
  const int t2g = int(grp % ngz);
  const int64_t t01 = grp / ngz;
  const int t1 = int(t01 % g.nty);
  const int t0 = int(t01 / g.nty);
  const int ez = g.tz + 1, ey = g.ty + 1;
  const int fx = ey * ez, fy = g.tx * ez;
  const int lw = g.ltz + lpz;   // log2 of a face row across the group
  const int nA = g.ty << lw, nB = (g.tx - 1) << lw, nC = (g.tx - 1) * (g.ty - 1);
  const int nb = nA + nB + (DEFER ? 0 : nC << lpz);
  for (int i = threadIdx.x; i < nb; i += kThreads) {
    int lx, ly, lzz;
    if (i < nA) { lx = 0; ly = i >> lw; lzz = i & ((1 << lw) - 1); }
    else if (i < nA + nB) { const int k = i - nA; lx = 1 + (k >> lw); ly = 0; lzz = k & ((1 << lw) - 1); }
    else {
      const int k = i - nA - nB, sub = k / nC, r = k - sub * nC;
      lx = 1 + r / (g.ty - 1);
      ly = 1 + r % (g.ty - 1);
      lzz = sub << g.ltz;
    }
    const int t2 = (t2g << lpz) + (lzz >> g.ltz);
    const int lz = lzz & (g.tz - 1);
    const int64_t cell = (int64_t(t0 * g.tx + lx) * g.n1 + (t1 * g.ty + ly)) * g.n2 + (t2 * g.tz + lz);
    // every load is issued before any is used: the cell's own values, then
    // the halo entry of each neighbour d (a neighbour that does not touch
    // this cell reads its own first entry and contributes +0)
    T own[NCH], hv[7][NCH];
    bool use[7];
#pragma unroll
    for (int c = 0; c < NCH; ++c) own[c] = mesh[c * g.ncell + cell];
#pragma unroll
    for (int d = 1; d < 8; ++d) {
      const int dx = d >> 2, dy = (d >> 1) & 1, dz = d & 1;
      use[d - 1] = !((dx && lx) || (dy && ly) || (dz && lz)) && !(DEFER && d == 1);
      const int u0 = (t0 - dx + g.ntx) % g.ntx, u1 = (t1 - dy + g.nty) % g.nty, u2 = (t2 - dz + g.ntz) % g.ntz;
      const int64_t u = (int64_t(u0) * g.nty + u1) * g.ntz + u2;
      const int e1 = dy ? g.ty : ly, e2 = dz ? g.tz : lz;
      int h;
      if (dx) h = e1 * ez + e2;
      else if (dy) h = fx + lx * ez + e2;
      else h = fx + fy + lx * g.ty + ly;
      if (!use[d - 1]) h = 0;
#pragma unroll
      for (int c = 0; c < NCH; ++c) hv[d - 1][c] = halo[(int64_t(c) * g.ntiles + u) * g.hc + h];
    }
#pragma unroll
    for (int c = 0; c < NCH; ++c) {
      T add = T(0);
#pragma unroll
      for (int d = 0; d < 7; ++d) add += use[d] ? hv[d][c] : T(0);
      mesh[c * g.ncell + cell] = own[c] + add;
    }
  }
}

template <typename S, typename T>
int bin_typed(Plan* p, DriftMode mode, const PaintArgs& in, hipStream_t st) {
  const TileGeo g = tile_geo(p);
  const dim3 block(kThreads);
  const int pblocks = blocks_for_particles(p);
  PM_HIP_CHECK(p, hipMemsetAsync(p->bin_counts, 0, size_t(g.ntiles) * sizeof(unsigned), st));
  BinP<S, T> b;
  b.g = g;
  b.s = static_cast<S*>(const_cast<void*>(in.s));
  b.p = static_cast<S*>(const_cast<void*>(in.p));
  b.xi = static_cast<T*>(const_cast<void*>(in.xi));
  b.pi = static_cast<T*>(in.pi);
  b.D = S(in.D);
  b.counts = p->bin_counts;
  b.keys = static_cast<uint2*>(p->bin_keys);
  b.partials = in.partials;
  b.s_set = static_cast<const S*>(in.s_set);
  b.ka = static_cast<const T*>(in.kick_a);
  b.kal = static_cast<const T*>(in.kick_al);
  b.Kp = S(in.Kp);
  b.Kx = T(in.Kx);
  b.kick_sorted = in.kick_sorted;
  b.offs = p->bin_offs;
  b.rec = static_cast<float4*>(p->bin_rec);
  const bool kick = in.kick_a != nullptr;
  const bool adj = mode == DRIFT_ADJ || mode == DRIFT_SET;
  // a particle-major pi is the native adjoint loop's: its kicks are pending
  // in tile order, or there is none yet
  if (in.pi_pm && (!adj || (kick && !in.kick_sorted)))
    return set_error(p, PM_EINVAL, "particle-major pi needs the adjoint drift with tile-order kicks");
  timing_begin(p, PM_K_BIN, st);
#define PM_BIN(MODE, KICK, PM) hipLaunchKernelGGL((k_bin<S, T, MODE, KICK, PM>), dim3(pblocks), block, 0, st, b)
#define PM_BIN_K(MODE)                      \
  do {                                      \
    if (!kick) PM_BIN(MODE, 0, false);      \
    else if (in.kick_sorted) PM_BIN(MODE, 2, false); \
    else PM_BIN(MODE, 1, false);            \
  } while (0)
#define PM_BIN_ADJ(MODE)                    \
  do {                                      \
    if (!in.pi_pm) PM_BIN_K(MODE);          \
    else if (!kick) PM_BIN(MODE, 0, true);  \
    else PM_BIN(MODE, 2, true);             \
  } while (0)
  if (mode == DRIFT_FWD) PM_BIN_K(DRIFT_FWD);
  else if (mode == DRIFT_ADJ) PM_BIN_ADJ(DRIFT_ADJ);
  else if (mode == DRIFT_SET) PM_BIN_ADJ(DRIFT_SET);
  else PM_BIN(DRIFT_NONE, 0, false);
#undef PM_BIN_ADJ
#undef PM_BIN_K
#undef PM_BIN
  {
    // s (or s_set) read (+ p read, s write; adjoint: xi read, pi read/write),
    // key write; a pending kick reads a (and alpha) and writes p (and xi)
    const double N = double(g.N), sb = sizeof(S), mb = sizeof(T);
    double method = 3 * N * sb;
    if (mode == DRIFT_FWD) method += 6 * N * sb;
    if (adj) method += 6 * N * sb + 9 * N * mb;
    if (kick) method += 3 * N * (mb + sb) + (adj ? 6 * N * mb : 0.0);
    // the implementation adds the (tile, rank) keys (also read, for a kick
    // stored in tile order) and the CIC records
    timing_end(p, PM_K_BIN, st, method + 8 * N + (kick && in.kick_sorted ? 8 * N : 0.0) + (b.rec ? 16 * N : 0.0),
               method);
  }
  const int64_t nt = g.ntiles;
  const int nsb = int((nt + 4 * kThreads - 1) / (4 * kThreads));
  hipLaunchKernelGGL(k_scan_local, dim3(nsb), block, 0, st, p->bin_counts, p->bin_offs, p->bin_bsum, nt);
  hipLaunchKernelGGL(k_scan_blocks, dim3(1), block, 0, st, p->bin_bsum, nsb);
  hipLaunchKernelGGL(k_scan_add, dim3(unsigned((nt + 1 + kThreads - 1) / kThreads)), block, 0, st, p->bin_offs,
                     p->bin_bsum, nt, unsigned(g.N));
  timing_begin(p, PM_K_SCATTER, st);
  hipLaunchKernelGGL(k_scatter, dim3(pblocks), block, 0, st, static_cast<const uint2*>(p->bin_keys), p->bin_offs,
                     p->bin_list, g.N);
  timing_end(p, PM_K_SCATTER, st, 12.0 * double(g.N), 0.0);  // key read, list write: intermediates only
  PM_HIP_CHECK(p, hipGetLastError());
  return PM_OK;
}

template <typename S, typename T>
int paint_typed(Plan* p, DriftMode mode, const PaintArgs& in, hipStream_t st) {
  const TileGeo g = tile_geo(p);
  const int nch = in.unit + in.nw;
  const dim3 block(kThreads);
  const int64_t nt = g.ntiles;
  if (in.pi_pm && !(in.unit && nch == 4 && (mode == DRIFT_ADJ || mode == DRIFT_SET)))
    return set_error(p, PM_EINVAL, "particle-major weights are the adjoint drift's pi");
  if (int rc = bin_typed<S, T>(p, mode, in, st)) return rc;
  const S* s = static_cast<const S*>(in.s);
  // in the adjoint drift the weighted channels are the updated pi, whose
  // per-channel maxima the drift left in the block partials
  const bool adj = mode == DRIFT_ADJ || mode == DRIFT_SET;
  const T* w = static_cast<const T*>(adj ? in.pi : in.w);
  // the fixed-point (bitwise reproducible) paint unless the plan asks for
  // floating-point LDS atomics
  const bool fixed = p->cfg.deterministic != 0;
  const double* wglob = nullptr;
  if (fixed && adj && in.nw == 3) {
    hipLaunchKernelGGL(k_wmax, dim3(1), block, 0, st, in.partials, blocks_for_particles(p), p->scalars);
    wglob = p->scalars;
  }
  T* mesh = static_cast<T*>(in.mesh);
  T* halo = static_cast<T*>(p->bin_halo);
  const dim3 tg{unsigned(nt), 1, 1};
  const double N = double(g.N), sb = sizeof(S), mb = sizeof(T);
  const double core_bytes = double(nch) * double(p->ncell) * mb;
  const double halo_bytes = double(nch) * double(nt) * g.hc * mb;
  // tiles: list + positions (the CIC records with FP32 meshes, else s) +
  // weights read, core and halo faces written
  const double pos_bytes = p->bin_rec ? 16 * N : 3 * N * sb;
  const double tile_bytes = 4 * N + pos_bytes + double(nch - in.unit) * N * mb + core_bytes + halo_bytes;
  // method: the painted mesh written, and the weights read unless the fused
  // adjoint drift has just read them (the positions are charged to the bin)
  const double tile_method = core_bytes + (adj ? 0.0 : double(nch - in.unit) * N * mb);
  // halo: halo faces read (but the z faces when deferred), the lower-face
  // core cells read and written
  const int zc = g.tx * g.ty;
  const int nlow = g.ty * g.tz + (g.tx - 1) * g.tz + (in.defer_z ? 0 : (g.tx - 1) * (g.ty - 1));
  const double lower = double(nlow) / (g.tx * g.ty * g.tz);
  const double hadd_bytes = halo_bytes * (in.defer_z ? double(g.hc - zc) / g.hc : 1.0) + 2.0 * lower * core_bytes;
  // the halo fold takes tiles in pairs along z where their number is even
  const int lpz = g.ntz % 2 == 0 ? 1 : 0;
  const dim3 hg(unsigned(g.ntiles >> lpz));
#define PM_TILES_W(NCH, UNIT, WPM)                                                                         \
  timing_begin(p, PM_K_PAINT_TILES, st);                                                                   \
  if (fixed)                                                                                               \
    hipLaunchKernelGGL((k_paint_tiles<S, T, NCH, UNIT, true, WPM>), tg, dim3(kPaintThreads), 0, st, g, s, w, \
                       p->bin_offs, p->bin_list, mesh, halo, wglob, static_cast<const float4*>(p->bin_rec)); \
  else                                                                                                     \
    hipLaunchKernelGGL((k_paint_tiles<S, T, NCH, UNIT, false, WPM>), tg, dim3(kPaintThreads), 0, st, g, s, w, \
                       p->bin_offs, p->bin_list, mesh, halo, wglob, static_cast<const float4*>(p->bin_rec)); \
  timing_end(p, PM_K_PAINT_TILES, st, tile_bytes, tile_method);                                            \
  timing_begin(p, PM_K_HALO, st);                                                                          \
  if (in.defer_z) hipLaunchKernelGGL((k_halo_add<T, NCH, true>), hg, block, 0, st, g, mesh, halo, lpz);   \
  else hipLaunchKernelGGL((k_halo_add<T, NCH, false>), hg, block, 0, st, g, mesh, halo, lpz);             \
  timing_end(p, PM_K_HALO, st, hadd_bytes, 0.0)
#define PM_TILES(NCH, UNIT) PM_TILES_W(NCH, UNIT, false)
  if (in.pi_pm) {
    PM_TILES_W(4, true, true);
  } else if (in.unit) {
    switch (nch) {
      case 1: PM_TILES(1, true); break;
      case 2: PM_TILES(2, true); break;
      case 3: PM_TILES(3, true); break;
      default: PM_TILES(4, true); break;
    }
  } else {
    switch (nch) {
      case 1: PM_TILES(1, false); break;
      case 2: PM_TILES(2, false); break;
      case 3: PM_TILES(3, false); break;
      default: PM_TILES(4, false); break;
    }
  }
#undef PM_TILES
#undef PM_TILES_W
  (void)sb;
  PM_HIP_CHECK(p, hipGetLastError());
  return PM_OK;
}

}  // namespace

int bin_launch(Plan* p, DriftMode mode, const PaintArgs& a, hipStream_t st) {
  const bool s64 = p->cfg.state_dtype == PM_F64, m64 = p->cfg.mesh_dtype == PM_F64;
  if (m64) return bin_typed<double, double>(p, mode, a, st);
  if (s64) return bin_typed<double, float>(p, mode, a, st);
  return bin_typed<float, float>(p, mode, a, st);
}

int paint_launch(Plan* p, DriftMode mode, const PaintArgs& a, hipStream_t st) {
  const bool s64 = p->cfg.state_dtype == PM_F64, m64 = p->cfg.mesh_dtype == PM_F64;
  if (m64) return paint_typed<double, double>(p, mode, a, st);
  if (s64) return paint_typed<double, float>(p, mode, a, st);
  return paint_typed<float, float>(p, mode, a, st);
}

ZFold paint_zfold(const Plan* p) {
  const TileGeo g = tile_geo(p);
  ZFold z{};
  z.halo = p->bin_halo;
  z.ntiles = g.ntiles;
  z.hc = g.hc;
  z.face = (g.ty + 1) * (g.tz + 1) + g.tx * (g.tz + 1);   // after the x and y faces
  z.ln1 = ilog2(g.n1);
  z.ltx = g.ltx;
  z.lty = g.lty;
  z.ltz = g.ltz;
  z.nty = g.nty;
  z.ntz = g.ntz;
  return z;
}

void tile_dims(const int n[3], int tile[3], int64_t& ntiles, int& halo_cells) {
  tile[0] = n[0] < 8 ? n[0] : 8;
  tile[1] = n[1] < 8 ? n[1] : 8;
  tile[2] = n[2] < 16 ? n[2] : 16;
  ntiles = int64_t(n[0] / tile[0]) * (n[1] / tile[1]) * (n[2] / tile[2]);
  halo_cells = (tile[1] + 1) * (tile[2] + 1) + tile[0] * (tile[2] + 1) + tile[0] * tile[1];
}

}  // namespace pmx
