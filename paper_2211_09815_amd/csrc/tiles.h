// Device helpers shared by the tiled paint (paint.hip) and the tiled gather
// (particles.hip).  The mesh is cut into tiles of tx * ty * tz cells; every
// particle belongs to the tile that holds its CIC base node floor(x), so its
// 8 CIC corners lie in the tile's "box" of (tx+1)(ty+1)(tz+1) cells.
#pragma once

#include "pm_internal.h"

namespace pmx {

constexpr int kBoxMax = 9 * 9 * 17;  // box cells for the largest tile (8 x 8 x 16)

struct TileGeo {
  int64_t N;
  int np1, np2;
  double inv_np1, inv_np2;   // 1/np1, 1/np2 (quotient estimates, corrected)
  double r0, r1, r2, off;
  int n0, n1, n2;
  int64_t ncell;
  int tx, ty, tz;        // tile dims (cells), powers of two
  int ltx, lty, ltz;     // their log2
  int ntx, nty, ntz;     // tiles per axis
  int64_t ntiles;
  int hc;                // halo cells per tile (the three upper faces of the box)
};

inline TileGeo tile_geo(const Plan* p) {
  TileGeo g;
  g.N = p->nptcl;
  g.np1 = p->np[1];
  g.np2 = p->np[2];
  g.inv_np1 = 1.0 / double(g.np1);
  g.inv_np2 = 1.0 / double(g.np2);
  g.r0 = p->r[0];
  g.r1 = p->r[1];
  g.r2 = p->r[2];
  g.off = p->cfg.lattice_offset;
  g.n0 = p->n[0];
  g.n1 = p->n[1];
  g.n2 = p->n[2];
  g.ncell = p->ncell;
  g.tx = p->tile[0];
  g.ty = p->tile[1];
  g.tz = p->tile[2];
  g.ltx = ilog2(g.tx);
  g.lty = ilog2(g.ty);
  g.ltz = ilog2(g.tz);
  g.ntx = g.n0 / g.tx;
  g.nty = g.n1 / g.ty;
  g.ntz = g.n2 / g.tz;
  g.ntiles = p->ntiles;
  g.hc = p->halo_cells;
  return g;
}

// q = n / d and n - q d for 0 <= n < 2^31: the FP64 estimate n * (1/d) is
// within one of the quotient, and one correction step makes it exact
__device__ __forceinline__ int divmod_small(int n, int d, double inv, int& rem) {
  int q = int(double(n) * inv);
  int r = n - q * d;
  if (r < 0) { --q; r += d; }
  if (r >= d) { ++q; r -= d; }
  rem = r;
  return q;
}

// Lagrangian position q = (i, j, k) r + offset of particle n (row-major lattice)
__device__ __forceinline__ void lattice_pos(const TileGeo& g, int64_t n, double q[3]) {
  int k, j;
  const int row = divmod_small(int(n), g.np2, g.inv_np2, k);
  const int i = divmod_small(row, g.np1, g.inv_np1, j);
  q[0] = double(i) * g.r0 + g.off;
  q[1] = double(j) * g.r1 + g.off;
  q[2] = double(k) * g.r2 + g.off;
}

// r / d for 0 <= r < 2^20 and 1 <= d < 2^10 with m = 0xffffffff / d + 1:
// the high word of r m is exact in that range
__device__ __forceinline__ int fdiv_small(int r, unsigned m) { return int(__umulhi(unsigned(r), m)); }

// Per-particle CIC record, written by the binning for FP32 meshes and read
// by the paint and the gather instead of the displacement: the base node
// (floor of the FP64 position, wrapped; 10 bits per axis, meshes up to 1024)
// and the in-cell fractions rounded to float, i.e. exactly the values those
// kernels would form from the FP64 position themselves.  The 10-bit fields
// and the two-level scan of the tile offsets (at most (4 kThreads)^2 tiles)
// tie the mesh to sides <= 1024 with tiles of at least 8x8x16 cells;
// pm_plan_create refuses any plan beyond them.
template <typename T> constexpr bool kUseRec = sizeof(T) == 4;

// three components of one particle, stored particle-major (the pending kicks
// in tile order): one 12- or 24-byte access per lane instead of three strided
// ones
template <typename T>
struct Comp3 {
  T c[3];
};

__device__ __forceinline__ unsigned pack_cell(int b0, int b1, int b2) {
  return (unsigned(b0) << 20) | (unsigned(b1) << 10) | unsigned(b2);
}

template <typename T>
__device__ __forceinline__ void unpack_rec(const float4 r, int o0, int o1, int o2, int& l0, int& l1, int& l2, T& d0,
                                           T& d1, T& d2) {
  const unsigned c = __float_as_uint(r.x);
  l0 = int(c >> 20) - o0;
  l1 = int((c >> 10) & 1023u) - o1;
  l2 = int(c & 1023u) - o2;
  d0 = T(r.y);
  d1 = T(r.z);
  d2 = T(r.w);
}

// tile coordinates and origin cell of a tile index
__device__ __forceinline__ void tile_origin(const TileGeo& g, int64_t tile, int& o0, int& o1, int& o2) {
  const int t2 = int(tile % g.ntz);
  const int64_t t01 = tile / g.ntz;
  const int t1 = int(t01 % g.nty);
  const int t0 = int(t01 / g.nty);
  o0 = t0 * g.tx;
  o1 = t1 * g.ty;
  o2 = t2 * g.tz;
}

// Dispatch order of the tiles: groups of kOrderX x kOrderY columns of tiles
// (x, y) are interleaved at every z, so the x and y neighbours of most tiles
// run at about the same time on the same XCD and share its L2 (boxes overlap
// by one cell plane, and particle cache lines straddle tile faces).
// pos -> tile id; identity when the tile grid does not divide into groups.
constexpr int kOrderX = 2, kOrderY = 2;
__device__ __forceinline__ int64_t tile_order(const TileGeo& g, int64_t pos) {
  if (g.ntx % kOrderX || g.nty % kOrderY) return pos;
  constexpr int G = kOrderX * kOrderY;
  const int64_t blk = pos / (G * g.ntz);
  const int w = int(pos - blk * G * g.ntz);
  const int t2 = w / G, d = w % G;
  const int d0 = d / kOrderY, d1 = d % kOrderY;
  const int hy = g.nty / kOrderY;
  const int m0 = int(blk / hy), m1 = int(blk - int64_t(m0) * hy);
  return (int64_t(kOrderX * m0 + d0) * g.nty + (kOrderY * m1 + d1)) * g.ntz + t2;
}

// contiguous particle chunk of this workgroup (consecutive chunks on one XCD)
__device__ __forceinline__ void chunk_of(int64_t N, int64_t& start, int64_t& end) {
  const int64_t nb = gridDim.x;
  const int64_t per = ((N + nb - 1) / nb + kThreads - 1) / kThreads * kThreads;
  start = xcd_tile(blockIdx.x, nb) * per;
  end = start + per < N ? start + per : N;
}

// sum over a workgroup of NT threads; the result is valid in thread 0
template <int NT = kThreads>
__device__ __forceinline__ double block_sum_d(double v) {
  __shared__ double ws[NT / 64];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) ws[wid] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < NT / 64; ++w) t += ws[w];
  return t;
}

// largest of v over a workgroup of NT threads, NaN if any v is NaN; the
// result is valid in thread 0
template <int NT = kThreads>
__device__ __forceinline__ double block_max_d(double v) {
  __shared__ double wm[NT / 64];
  auto fold = [](double m, double a) { return (a > m || a != a) ? a : m; };
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v = fold(v, __shfl_down(v, off, 64));
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) wm[wid] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int w = 0; w < NT / 64; ++w) t = fold(t, wm[w]);
  return t;
}

}  // namespace pmx
