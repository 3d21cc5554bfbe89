// Particle kernels: CIC gather with fused kick (Sec. 2.2 and eq. KDFK), the
// force-VJP gather (Sec. 3.6, eq. KDFKO_adj) and the density-MSE mesh kernel
// (Sec. 4.2).  The paint and the particle binning live in paint.hip.
//
// The gather reuses the paint's tile binning: one workgroup per mesh tile
// loads the tile's box of (tx+1)(ty+1)(tz+1) cells of every field into LDS
// with coalesced row reads, then serves the 8 CIC corners of each of its
// particles from LDS, so the random part of the access pattern never reaches
// HBM or L2.  Positions are formed in FP64 from the exact lattice coordinate
// and the stored displacement, then the in-cell fraction is rounded to the
// mesh type; with FP32 meshes the binning has stored exactly those values per
// particle (base node and fractions, 16 bytes), and the gather reads that
// record instead of the displacement.  Reductions that feed gradients (pi.a, (delta - target)^2) are
// written as per-workgroup FP64 partial sums and combined in a fixed order,
// so they are deterministic.
#include <type_traits>

#include "tiles.h"

namespace pmx {

namespace {

__device__ __forceinline__ double block_sum(double v) { return block_sum_d<kThreads>(v); }

// ---------------------------------------------------------------------------
// gather (+ kick / VJP)
// ---------------------------------------------------------------------------
template <typename S, typename T>
struct GatherP {
  TileGeo g;
  const S* s;
  const T* mesh;   // [nf][ncell]
  T* out;          // plain: [nf][N]; VJP/MSE: xbar [3][N]
  T* acc;          // optional acceleration output
  S* p;            // kick target
  T* xi;           // adjoint kick target
  const T* cot;    // cotangent [3][N]
  const T* acc_in; // if set, the kick and cot.a use these accelerations
  S K;             // kick coefficient
  const unsigned* offs;
  const unsigned* list;
  double* partials;  // per tile, slot 1: sum cot.a
  const float4* rec; // FP32 meshes: the binning's CIC records
  bool vec_box;      // the box rows can be read as 16-byte vectors (see load_box)
  bool sorted;       // PLAIN / VJP outputs particle-major at the list position (GatherArgs::sorted_out)
};

constexpr int kGatherThreads = 512;  // threads per tile workgroup of the gather

// The tile's box of NF fields into LDS, [c][lx][ly][lz] with rows of
// ez = tz + 1 cells.  With VEC (tz a multiple of the 16-byte vector and the
// fields 16-byte aligned) the tz core cells of a row, which start on a
// multiple of tz and never wrap, are read as 16-byte vectors and the last
// cell (z wrapped) on its own; otherwise one cell at a time.  Every load of a
// thread is issued before its first LDS store, so the box costs one memory
// round trip.
template <typename T, int NF>
__device__ __forceinline__ void load_box(const TileGeo& g, const T* __restrict__ mesh, T* box, int o0, int o1,
                                         int o2, bool vec) {
  const int tid = threadIdx.x;
  const int ex = g.tx + 1, ey = g.ty + 1, ez = g.tz + 1;
  const int nrow = ex * ey;                      // rows per field
  const unsigned mrow = 0xffffffffu / unsigned(nrow) + 1u, mey = 0xffffffffu / unsigned(ey) + 1u;
  auto row_base = [&](int row, int& slot) -> int64_t {
    const int c = fdiv_small(row, mrow);
    const int rr = row - c * nrow;
    const int lx = fdiv_small(rr, mey);
    const int ly = rr - lx * ey;
    slot = c * kBoxMax + rr * ez;
    return int64_t(c) * g.ncell + (int64_t((o0 + lx) & (g.n0 - 1)) * g.n1 + ((o1 + ly) & (g.n1 - 1))) * g.n2;
  };
  constexpr int VW = 16 / sizeof(T);             // cells per 16-byte vector
  using V = typename std::conditional<sizeof(T) == 4, float4, double2>::type;
  constexpr int kRowsMax = 9 * 9;                // rows of the largest box
  if (vec) {
    const int lvr = g.ltz - ilog2c(VW);          // log2 of vectors per row core
    constexpr int ITV = (NF * kRowsMax * (16 / VW) + kGatherThreads - 1) / kGatherThreads;
    constexpr int ITT = (NF * kRowsMax + kGatherThreads - 1) / kGatherThreads;
    V vv[ITV];
    T tv[ITT];
    int vslot[ITV], tslot[ITT];
#pragma unroll
    for (int it = 0; it < ITV; ++it) {
      const int v = tid + it * kGatherThreads;
      vslot[it] = -1;
      if (v < (NF * nrow) << lvr) {
        const int row = v >> lvr, q = v & ((1 << lvr) - 1);
        int slot;
        const int64_t base = row_base(row, slot);
        vv[it] = *reinterpret_cast<const V*>(mesh + base + o2 + q * VW);
        vslot[it] = slot + q * VW;
      }
    }
#pragma unroll
    for (int it = 0; it < ITT; ++it) {
      const int row = tid + it * kGatherThreads;
      tslot[it] = -1;
      if (row < NF * nrow) {
        int slot;
        const int64_t base = row_base(row, slot);
        tv[it] = mesh[base + ((o2 + g.tz) & (g.n2 - 1))];
        tslot[it] = slot + g.tz;
      }
    }
#pragma unroll
    for (int it = 0; it < ITV; ++it)
      if (vslot[it] >= 0) {
        const T* e = reinterpret_cast<const T*>(&vv[it]);
#pragma unroll
        for (int k = 0; k < VW; ++k) box[vslot[it] + k] = e[k];
      }
#pragma unroll
    for (int it = 0; it < ITT; ++it)
      if (tslot[it] >= 0) box[tslot[it]] = tv[it];
    return;
  }
  constexpr int ITER = (NF * kBoxMax + kGatherThreads - 1) / kGatherThreads;
  const int nbox = nrow * ez;
  const unsigned mez = 0xffffffffu / unsigned(ez) + 1u;
  const unsigned mbox = 0xffffffffu / unsigned(nbox) + 1u;
  T bv[ITER];
  int slot[ITER];
#pragma unroll
  for (int it = 0; it < ITER; ++it) {
    const int i = tid + it * kGatherThreads;
    slot[it] = -1;
    if (i < NF * nbox) {
      const int c = fdiv_small(i, mbox);
      const int r = i - c * nbox;
      const int lxy = fdiv_small(r, mez);
      const int lz = r - lxy * ez;
      const int lx = fdiv_small(lxy, mey);
      const int ly = lxy - lx * ey;
      const int64_t cell = (int64_t((o0 + lx) & (g.n0 - 1)) * g.n1 + ((o1 + ly) & (g.n1 - 1))) * g.n2 +
                           ((o2 + lz) & (g.n2 - 1));
      bv[it] = mesh[c * g.ncell + cell];
      slot[it] = c * kBoxMax + r;
    }
  }
#pragma unroll
  for (int it = 0; it < ITER; ++it)
    if (slot[it] >= 0) box[slot[it]] = bv[it];
}

// CPM: the cotangent is particle-major, [N][3] (GatherArgs::cot_pm).
template <typename S, typename T, int MODE, int NF, bool CPM = false>
// the VJP gather keeps three workgroups per CU (six waves per SIMD)
__global__ __launch_bounds__(kGatherThreads, MODE == GATHER_VJP ? 6 : 1) void k_gather_tiles(GatherP<S, T> a) {
  // particles per thread per chunk: one for the adjoint modes, whose register
  // use would otherwise hold the CU to two workgroups
  constexpr int P = (MODE == GATHER_KICK_ADJ || MODE == GATHER_VJP ? 512 : 1024) / kGatherThreads;
  constexpr unsigned CHUNK = P * kGatherThreads;
  constexpr unsigned NONE = 0xffffffffu;
  constexpr bool KICKF = MODE == GATHER_KICK_FWD, KICKA = MODE == GATHER_KICK_ADJ;
  constexpr bool COT = MODE == GATHER_VJP || KICKA;
  const TileGeo& g = a.g;
  __shared__ T box[NF * kBoxMax];
  const int64_t tile = tile_order(g, xcd_tile(blockIdx.x, int64_t(gridDim.x)));
  const int ey = g.ty + 1, ez = g.tz + 1;
  int o0, o1, o2;
  tile_origin(g, tile, o0, o1, o2);
  const unsigned beg = a.offs[tile], fin = a.offs[tile + 1];
  const int tid = threadIdx.x;
  double ca = 0.0;
  if (fin > beg) {
    // particle chunk: all loads issued before any is used
    constexpr bool REC = kUseRec<T>;
    unsigned nn[P];
    S xs[P][REC ? 1 : 3], ps[P][KICKF || KICKA ? 3 : 1];
    float4 rs[P];
    T cs[P][COT ? 3 : 1], xis[P][KICKA ? 3 : 1];
    auto load = [&](unsigned c0) {
#pragma unroll
      for (int k = 0; k < P; ++k) {
        const unsigned i = c0 + tid + k * kGatherThreads;
        nn[k] = i < fin ? a.list[i] : NONE;
      }
#pragma unroll
      for (int k = 0; k < P; ++k) {
        if (nn[k] == NONE) continue;
        const int64_t n = nn[k];
        if constexpr (REC) rs[k] = a.rec[n];
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
          if (!REC) xs[k][ax] = a.s[ax * g.N + n];
          if (KICKF || KICKA) ps[k][ax] = a.p[ax * g.N + n];
          if (COT) cs[k][ax] = a.cot[CPM ? 3 * n + ax : ax * g.N + n];
          if (KICKA) xis[k][ax] = a.xi[ax * g.N + n];
        }
      }
    };
    load(beg);
    load_box<T, NF>(g, a.mesh, box, o0, o1, o2, a.vec_box);
    __syncthreads();
    for (unsigned c0 = beg;;) {
#pragma unroll
      for (int k = 0; k < P; ++k) {
        if (nn[k] == NONE) continue;
        const int64_t n = nn[k];
        // where this particle's PLAIN / VJP outputs go: its lattice index
        // ([c][N]), or its position in the tile lists, particle-major
        // ([pos][3], contiguous per tile)
        const int64_t o = a.sorted ? int64_t(c0) + tid + k * kGatherThreads : n;
        int l0, l1, l2;
        T d0, d1, d2;
        if constexpr (REC) {
          unpack_rec(rs[k], o0, o1, o2, l0, l1, l2, d0, d1, d2);
        } else {
          double q[3];
          lattice_pos(g, n, q);
          const double x0 = q[0] + double(xs[k][0]), x1 = q[1] + double(xs[k][1]), x2 = q[2] + double(xs[k][2]);
          const double f0 = floor(x0), f1 = floor(x1), f2 = floor(x2);
          l0 = int(int64_t(f0) & (g.n0 - 1)) - o0;
          l1 = int(int64_t(f1) & (g.n1 - 1)) - o1;
          l2 = int(int64_t(f2) & (g.n2 - 1)) - o2;
          d0 = T(x0 - f0);
          d1 = T(x1 - f1);
          d2 = T(x2 - f2);
        }
        const T wx[2] = {T(1) - d0, d0}, wy[2] = {T(1) - d1, d1}, wz[2] = {T(1) - d2, d2};
        T v[NF];
#pragma unroll
        for (int c = 0; c < NF; ++c) v[c] = T(0);
        T cot[3] = {T(0), T(0), T(0)};
        if (COT) {
#pragma unroll
          for (int ax = 0; ax < 3; ++ax) cot[ax] = cs[k][ax];
        }
        T dv[3] = {T(0), T(0), T(0)};  // sum_corner dW_k * h(corner)
#pragma unroll
        for (int i0 = 0; i0 < 2; ++i0)
#pragma unroll
          for (int i1 = 0; i1 < 2; ++i1)
#pragma unroll
            for (int i2 = 0; i2 < 2; ++i2) {
              const int r = ((l0 + i0) * ey + (l1 + i1)) * ez + (l2 + i2);
              const T w = wx[i0] * wy[i1] * wz[i2];
              T m[NF];
#pragma unroll
              for (int c = 0; c < NF; ++c) m[c] = box[c * kBoxMax + r];
              if (MODE == GATHER_PLAIN || KICKF || COT) {
#pragma unroll
                for (int c = 0; c < (MODE == GATHER_PLAIN || KICKF ? NF : 3); ++c) v[c] += w * m[c];
              }
              if (COT || MODE == GATHER_MSE) {
                // h = sum_j cot_j g_j + rhobar   (VJP)   or   h = mbar   (MSE)
                T h;
                if (MODE == GATHER_MSE) h = m[0];
                else h = cot[0] * m[0] + cot[1] * m[1] + cot[2] * m[2] + m[3];
                const T sx = i0 ? T(1) : T(-1), sy = i1 ? T(1) : T(-1), sz = i2 ? T(1) : T(-1);
                dv[0] += sx * wy[i1] * wz[i2] * h;
                dv[1] += sy * wx[i0] * wz[i2] * h;
                dv[2] += sz * wx[i0] * wy[i1] * h;
              }
            }
        if (MODE == GATHER_PLAIN) {
          if (NF == 3 && a.sorted) {
            Comp3<T> r;
#pragma unroll
            for (int c = 0; c < 3; ++c) r.c[c] = v[c];
            reinterpret_cast<Comp3<T>*>(a.out)[o] = r;
          } else {
#pragma unroll
            for (int c = 0; c < NF; ++c) a.out[c * g.N + o] = v[c];
          }
        } else if (KICKF) {
#pragma unroll
          for (int ax = 0; ax < 3; ++ax) {
            // fused multiply-add, as a drift applying this kick later does
            a.p[ax * g.N + n] = fma(S(v[ax]), a.K, ps[k][ax]);
            if (a.acc) a.acc[ax * g.N + n] = v[ax];
          }
        } else if (MODE == GATHER_VJP) {
#pragma unroll
          for (int ax = 0; ax < 3; ++ax) ca += double(cot[ax]) * double(v[ax]);
          if (a.sorted) {
            Comp3<T> r, q;
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
              r.c[ax] = dv[ax];
              q.c[ax] = v[ax];
            }
            reinterpret_cast<Comp3<T>*>(a.out)[o] = r;
            if (a.acc) reinterpret_cast<Comp3<T>*>(a.acc)[o] = q;
          } else {
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
              a.out[ax * g.N + o] = dv[ax];
              if (a.acc) a.acc[ax * g.N + o] = v[ax];
            }
          }
        } else if (KICKA) {
          if (a.acc_in) {
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) v[ax] = a.acc_in[ax * g.N + n];
          }
#pragma unroll
          for (int ax = 0; ax < 3; ++ax) {
            ca += double(cot[ax]) * double(v[ax]);
            a.p[ax * g.N + n] = fma(-S(v[ax]), a.K, ps[k][ax]);
            a.xi[ax * g.N + n] = fma(dv[ax], T(a.K), xis[k][ax]);
            if (a.acc) a.acc[ax * g.N + n] = v[ax];
          }
        } else if (MODE == GATHER_MSE) {
#pragma unroll
          for (int ax = 0; ax < 3; ++ax) a.out[ax * g.N + n] = dv[ax];
        }
      }
      c0 += CHUNK;
      if (c0 >= fin) break;
      load(c0);
    }
  }
  if (COT) {
    const double t = block_sum_d<kGatherThreads>(ca);
    if (threadIdx.x == 0) a.partials[tile * 4 + 1] = t;
  }
}

// (delta - target) on the mesh: mesh <- 2 (rho Nc/Np - 1 - target) / Np,
// partial sums of (delta - target)^2 in slot 2
template <typename T>
__global__ __launch_bounds__(kThreads) void k_mse_mesh(T* mesh, const T* target, int64_t ncell, double ratio,
                                                       double inv_np, double* partials) {
  const int64_t stride = int64_t(gridDim.x) * kThreads;
  double acc = 0.0;
  for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < ncell; i += stride) {
    const double d = double(mesh[i]) * ratio - 1.0 - double(target[i]);
    acc += d * d;
    mesh[i] = T(2.0 * d * inv_np);
  }
  const double t = block_sum(acc);
  if (threadIdx.x == 0) partials[blockIdx.x * 4 + 2] = t;
}

// density contrast in place: mesh <- mesh * ratio - 1
template <typename T>
__global__ __launch_bounds__(kThreads) void k_contrast(T* mesh, int64_t ncell, double ratio) {
  const int64_t stride = int64_t(gridDim.x) * kThreads;
  for (int64_t i = int64_t(blockIdx.x) * kThreads + threadIdx.x; i < ncell; i += stride)
    mesh[i] = T(double(mesh[i]) * ratio - 1.0);
}

// out[0] (+)= sum_k f[k] * sum_b part[b*4 + k], summed in a fixed order in
// two levels: workgroup w of kReduceBlocks sums the slots of a contiguous
// range of b into stage[w], then one workgroup sums stage (slots whose factor
// is zero are skipped, so stale slots never contribute)
__global__ __launch_bounds__(kThreads) void k_reduce(const double* part, int64_t nblocks, double f0, double f1,
                                                     double f2, double f3, double* stage) {
  const double f[4] = {f0, f1, f2, f3};
  const int64_t per = (nblocks + gridDim.x - 1) / gridDim.x;
  const int64_t b0 = int64_t(blockIdx.x) * per;
  const int64_t b1 = b0 + per < nblocks ? b0 + per : nblocks;
  double v = 0.0;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    if (f[k] == 0.0) continue;
    double s = 0.0;
    for (int64_t b = b0 + threadIdx.x; b < b1; b += kThreads) s += part[b * 4 + k];
    v += f[k] * s;
  }
  const double t = block_sum(v);
  if (threadIdx.x == 0) stage[blockIdx.x] = t;
}

__global__ __launch_bounds__(kThreads) void k_reduce_stage(const double* stage, int n, double* out, int accumulate) {
  const double t = block_sum(threadIdx.x < n ? stage[threadIdx.x] : 0.0);
  if (threadIdx.x == 0) out[0] = accumulate ? out[0] + t : t;
}

template <typename S, typename T>
int gather_typed(Plan* p, GatherMode mode, const GatherArgs& in, hipStream_t st) {
  if (in.sorted_out && !((mode == GATHER_PLAIN && in.nf == 3) || mode == GATHER_VJP))
    return set_error(p, PM_EINVAL, "tile-order outputs are three components per particle");
  if (in.cot_pm && mode != GATHER_VJP) return set_error(p, PM_EINVAL, "a particle-major cotangent is the VJP's");
  GatherP<S, T> a;
  a.g = tile_geo(p);
  a.s = static_cast<const S*>(in.s);
  a.mesh = static_cast<const T*>(in.mesh);
  a.out = static_cast<T*>(in.out);
  a.acc = static_cast<T*>(in.acc);
  a.p = static_cast<S*>(in.p);
  a.xi = static_cast<T*>(in.xi);
  a.cot = static_cast<const T*>(in.cot);
  a.acc_in = static_cast<const T*>(in.acc_in);
  a.K = S(in.K);
  a.offs = p->bin_offs;
  a.list = p->bin_list;
  a.partials = p->tile_partials;
  a.rec = static_cast<const float4*>(p->bin_rec);
  a.sorted = in.sorted_out;
  // vector box rows need the row cores to hold whole 16-byte vectors and the
  // fields (each ncell long, so all of them) to start 16-byte aligned
  a.vec_box = (p->tile[2] * sizeof(T)) % 16 == 0 && (reinterpret_cast<uintptr_t>(in.mesh) & 15) == 0 &&
              (p->ncell * sizeof(T)) % 16 == 0;
  const dim3 grid(unsigned(p->ntiles)), block(kGatherThreads);
  timing_begin(p, PM_K_GATHER, st);
#define PM_GATHER(MODE, NF) hipLaunchKernelGGL((k_gather_tiles<S, T, MODE, NF>), grid, block, 0, st, a)
#define PM_GATHER_CPM(MODE, NF) hipLaunchKernelGGL((k_gather_tiles<S, T, MODE, NF, true>), grid, block, 0, st, a)
  switch (mode) {
    case GATHER_PLAIN:
      switch (in.nf) {
        case 1: PM_GATHER(GATHER_PLAIN, 1); break;
        case 2: PM_GATHER(GATHER_PLAIN, 2); break;
        case 3: PM_GATHER(GATHER_PLAIN, 3); break;
        default: PM_GATHER(GATHER_PLAIN, 4); break;
      }
      break;
    case GATHER_KICK_FWD: PM_GATHER(GATHER_KICK_FWD, 3); break;
    case GATHER_VJP:
      if (in.cot_pm) PM_GATHER_CPM(GATHER_VJP, 4);
      else PM_GATHER(GATHER_VJP, 4);
      break;
    case GATHER_KICK_ADJ: PM_GATHER(GATHER_KICK_ADJ, 4); break;
    case GATHER_MSE: PM_GATHER(GATHER_MSE, 1); break;
  }
#undef PM_GATHER_CPM
#undef PM_GATHER
  {
    // list, positions (the CIC records with FP32 meshes, else s) and the
    // gathered mesh fields once, plus the per-mode particle traffic
    // (method bytes: the positions as the state stores them, 3 N s_b, in
    // place of the list and the records)
    const double N = double(p->nptcl), sb = sizeof(S), mb = sizeof(T);
    double part = 0.0;
    if (mode == GATHER_PLAIN) part = double(in.nf) * N * mb;
    if (mode == GATHER_KICK_FWD) part = 6 * N * sb + (in.acc ? 3 * N * mb : 0.0);
    if (mode == GATHER_VJP) part = 6 * N * mb + (in.acc ? 3 * N * mb : 0.0);
    if (mode == GATHER_KICK_ADJ) part = 6 * N * sb + 9 * N * mb + (in.acc_in ? 3 * N * mb : 0.0);
    if (mode == GATHER_MSE) part = 3 * N * mb;
    const double fields = double(in.nf) * double(p->ncell) * mb;
    timing_end(p, PM_K_GATHER, st, 4 * N + (p->bin_rec ? 16 * N : 3 * N * sb) + fields + part,
               3 * N * sb + fields + part);
  }
  PM_HIP_CHECK(p, hipGetLastError());
  return PM_OK;
}

}  // namespace

// p += a Kp (or -=, adjoint) and xi += alpha Kx: a kick left pending by the
// last gather of a native loop, with the fused multiply-adds of the drift.
// a and al are particle-major in the tile order of the last binning:
// particle n's values sit at 3 (offs[key.x] + key.y) + 0..2.  acc_out
// (forward, optional) receives a in lattice order.
template <typename S, typename T, bool ADJ>
__global__ __launch_bounds__(kThreads) void k_kick_flush(S* __restrict__ p, const T* __restrict__ a, S Kp,
                                                         T* __restrict__ xi, const T* __restrict__ al, T Kx,
                                                         const uint2* __restrict__ keys,
                                                         const unsigned* __restrict__ offs, T* __restrict__ acc_out,
                                                         int64_t N) {
  const int64_t stride = int64_t(gridDim.x) * kThreads;
  for (int64_t n = int64_t(blockIdx.x) * kThreads + threadIdx.x; n < N; n += stride) {
    const uint2 key = keys[n];
    const int64_t q = int64_t(offs[key.x]) + key.y;
    const Comp3<T> a3 = reinterpret_cast<const Comp3<T>*>(a)[q];
    Comp3<T> l3{};
    if (ADJ) l3 = reinterpret_cast<const Comp3<T>*>(al)[q];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const T av = a3.c[ax];
      p[ax * N + n] = fma(ADJ ? -S(av) : S(av), Kp, p[ax * N + n]);
      if (ADJ) xi[ax * N + n] = fma(l3.c[ax], Kx, xi[ax * N + n]);
      if (acc_out) acc_out[ax * N + n] = av;
    }
  }
}

template <typename S, typename T>
void kick_flush_typed(Plan* p, void* ps, const void* a, double Kp, bool adjoint, void* xi, const void* al,
                      double Kx, void* acc_out, hipStream_t st) {
  const int64_t N = p->nptcl;
  const int64_t need = (N + kThreads - 1) / kThreads;
  const int blocks = int(need < 4096 ? need : 4096);
  const uint2* keys = static_cast<const uint2*>(p->bin_keys);
  if (adjoint)
    hipLaunchKernelGGL((k_kick_flush<S, T, true>), dim3(blocks), dim3(kThreads), 0, st, static_cast<S*>(ps),
                       static_cast<const T*>(a), S(Kp), static_cast<T*>(xi), static_cast<const T*>(al), T(Kx), keys,
                       p->bin_offs, static_cast<T*>(acc_out), N);
  else
    hipLaunchKernelGGL((k_kick_flush<S, T, false>), dim3(blocks), dim3(kThreads), 0, st, static_cast<S*>(ps),
                       static_cast<const T*>(a), S(Kp), static_cast<T*>(xi), static_cast<const T*>(al), T(Kx), keys,
                       p->bin_offs, static_cast<T*>(acc_out), N);
}

int kick_flush(Plan* p, void* ps, const void* a, double Kp, bool adjoint, void* xi, const void* al, double Kx,
               void* acc_out, hipStream_t st) {
  const bool s64 = p->cfg.state_dtype == PM_F64, m64 = p->cfg.mesh_dtype == PM_F64;
  if (m64) kick_flush_typed<double, double>(p, ps, a, Kp, adjoint, xi, al, Kx, acc_out, st);
  else if (s64) kick_flush_typed<double, float>(p, ps, a, Kp, adjoint, xi, al, Kx, acc_out, st);
  else kick_flush_typed<float, float>(p, ps, a, Kp, adjoint, xi, al, Kx, acc_out, st);
  PM_HIP_CHECK(p, hipGetLastError());
  return PM_OK;
}

// dst <- src with pi's layout changed: [3][N] to particle-major [N][3]
// (TO_PM) or back
template <typename T, bool TO_PM>
__global__ __launch_bounds__(kThreads) void k_pi_layout(const T* __restrict__ src, T* __restrict__ dst, int64_t N) {
  const int64_t stride = int64_t(gridDim.x) * kThreads;
  for (int64_t n = int64_t(blockIdx.x) * kThreads + threadIdx.x; n < N; n += stride) {
    T v[3];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) v[ax] = TO_PM ? src[ax * N + n] : src[3 * n + ax];
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) (TO_PM ? dst[3 * n + ax] : dst[ax * N + n]) = v[ax];
  }
}

template <typename T>
void pi_layout_launch(const void* src, void* dst, int64_t N, bool to_pm, hipStream_t st) {
  const int64_t need = (N + kThreads - 1) / kThreads;
  const dim3 grid(unsigned(need < 4096 ? need : 4096)), block(kThreads);
  const T* x = static_cast<const T*>(src);
  T* y = static_cast<T*>(dst);
  if (to_pm) hipLaunchKernelGGL((k_pi_layout<T, true>), grid, block, 0, st, x, y, N);
  else hipLaunchKernelGGL((k_pi_layout<T, false>), grid, block, 0, st, x, y, N);
}

bool pi_layout_fits(const Plan* p) { return 3 * p->nptcl <= 4 * p->ncell; }

int pi_layout(Plan* p, void* pi, bool to_pm, hipStream_t st) {
  if (!pi_layout_fits(p)) return set_error(p, PM_EINVAL, "pi does not fit the mesh workspace");
  const size_t rb = p->cfg.mesh_dtype == PM_F64 ? 8 : 4;
  const int64_t N = p->nptcl;
  // the plan's meshes are one allocation of 4 ncell values, free between steps
  void* ws = p->mesh[0];
  PM_HIP_CHECK(p, hipMemcpyAsync(ws, pi, size_t(3) * size_t(N) * rb, hipMemcpyDeviceToDevice, st));
  if (rb == 8) pi_layout_launch<double>(ws, pi, N, to_pm, st);
  else pi_layout_launch<float>(ws, pi, N, to_pm, st);
  PM_HIP_CHECK(p, hipGetLastError());
  return PM_OK;
}

int blocks_for_particles(const Plan* p) {
  const int64_t need = (p->nptcl + kThreads - 1) / kThreads;
  const int64_t cap = 2048;  // 8 workgroups per CU on 256 CUs; <= kMaxPartials
  return int(need < cap ? (need < 1 ? 1 : need) : cap);
}

int gather_launch(Plan* p, GatherMode mode, const GatherArgs& a, hipStream_t st) {
  if (!a.binned) {
    // bin the particles by their current positions (no paint precedes this call)
    PaintArgs b{};
    b.s = a.s;
    if (int rc = bin_launch(p, DRIFT_NONE, b, st)) return rc;
  }
  const bool s64 = p->cfg.state_dtype == PM_F64, m64 = p->cfg.mesh_dtype == PM_F64;
  if (m64) return gather_typed<double, double>(p, mode, a, st);
  if (s64) return gather_typed<double, float>(p, mode, a, st);
  return gather_typed<float, float>(p, mode, a, st);
}

int mse_mesh_launch(Plan* p, void* mesh, const void* target, double* partials, hipStream_t st) {
  const double ratio = double(p->ncell) / double(p->nptcl);
  const double inv_np = 1.0 / double(p->nptcl);
  const int64_t need = (p->ncell + kThreads - 1) / kThreads;
  const int blocks = int(need < 2048 ? need : 2048);
  if (p->cfg.mesh_dtype == PM_F64)
    hipLaunchKernelGGL((k_mse_mesh<double>), dim3(blocks), dim3(kThreads), 0, st, static_cast<double*>(mesh),
                       static_cast<const double*>(target), p->ncell, ratio, inv_np, partials);
  else
    hipLaunchKernelGGL((k_mse_mesh<float>), dim3(blocks), dim3(kThreads), 0, st, static_cast<float*>(mesh),
                       static_cast<const float*>(target), p->ncell, ratio, inv_np, partials);
  PM_HIP_CHECK(p, hipGetLastError());
  return blocks;
}

int contrast_launch(Plan* p, void* mesh, hipStream_t st) {
  const double ratio = double(p->ncell) / double(p->nptcl);
  const int64_t need = (p->ncell + kThreads - 1) / kThreads;
  const int blocks = int(need < 2048 ? need : 2048);
  if (p->cfg.mesh_dtype == PM_F64)
    hipLaunchKernelGGL((k_contrast<double>), dim3(blocks), dim3(kThreads), 0, st, static_cast<double*>(mesh), p->ncell,
                       ratio);
  else
    hipLaunchKernelGGL((k_contrast<float>), dim3(blocks), dim3(kThreads), 0, st, static_cast<float*>(mesh), p->ncell,
                       ratio);
  PM_HIP_CHECK(p, hipGetLastError());
  return PM_OK;
}

int reduce_partials(Plan* p, int nblocks, const double* f, double* out, bool accumulate, hipStream_t st) {
  return reduce_buffer(p, p->partials, nblocks, f, out, accumulate, st);
}

int reduce_buffer(Plan* p, const double* buf, int64_t nblocks, const double* f, double* out, bool accumulate,
                  hipStream_t st) {
  static_assert(kReduceBlocks <= kThreads, "one thread per staged sum");
  double* stage = p->scalars + 16;
  hipLaunchKernelGGL(k_reduce, dim3(kReduceBlocks), dim3(kThreads), 0, st, buf, nblocks, f[0], f[1], f[2], f[3],
                     stage);
  hipLaunchKernelGGL(k_reduce_stage, dim3(1), dim3(kThreads), 0, st, stage, kReduceBlocks, out, accumulate ? 1 : 0);
  PM_HIP_CHECK(p, hipGetLastError());
  return PM_OK;
}

}  // namespace pmx
