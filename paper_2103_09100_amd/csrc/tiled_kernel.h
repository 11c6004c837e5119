// Owner-tile kernel templates (included by the per-precision translation units).
#pragma once

#include "device_common.h"

// =============================================================================================
// Owner-tile step: one block per tile, everything in one pass (Alg. 1 time loop).
//   1. stage u_n of the tile's local nodes in LDS, clear the owned forces;
//   2. add -P(t_n) b on owned load dofs;
//   3. each wave takes cell items: gather u_e from LDS, multiply by the master
//      matrix (eqs. Rinte, Rintep, KM_scale), add the rows of owned nodes into
//      the LDS force array with FP64 LDS atomics;
//   4. central-difference update of the owned dofs (eq. DnMdiag), or, force-only,
//      write R_int of the owned dofs.
// Blocks are mapped so that each XCD (blocks b, b+8, ...) walks a contiguous run
// of tiles, which keeps neighbouring tiles' shared nodes in one L2.

namespace sbfem {

template <bool FP32>
struct LdsType {
  using T = double;
};
template <>
struct LdsType<true> {
  using T = float;
};

template <typename T>
__device__ __forceinline__ T pick3t(int i, T x, T y, T z) {
  return i == 0 ? x : (i == 1 ? y : z);
}

// The regular 8-node cell is symmetric under the three mirror planes, so in the
// basis of Walsh functions over its corners (per displacement component) its
// master matrix splits into 8 blocks of 3x3: mode (a, s) of component a and
// corner character s couples only to modes of the same parity type s ^ (1 << a).
// f = K u becomes: forward butterflies (24 adds per component), 72 products,
// inverse butterflies.  Corner k = i + 2j + 4l sits at (2i-1, 2j-1, 2l-1);
// W holds the blocks with the 1/64 normalisation (and, for pure 8-node tiles,
// the cell scale) folded in.
template <typename T>
__device__ __forceinline__ void walsh8_apply(cptr_t<T> W, const T (&ue)[24], T (&fe)[24]) {
  T x[3][8];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int k = 0; k < 8; ++k) x[a][k] = ue[3 * k + a];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
      for (int k = 0; k < 8; ++k)
        if (!((k >> b) & 1)) {
          const T lo = x[a][k], hi = x[a][k | (1 << b)];
          x[a][k] = lo + hi;
          x[a][k | (1 << b)] = hi - lo;
        }
  T y[3][8];
#pragma unroll
  for (int t = 0; t < 8; ++t)
#pragma unroll
    for (int a2 = 0; a2 < 3; ++a2) {
      T acc = W[t * 9 + a2 * 3 + 0] * x[0][t ^ 1];
      acc = fma(W[t * 9 + a2 * 3 + 1], x[1][t ^ 2], acc);
      acc = fma(W[t * 9 + a2 * 3 + 2], x[2][t ^ 4], acc);
      y[a2][t ^ (1 << a2)] = acc;
    }
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
      for (int k = 0; k < 8; ++k)
        if (!((k >> b) & 1)) {
          const T A = y[a][k], B = y[a][k | (1 << b)];
          y[a][k] = A - B;
          y[a][k | (1 << b)] = A + B;
        }
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int k = 0; k < 8; ++k) fe[3 * k + a] = y[a][k];
}

// The block's tile: which mesh (single or batched launch), its argument block for
// this step (u and u_prev swap roles every step) and the tile index.  false: no tile.
__device__ __forceinline__ bool block_tile(const MeshRef& single, const MeshRef* refs, const TileWork* work,
                                           int64_t first, int64_t count, int64_t k, TiledArgs& a,
                                           int64_t& ti, int64_t& step) {
  // XCD-contiguous block -> tile map
  const int64_t per = (count + 7) / 8;
  const int64_t b = blockIdx.x;
  const int64_t t = (b % 8) * per + b / 8;
  if (t >= count) return false;
  MeshRef r = single;
  ti = first + t;
  if (work) {
    const TileWork w = load_const(as_const(work) + (first + t));
    r = load_const(as_const(refs) + w.mesh);
    ti = w.tile;
  }
  // k steps after the step recorded in the mesh ref (batched calls advance every mesh together)
  step = r.step + k;
  a = load_const(as_const(r.args) + ((r.parity + k) & 1));
  return true;
}

// Generic cell of NN nodes (any pattern): orientation per cell, dense master matrix
// (or the Walsh form for the 8-node pattern), scale s_e per cell.
template <int NN, bool FP32>
__device__ __forceinline__ void tile_cell(const TiledArgs& a, const CellItem& it, int lane, int n_own,
                                          const typename LdsType<FP32>::T* __restrict__ ul,
                                          double* __restrict__ fl) {
  constexpr int ND = 3 * NN;
  using T = typename LdsType<FP32>::T;
  const int64_t cell = it.cell0 + lane;
  int p0, p1, p2;
  double s0, s1, s2;
  decode_orient(as_global(a.orient)[cell], p0, p1, p2, s0, s1, s2);
  const double se = as_const(a.matE)[as_global(a.material)[cell]] * ldexp(a.h0, -(int)as_global(a.level)[cell]);
  int li[NN];
  gptr_t<uint16_t> lidx = as_global(a.lidx);
#pragma unroll
  for (int k = 0; k < NN; ++k) li[k] = lidx[it.lidx0 + (int64_t)k * it.count + lane];
  const uint32_t mask = it.mask;
  // oriented nodal displacements; the FP32 path also removes the rigid translation of
  // node 0 (K_p annihilates it) so that only differences across the cell are rounded
  T ue[ND];
  {
    T rx = 0, ry = 0, rz = 0;
    if constexpr (FP32) {
      const T* q0 = ul + 3 * li[0];
      rx = q0[0];
      ry = q0[1];
      rz = q0[2];
    }
#pragma unroll
    for (int k = 0; k < NN; ++k) {
      const T* q = ul + 3 * li[k];
      const T x = q[0] - rx, y = q[1] - ry, z = q[2] - rz;
      ue[3 * k + 0] = (T)s0 * pick3t<T>(p0, x, y, z);
      ue[3 * k + 1] = (T)s1 * pick3t<T>(p1, x, y, z);
      ue[3 * k + 2] = (T)s2 * pick3t<T>(p2, x, y, z);
    }
  }
  if constexpr (NN == 8) {
    if (it.koff == a.walsh_koff) {  // uniform in the wave
      T fe[24];
      walsh8_apply<T>(as_const(FP32 ? (const T*)a.W32 : (const T*)a.W64), ue, fe);
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        if (!((mask >> k) & 1u)) continue;
        if (li[k] >= n_own) continue;
        // forces are summed in FP64 (LDS FP64 atomics are also the fast ones here)
        atomicAdd(fl + 3 * li[k] + p0, s0 * se * (double)fe[3 * k + 0]);
        atomicAdd(fl + 3 * li[k] + p1, s1 * se * (double)fe[3 * k + 1]);
        atomicAdd(fl + 3 * li[k] + p2, s2 * se * (double)fe[3 * k + 2]);
      }
      return;
    }
  }
  cptr_t<T> Kp = as_const(FP32 ? (const T*)(a.K32 + it.koff) : (const T*)(a.K64 + it.koff));
#pragma unroll
  for (int k = 0; k < NN; ++k) {
    if (!((mask >> k) & 1u)) continue;  // uniform in the wave
    const bool own = li[k] < n_own;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int i = 3 * k + c;
      T acc = 0;
#pragma unroll
      for (int j = 0; j < ND; ++j) acc = fma(Kp[i * ND + j], ue[j], acc);
      const int pc = c == 0 ? p0 : (c == 1 ? p1 : p2);
      const double sc = c == 0 ? s0 : (c == 1 ? s1 : s2);
      if (own) atomicAdd(fl + 3 * li[k] + pc, sc * se * (double)acc);
    }
  }
}

// Owned forces start at -P(t_n) b on the tile's load dofs.
__device__ __forceinline__ void tile_loads(const TiledArgs& a, const OwnerTile& tile, int64_t step, double* fl,
                                           int tid, int nt) {
  for (int i = tid; i < tile.n_load; i += nt) {
    const LoadEntry e = load_const(as_const(a.loads) + (tile.load0 + i));
    atomicAdd(fl + e.ldof, -load_time(a.L, (double)step * a.dt) * e.val);
  }
}

// Central-difference update of the owned dofs written over u_{n-1} (or R_int, force-only).
// un_lds: u_n of the owned dofs as staged (FP64 staging holds u_n itself).
template <bool FP32>
__device__ __forceinline__ void tile_update(const TiledArgs& a, const OwnerTile& tile, const double* fl,
                                            const double* un_lds, int force_only, int tid, int nt) {
  const int64_t d0 = 3 * tile.own0;
  const int n = 3 * tile.n_own;
  if (force_only) {
    gmut_t<double> f = as_global_mut(a.f);
    for (int i = tid; i < n; i += nt) f[d0 + i] = fl[i];
    return;
  }
  gptr_t<double> u = as_global(a.u);
  gptr_t<double> minv = as_global(a.minv);
  gmut_t<double> um1 = as_global_mut(a.um1);
  const double inv = 1.0 / (1.0 + a.c);
  for (int i = tid; i < n; i += nt) {
    const int64_t d = d0 + i;
    const double un = FP32 ? u[d] : un_lds[i];
    um1[d] = (a.dt2 * minv[d] * (-fl[i]) + 2.0 * un - (1.0 - a.c) * um1[d]) * inv;
  }
}

// Tiles with cells of any pattern.  LDS: the owned forces (FP64), then u of the local nodes,
// 3 values per node: FP64 for FP64 products; for FP32 products u minus the displacement of
// the tile's first owned node, in FP32.
template <bool FP32>
__global__ void __launch_bounds__(512) tiled_step(MeshRef single, const MeshRef* __restrict__ refs,
                                                  const TileWork* __restrict__ work, int64_t first, int64_t count,
                                                  int64_t k, int force_only) {
  using T = typename LdsType<FP32>::T;
  extern __shared__ double lds[];
  TiledArgs a;
  int64_t ti, step;
  if (!block_tile(single, refs, work, first, count, k, a, ti, step)) return;
  const OwnerTile tile = load_const(as_const(a.tiles) + ti);
  const int n_own = tile.n_own, n_local = tile.n_local;
  double* fl = lds;
  T* ul = (T*)(lds + 3 * (int64_t)n_own);
  const int tid = threadIdx.x;
  const int nt = blockDim.x;
  gptr_t<double> u = as_global(a.u);
  gptr_t<int32_t> nodelist = as_global(a.nodelist);
  double ref[3] = {0.0, 0.0, 0.0};
  if constexpr (FP32) {
#pragma unroll
    for (int c = 0; c < 3; ++c) ref[c] = u[3 * tile.own0 + c];
  }
  for (int i = tid; i < 3 * n_local; i += nt) {
    const int l = i / 3, c = i - 3 * l;
    const int64_t g = l < n_own ? tile.own0 + l : (int64_t)nodelist[tile.node0 + l - n_own];
    ul[i] = (T)(u[3 * g + c] - ref[c]);
  }
  for (int i = tid; i < 3 * n_own; i += nt) fl[i] = 0;
  __syncthreads();
  if (!force_only) tile_loads(a, tile, step, fl, tid, nt);
  // the wave index is uniform in a wave: say so, so item fields (and K_p) come through scalar loads
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int n_waves = nt >> 6;
  cptr_t<CellItem> items = as_const(a.items) + tile.item0;
  for (int w = wave; w < tile.n_items; w += n_waves) {
    const CellItem it = load_const(items + w);
    if (lane >= it.count) continue;
#define SBFEM_TCASE(N) \
  case N:              \
    tile_cell<N, FP32>(a, it, lane, n_own, ul, fl); \
    break;
    switch (it.nn) {
      SBFEM_TCASE(8) SBFEM_TCASE(9) SBFEM_TCASE(10) SBFEM_TCASE(11) SBFEM_TCASE(12) SBFEM_TCASE(13)
      SBFEM_TCASE(14) SBFEM_TCASE(15) SBFEM_TCASE(16) SBFEM_TCASE(17) SBFEM_TCASE(18) SBFEM_TCASE(19)
      SBFEM_TCASE(20) SBFEM_TCASE(21) SBFEM_TCASE(22) SBFEM_TCASE(23) SBFEM_TCASE(24) SBFEM_TCASE(25)
      SBFEM_TCASE(26)
      default:
        break;
    }
#undef SBFEM_TCASE
  }
  __syncthreads();
  tile_update<FP32>(a, tile, fl, (const double*)ul, force_only, tid, nt);
}

// Tiles whose cells are all regular 8-node cells in identity orientation (the master
// matrix is invariant under the 48 cube transformations, so the set-up maps every such
// cell onto it without a transformation).  Per cell: one 16-byte record of local node
// indices, the Walsh-form product with the blocks pre-scaled by the item's scale class,
// FP64 LDS atomics for the owned rows.  LDS: owned forces (FP64), then u of the local
// nodes: FP32 products 4 floats per node (x, y, z minus the tile reference, pad) so
// one 16-byte read fetches a node; FP64 products 3 doubles per node.
template <bool FP32>
__global__ void __launch_bounds__(512) tiled_step8(MeshRef single, const MeshRef* __restrict__ refs,
                                                   const TileWork* __restrict__ work, int64_t first,
                                                   int64_t count, int64_t k, int force_only) {
  using T = typename LdsType<FP32>::T;
  extern __shared__ double lds[];
  TiledArgs a;
  int64_t ti, step;
  if (!block_tile(single, refs, work, first, count, k, a, ti, step)) return;
  const OwnerTile tile = load_const(as_const(a.tiles) + ti);
  const int n_own = tile.n_own, n_local = tile.n_local;
  double* fl = lds;
  T* ul = (T*)(lds + 3 * (int64_t)n_own);
  const int tid = threadIdx.x;
  const int nt = blockDim.x;
  gptr_t<double> u = as_global(a.u);
  gptr_t<int32_t> nodelist = as_global(a.nodelist);
  double r0 = 0.0, r1 = 0.0, r2 = 0.0;
  if constexpr (FP32) {
    r0 = u[3 * tile.own0 + 0];
    r1 = u[3 * tile.own0 + 1];
    r2 = u[3 * tile.own0 + 2];
  }
  for (int l = tid; l < n_local; l += nt) {
    const int64_t g = l < n_own ? tile.own0 + l : (int64_t)nodelist[tile.node0 + l - n_own];
    const double x = u[3 * g + 0], y = u[3 * g + 1], z = u[3 * g + 2];
    if constexpr (FP32) {
      reinterpret_cast<float4*>(ul)[l] = make_float4((float)(x - r0), (float)(y - r1), (float)(z - r2), 0.0f);
    } else {
      ul[3 * l + 0] = x;
      ul[3 * l + 1] = y;
      ul[3 * l + 2] = z;
    }
  }
  for (int i = tid; i < 3 * n_own; i += nt) fl[i] = 0;
  __syncthreads();
  if (!force_only) tile_loads(a, tile, step, fl, tid, nt);
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int n_waves = nt >> 6;
  cptr_t<CellItem> items = as_const(a.items) + tile.item0;
  gptr_t<uint4> lrec = as_global(reinterpret_cast<const uint4*>(a.lidx));
  cptr_t<T> Ws = as_const(FP32 ? (const T*)a.Ws32 : (const T*)a.Ws64);
  for (int w = wave; w < tile.n_items; w += n_waves) {
    const CellItem it = load_const(items + w);
    if (lane >= it.count) continue;
    const uint4 q = load_global(lrec + ((it.lidx0 >> 3) + lane));
    const int li[8] = {(int)(q.x & 0xFFFFu), (int)(q.x >> 16), (int)(q.y & 0xFFFFu), (int)(q.y >> 16),
                       (int)(q.z & 0xFFFFu), (int)(q.z >> 16), (int)(q.w & 0xFFFFu), (int)(q.w >> 16)};
    T ue[24];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      if constexpr (FP32) {
        const float4 v = reinterpret_cast<const float4*>(ul)[li[c]];
        ue[3 * c + 0] = v.x;
        ue[3 * c + 1] = v.y;
        ue[3 * c + 2] = v.z;
      } else {
        ue[3 * c + 0] = ul[3 * li[c] + 0];
        ue[3 * c + 1] = ul[3 * li[c] + 1];
        ue[3 * c + 2] = ul[3 * li[c] + 2];
      }
    }
    T fe[24];
    walsh8_apply<T>(Ws + it.koff, ue, fe);
    const uint32_t mask = it.mask;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      if (!((mask >> c) & 1u)) continue;  // uniform in the wave
      if (li[c] >= n_own) continue;
      double* fp = fl + 3 * li[c];
      atomicAdd(fp + 0, (double)fe[3 * c + 0]);
      atomicAdd(fp + 1, (double)fe[3 * c + 1]);
      atomicAdd(fp + 2, (double)fe[3 * c + 2]);
    }
  }
  __syncthreads();
  // FP64 staging keeps u_n of the owned nodes at the start of ul (owned nodes come first)
  tile_update<FP32>(a, tile, fl, (const double*)ul, force_only, tid, nt);
}

}  // namespace sbfem
