// Owner-tile kernel template (included by the per-precision translation units).
#pragma once

#include "device_common.h"

// =============================================================================================
// Owner-tile step: one block per tile, everything in one pass.
//   1. stage u_n of the tile's local nodes in LDS, clear the owned forces;
//   2. add -P(t_n) b on owned load dofs;
//   3. each wave takes cell items: gather u_e from LDS, orient, accumulate the
//      master rows of owned nodes (K_p through the scalar cache), LDS atomics;
//   4. central-difference update of the owned dofs (or, force-only, write R_int).
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
// W holds the blocks with the 1/64 normalisation folded in.
template <typename T>
__device__ __forceinline__ void walsh8_apply(const T* __restrict__ W, const T (&ue)[24], T (&fe)[24]) {
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

template <int NN, bool FP32, int WALSH = 0>  // WALSH: 0 runtime choice, 1 always (8-node only)
__device__ __forceinline__ void tile_cell(const TiledArgs& a, const CellItem& it, int lane, int n_own,
                                          const typename LdsType<FP32>::T* __restrict__ ul,
                                          double* __restrict__ fl) {
  constexpr int ND = 3 * NN;
  using T = typename LdsType<FP32>::T;
  const int64_t cell = it.cell0 + lane;
  int p0, p1, p2;
  double s0, s1, s2;
  decode_orient(a.orient[cell], p0, p1, p2, s0, s1, s2);
  const double se = a.matE[a.material[cell]] * ldexp(a.h0, -(int)a.level[cell]);
  int li[NN];
#pragma unroll
  for (int k = 0; k < NN; ++k) li[k] = a.lidx[it.lidx0 + (int64_t)k * it.count + lane];
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
    if (WALSH == 1 || it.koff == a.walsh_koff) {  // uniform in the wave
      T fe[24];
      walsh8_apply<T>(FP32 ? (const T*)a.W32 : (const T*)a.W64, ue, fe);
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
  if constexpr (WALSH == 1) return;
  const T* Kp = FP32 ? (const T*)(a.K32 + it.koff) : (const T*)(a.K64 + it.koff);
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

// PURE8: tiles of 8-node cells only; WALSH (with PURE8): use the block form of the 8-node matrix.
// LDS holds the owned forces (FP64) and u of the local nodes: FP64 for FP64 products, and for
// FP32 products u minus the displacement of the tile's first owned node, in FP32.
template <bool PURE8, bool FP32, bool WALSH = false>
__global__ void __launch_bounds__(512) tiled_step(MeshRef single, const MeshRef* __restrict__ refs,
                                                  const TileWork* __restrict__ work, int64_t first, int64_t count,
                                                  int64_t k, int force_only) {
  using T = typename LdsType<FP32>::T;
  extern __shared__ double lds[];
  // XCD-contiguous block -> tile map
  const int64_t per = (count + 7) / 8;
  const int64_t b = blockIdx.x;
  const int64_t t = (b % 8) * per + b / 8;
  if (t >= count) return;
  MeshRef r = single;
  int64_t ti = first + t;
  if (work) {
    const TileWork w = work[first + t];
    r = refs[w.mesh];
    ti = w.tile;
  }
  // k steps after the step recorded in the mesh ref (batched calls advance every mesh together)
  r.step += k;
  const TiledArgs a = r.args[(r.parity + k) & 1];
  const OwnerTile tile = a.tiles[ti];
  const int n_own = tile.n_own, n_local = tile.n_local;
  double* fl = lds;
  T* ul = (T*)(lds + 3 * (int64_t)n_own);
  const int tid = threadIdx.x;
  const int nt = blockDim.x;
  double ref[3] = {0.0, 0.0, 0.0};
  if constexpr (FP32) {
#pragma unroll
    for (int c = 0; c < 3; ++c) ref[c] = a.u[3 * tile.own0 + c];
  }
  for (int i = tid; i < 3 * n_local; i += nt) {
    const int l = i / 3, c = i - 3 * l;
    const int64_t g = l < n_own ? tile.own0 + l : (int64_t)a.nodelist[tile.node0 + l - n_own];
    ul[i] = (T)(a.u[3 * g + c] - ref[c]);
  }
  for (int i = tid; i < 3 * n_own; i += nt) fl[i] = 0;
  __syncthreads();
  if (!force_only)
    for (int i = tid; i < tile.n_load; i += nt) {
      const LoadEntry e = a.loads[tile.load0 + i];
      atomicAdd(fl + e.ldof, -load_time(a.L, (double)r.step * a.dt) * e.val);
    }
  // the wave index is uniform in a wave: say so, so item fields (and K_p) come through scalar loads
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int n_waves = nt >> 6;
  for (int w = wave; w < tile.n_items; w += n_waves) {
    const CellItem it = a.items[tile.item0 + w];
    if (lane >= it.count) continue;
    if constexpr (PURE8) {
      tile_cell<8, FP32, WALSH ? 1 : 0>(a, it, lane, n_own, ul, fl);
    } else {
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
  }
  __syncthreads();
  const int64_t d0 = 3 * tile.own0;
  if (force_only) {
    for (int i = tid; i < 3 * n_own; i += nt) a.f[d0 + i] = fl[i];
  } else {
    const double inv = 1.0 / (1.0 + a.c);
    for (int i = tid; i < 3 * n_own; i += nt) {
      const int64_t d = d0 + i;
      const double un = FP32 ? a.u[d] : (double)ul[i];  // FP32 staging holds differences only
      a.um1[d] = (a.dt2 * a.minv[d] * (-fl[i]) + 2.0 * un - (1.0 - a.c) * a.um1[d]) * inv;
    }
  }
}

}  // namespace sbfem
