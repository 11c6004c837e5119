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

template <int NN, bool FP32>
__device__ __forceinline__ void tile_cell(const TiledArgs& a, const CellItem& it, int lane, int n_own,
                                          const double* __restrict__ ul, double* __restrict__ fl) {
  constexpr int ND = 3 * NN;
  const int64_t cell = it.cell0 + lane;
  int p0, p1, p2;
  double s0, s1, s2;
  decode_orient(a.orient[cell], p0, p1, p2, s0, s1, s2);
  const double se = a.matE[a.material[cell]] * ldexp(a.h0, -(int)a.level[cell]);
  int li[NN];
#pragma unroll
  for (int k = 0; k < NN; ++k) li[k] = a.lidx[it.lidx0 + (int64_t)k * it.count + lane];
  const uint32_t mask = it.mask;
  if constexpr (!FP32) {
    double ue[ND];
#pragma unroll
    for (int k = 0; k < NN; ++k) {
      const double* q = ul + 3 * li[k];
      const double x = q[0], y = q[1], z = q[2];
      ue[3 * k + 0] = s0 * pick3(p0, x, y, z);
      ue[3 * k + 1] = s1 * pick3(p1, x, y, z);
      ue[3 * k + 2] = s2 * pick3(p2, x, y, z);
    }
    const double* Kp = a.K64 + it.koff;
#pragma unroll
    for (int k = 0; k < NN; ++k) {
      if (!((mask >> k) & 1u)) continue;  // uniform in the wave
      const bool own = li[k] < n_own;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const int i = 3 * k + c;
        double acc = 0.0;
#pragma unroll
        for (int j = 0; j < ND; ++j) acc = fma(Kp[i * ND + j], ue[j], acc);
        const int pc = c == 0 ? p0 : (c == 1 ? p1 : p2);
        const double sc = c == 0 ? s0 : (c == 1 ? s1 : s2);
        if (own) atomicAdd(fl + 3 * li[k] + pc, sc * se * acc);
      }
    }
  } else {
    const double* q0 = ul + 3 * li[0];
    const double rx = q0[0], ry = q0[1], rz = q0[2];
    float ue[ND];
#pragma unroll
    for (int k = 0; k < NN; ++k) {
      const double* q = ul + 3 * li[k];
      const double x = q[0] - rx, y = q[1] - ry, z = q[2] - rz;
      ue[3 * k + 0] = (float)(s0 * pick3(p0, x, y, z));
      ue[3 * k + 1] = (float)(s1 * pick3(p1, x, y, z));
      ue[3 * k + 2] = (float)(s2 * pick3(p2, x, y, z));
    }
    const float* Kp = a.K32 + it.koff;
#pragma unroll
    for (int k = 0; k < NN; ++k) {
      if (!((mask >> k) & 1u)) continue;
      const bool own = li[k] < n_own;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const int i = 3 * k + c;
        float acc = 0.0f;
#pragma unroll
        for (int j = 0; j < ND; ++j) acc = fmaf(Kp[i * ND + j], ue[j], acc);
        const int pc = c == 0 ? p0 : (c == 1 ? p1 : p2);
        const double sc = c == 0 ? s0 : (c == 1 ? s1 : s2);
        if (own) atomicAdd(fl + 3 * li[k] + pc, sc * se * (double)acc);
      }
    }
  }
}

template <bool PURE8, bool FP32, bool FORCE_ONLY>
__global__ void __launch_bounds__(256) tiled_step(TiledArgs a, int64_t first, int64_t count) {
  extern __shared__ double lds[];
  // XCD-contiguous block -> tile map
  const int64_t per = (count + 7) / 8;
  const int64_t b = blockIdx.x;
  const int64_t t = (b % 8) * per + b / 8;
  if (t >= count) return;
  const OwnerTile tile = a.tiles[first + t];
  const int n_own = tile.n_own, n_local = tile.n_local;
  double* ul = lds;
  double* fl = lds + 3 * (int64_t)n_local;
  const int tid = threadIdx.x;
  for (int i = tid; i < 3 * n_local; i += 256) {
    const int l = i / 3, c = i - 3 * l;
    const int64_t g = l < n_own ? tile.own0 + l : (int64_t)a.nodelist[tile.node0 + l - n_own];
    ul[i] = a.u[3 * g + c];
  }
  for (int i = tid; i < 3 * n_own; i += 256) fl[i] = 0.0;
  __syncthreads();
  if (!FORCE_ONLY)
    for (int i = tid; i < tile.n_load; i += 256) {
      const LoadEntry e = a.loads[tile.load0 + i];
      atomicAdd(fl + e.ldof, -a.P * e.val);
    }
  // the wave index is uniform in a wave: say so, so item fields (and K_p) come through scalar loads
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  for (int w = wave; w < tile.n_items; w += 4) {
    const CellItem it = a.items[tile.item0 + w];
    if (lane >= it.count) continue;
    if constexpr (PURE8) {
      tile_cell<8, FP32>(a, it, lane, n_own, ul, fl);
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
  if (FORCE_ONLY) {
    for (int i = tid; i < 3 * n_own; i += 256) a.f[d0 + i] = fl[i];
  } else {
    const double inv = 1.0 / (1.0 + a.c);
    for (int i = tid; i < 3 * n_own; i += 256) {
      const int64_t d = d0 + i;
      a.um1[d] = (a.dt2 * a.minv[d] * (-fl[i]) + 2.0 * ul[i] - (1.0 - a.c) * a.um1[d]) * inv;
    }
  }
}

}  // namespace sbfem
