// Owner-tile kernel templates (included by the per-precision translation units).
#pragma once

#include "device_common.h"

// =============================================================================================
// A time step (Alg. 1 time loop) is two passes.
//  Hanging-cell pass: every cell that is not a regular 8-node cell, once, in items of one
//    pattern: gather u_e, orient (Sec. 3.2.2), dense master product (eqs. Rinte, Rintep,
//    KM_scale); the force of every row is stored (no atomics) for the owner tiles.
//  Owner-tile pass, one block per tile:
//   1. stage u_n of the tile's local nodes in LDS, clear the owned forces;
//   2. add -P(t_n) b on owned load dofs;
//   3. each wave takes items of regular 8-node cells: gather u_e from LDS, Walsh-form
//      product, add the rows of owned nodes with FP64 LDS atomics;
//   4. add the hanging-cell forces of its owned dofs (a list of (dof, result) pairs), then
//      the central-difference update of the owned dofs (eq. DnMdiag), or, force-only, write
//      R_int of the owned dofs.
// Blocks are mapped so that each XCD (blocks b, b+8, ...) walks a contiguous run of tiles,
// which keeps neighbouring tiles' shared nodes in one L2.

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
// corner character s couples only to modes of the same type t = s ^ (1 << a).
// Corner k = i + 2j + 4l sits at (2i-1, 2j-1, 2l-1).  The full cube symmetry
// fixes more: the translation modes (s = 0) carry no force, block t = 1 << m
// couples only the two axes other than m, block t = 7 ^ (1 << m) couples the two
// axes of t and keeps axis m on its own, and blocks 0 and 7 have the form
// (d - o) I + o J.  The table C holds the 31 remaining coefficients (with the
// 1/64 normalisation and the cell scale s_e folded in):
//   [0] d0 - o0, [1] o0, [2] d7 - o7, [3] o7,
//   [4 + 4m]  t = 1 << m:       B_ii, B_ij, B_ji, B_jj over the axes i < j other than m,
//   [16 + 5m] t = 7 ^ (1 << m): B_ii, B_ij, B_ji, B_jj, B_mm.
// f = K u: forward butterflies, 39 products, inverse butterflies (174 operations).
__device__ __forceinline__ constexpr int other_lo(int m) { return m == 0 ? 1 : 0; }
__device__ __forceinline__ constexpr int other_hi(int m) { return m == 2 ? 1 : 2; }

// With 16-bit products (rmode != 0, FP32 only) the transformed displacements are scaled by a
// power of two and rounded to FP16 / BF16, the table holds the unscaled coefficients rounded
// to 16 bits with s_e in C[31], and the products are scaled back by s_e / scale.
template <typename T>
__device__ __forceinline__ void walsh8_sym(cptr_t<T> C, const T (&ue)[24], T (&fe)[24], int32_t rmode = 0) {
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
          if (b < 2 || k != 0) x[a][k] = lo + hi;  // the translation sum x[a][0] is never used
          x[a][k | (1 << b)] = hi - lo;
        }
  T back = T(1);
  if constexpr (sizeof(T) == 4) {
    if (rmode) {
      float mx = 0.0f;
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int k = 1; k < 8; ++k) mx = fmaxf(mx, fabsf(x[a][k]));
      const float sx = pow2_scale(mx);
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int k = 1; k < 8; ++k) x[a][k] = round16(x[a][k] * sx, rmode);
      back = C[31] / sx;
    }
  }
  T y[3][8];
#pragma unroll
  for (int a = 0; a < 3; ++a) y[a][0] = T(0);
#pragma unroll
  for (int h = 0; h < 2; ++h) {  // t = 0 and t = 7
    const int t = 7 * h;
    const T dm = C[2 * h], o = C[2 * h + 1];
    const T x0 = x[0][t ^ 1], x1 = x[1][t ^ 2], x2 = x[2][t ^ 4];
    T sum = x0 + x1 + x2;
    if constexpr (sizeof(T) == 4) {
      if (rmode) sum = round16(sum, rmode);  // a product operand too
    }
    const T os = o * sum;
    y[0][t ^ 1] = fma(dm, x0, os);
    y[1][t ^ 2] = fma(dm, x1, os);
    y[2][t ^ 4] = fma(dm, x2, os);
  }
#pragma unroll
  for (int m = 0; m < 3; ++m) {
    const int i = other_lo(m), j = other_hi(m);
    {
      const int t = 1 << m;
      cptr_t<T> B = C + 4 + 4 * m;
      const T xi = x[i][t ^ (1 << i)], xj = x[j][t ^ (1 << j)];
      y[i][t ^ (1 << i)] = fma(B[1], xj, B[0] * xi);
      y[j][t ^ (1 << j)] = fma(B[3], xj, B[2] * xi);
    }
    {
      const int t = 7 ^ (1 << m);
      cptr_t<T> B = C + 16 + 5 * m;
      const T xi = x[i][t ^ (1 << i)], xj = x[j][t ^ (1 << j)];
      y[i][t ^ (1 << i)] = fma(B[1], xj, B[0] * xi);
      y[j][t ^ (1 << j)] = fma(B[3], xj, B[2] * xi);
      y[m][t ^ (1 << m)] = B[4] * x[m][t ^ (1 << m)];
    }
  }
  if constexpr (sizeof(T) == 4) {
    if (rmode) {
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int k = 1; k < 8; ++k) y[a][k] *= back;
    }
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

// the lane's 16-byte record of local node indices in a regular-cell item
__device__ __forceinline__ uint4 cell8_record(const TiledArgs& a, const CellItem& it, int lane) {
  typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
  const u32x4 v = ld_nt(as_global(reinterpret_cast<const u32x4*>(a.lidx)) + ((it.lidx0 >> 3) + lane));
  return make_uint4(v.x, v.y, v.z, v.w);
}

// Precision forms of the hanging-cell pass with one lane per cell: kernels instantiated with
// RED = false take FP64 state and no 16-bit rounding as compile-time constants; RED = true
// reads them from the argument block.  (The owner-tile pass and the matrix-core hanging pass
// take the product precision and the state storage as template parameters.)
template <bool RED>
__device__ __forceinline__ int32_t state_of(const TiledArgs& a) {
  return RED ? a.state : 0;
}
template <bool RED>
__device__ __forceinline__ int32_t round_of(const TiledArgs& a) {
  return RED ? a.round16 : 0;
}

// product precision (sbfem_prod) -> 16-bit operand rounding of the Walsh product (0 none,
// 1 FP16, 2 BF16)
template <int PROD>
__host__ __device__ constexpr int round_mode() {
  return PROD == 2 ? 1 : (PROD == 3 ? 2 : 0);
}

// A regular 8-node cell: gather from the staged u (FP32: 16-byte float4 nodes, FP64: 3
// doubles), structured Walsh product with the class-scaled table, FP64 LDS atomics into the
// rows of owned corners.
template <bool FP32, int RM>
__device__ __forceinline__ void cell8(const TiledArgs& a, const CellItem& it, const uint4 q, int n_own,
                                      const typename LdsType<FP32>::T* __restrict__ ul, double* __restrict__ fl) {
  using T = typename LdsType<FP32>::T;
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
  walsh8_sym<T>(as_const(FP32 ? (const T*)a.Ws32 : (const T*)a.Ws64) + it.koff, ue, fe, RM);
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

// The mesh of a block (single or batched launch), its argument block for this step (u and
// u_prev swap roles every step), the index of its work unit (tile or hanging-cell item),
// and the step number.  unit_of_block: XCD-contiguous map of blocks onto units.
__device__ __forceinline__ bool block_unit(const MeshRef& single, const MeshRef* refs, const TileWork* work,
                                           int64_t first, int64_t count, int64_t k, int64_t t, TiledArgs& a,
                                           int64_t& ui, int64_t& step) {
  if (t >= count) return false;
  MeshRef r = single;
  ui = first + t;
  if (work) {
    const TileWork w = load_const(as_const(work) + (first + t));
    r = load_const(as_const(refs) + w.mesh);
    ui = w.tile;
  } else if (refs) {
    r = load_const(as_const(refs));
  }
  // k steps after the step recorded in the mesh ref (batched calls advance every mesh together)
  step = r.step + k;
  a = load_const(as_const(r.args) + ((r.parity + k) & 1));
  return true;
}
__device__ __forceinline__ int64_t xcd_unit(int64_t count) {
  const int64_t per = (count + 7) / 8;
  const int64_t b = blockIdx.x;
  return (b % 8) * per + b / 8;
}

// Owned forces start at -P(t_n) b on the tile's load dofs.
__device__ __forceinline__ void tile_loads(const TiledArgs& a, const OwnerTile& tile, int64_t step, double* fl,
                                           int tid, int nt) {
  for (int i = tid; i < tile.n_load; i += nt) {
    const LoadEntry e = load_const(as_const(a.loads) + (tile.load0 + i));
    atomicAdd(fl + e.ldof, -load_time(a.L, (double)step * a.dt) * e.val);
  }
}

// Forces of hanging-node cells on the tile's owned dofs, from the hanging-cell pass (stored
// in FP64 for FP64 products, else in FP32).  A tile next to refined regions holds thousands
// of such rows.  With ROWS > 1 each thread takes ROWS pairs at a time (their loads, then their
// forces, then the sums), so that a round trip serves ROWS rows.  The best ROWS was measured
// per kernel on the pattern-rich and the inclusion meshes (it changes the code the compiler
// schedules around the item loop): four for FP64 products, the compensated state and FP32
// products with FP32 state, two for FP32 products with FP64 state, one for the 16-bit forms
// with FP64 or FP32 state.
template <int PROD, int STATE>
__host__ __device__ constexpr int hang_rows_per_round() {
  return PROD == 0 || STATE == 2 || (PROD == 1 && STATE == 1) ? 4 : (PROD == 1 ? 2 : 1);
}
template <bool FP32, int ROWS>
__device__ __forceinline__ void tile_hang_forces(const TiledArgs& a, const OwnerTile& tile, double* fl, int tid,
                                                 int nt) {
  using RT = typename LdsType<FP32>::T;
  const gptr_t<HangPair> pr = as_global(a.hpairs) + tile.hpair0;
  const gptr_t<RT> res = as_global((const RT*)a.hres);
  const int n = tile.n_hpair;
  if constexpr (ROWS == 1) {
    for (int i = tid; i < n; i += nt) {
      const HangPair h = load_global(pr + i);
      atomicAdd(fl + h.ldof, (double)res[h.res]);
    }
  } else {
    for (int i0 = tid; i0 < n; i0 += ROWS * nt) {
      HangPair h[ROWS];
      RT f[ROWS];
#pragma unroll
      for (int r = 0; r < ROWS; ++r) {
        h[r] = HangPair{-1, 0};
        if (i0 + r * nt < n) h[r] = load_global(pr + (i0 + r * nt));
      }
#pragma unroll
      for (int r = 0; r < ROWS; ++r) f[r] = h[r].ldof >= 0 ? res[h[r].res] : RT(0);
#pragma unroll
      for (int r = 0; r < ROWS; ++r)
        if (h[r].ldof >= 0) atomicAdd(fl + h[r].ldof, (double)f[r]);
    }
  }
}

// Probe histories: if owned dof ldof of the tile is a probe, its u_{n+1} and the central-
// difference acceleration of step n go to the history row of the step.  [e0, e1): the tile's
// probe entries (a handful at most, so they are scanned).
__device__ __forceinline__ void probe_record(const TiledArgs& a, int32_t e0, int32_t e1, int ldof, int64_t step,
                                             double unew, double un, double up) {
  for (int32_t e = e0; e < e1; ++e) {
    const int2 pe = a.probes[e];
    if (pe.x != ldof) continue;
    const int64_t row = step - a.probe_step0;
    if (row < 0 || row >= a.probe_rows) continue;
    const int64_t o = row * a.n_probes + pe.y;
    as_global_mut(a.probe_u)[o] = unew;
    as_global_mut(a.probe_a)[o] = (unew - 2.0 * un + up) / a.dt2;
  }
}

// u_{n+1} of one owned node from its forces, u_n, u_{n-1} and inverse mass (eq. DnMdiag),
// written over u_{n-1}; false if a stored value is not finite
template <int STATE>
__device__ __forceinline__ bool node_update(const TiledArgs& a, int64_t node, const double* f, double un0, double un1,
                                            double un2, double up0, double up1, double up2, double m0, double m1,
                                            double m2, double (&v)[3]) {
  const double inv = 1.0 / (1.0 + a.c), cm = 1.0 - a.c;
  const double v0 = (a.dt2 * m0 * (-f[0]) + 2.0 * un0 - cm * up0) * inv;
  const double v1 = (a.dt2 * m1 * (-f[1]) + 2.0 * un1 - cm * up1) * inv;
  const double v2 = (a.dt2 * m2 * (-f[2]) + 2.0 * un2 - cm * up2) * inv;
  v[0] = v0, v[1] = v1, v[2] = v2;
  state_store(a.um1, STATE, a.ndof, 3 * node + 0, v0);
  state_store(a.um1, STATE, a.ndof, 3 * node + 1, v1);
  state_store(a.um1, STATE, a.ndof, 3 * node + 2, v2);
  return state_finite(STATE, v0) && state_finite(STATE, v1) && state_finite(STATE, v2);
}

// Central-difference update of the owned nodes written over u_{n-1} (or R_int, force-only),
// node by node, with every operand loaded here (tiles that the block does not cover one node
// per thread).  un_lds: u_n of the owned dofs as staged (FP64 staging holds u_n itself).
template <bool FP32, int STATE>
__device__ __forceinline__ void tile_update(const TiledArgs& a, const OwnerTile& tile, int64_t ti, const double* fl,
                                            const double* un_lds, int force_only, int64_t step, int tid, int nt) {
  if (force_only) {
    const int64_t d0 = 3 * tile.own0;
    gmut_t<double> f = as_global_mut(a.f);
    for (int i = tid; i < 3 * tile.n_own; i += nt) f[d0 + i] = fl[i];
    return;
  }
  bool ok = true;
  for (int l = tid; l < tile.n_own; l += nt) {
    const int64_t node = tile.own0 + l;
    const double m0 = minv_load(a.minv, STATE, 3 * node + 0), m1 = minv_load(a.minv, STATE, 3 * node + 1),
                 m2 = minv_load(a.minv, STATE, 3 * node + 2);
    double un[3], up[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      un[c] = FP32 ? state_load(a.u, STATE, a.ndof, 3 * node + c) : un_lds[3 * l + c];
      up[c] = state_load(a.um1, STATE, a.ndof, 3 * node + c);
    }
    double v[3];
    ok &= node_update<STATE>(a, node, fl + 3 * l, un[0], un[1], un[2], up[0], up[1], up[2], m0, m1, m2, v);
    if (a.n_probes) {
      const int32_t e0 = a.probe_ptr[ti], e1 = a.probe_ptr[ti + 1];
#pragma unroll
      for (int c = 0; c < 3; ++c)
        if (e1 > e0) probe_record(a, e0, e1, 3 * l + c, step, v[c], un[c], up[c]);
    }
  }
  if (!ok) atomicMin(a.flag, (unsigned long long)step);
}

// Stage u_n of the tile's local nodes in LDS (owned nodes first, then the tile's node list)
// and clear the owned forces.  FP32 products keep u minus the displacement of the tile's
// first owned node, so that only variations across the tile are rounded.
template <bool FP32, int STATE>
__device__ __forceinline__ void tile_stage(const TiledArgs& a, const OwnerTile& tile, typename LdsType<FP32>::T* ul,
                                           double* fl, int tid, int nt) {
  gptr_t<int32_t> nodelist = as_global(a.nodelist);
  const int n_own = tile.n_own;
  constexpr int32_t sm = STATE;
  double r0 = 0.0, r1 = 0.0, r2 = 0.0;
  if constexpr (FP32) {
    r0 = state_load(a.u, sm, a.ndof, 3 * tile.own0 + 0);
    r1 = state_load(a.u, sm, a.ndof, 3 * tile.own0 + 1);
    r2 = state_load(a.u, sm, a.ndof, 3 * tile.own0 + 2);
  }
  for (int l = tid; l < tile.n_local; l += nt) {
    const int64_t g = l < n_own ? tile.own0 + l : (int64_t)nodelist[tile.node0 + l - n_own];
    const double x = state_load(a.u, sm, a.ndof, 3 * g + 0);
    const double y = state_load(a.u, sm, a.ndof, 3 * g + 1);
    const double z = state_load(a.u, sm, a.ndof, 3 * g + 2);
    if constexpr (FP32) {
      reinterpret_cast<float4*>(ul)[l] = make_float4((float)(x - r0), (float)(y - r1), (float)(z - r2), 0.0f);
    } else {
      ul[3 * l + 0] = x;
      ul[3 * l + 1] = y;
      ul[3 * l + 2] = z;
    }
  }
  for (int i = tid; i < 3 * n_own; i += nt) fl[i] = 0;
}

// The same staging with every global load issued up front, for tiles whose owned nodes fit
// one per thread and whose other local nodes two per thread: the caller has loaded the
// thread's halo node ids (h0 = halo entry tid, h1 = entry tid + nt, -1 if none) as its
// first loads, so a tile costs two dependent round trips to memory (ids, then u), not two
// per node a thread stages.  In two halves (loads, then LDS stores) so that the caller can
// request its first cell record in between.
struct StagedNodes {
  double r[3], vo[3], v0[3], v1[3];
};

// u_n at a block-uniform index through the constant space (scalar loads): u_n is read-only
// during the pass (u_{n+1} goes to the other buffer)
template <int STATE>
__device__ __forceinline__ double state_load_uniform(const void* p, int64_t ndof, int64_t i) {
  if constexpr (STATE == 0) return as_const((const double*)p)[i];
  const cptr_t<float> q = as_const((const float*)p);
  if constexpr (STATE == 1) return (double)q[i];
  return (double)q[i] + (double)q[ndof + i];
}

template <bool FP32, int STATE>
__device__ __forceinline__ StagedNodes stage_loads(const TiledArgs& a, int64_t own0, int n_own, int32_t h0,
                                                   int32_t h1, int tid) {
  constexpr int32_t sm = STATE;
  StagedNodes v{};
  if constexpr (FP32) {
#pragma unroll
    for (int c = 0; c < 3; ++c) v.r[c] = state_load_uniform<STATE>(a.u, a.ndof, 3 * own0 + c);
  }
  if (tid < n_own) {
#pragma unroll
    for (int c = 0; c < 3; ++c) v.vo[c] = state_load(a.u, sm, a.ndof, 3 * (own0 + tid) + c);
  }
  if (h0 >= 0) {
#pragma unroll
    for (int c = 0; c < 3; ++c) v.v0[c] = state_load(a.u, sm, a.ndof, 3 * (int64_t)h0 + c);
  }
  if (h1 >= 0) {
#pragma unroll
    for (int c = 0; c < 3; ++c) v.v1[c] = state_load(a.u, sm, a.ndof, 3 * (int64_t)h1 + c);
  }
  return v;
}

template <bool FP32>
__device__ __forceinline__ void stage_stores(const StagedNodes& v, int n_own, int32_t h0, int32_t h1,
                                             typename LdsType<FP32>::T* ul, double* fl, int tid, int nt) {
  auto put = [&](int l, double x, double y, double z) {
    if constexpr (FP32) {
      reinterpret_cast<float4*>(ul)[l] =
          make_float4((float)(x - v.r[0]), (float)(y - v.r[1]), (float)(z - v.r[2]), 0.0f);
    } else {
      ul[3 * l + 0] = x;
      ul[3 * l + 1] = y;
      ul[3 * l + 2] = z;
    }
  };
  if (tid < n_own) put(tid, v.vo[0], v.vo[1], v.vo[2]);
  if (h0 >= 0) put(n_own + tid, v.v0[0], v.v0[1], v.v0[2]);
  if (h1 >= 0) put(n_own + nt + tid, v.v1[0], v.v1[1], v.v1[2]);
  for (int i = tid; i < 3 * n_own; i += nt) fl[i] = 0;
}

// Hanging-node cell of NN nodes in the hanging-cell pass: u_e gathered from global memory,
// oriented, 16-bit operands if asked, dense master product over all rows scaled by s_e;
// row i of the item's lane goes to hres[res0 + 64 i + lane] (the owner tiles add it).
template <int NN>
constexpr int k_row_stride() {
  return (3 * NN + 3) & ~3;
}

template <int NN, bool FP32, bool RED>
__device__ __forceinline__ void hang_cell(const TiledArgs& a, const HangItem& it, int lane,
                                          const typename LdsType<FP32>::T* __restrict__ Kl) {
  constexpr int ND = 3 * NN;
  constexpr int NDP = k_row_stride<NN>();
  using T = typename LdsType<FP32>::T;
  const int64_t cell = it.cell0 + lane;
  int p0, p1, p2;
  double s0, s1, s2;
  decode_orient(as_global(a.horient)[cell], p0, p1, p2, s0, s1, s2);
  const double se = as_const(a.matE)[as_global(a.hmaterial)[cell]] * ldexp(a.h0, -(int)as_global(a.hlevel)[cell]);
  const gptr_t<int32_t> conn = as_global(a.hconn);
  const int32_t sm = state_of<RED>(a);
  int64_t g[NN];
#pragma unroll
  for (int k = 0; k < NN; ++k) g[k] = conn[it.conn0 + (int64_t)k * it.count + lane];
  // oriented nodal displacements; reduced products take differences to node 0 (K_p
  // annihilates translations) so that only variations across the cell are rounded
  T ue[ND];
  {
    double r[3] = {0.0, 0.0, 0.0};
    if constexpr (FP32) {
#pragma unroll
      for (int c = 0; c < 3; ++c) r[c] = state_load(a.u, sm, a.ndof, 3 * g[0] + c);
    }
#pragma unroll
    for (int k = 0; k < NN; ++k) {
      const T x = (T)(state_load(a.u, sm, a.ndof, 3 * g[k] + 0) - r[0]);
      const T y = (T)(state_load(a.u, sm, a.ndof, 3 * g[k] + 1) - r[1]);
      const T z = (T)(state_load(a.u, sm, a.ndof, 3 * g[k] + 2) - r[2]);
      ue[3 * k + 0] = (T)s0 * pick3t<T>(p0, x, y, z);
      ue[3 * k + 1] = (T)s1 * pick3t<T>(p1, x, y, z);
      ue[3 * k + 2] = (T)s2 * pick3t<T>(p2, x, y, z);
    }
  }
  double post = se;  // applied to each product row
  if constexpr (FP32) {
    const int32_t rm = round_of<RED>(a);
    if (rm) {  // 16-bit operands: scale by a power of two, round, undo the scale after
      float mx = 0.0f;
#pragma unroll
      for (int j = 0; j < ND; ++j) mx = fmaxf(mx, fabsf(ue[j]));
      const float su = pow2_scale(mx);
#pragma unroll
      for (int j = 0; j < ND; ++j) ue[j] = round16(ue[j] * su, rm);
      post = se / (double)su;
    }
  }
  const gmut_t<T> res = as_global_mut((T*)a.hres) + it.res0 + lane;
#pragma unroll
  for (int k = 0; k < NN; ++k) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const int i = 3 * k + c;
      T acc = 0;
#pragma unroll
      for (int j = 0; j < ND; ++j) acc = fma(Kl[i * NDP + j], ue[j], acc);
      const double sc = c == 0 ? s0 : (c == 1 ? s1 : s2);
      res[(int64_t)i * 64] = (T)(sc * post * (double)acc);  // to node k, component pi(c)
    }
  }
}

// Hanging-cell pass: one wave per item; the items of a block share one pattern (the set-up
// pads every pattern's items to whole blocks), whose master matrix the block stages in LDS
// once (rows padded to a multiple of 4 entries) so the waves read its rows as LDS broadcasts.
// FP32 products are held to 128 VGPRs (4 waves per SIMD); the FP64 variant keeps the register
// file (its spills would cost more).
template <bool FP32, bool RED>
__global__ void __launch_bounds__(512, FP32 ? 4 : 1) tiled_hang(MeshRef single, const MeshRef* __restrict__ refs,
                                                                 const TileWork* __restrict__ work, int64_t first,
                                                                 int64_t count, int64_t k) {
  using T = typename LdsType<FP32>::T;
  extern __shared__ double lds[];
  T* Kl = (T*)lds;
  const int per_block = blockDim.x >> 6;
  const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6)), lane = threadIdx.x & 63;
  const int64_t t0 = (int64_t)blockIdx.x * per_block;
  TiledArgs a;
  int64_t ii, step;
  if (!block_unit(single, refs, work, first, count, k, t0, a, ii, step)) return;  // uniform in the block
  {
    // the block's pattern: that of its first item (every item of the block has it)
    const HangItem i0 = load_const(as_const(a.hitems) + ii);
    const int nd = 3 * i0.nn, ndp = (nd + 3) & ~3;
    const gptr_t<T> K = as_global(FP32 ? (const T*)(a.K32 + i0.koff) : (const T*)(a.K64 + i0.koff));
    for (int e = threadIdx.x; e < nd * ndp; e += blockDim.x) {
      const int r = e / ndp, c = e - r * ndp;
      Kl[e] = c < nd ? K[r * nd + c] : T(0);
    }
  }
  __syncthreads();
  if (!block_unit(single, refs, work, first, count, k, t0 + wave, a, ii, step)) return;
  const HangItem it = load_const(as_const(a.hitems) + ii);
  if (lane >= it.count) return;
#define SBFEM_TCASE(N) \
  case N:              \
    hang_cell<N, FP32, RED>(a, it, lane, Kl); \
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

// One owner tile (steps 1-4 of the pass).  own0 and n_own come from the tile index and the
// tile size, so that the loads that need nothing else (the update operands of the thread's
// owned node -- u_{n-1} and its inverse mass -- and, with `ids`, the staging of the owned node
// and of the halo nodes h0, h1) are issued while the tile record is still on its way; the
// record feeds the item loop, the loads and the hanging-cell forces.  With `ids` each thread
// owns one node, whose staged u_n also serves the update.
template <int PROD, int STATE>
__device__ __forceinline__ void owner_tile(const TiledArgs& a, const OwnerTile& tile, int64_t ti, int64_t own0,
                                           int n_own, int64_t step, int force_only, bool ids, int32_t h0, int32_t h1,
                                           double* lds) {
  constexpr bool FP32 = PROD != 0;
  using T = typename LdsType<FP32>::T;
  double* fl = lds;
  // the staged u starts 16-byte aligned (FP32 staging reads float4 nodes)
  T* ul = (T*)(lds + ((3 * (int64_t)n_own + 1) & ~(int64_t)1));
  const int tid = threadIdx.x;
  const int nt = blockDim.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int n_waves = nt >> 6;
  // update operands of the thread's owned dofs tid, tid + nt, tid + 2 nt (consecutive dofs in
  // consecutive lanes): u_{n-1}, the inverse mass and, for FP32 products, u_n
  constexpr int kPre = 3;
  const int n_dof = 3 * n_own;
  const bool pre = !force_only && n_dof <= kPre * nt;  // uniform
  double pu[kPre], pp[kPre], pm[kPre];
  if (pre) {
    const int64_t d0 = 3 * own0;
#pragma unroll
    for (int j = 0; j < kPre; ++j) {
      const int i = tid + j * nt;
      pu[j] = pp[j] = pm[j] = 0.0;
      if (i < n_dof) {
        if constexpr (FP32) pu[j] = state_load(a.u, STATE, a.ndof, d0 + i);
        pp[j] = state_load_nt(a.um1, STATE, a.ndof, d0 + i);
        pm[j] = minv_load_nt(a.minv, STATE, d0 + i);
      }
    }
  }
  StagedNodes sv{};
  if (ids) sv = stage_loads<FP32, STATE>(a, own0, n_own, h0, h1, tid);
  cptr_t<CellItem> items = as_const(a.items) + tile.item0;
  int w = wave;
  CellItem it{};
  uint4 q = make_uint4(0, 0, 0, 0);
  if (w < tile.n_items) {
    it = load_const(items + w);
    if (lane < it.count) q = cell8_record(a, it, lane);
  }
  if (ids)
    stage_stores<FP32>(sv, n_own, h0, h1, ul, fl, tid, nt);
  else
    tile_stage<FP32, STATE>(a, tile, ul, fl, tid, nt);
  __syncthreads();
  if (!force_only) tile_loads(a, tile, step, fl, tid, nt);
  tile_hang_forces<FP32, hang_rows_per_round<PROD, STATE>()>(a, tile, fl, tid, nt);
  while (w < tile.n_items) {
    // the next record is requested before this cell's work
    const int wn = w + n_waves;
    CellItem itn{};
    uint4 qn = make_uint4(0, 0, 0, 0);
    if (wn < tile.n_items) {
      itn = load_const(items + wn);
      if (lane < itn.count) qn = cell8_record(a, itn, lane);
    }
    if (lane < it.count) cell8<FP32, round_mode<PROD>()>(a, it, q, n_own, ul, fl);
    w = wn;
    it = itn;
    q = qn;
  }
  __syncthreads();
  if (pre) {
    const int64_t d0 = 3 * own0;
    const double inv = 1.0 / (1.0 + a.c), cm = 1.0 - a.c;
    bool ok = true;
#pragma unroll
    for (int j = 0; j < kPre; ++j) {
      const int i = tid + j * nt;
      if (i < n_dof) {
        const double un = FP32 ? pu[j] : (double)ul[i];
        const double v = (a.dt2 * pm[j] * (-fl[i]) + 2.0 * un - cm * pp[j]) * inv;
        state_store_nt(a.um1, STATE, a.ndof, d0 + i, v);
        ok &= state_finite(STATE, v);
        if (a.n_probes) {  // uniform
          const int32_t e0 = a.probe_ptr[ti], e1 = a.probe_ptr[ti + 1];
          if (e1 > e0) probe_record(a, e0, e1, i, step, v, un, pp[j]);
        }
      }
    }
    if (!ok) atomicMin(a.flag, (unsigned long long)step);
  } else {
    tile_update<FP32, STATE>(a, tile, ti, fl, (const double*)ul, force_only, step, tid, nt);
  }
}

// Owner-tile pass, one block per work unit (a tile; in a batched launch a (mesh, tile)).
// With halo lists at a fixed stride and tiles that fit the block (owned nodes one per
// thread, halo nodes two per thread), the halo ids are the block's first loads.
// PROD: sbfem_prod of the Walsh product (FP64; FP32; FP16 / BF16 operands with FP32
// arithmetic); STATE: sbfem_state of u_n, u_{n-1} (and of the inverse mass: FP32 with FP32
// state, else FP64).  The reduced-product forms fit 80 VGPRs (6 waves per SIMD: three blocks
// per CU); the compensated state asks for that bound, which it would otherwise just miss.
template <int PROD, int STATE>
__global__ void __launch_bounds__(512, PROD != 0 && STATE == 2 ? 6 : 1) tiled_step8(MeshRef single, const MeshRef* __restrict__ refs,
                                                   const TileWork* __restrict__ work, int64_t first,
                                                   int64_t count, int64_t k, int force_only) {
  extern __shared__ double lds[];
  TiledArgs a;
  int64_t ti, step;
  if (!block_unit(single, refs, work, first, count, k, xcd_unit(count), a, ti, step)) return;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int64_t own0 = ti * a.tile_nodes;
  const int64_t n_nodes = a.ndof / 3;
  const int n_own = (int)(n_nodes - own0 < a.tile_nodes ? n_nodes - own0 : a.tile_nodes);
  const int64_t H = a.halo_stride;
  const bool ids = H > 0 && n_own <= nt && H <= 2 * nt;
  int32_t h0 = -1, h1 = -1;
  if (ids) {
    const gptr_t<int32_t> nl = as_global(a.nodelist) + ti * H;
    if (tid < H) h0 = nl[tid];
    if (tid + nt < H) h1 = nl[tid + nt];
  }
  const OwnerTile tile = load_const(as_const(a.tiles) + ti);
  owner_tile<PROD, STATE>(a, tile, ti, own0, n_own, step, force_only, ids, h0, h1, lds);
}

}  // namespace sbfem
