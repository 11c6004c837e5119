// Hanging-cell pass on the matrix cores (included by the per-precision translation units).
#pragma once

#include <type_traits>
#include <utility>

#include "tiled_kernel.h"

// =============================================================================================
// Every cell that is not a regular 8-node cell is computed once per step, in items of up to
// 64 cells of one pattern (eqs. Rinte, Rintep, KM_scale; orientation as in Sec. 3.2.2).  An
// item is the dense product F = K_p U, K_p the n x n master matrix (n = 3 x nodes, 33..78)
// and U the oriented displacements of the item's cells (n x 64): one block of four waves per
// item, wave w taking cells 16w .. 16w + 15 as the columns of 16 x 16 output tiles.
//
// Operand layouts (16 x 16 tiles, lane l, q = l & 15, p = l >> 4):
//  * FP64 / FP32 products, 16x16x4 steps: A = K[16 rt + q][4 t + p], B = U[4 t + p][q],
//    so lane l gathers the dofs j = 4 t + p of its cell; D (value v of the lane): column q,
//    row 16 rt + 4 p + v for FP32 and 16 rt + p + 4 v for FP64 (checked on the device).
//  * FP16 / BF16 products (FP32 accumulation), 16x16x32 steps: A = K[16 rt + q][32 t + 8 p + i]
//    and B = U[32 t + 8 p + i][q] for i < 8 (one 16-byte LDS read of a K row).
// The column of a lane's D values is its own cell, so the signs of the back-transformation
// and the cell scale s_e = E h apply in the lane that gathered the cell.  The master matrix is
// staged in LDS once per block (zero-padded to whole tiles); U stays in registers.
// Row i of cell c goes to hres[res0 + 64 i + c] (FP64 for FP64 products, else FP32), which
// the owner tiles add to their owned dofs.

namespace sbfem {

typedef float mma_f4 __attribute__((ext_vector_type(4)));
typedef double mma_d4 __attribute__((ext_vector_type(4)));
typedef __bf16 mma_bf8 __attribute__((ext_vector_type(8)));
typedef _Float16 mma_h8 __attribute__((ext_vector_type(8)));

constexpr int kHangMaxDof = 78;
constexpr int kHangRowTiles = (kHangMaxDof + 15) / 16;  // 5

// Row stride (elements) of the staged master matrix: FP64/FP32 one column past a multiple of
// 4 (A reads of 16 rows x 4 columns fall in distinct banks), 16-bit a multiple of 32 plus 8
// (16-byte aligned rows).
template <int PREC>
__host__ __device__ constexpr int hang_kstride(int nd) {
  return PREC <= 1 ? ((nd + 3) & ~3) + 1 : ((nd + 31) & ~31) + 8;
}
template <int PREC>
__host__ __device__ constexpr int hang_lds_bytes(int nd) {
  return 16 * ((nd + 15) / 16) * hang_kstride<PREC>(nd) * (PREC == 0 ? 8 : (PREC == 1 ? 4 : 2));
}

template <int PREC>
struct HangTypes;
template <>
struct HangTypes<0> {
  using K = double;
  using Res = double;
};
template <>
struct HangTypes<1> {
  using K = float;
  using Res = float;
};
template <>
struct HangTypes<2> {
  using K = _Float16;
  using Res = float;
};
template <>
struct HangTypes<3> {
  using K = __bf16;
  using Res = float;
};

// the oriented displacement of dof j (= 3 node + a) of the lane's cell, FP64, minus node 0's
// when `centre` (reduced products: only the variation across the cell is rounded)
// A lane's dofs j cycle through the three components a = j mod 3 in a fixed order, so the
// orientation of its cell is held rotated: component slot k (k = 0, 1, 2) carries the source
// axis pi(a), the sign s_a and the oriented displacement of node 0, for a = (base + k) mod 3.
// Only the rotation is chosen at run time; slot k is then a compile-time register.
struct HangRot {
  int src0, src1, src2;
  double sg0, sg1, sg2;
  double r0, r1, r2;
};
__device__ __forceinline__ int pick3i(int a, int x, int y, int z) { return a == 0 ? x : (a == 1 ? y : z); }
__device__ __forceinline__ double pick3d(int a, double x, double y, double z) { return a == 0 ? x : (a == 1 ? y : z); }

template <int STATE, bool CENTRE>
__device__ __forceinline__ HangRot hang_rot(const TiledArgs& a, int base, int p0, int p1, int p2, double s0, double s1,
                                            double s2, int64_t g0, bool live) {
  HangRot h;
  const int a0 = base, a1 = (base + 1) % 3, a2 = (base + 2) % 3;
  h.src0 = pick3i(a0, p0, p1, p2);
  h.src1 = pick3i(a1, p0, p1, p2);
  h.src2 = pick3i(a2, p0, p1, p2);
  h.sg0 = pick3d(a0, s0, s1, s2);
  h.sg1 = pick3d(a1, s0, s1, s2);
  h.sg2 = pick3d(a2, s0, s1, s2);
  h.r0 = h.r1 = h.r2 = 0.0;
  if (CENTRE && live) {
    h.r0 = h.sg0 * state_load(a.u, STATE, a.ndof, 3 * g0 + h.src0);
    h.r1 = h.sg1 * state_load(a.u, STATE, a.ndof, 3 * g0 + h.src1);
    h.r2 = h.sg2 * state_load(a.u, STATE, a.ndof, 3 * g0 + h.src2);
  }
  return h;
}
// f(std::integral_constant<int, I>) for I = 0 .. N-1, unrolled at compile time
template <class F, int... I>
__device__ __forceinline__ void static_for_impl(F&& f, std::integer_sequence<int, I...>) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(f, std::make_integer_sequence<int, N>{});
}

template <int K>
__device__ __forceinline__ void rot_slot(const HangRot& h, int& src, double& sg, double& r) {
  if constexpr (K == 0) {
    src = h.src0, sg = h.sg0, r = h.r0;
  } else if constexpr (K == 1) {
    src = h.src1, sg = h.sg1, r = h.r1;
  } else {
    src = h.src2, sg = h.sg2, r = h.r2;
  }
}
template <int K>
__device__ __forceinline__ double rot_sign(const HangRot& h) {
  return K == 0 ? h.sg0 : (K == 1 ? h.sg1 : h.sg2);
}

// the oriented (and, for reduced products, centred) displacement of a dof of the lane's cell
// at node g, its component taken from rotation slot K
template <int STATE, int K>
__device__ __forceinline__ double hang_dof_at(const TiledArgs& a, int32_t g, const HangRot& h) {
  int src;
  double sg, r;
  rot_slot<K>(h, src, sg, r);
  return sg * state_load(a.u, STATE, a.ndof, 3 * (int64_t)g + src) - r;
}

template <int PREC, int STATE>
__global__ void __launch_bounds__(256) tiled_hang_mma(MeshRef single, const MeshRef* __restrict__ refs,
                                                      const TileWork* __restrict__ work, int64_t first,
                                                      int64_t count, int64_t kstep) {
  using KT = typename HangTypes<PREC>::K;
  using RT = typename HangTypes<PREC>::Res;
  extern __shared__ double lds_raw[];
  KT* Kl = (KT*)lds_raw;
  TiledArgs a;
  int64_t ii, step;
  if (!block_unit(single, refs, work, first, count, kstep, blockIdx.x, a, ii, step)) return;
  const HangItem it = load_const(as_const(a.hitems) + ii);
  if (it.count == 0) return;  // padding item (uniform in the block)
  const int nd = 3 * it.nn;
  const int KP = hang_kstride<PREC>(nd);
  const int rows = 16 * ((nd + 15) / 16);
  const int tid = threadIdx.x;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int q = lane & 15, p = lane >> 4;
  const int c = 16 * wave + q;  // the lane's cell in the item
  const bool live = c < it.count;

  // the lane's cell: orientation, scale, and (reduced products) node 0 for centring
  int p0 = 0, p1 = 1, p2 = 2;
  double s0 = 1.0, s1 = 1.0, s2 = 1.0, se = 0.0;
  int64_t g0 = 0;
  const gptr_t<int32_t> conn = as_global(a.hconn);
  if (live) {
    const int64_t cell = it.cell0 + c;
    decode_orient(as_global(a.horient)[cell], p0, p1, p2, s0, s1, s2);
    se = as_const(a.matE)[as_global(a.hmaterial)[cell]] * ldexp(a.h0, -(int)as_global(a.hlevel)[cell]);
    g0 = conn[it.conn0 + c];
  }
  // output rows i = 16 rt + 4 p + v have component (p + rt + v) mod 3
  const HangRot ho = hang_rot<STATE, false>(a, p % 3, p0, p1, p2, s0, s1, s2, g0, live);

  // K_p is staged in LDS first, in batches of a few elements per thread (few registers: a CU
  // then holds six blocks, so the items of a step mostly fit in one round of blocks), then the
  // lane gathers its cell's displacements.
  const int n_k = nd * nd;
  using GT = typename std::conditional<PREC == 0, double, float>::type;  // K32: FP32 or 16-bit-rounded
  const float inv_nd = 1.0f / (float)nd;
  auto put_k = [&](int e, GT v) {
    const int r = (int)(((float)e + 0.5f) * inv_nd);  // exact for e < 2^22
    Kl[r * KP + (e - r * nd)] = (KT)v;
  };
  auto pad_k = [&]() {  // zero padding: columns nd .. KP-1 of every row, and rows nd .. rows-1
    const int padc = KP - nd;
    for (int e = tid; e < rows * padc; e += 256) {
      const int r = e / padc;
      Kl[r * KP + nd + (e - r * padc)] = KT(0);
    }
    for (int e = tid; e < (rows - nd) * nd; e += 256) Kl[(nd + e / nd) * KP + e % nd] = KT(0);
  };
  // K_p into LDS, rows and columns zero-padded to whole tiles, 8 elements per thread at a time
  auto stage_k_batched = [&]() {
    const gptr_t<GT> K = as_global(PREC == 0 ? (const GT*)(a.K64 + it.koff) : (const GT*)(a.K32 + it.koff));
    constexpr int kBatch = 8;
    for (int e0 = 0; e0 < n_k; e0 += 256 * kBatch) {
      GT v[kBatch];
#pragma unroll
      for (int b = 0; b < kBatch; ++b) {
        const int e = e0 + b * 256 + tid;
        v[b] = e < n_k ? K[e] : GT(0);
      }
#pragma unroll
      for (int b = 0; b < kBatch; ++b) {
        const int e = e0 + b * 256 + tid;
        if (e < n_k) put_k(e, v[b]);
      }
    }
    pad_k();
  };

  const gmut_t<RT> res = as_global_mut((RT*)a.hres) + it.res0 + c;
  if constexpr (PREC <= 1) {
    // ---- FP64 / FP32: 16x16x4 steps over the columns j = 4 t + p ----
    constexpr int TMAX = (kHangMaxDof + 3) / 4;  // 20
    using VT = typename HangTypes<PREC>::K;
    VT b[TMAX];
    const int T = (nd + 3) / 4;
    // dofs j = 4 t + p have component (t + p) mod 3: the output rotation
    const HangRot hi = hang_rot<STATE, PREC != 0>(a, p % 3, p0, p1, p2, s0, s1, s2, g0, live);
    const int jmax = live ? nd : 0;
    stage_k_batched();
    int32_t gi[TMAX];
    static_for<TMAX>([&](auto tc) {
      constexpr int t = decltype(tc)::value;
      const int j = 4 * t + p;
      gi[t] = t < T && j < jmax ? conn[it.conn0 + (int64_t)(j / 3) * it.count + c] : -1;
    });
    static_for<TMAX>([&](auto tc) {
      constexpr int t = decltype(tc)::value;
      b[t] = VT(0);
      if (gi[t] >= 0) b[t] = (VT)hang_dof_at<STATE, t % 3>(a, gi[t], hi);
    });
    __syncthreads();  // K staged
    using AT = typename std::conditional<PREC == 0, mma_d4, mma_f4>::type;
    AT acc[kHangRowTiles];
#pragma unroll
    for (int rt = 0; rt < kHangRowTiles; ++rt) acc[rt] = AT{0, 0, 0, 0};
    const int R = rows / 16;
#pragma unroll
    for (int t = 0; t < TMAX; ++t) {
      if (t < T) {  // uniform
#pragma unroll
        for (int rt = 0; rt < kHangRowTiles; ++rt) {
          if (rt < R) {  // uniform
            const VT av = Kl[(16 * rt + q) * KP + 4 * t + p];
            if constexpr (PREC == 0)
              acc[rt] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, b[t], acc[rt], 0, 0, 0);
            else
              acc[rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, b[t], acc[rt], 0, 0, 0);
          }
        }
      }
    }
    if (!live) return;
    static_for<kHangRowTiles>([&](auto rc) {
      constexpr int rt = decltype(rc)::value;
      if (rt < R) {
        static_for<4>([&](auto vc) {
          constexpr int v = decltype(vc)::value;
          // D rows of lane l: 4 p + v (FP32 16x16x4), p + 4 v (FP64 16x16x4); both have
          // component (rt + p + v) mod 3
          const int i = 16 * rt + (PREC == 0 ? p + 4 * v : 4 * p + v);
          if (i < nd) res[(int64_t)i * 64] = (RT)(rot_sign<(rt + v) % 3>(ho) * se * (double)acc[rt][v]);
        });
      }
    });
  } else {
    // ---- FP16 / BF16 operands, FP32 accumulation: 16x16x32 steps over j = 32 t + 8 p + i ----
    constexpr int TMAX = (kHangMaxDof + 31) / 32;  // 3
    float u[TMAX][8];
    const int T = (nd + 31) / 32;
    float mx = 0.0f;
    // dofs j = 32 t + 8 p + i have component (2 p + 2 t + i) mod 3
    const HangRot hi = hang_rot<STATE, true>(a, (2 * p) % 3, p0, p1, p2, s0, s1, s2, g0, live);
    const int jmax = live ? nd : 0;
    int32_t gi[TMAX][8];
    static_for<TMAX>([&](auto tc) {
      constexpr int t = decltype(tc)::value;
      static_for<8>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        const int j = 32 * t + 8 * p + i;
        gi[t][i] = t < T && j < jmax ? conn[it.conn0 + (int64_t)(j / 3) * it.count + c] : -1;
      });
    });
    stage_k_batched();
    static_for<TMAX>([&](auto tc) {
      constexpr int t = decltype(tc)::value;
      static_for<8>([&](auto ic) {
        constexpr int i = decltype(ic)::value;
        u[t][i] = 0.0f;
        if (gi[t][i] >= 0) u[t][i] = (float)hang_dof_at<STATE, (2 * t + i) % 3>(a, gi[t][i], hi);
        mx = fmaxf(mx, fabsf(u[t][i]));
      });
    });
    // FP16: a power of two per cell brings its largest value into [1, 2) (the cell's dofs are
    // spread over the lanes q, q + 16, q + 32, q + 48)
    float scale = 1.0f;
    if constexpr (PREC == 2) {
      mx = fmaxf(mx, __shfl_xor(mx, 16));
      mx = fmaxf(mx, __shfl_xor(mx, 32));
      scale = pow2_scale(mx);
    }
    using BT = typename std::conditional<PREC == 2, mma_h8, mma_bf8>::type;
    BT b[TMAX];
#pragma unroll
    for (int t = 0; t < TMAX; ++t)
#pragma unroll
      for (int i = 0; i < 8; ++i) b[t][i] = (KT)(u[t][i] * scale);
    __syncthreads();  // K staged
    mma_f4 acc[kHangRowTiles];
#pragma unroll
    for (int rt = 0; rt < kHangRowTiles; ++rt) acc[rt] = mma_f4{0, 0, 0, 0};
    const int R = rows / 16;
#pragma unroll
    for (int t = 0; t < TMAX; ++t) {
      if (t < T) {  // uniform
#pragma unroll
        for (int rt = 0; rt < kHangRowTiles; ++rt) {
          if (rt < R) {  // uniform
            const BT av = *reinterpret_cast<const BT*>(Kl + (16 * rt + q) * KP + 32 * t + 8 * p);
            if constexpr (PREC == 2)
              acc[rt] = __builtin_amdgcn_mfma_f32_16x16x32_f16(av, b[t], acc[rt], 0, 0, 0);
            else
              acc[rt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, b[t], acc[rt], 0, 0, 0);
          }
        }
      }
    }
    if (!live) return;
    const double post = se / (double)scale;
    static_for<kHangRowTiles>([&](auto rc) {
      constexpr int rt = decltype(rc)::value;
      if (rt < R) {
        static_for<4>([&](auto vc) {
          constexpr int v = decltype(vc)::value;
          const int i = 16 * rt + 4 * p + v;
          if (i < nd) res[(int64_t)i * 64] = (RT)(rot_sign<(rt + v) % 3>(ho) * post * (double)acc[rt][v]);
        });
      }
    });
  }
}

}  // namespace sbfem
