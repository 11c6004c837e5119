// Element kernels of the atomic and colour assemblies (template, included by the units).
#pragma once

#include "device_common.h"

namespace sbfem {

// One cell: gather + orient, K_p u_e (FP64 or FP32), inverse orient, scatter.
template <int NN, bool FP32, bool ATOMIC>
__device__ __forceinline__ void cell_force(const Tile& t, int lane, const double* __restrict__ u,
                                           double* __restrict__ f, const int32_t* __restrict__ conn,
                                           const uint8_t* __restrict__ orient,
                                           const uint8_t* __restrict__ level,
                                           const uint8_t* __restrict__ material,
                                           const double* __restrict__ matE, double h0,
                                           const double* __restrict__ K64,
                                           const float* __restrict__ K32) {
  constexpr int ND = 3 * NN;
  const int64_t cell = t.cell0 + lane;
  int p0, p1, p2;
  double s0, s1, s2;
  decode_orient(orient[cell], p0, p1, p2, s0, s1, s2);
  const double se = matE[material[cell]] * ldexp(h0, -(int)level[cell]);
  int32_t nd[NN];
#pragma unroll
  for (int k = 0; k < NN; ++k) nd[k] = conn[t.conn0 + (int64_t)k * t.stride + lane];

  if constexpr (!FP32) {
    double ue[ND];
#pragma unroll
    for (int k = 0; k < NN; ++k) {
      const double* q = u + 3 * (int64_t)nd[k];
      const double x = q[0], y = q[1], z = q[2];
      ue[3 * k + 0] = s0 * pick3(p0, x, y, z);
      ue[3 * k + 1] = s1 * pick3(p1, x, y, z);
      ue[3 * k + 2] = s2 * pick3(p2, x, y, z);
    }
    const double* Kp = K64 + t.koff;
#pragma unroll
    for (int k = 0; k < NN; ++k) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const int i = 3 * k + a;
        double acc = 0.0;
#pragma unroll
        for (int j = 0; j < ND; ++j) acc = fma(Kp[i * ND + j], ue[j], acc);
        const int pa = a == 0 ? p0 : (a == 1 ? p1 : p2);
        const double sa = a == 0 ? s0 : (a == 1 ? s1 : s2);
        add_force(f, 3 * (int64_t)nd[k] + pa, sa * se * acc, ATOMIC);
      }
    }
  } else {
    // rigid translation removed before rounding to FP32 (K_p annihilates it)
    const double* q0 = u + 3 * (int64_t)nd[0];
    const double rx = q0[0], ry = q0[1], rz = q0[2];
    float ue[ND];
#pragma unroll
    for (int k = 0; k < NN; ++k) {
      const double* q = u + 3 * (int64_t)nd[k];
      const double x = q[0] - rx, y = q[1] - ry, z = q[2] - rz;
      ue[3 * k + 0] = (float)(s0 * pick3(p0, x, y, z));
      ue[3 * k + 1] = (float)(s1 * pick3(p1, x, y, z));
      ue[3 * k + 2] = (float)(s2 * pick3(p2, x, y, z));
    }
    const float* Kp = K32 + t.koff;
#pragma unroll
    for (int k = 0; k < NN; ++k) {
#pragma unroll
      for (int a = 0; a < 3; ++a) {
        const int i = 3 * k + a;
        float acc = 0.0f;
#pragma unroll
        for (int j = 0; j < ND; ++j) acc = fmaf(Kp[i * ND + j], ue[j], acc);
        const int pa = a == 0 ? p0 : (a == 1 ? p1 : p2);
        const double sa = a == 0 ? s0 : (a == 1 ? s1 : s2);
        add_force(f, 3 * (int64_t)nd[k] + pa, sa * se * (double)acc, ATOMIC);
      }
    }
  }
}

// Tiles of one node count.
template <int NN, bool FP32, bool ATOMIC>
__global__ void __launch_bounds__(kTile) ebe_fixed(const Tile* __restrict__ tiles, const double* __restrict__ u,
                                                   double* __restrict__ f, const int32_t* __restrict__ conn,
                                                   const uint8_t* __restrict__ orient,
                                                   const uint8_t* __restrict__ level,
                                                   const uint8_t* __restrict__ material,
                                                   const double* __restrict__ matE, double h0,
                                                   const double* __restrict__ K64,
                                                   const float* __restrict__ K32) {
  const Tile t = tiles[blockIdx.x];
  const int lane = threadIdx.x;
  if (lane >= t.count) return;
  cell_force<NN, FP32, ATOMIC>(t, lane, u, f, conn, orient, level, material, matE, h0, K64, K32);
}

// Tiles of any node count 9..26 (the node count is uniform in a block).
template <bool FP32, bool ATOMIC>
__global__ void __launch_bounds__(kTile) ebe_mixed(const Tile* __restrict__ tiles, const double* __restrict__ u,
                                                   double* __restrict__ f, const int32_t* __restrict__ conn,
                                                   const uint8_t* __restrict__ orient,
                                                   const uint8_t* __restrict__ level,
                                                   const uint8_t* __restrict__ material,
                                                   const double* __restrict__ matE, double h0,
                                                   const double* __restrict__ K64,
                                                   const float* __restrict__ K32) {
  const Tile t = tiles[blockIdx.x];
  const int lane = threadIdx.x;
  if (lane >= t.count) return;
#define SBFEM_CASE(N)                                                                                     \
  case N:                                                                                                 \
    cell_force<N, FP32, ATOMIC>(t, lane, u, f, conn, orient, level, material, matE, h0, K64, K32); \
    break;
  switch (t.nn) {
    SBFEM_CASE(9) SBFEM_CASE(10) SBFEM_CASE(11) SBFEM_CASE(12) SBFEM_CASE(13) SBFEM_CASE(14)
    SBFEM_CASE(15) SBFEM_CASE(16) SBFEM_CASE(17) SBFEM_CASE(18) SBFEM_CASE(19) SBFEM_CASE(20)
    SBFEM_CASE(21) SBFEM_CASE(22) SBFEM_CASE(23) SBFEM_CASE(24) SBFEM_CASE(25) SBFEM_CASE(26)
    default:
      break;
  }
#undef SBFEM_CASE
}

}  // namespace sbfem
