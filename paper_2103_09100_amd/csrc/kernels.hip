// Device kernels of the explicit octree-SBFEM stepper (gfx950).
//
// Per time step (Alg. 1 time loop):
//   load_kernel     f[b.idx] -= P(t_n) * b.val          (R_ext, eq. Ricker/Triangle/Lamb)
//   ebe kernels     f += s_e R_e^T K_p R_e u_e          (eqs. Rinte, Rintep, KM_scale)
//   update_kernel   u_{n+1} = (dt^2 M^-1 (-f) + 2 u_n - (1 - a dt/2) u_{n-1}) / (1 + a dt/2)
//                   (eq. DnMdiag), written over u_{n-1}; f is cleared for the next step.
//
// Element kernels run one cell per thread.  A block covers one tile: up to
// 256 cells of a single pattern, so the master matrix pointer is uniform in
// the block and its entries are fetched through the scalar cache.  The cell's
// node ids are stored slot-major inside its pattern segment so that the
// threads of a wave read consecutive ids.

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace sbfem {

// orientation code -> axis permutation pi and signs s:  u_master[k][a] = s_a u[node][pi(a)]
__device__ __forceinline__ void decode_orient(int code, int& p0, int& p1, int& p2,
                                              double& s0, double& s1, double& s2) {
  const int p = code >> 3;
  p0 = p >> 1;
  const int lo = (p0 == 0) ? 1 : 0;
  const int hi = (p0 == 2) ? 1 : 2;
  p1 = (p & 1) ? hi : lo;
  p2 = (p & 1) ? lo : hi;
  s0 = (code & 1) ? -1.0 : 1.0;
  s1 = (code & 2) ? -1.0 : 1.0;
  s2 = (code & 4) ? -1.0 : 1.0;
}

__device__ __forceinline__ double pick3(int i, double x, double y, double z) {
  return i == 0 ? x : (i == 1 ? y : z);
}

__device__ __forceinline__ double load_time(const LoadParams& L, double t) {
  if (L.kind == 0) {  // Ricker
    const double tau = (t - L.t1) / (L.t1 / 5.0);
    return (1.0 - tau * tau) * exp(-0.5 * tau * tau) * L.P0;
  }
  if (L.kind == 1) {  // triangle
    if (t < 0.0 || t > 2.0 * L.t1) return 0.0;
    return (1.0 - fabs(t / L.t1 - 1.0)) * L.P0;
  }
  // Hann-windowed sine burst
  if (t < 0.0 || t > L.t1) return 0.0;
  const double pi = 3.14159265358979323846;
  const double w = sin(pi * t / L.t1);
  return sin(2.0 * pi * L.cycles * t / L.t1) * w * w * L.P0;
}

__device__ __forceinline__ void add_force(double* f, int64_t dof, double v, bool atomic) {
  if (atomic) {
    atomicAdd(f + dof, v);
  } else {
    f[dof] += v;
  }
}

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

__global__ void load_kernel(double* __restrict__ f, const int64_t* __restrict__ idx,
                            const double* __restrict__ val, int64_t nnz, LoadParams L, double t) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nnz) return;
  const double P = load_time(L, t);
  atomicAdd(f + idx[i], -P * val[i]);
}

// u_{n+1} written over u_{n-1}; f cleared.
__global__ void update_kernel(const double* __restrict__ un, double* __restrict__ unm1,
                              double* __restrict__ f, const double* __restrict__ minv, int64_t ndof,
                              double dt2, double c) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const double inv = 1.0 / (1.0 + c);
  for (int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; d < ndof; d += stride) {
    const double r = -f[d];
    const double v = (dt2 * minv[d] * r + 2.0 * un[d] - (1.0 - c) * unm1[d]) * inv;
    unm1[d] = v;
    f[d] = 0.0;
  }
}

__global__ void fill_kernel(double* __restrict__ a, int64_t n, double v) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) a[i] = v;
}

// flag[0] |= 1 if any entry is not finite
__global__ void finite_kernel(const double* __restrict__ a, int64_t n, int32_t* __restrict__ flag) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
    bad |= !isfinite(a[i]);
  if (bad) atomicOr(flag, 1);
}

// ---------------------------------------------------------------------------------------------
// host-side launchers

template <bool FP32, bool ATOMIC>
static hipError_t launch_ebe_t(const ElementArgs& a, const TileRange& r, hipStream_t s) {
  if (r.n_fixed8)
    hipLaunchKernelGGL((ebe_fixed<8, FP32, ATOMIC>), dim3(r.n_fixed8), dim3(kTile), 0, s, a.tiles + r.first,
                       a.u, a.f, a.conn, a.orient, a.level, a.material, a.matE, a.h0, a.K64, a.K32);
  if (r.n_mixed)
    hipLaunchKernelGGL((ebe_mixed<FP32, ATOMIC>), dim3(r.n_mixed), dim3(kTile), 0, s,
                       a.tiles + r.first + r.n_fixed8, a.u, a.f, a.conn, a.orient, a.level, a.material,
                       a.matE, a.h0, a.K64, a.K32);
  return hipGetLastError();
}

hipError_t launch_ebe(const ElementArgs& a, const TileRange& r, bool fp32, bool atomic, hipStream_t s) {
  if (fp32) return atomic ? launch_ebe_t<true, true>(a, r, s) : launch_ebe_t<true, false>(a, r, s);
  return atomic ? launch_ebe_t<false, true>(a, r, s) : launch_ebe_t<false, false>(a, r, s);
}

hipError_t launch_load(double* f, const int64_t* idx, const double* val, int64_t nnz, const LoadParams& L,
                       double t, hipStream_t s) {
  if (nnz <= 0) return hipSuccess;
  const int blocks = (int)((nnz + 255) / 256);
  hipLaunchKernelGGL(load_kernel, dim3(blocks), dim3(256), 0, s, f, idx, val, nnz, L, t);
  return hipGetLastError();
}

static int grid_for(int64_t n) {
  int64_t b = (n + 255) / 256;
  if (b > 8192) b = 8192;
  if (b < 1) b = 1;
  return (int)b;
}

hipError_t launch_update(const double* un, double* unm1, double* f, const double* minv, int64_t ndof,
                         double dt2, double c, hipStream_t s) {
  hipLaunchKernelGGL(update_kernel, dim3(grid_for(ndof)), dim3(256), 0, s, un, unm1, f, minv, ndof, dt2, c);
  return hipGetLastError();
}

hipError_t launch_fill(double* a, int64_t n, double v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_kernel, dim3(grid_for(n)), dim3(256), 0, s, a, n, v);
  return hipGetLastError();
}

hipError_t launch_finite(const double* a, int64_t n, int32_t* flag, hipStream_t s) {
  hipLaunchKernelGGL(finite_kernel, dim3(grid_for(n)), dim3(256), 0, s, a, n, flag);
  return hipGetLastError();
}

}  // namespace sbfem
