// Device kernels of the explicit octree-SBFEM stepper (gfx950): element kernels of the
// atomic and colour assemblies, load, update and utility kernels.
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

#include "classic_kernel.h"
#include "tiled_kernel.h"

namespace sbfem {

__global__ void load_kernel(double* __restrict__ f, const int64_t* __restrict__ idx,
                            const double* __restrict__ val, int64_t nnz, LoadParams L, double t) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nnz) return;
  const double P = load_time(L, t);
  atomicAdd(f + idx[i], -P * val[i]);
}

// u_{n+1} written over u_{n-1}; f cleared; the first step with a non-finite result is recorded.
__global__ void update_kernel(const double* __restrict__ un, double* __restrict__ unm1,
                              double* __restrict__ f, const double* __restrict__ minv, int64_t ndof,
                              double dt2, double c, unsigned long long* __restrict__ flag, int64_t step) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const double inv = 1.0 / (1.0 + c);
  bool bad = false;
  for (int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; d < ndof; d += stride) {
    const double r = -f[d];
    const double v = (dt2 * minv[d] * r + 2.0 * un[d] - (1.0 - c) * unm1[d]) * inv;
    unm1[d] = v;
    f[d] = 0.0;
    bad |= !isfinite(v);
  }
  if (bad) atomicMin(flag, (unsigned long long)step);
}

__global__ void fill_kernel(double* __restrict__ a, int64_t n, double v) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) a[i] = v;
}


// ---------------------------------------------------------------------------------------------
// host-side launchers

hipError_t launch_ebe(const ElementArgs& a, const TileRange& r, bool fp32, bool atomic, hipStream_t s,
                      const LaunchHook& hook) {
  if (r.n_fixed8) {
    hook(1, true, s);
    ebe8_launch(a, a.tiles + r.first, r.n_fixed8, fp32, atomic, s);
    hook(1, false, s);
  }
  if (r.n_mixed) {
    hook(2, true, s);
    if (fp32)
      ebe_mixed_fp32_launch(a, a.tiles + r.first + r.n_fixed8, r.n_mixed, atomic, s);
    else
      ebe_mixed_fp64_launch(a, a.tiles + r.first + r.n_fixed8, r.n_mixed, atomic, s);
    hook(2, false, s);
  }
  return hipGetLastError();
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
                         double dt2, double c, unsigned long long* flag, int64_t step, hipStream_t s) {
  hipLaunchKernelGGL(update_kernel, dim3(grid_for(ndof)), dim3(256), 0, s, un, unm1, f, minv, ndof, dt2, c, flag,
                     step);
  return hipGetLastError();
}

hipError_t launch_fill(double* a, int64_t n, double v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_kernel, dim3(grid_for(n)), dim3(256), 0, s, a, n, v);
  return hipGetLastError();
}


hipError_t launch_tiled(const TiledLaunch& L, hipStream_t s, const LaunchHook& hook) {
  // hanging-node cells first: they store their row forces for the owner tiles
  if (L.n_hang > 0 && L.hang_mma) {
    hook(2, true, s);
    switch (L.prec) {
      case 0: hang_mma_fp64_launch(L, L.work_hang, L.n_hang, s); break;
      case 1: hang_mma_fp32_launch(L, L.work_hang, L.n_hang, s); break;
      case 2: hang_mma_fp16_launch(L, L.work_hang, L.n_hang, s); break;
      default: hang_mma_bf16_launch(L, L.work_hang, L.n_hang, s); break;
    }
    hook(2, false, s);
  } else if (L.n_hang > 0) {
    hook(2, true, s);
    if (L.fp32)
      (L.reduced ? tiled_hang_fp32r_launch : tiled_hang_fp32_launch)(L, L.work_hang, 0, L.n_hang, s);
    else
      (L.reduced ? tiled_hang_fp64r_launch : tiled_hang_fp64_launch)(L, L.work_hang, 0, L.n_hang, s);
    hook(2, false, s);
  }
  // then every owner tile: regular cells, the hanging-cell rows of its dofs, the update
  if (L.n_tiles > 0) {
    hook(1, true, s);
    owner_pass_launch(L, L.work8, 0, L.n_tiles, s);
    hook(1, false, s);
  }
  return hipGetLastError();
}

// Device mesh refs advanced by a number of steps (u and u_prev swap roles every step).
__global__ void refs_advance_kernel(MeshRef* refs, int32_t n, int64_t steps) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  MeshRef r = refs[i];
  r.step += steps;
  r.parity = (int32_t)((r.parity + steps) & 1);
  refs[i] = r;
}

hipError_t launch_refs_advance(MeshRef* refs, int32_t n, int64_t steps, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(refs_advance_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, refs, n, steps);
  return hipGetLastError();
}

__global__ void ref_set_kernel(MeshRef* ref, MeshRef v) { *ref = v; }

hipError_t launch_ref_set(MeshRef* ref, const MeshRef& v, hipStream_t s) {
  hipLaunchKernelGGL(ref_set_kernel, dim3(1), dim3(1), 0, s, ref, v);
  return hipGetLastError();
}

// 8-node element kernels of the classic assemblies
void ebe8_launch(const ElementArgs& a, const Tile* tiles, int64_t n, bool fp32, bool atomic, hipStream_t s) {
#define SBFEM_L(F, A)                                                                                      \
  hipLaunchKernelGGL((ebe_fixed<8, F, A>), dim3((unsigned)n), dim3(kTile), 0, s, tiles, a.u, a.f, a.conn, \
                     a.orient, a.level, a.material, a.matE, a.h0, a.K64, a.K32)
  if (fp32) {
    if (atomic) SBFEM_L(true, true); else SBFEM_L(true, false);
  } else {
    if (atomic) SBFEM_L(false, true); else SBFEM_L(false, false);
  }
#undef SBFEM_L
}

// owner-tile pass: one block per tile (per (mesh, tile) in a batch)
void owner_pass_launch(const TiledLaunch& L, const TileWork* work, int64_t first, int64_t count, hipStream_t s) {
  switch (L.prec) {
    case 0: owner_fp64_launch(L, work, first, count, s); break;
    case 1: owner_fp32_launch(L, work, first, count, s); break;
    case 2: owner_fp16_launch(L, work, first, count, s); break;
    default: owner_bf16_launch(L, work, first, count, s); break;
  }
}

}  // namespace sbfem
