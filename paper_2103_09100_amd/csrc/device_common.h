// Device helpers shared by the kernel translation units.
#pragma once

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

}  // namespace sbfem
