// Device helpers shared by the kernel translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "kernels.h"

namespace sbfem {

// Address-space views.  Pointers that arrive through a struct in device memory are
// generic (flat) pointers to the compiler; a flat load waits on both the vector and
// the LDS counters and may alias LDS.  Data that no kernel writes during the launch
// (tables, layouts, master matrices) is read through the constant space (scalar
// loads when the address is uniform), other device arrays through the global space.
template <class T>
using cptr_t = const __attribute__((address_space(4))) T*;
template <class T>
using gptr_t = const __attribute__((address_space(1))) T*;
template <class T>
using gmut_t = __attribute__((address_space(1))) T*;

template <class T>
__device__ __forceinline__ cptr_t<T> as_const(const T* p) {
  return (cptr_t<T>)p;
}
template <class T>
__device__ __forceinline__ gptr_t<T> as_global(const T* p) {
  return (gptr_t<T>)p;
}
template <class T>
__device__ __forceinline__ gmut_t<T> as_global_mut(T* p) {
  return (gmut_t<T>)p;
}

// Copy of a struct read through such a view, dword by dword (the compiler merges the loads).
template <class T>
__device__ __forceinline__ T load_const(cptr_t<T> p) {
  static_assert(sizeof(T) % 4 == 0, "dword-sized structs only");
  T v;
  const cptr_t<uint32_t> q = (cptr_t<uint32_t>)p;
  uint32_t* d = reinterpret_cast<uint32_t*>(&v);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) / 4); ++i) d[i] = q[i];
  return v;
}
template <class T>
__device__ __forceinline__ T load_global(gptr_t<T> p) {
  static_assert(sizeof(T) % 4 == 0, "dword-sized structs only");
  T v;
  const gptr_t<uint32_t> q = (gptr_t<uint32_t>)p;
  uint32_t* d = reinterpret_cast<uint32_t*>(&v);
#pragma unroll
  for (int i = 0; i < (int)(sizeof(T) / 4); ++i) d[i] = q[i];
  return v;
}

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
