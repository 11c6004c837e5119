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

// State storage (TiledArgs::state): FP64; FP32; or a compensated pair of FP32 values whose
// sum carries the value (hi = fl32(v), lo = fl32(v - hi)), hi at p[i] and lo at p[ndof + i].
// Arithmetic on the state is done in FP64 registers.
__device__ __forceinline__ double state_load(const void* p, int32_t mode, int64_t ndof, int64_t i) {
  if (mode == 0) return as_global((const double*)p)[i];
  const gptr_t<float> q = as_global((const float*)p);
  if (mode == 1) return (double)q[i];
  return (double)q[i] + (double)q[ndof + i];
}
__device__ __forceinline__ void state_store(void* p, int32_t mode, int64_t ndof, int64_t i, double v) {
  if (mode == 0) {
    as_global_mut((double*)p)[i] = v;
    return;
  }
  const gmut_t<float> q = as_global_mut((float*)p);
  const float hi = (float)v;
  q[i] = hi;
  if (mode == 2) q[ndof + i] = (float)(v - (double)hi);
}
// false if v, or the value the state storage keeps of it, is not finite
__device__ __forceinline__ bool state_finite(int32_t mode, double v) {
  return mode == 0 ? isfinite(v) : isfinite((float)v);
}
__device__ __forceinline__ double minv_load(const void* p, int32_t mode, int64_t i) {
  return mode == 1 ? (double)as_global((const float*)p)[i] : as_global((const double*)p)[i];
}

// Streaming forms for data a pass touches once (u_{n-1}, the inverse mass, u_{n+1}, cell
// records): non-temporal accesses, so that they do not displace from L2 the displacements that
// neighbouring tiles read again.
template <class T>
__device__ __forceinline__ T ld_nt(gptr_t<T> p) {
  return __builtin_nontemporal_load(p);
}
template <class T>
__device__ __forceinline__ void st_nt(gmut_t<T> p, T v) {
  __builtin_nontemporal_store(v, p);
}
// (the compensated pair, two FP32 arrays per value, keeps ordinary accesses)
__device__ __forceinline__ double state_load_nt(const void* p, int32_t mode, int64_t ndof, int64_t i) {
  if (mode == 0) return ld_nt(as_global((const double*)p) + i);
  if (mode == 1) return (double)ld_nt(as_global((const float*)p) + i);
  return state_load(p, mode, ndof, i);
}
__device__ __forceinline__ void state_store_nt(void* p, int32_t mode, int64_t ndof, int64_t i, double v) {
  if (mode == 0) {
    st_nt(as_global_mut((double*)p) + i, v);
  } else if (mode == 1) {
    st_nt(as_global_mut((float*)p) + i, (float)v);
  } else {
    state_store(p, mode, ndof, i, v);
  }
}
__device__ __forceinline__ double minv_load_nt(const void* p, int32_t mode, int64_t i) {
  return mode == 1 ? (double)ld_nt(as_global((const float*)p) + i) : ld_nt(as_global((const double*)p) + i);
}

// 16-bit product operands (values kept in FP32 registers; a product of two 16-bit values is
// exact in FP32, so FMAs on them are 16-bit products with FP32 accumulation).
__device__ __forceinline__ float round_fp16(float x) { return (float)(_Float16)x; }
__device__ __forceinline__ float round_bf16(float x) {  // round to nearest even on the FP32 bits
  uint32_t b = __float_as_uint(x);
  b += 0x7FFFu + ((b >> 16) & 1u);
  return __uint_as_float(b & 0xFFFF0000u);
}
__device__ __forceinline__ float round16(float x, int32_t mode) {
  return mode == 1 ? round_fp16(x) : round_bf16(x);
}
// power of two that brings max |x| into [1, 2) (1 for x = 0): FP16 operands are scaled by it
__device__ __forceinline__ float pow2_scale(float maxabs) {
  if (!(maxabs > 0.0f)) return 1.0f;
  int e;
  (void)frexpf(maxabs, &e);  // maxabs = f 2^e, f in [0.5, 1)
  return ldexpf(1.0f, 1 - e);
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
  if (L.kind == 3) {  // table of P(t_n): t is n dt up to rounding
    const double n = floor(t / L.dt + 0.5);
    return n >= 0.0 && n < (double)L.n_table ? as_global(L.table)[(int64_t)n] : 0.0;
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
