// Dense vector kernels of the eigenfrequency solver (Chebyshev-filtered subspace iteration):
// FP64; a block of p vectors of length n is stored column after column (column j at X + j n).
// Reductions run in a fixed order (one block per output, a fixed tree inside the block), so a
// result repeats bitwise from run to run.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "device_common.h"

namespace sbfem {

constexpr int kLinThreads = 256;

__device__ __forceinline__ double block_sum256(double v) {
  __shared__ double part[kLinThreads / 64];
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o);
  if ((threadIdx.x & 63) == 0) part[threadIdx.x >> 6] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < kLinThreads / 64; ++i) s += part[i];
  return s;  // valid in thread 0
}

// G[i * p + j] = X_i . Y_j (all i, j < p): one block per entry
__global__ void gram_kernel(const double* __restrict__ X, const double* __restrict__ Y, int64_t n, int p,
                            double* __restrict__ G) {
  const int i = blockIdx.x / p, j = blockIdx.x - (blockIdx.x / p) * p;
  const double* x = X + (int64_t)i * n;
  const double* y = Y + (int64_t)j * n;
  double s = 0.0;
  for (int64_t r = threadIdx.x; r < n; r += kLinThreads) s += x[r] * y[r];
  s = block_sum256(s);
  if (threadIdx.x == 0) G[blockIdx.x] = s;
}

// Y[:, j0 + jj] = sum_i X[:, i] Q[i * q + j0 + jj] for 16 columns per block row; Q (p x q) read
// through the constant space (uniform in the block)
constexpr int kGemmCols = 16;
__global__ void gemm_small_kernel(const double* __restrict__ X, int64_t n, int p, const double* __restrict__ Q,
                                  int q, double* __restrict__ Y) {
  const int64_t r = (int64_t)blockIdx.x * kLinThreads + threadIdx.x;
  const int j0 = blockIdx.y * kGemmCols;
  if (r >= n) return;
  const cptr_t<double> Qc = as_const(Q);
  double acc[kGemmCols];
#pragma unroll
  for (int jj = 0; jj < kGemmCols; ++jj) acc[jj] = 0.0;
  for (int i = 0; i < p; ++i) {
    const double x = X[(int64_t)i * n + r];
#pragma unroll
    for (int jj = 0; jj < kGemmCols; ++jj)
      if (j0 + jj < q) acc[jj] = fma(x, Qc[i * q + j0 + jj], acc[jj]);
  }
#pragma unroll
  for (int jj = 0; jj < kGemmCols; ++jj)
    if (j0 + jj < q) Y[(int64_t)(j0 + jj) * n + r] = acc[jj];
}

// z = a x + b y + c z (elementwise)
__global__ void axpbypcz_kernel(double a, const double* __restrict__ x, double b, const double* __restrict__ y,
                                double c, double* __restrict__ z, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kLinThreads + threadIdx.x;
  if (i < n) z[i] = a * x[i] + b * y[i] + c * z[i];
}

// Y[:, j] = S .* X[:, j] for the p columns (blockIdx.y = column)
__global__ void scale_cols_kernel(const double* __restrict__ S, const double* __restrict__ X, double* __restrict__ Y,
                                  int64_t n) {
  const int64_t r = (int64_t)blockIdx.x * kLinThreads + threadIdx.x;
  if (r >= n) return;
  const int64_t o = (int64_t)blockIdx.y * n + r;
  Y[o] = S[r] * X[o];
}

// z = a x + b y (elementwise)
__global__ void axpby_kernel(double a, const double* __restrict__ x, double b, const double* __restrict__ y,
                             double* __restrict__ z, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kLinThreads + threadIdx.x;
  if (i < n) z[i] = a * x[i] + b * y[i];
}

// y = s .* x (elementwise)
__global__ void vmul_kernel(const double* __restrict__ s, const double* __restrict__ x, double* __restrict__ y,
                            int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * kLinThreads + threadIdx.x;
  if (i < n) y[i] = s[i] * x[i];
}

// out[j] = |AX_j - theta_j X_j|^2 (one block per column)
__global__ void ritz_residual_kernel(const double* __restrict__ X, const double* __restrict__ AX, int64_t n,
                                     const double* __restrict__ theta, double* __restrict__ out) {
  const int j = blockIdx.x;
  const double t = theta[j];
  const double* x = X + (int64_t)j * n;
  const double* ax = AX + (int64_t)j * n;
  double s = 0.0;
  for (int64_t r = threadIdx.x; r < n; r += kLinThreads) {
    const double d = ax[r] - t * x[r];
    s += d * d;
  }
  s = block_sum256(s);
  if (threadIdx.x == 0) out[j] = s;
}

static unsigned lin_grid(int64_t n) { return (unsigned)((n + kLinThreads - 1) / kLinThreads); }

hipError_t launch_gram(const double* X, const double* Y, int64_t n, int p, double* G, hipStream_t s) {
  hipLaunchKernelGGL(gram_kernel, dim3((unsigned)(p * p)), dim3(kLinThreads), 0, s, X, Y, n, p, G);
  return hipGetLastError();
}
hipError_t launch_gemm_small(const double* X, int64_t n, int p, const double* Q, int q, double* Y, hipStream_t s) {
  hipLaunchKernelGGL(gemm_small_kernel, dim3(lin_grid(n), (unsigned)((q + kGemmCols - 1) / kGemmCols)),
                     dim3(kLinThreads), 0, s, X, n, p, Q, q, Y);
  return hipGetLastError();
}
hipError_t launch_axpbypcz(double a, const double* x, double b, const double* y, double c, double* z, int64_t n,
                           hipStream_t s) {
  hipLaunchKernelGGL(axpbypcz_kernel, dim3(lin_grid(n)), dim3(kLinThreads), 0, s, a, x, b, y, c, z, n);
  return hipGetLastError();
}
hipError_t launch_scale_cols(const double* S, const double* X, double* Y, int64_t n, int p, hipStream_t s) {
  hipLaunchKernelGGL(scale_cols_kernel, dim3(lin_grid(n), (unsigned)p), dim3(kLinThreads), 0, s, S, X, Y, n);
  return hipGetLastError();
}
hipError_t launch_axpby(double a, const double* x, double b, const double* y, double* z, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(axpby_kernel, dim3(lin_grid(n)), dim3(kLinThreads), 0, s, a, x, b, y, z, n);
  return hipGetLastError();
}
hipError_t launch_vmul(const double* sc, const double* x, double* y, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(vmul_kernel, dim3(lin_grid(n)), dim3(kLinThreads), 0, s, sc, x, y, n);
  return hipGetLastError();
}
hipError_t launch_ritz_residual(const double* X, const double* AX, int64_t n, int p, const double* theta,
                                double* out, hipStream_t s) {
  hipLaunchKernelGGL(ritz_residual_kernel, dim3((unsigned)p), dim3(kLinThreads), 0, s, X, AX, n, theta, out);
  return hipGetLastError();
}

}  // namespace sbfem
