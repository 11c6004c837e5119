// Kernels for cells of 9..26 nodes, FP64 element products (own unit: long compile).
#include "tiled_kernel.h"

namespace sbfem {

void tiled_mixed_fp64_launch(const TiledArgs& a, int64_t first, int64_t count, bool force_only, hipStream_t s) {
  const int64_t blocks = 8 * ((count + 7) / 8);
  const size_t lds = (size_t)a.lds_doubles * 8;
  if (force_only)
    hipLaunchKernelGGL((tiled_step<false, false, true>), dim3((unsigned)blocks), dim3(256), lds, s, a, first, count);
  else
    hipLaunchKernelGGL((tiled_step<false, false, false>), dim3((unsigned)blocks), dim3(256), lds, s, a, first, count);
}

}  // namespace sbfem
