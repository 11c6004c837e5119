// Kernels for cells of 9..26 nodes, FP64 element products (own unit: long compile).
#include "tiled_kernel.h"

namespace sbfem {

void tiled_mixed_fp64_launch(const TiledArgs& a, int64_t first, int64_t count, bool force_only, hipStream_t s) {
  const int64_t blocks = 8 * ((count + 7) / 8);
  const size_t lds = (size_t)a.lds_bytes;
  if (lds > 65536)
    (void)hipFuncSetAttribute((const void*)tiled_step<false, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds);
  hipLaunchKernelGGL((tiled_step<false, false>), dim3((unsigned)blocks), dim3(a.block_threads), lds, s, a, first,
                     count, (int)force_only);
}

}  // namespace sbfem
