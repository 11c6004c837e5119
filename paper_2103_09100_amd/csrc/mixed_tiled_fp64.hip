// Kernels for tiles with hanging-node cells, FP64 element products (own unit: long compile).
#include "tiled_kernel.h"

namespace sbfem {

void tiled_mixed_fp64_launch(const TiledLaunch& L, const TileWork* work, int64_t first, int64_t count,
                             hipStream_t s) {
  const int64_t blocks = 8 * ((count + 7) / 8);
  if (L.lds > 65536)
    (void)hipFuncSetAttribute((const void*)tiled_step<false, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)L.lds);
  hipLaunchKernelGGL((tiled_step<false, false>), dim3((unsigned)blocks), dim3(L.threads_mixed), L.lds, s, L.single,
                     L.refs, work, first, count, L.k, (int)L.force_only);
}

}  // namespace sbfem
