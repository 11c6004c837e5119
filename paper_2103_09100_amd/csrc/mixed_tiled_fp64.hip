// Hanging-cell pass, FP64 element products (own unit: long compile).
#include "tiled_kernel.h"

namespace sbfem {

void tiled_hang_fp64_launch(const TiledLaunch& L, const TileWork* work, int64_t first, int64_t count,
                              hipStream_t s) {
  const int64_t per_block = L.threads_mixed / 64;  // one wave per item
  const int64_t blocks = (count + per_block - 1) / per_block;
  if (L.lds_hang > 65536)
    (void)hipFuncSetAttribute((const void*)tiled_hang<false, false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)L.lds_hang);
  hipLaunchKernelGGL((tiled_hang<false, false>), dim3((unsigned)blocks), dim3(L.threads_mixed), L.lds_hang, s, L.single, L.refs,
                     work, first, count, L.k);
}

}  // namespace sbfem
