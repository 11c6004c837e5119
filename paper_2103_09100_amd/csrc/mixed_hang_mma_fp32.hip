// Hanging-cell pass on the matrix cores, FP32 products (own unit: long compile).
#include "hang_mma.h"

namespace sbfem {

void hang_mma_fp32_launch(const TiledLaunch& L, const TileWork* work, int64_t count, hipStream_t s) {
  auto launch = [&](auto kern) {
    if (L.lds_hang > 65536)
      (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)L.lds_hang);
    hipLaunchKernelGGL(kern, dim3((unsigned)count), dim3(256), L.lds_hang, s, L.single, L.refs, work, (int64_t)0,
                       count, L.k);
  };
  if (L.state == 0)
    launch(tiled_hang_mma<1, 0>);
  else if (L.state == 1)
    launch(tiled_hang_mma<1, 1>);
  else
    launch(tiled_hang_mma<1, 2>);
}

}  // namespace sbfem
