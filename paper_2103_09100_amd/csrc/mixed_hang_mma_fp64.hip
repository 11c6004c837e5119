// Hanging-cell pass on the matrix cores, FP64 products (own unit: long compile).
#include "hang_mma.h"

namespace sbfem {

void hang_mma_fp64_launch(const TiledLaunch& L, const TileWork* work, int64_t count, hipStream_t s) {
  auto launch = [&](auto kern) {
    if (L.lds_hang > 65536)
      (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)L.lds_hang);
    hipLaunchKernelGGL(kern, dim3((unsigned)count), dim3(256), L.lds_hang, s, L.single, L.refs, work, (int64_t)0,
                       count, L.k);
  };
  if (L.state == 0)
    launch(tiled_hang_mma<0, 0>);
  else if (L.state == 1)
    launch(tiled_hang_mma<0, 1>);
  else
    launch(tiled_hang_mma<0, 2>);
}

int hang_mma_lds_bytes(int prec, int nd) {
  switch (prec) {
    case 0: return hang_lds_bytes<0>(nd);
    case 1: return hang_lds_bytes<1>(nd);
    case 2: return hang_lds_bytes<2>(nd);
    default: return hang_lds_bytes<3>(nd);
  }
}

}  // namespace sbfem
