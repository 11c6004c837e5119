// Owner-tile pass, FP16 products, every state storage (own unit: long compile).
#include "tiled_kernel.h"

namespace sbfem {

void owner_fp16_launch(const TiledLaunch& L, const TileWork* work, int64_t first, int64_t count, hipStream_t s) {
  auto launch = [&](auto kern) {
    if (L.lds > 65536)
      (void)hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)L.lds);
    const int64_t blocks = 8 * ((count + 7) / 8);  // whole XCD rounds (see xcd_unit)
    hipLaunchKernelGGL(kern, dim3((unsigned)blocks), dim3(L.threads8), L.lds, s, L.single, L.refs, work, first,
                       count, L.k, (int)L.force_only);
  };
  if (L.state == 0)
    launch(tiled_step8<2, 0>);
  else if (L.state == 1)
    launch(tiled_step8<2, 1>);
  else
    launch(tiled_step8<2, 2>);
}

}  // namespace sbfem
