// Kernels for cells of 9..26 nodes, FP32 element products (own unit: long compile).
#include "classic_kernel.h"

namespace sbfem {

void ebe_mixed_fp32_launch(const ElementArgs& a, const Tile* tiles, int64_t n, bool atomic, hipStream_t s) {
  if (atomic)
    hipLaunchKernelGGL((ebe_mixed<true, true>), dim3((unsigned)n), dim3(kTile), 0, s, tiles, a.u, a.f, a.conn,
                       a.orient, a.level, a.material, a.matE, a.h0, a.K64, a.K32);
  else
    hipLaunchKernelGGL((ebe_mixed<true, false>), dim3((unsigned)n), dim3(kTile), 0, s, tiles, a.u, a.f, a.conn,
                       a.orient, a.level, a.material, a.matE, a.h0, a.K64, a.K32);
}

}  // namespace sbfem
