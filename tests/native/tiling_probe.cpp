// Test harness (host only): runs the owner-tile builder of the library on arrays handed in
// from Python and hands its output back, so that the index work of the tiling can be
// checked exactly on the CPU.  Built by the test with g++ together with csrc/tiling.cpp.
#include <cstring>
#include <vector>

#include "tiling.h"

namespace {
sbfem::TilingOutput g_out;
}

extern "C" {

void tiling_struct_sizes(int64_t* out) {
  out[0] = sizeof(sbfem::OwnerTile);
  out[1] = sizeof(sbfem::CellItem);
  out[2] = sizeof(sbfem::LoadEntry);
}

int tiling_run(int64_t n_nodes, int64_t n_cells, const int64_t* cptr, const int32_t* conn, const uint16_t* pattern,
               const uint8_t* level, const uint8_t* material, int32_t p8, int64_t n_load, const int64_t* load_dof,
               const double* load_val, int32_t tile_nodes) {
  sbfem::TilingInput in;
  in.n_nodes = n_nodes;
  in.n_cells = n_cells;
  in.cptr = cptr;
  in.conn = conn;
  in.pattern = pattern;
  in.level = level;
  in.material = material;
  static std::vector<int16_t> regular;
  regular.assign(1 << 16, -1);
  if (p8 >= 0) regular[p8] = 0;
  in.regular = regular.data();
  in.load_dof.assign(load_dof, load_dof + n_load);
  in.load_val.assign(load_val, load_val + n_load);
  return sbfem::build_owner_tiles(in, tile_nodes, g_out) ? 1 : 0;
}

// [n_tiles, n_items, n_lidx, n_nodelist, n_loads, n_scale_keys, halo_stride, tile_nodes, max_local,
//  local_entries, n_pure8, n_mixed]
void tiling_sizes(int64_t* out) {
  out[0] = (int64_t)g_out.tiles.size();
  out[1] = (int64_t)g_out.items.size();
  out[2] = (int64_t)g_out.lidx.size();
  out[3] = (int64_t)g_out.nodelist.size();
  out[4] = (int64_t)g_out.loads.size();
  out[5] = (int64_t)g_out.scale_keys.size();
  out[6] = g_out.halo_stride;
  out[7] = g_out.tile_nodes;
  out[8] = g_out.max_local;
  out[9] = g_out.local_entries;
  out[10] = g_out.n_pure8;
  out[11] = g_out.n_mixed;
}

void tiling_copy(void* tiles, void* items, void* lidx, void* nodelist, void* loads, void* scale_keys) {
  std::memcpy(tiles, g_out.tiles.data(), g_out.tiles.size() * sizeof(sbfem::OwnerTile));
  std::memcpy(items, g_out.items.data(), g_out.items.size() * sizeof(sbfem::CellItem));
  std::memcpy(lidx, g_out.lidx.data(), g_out.lidx.size() * sizeof(uint16_t));
  std::memcpy(nodelist, g_out.nodelist.data(), g_out.nodelist.size() * sizeof(int32_t));
  std::memcpy(loads, g_out.loads.data(), g_out.loads.size() * sizeof(sbfem::LoadEntry));
  std::memcpy(scale_keys, g_out.scale_keys.data(), g_out.scale_keys.size() * sizeof(int32_t));
}
}
