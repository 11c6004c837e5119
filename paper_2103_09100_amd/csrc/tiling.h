// Owner-tile layout: host builder interface.
#pragma once

#include <stdint.h>

#include <vector>

#include "kernels.h"

namespace sbfem {

struct TilingInput {
  int64_t n_nodes = 0, n_cells = 0;
  const int64_t* cptr = nullptr;       // [n_cells+1] offsets into conn
  const int32_t* conn = nullptr;       // internal node ids, master order
  const uint16_t* pattern = nullptr;
  const uint8_t* orient = nullptr;
  const uint8_t* level = nullptr;
  const uint8_t* material = nullptr;
  const int32_t* pattern_ndof = nullptr;
  const int64_t* pattern_koff = nullptr;
  // regular 8-node cells (identity orientation): per pattern id, the index of the pattern's
  // structured Walsh table (one per pattern library), -1 for hanging-node patterns; null: none
  const int16_t* regular = nullptr;
  std::vector<int64_t> load_dof;       // internal dofs
  std::vector<double> load_val;
};

struct TilingOutput {
  int32_t tile_nodes = 0;
  std::vector<OwnerTile> tiles;        // in node order; n_mixed of them own a hanging-cell node
  int64_t n_pure8 = 0, n_mixed = 0;
  int64_t max_local = 0;
  std::vector<CellItem> items;
  std::vector<int32_t> nodelist;       // halo node ids per tile (at halo_stride, -1 padded, if > 0)
  int64_t halo_stride = 0;
  int64_t local_entries = 0;           // local nodes over all tiles
  std::vector<uint16_t> lidx;
  std::vector<LoadEntry> loads;
  // scale classes of the regular cells: key = (Walsh table << 16) | (level << 8) | material, in
  // order of first use; an item of regular cells carries koff = kWalshC * class
  std::vector<int32_t> scale_keys;
};

// false if a tile would need more than 65535 local nodes
bool build_owner_tiles(const TilingInput& in, int32_t tile_nodes, TilingOutput& out);

}  // namespace sbfem
