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
  std::vector<int64_t> load_dof;       // internal dofs
  std::vector<double> load_val;
};

struct TilingOutput {
  int32_t tile_nodes = 0;
  std::vector<OwnerTile> tiles;        // n_pure8 tiles of 8-node cells only, then n_mixed
  int64_t n_pure8 = 0, n_mixed = 0;
  int64_t max_local = 0;
  std::vector<CellItem> items;
  std::vector<int32_t> nodelist;
  std::vector<uint16_t> lidx;
  std::vector<uint8_t> orient, level, material;
  std::vector<LoadEntry> loads;
};

// false if a tile would need more than 65535 local nodes
bool build_owner_tiles(const TilingInput& in, int32_t tile_nodes, TilingOutput& out);

}  // namespace sbfem
