// Internal interface between the C-ABI host code and the device kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sbfem {

constexpr int kTile = 256;  // cells per block (one cell per thread)

// A block's work: up to kTile consecutive cells of one pattern segment.
struct Tile {
  int64_t cell0;   // first cell (index into the sorted per-cell arrays)
  int64_t conn0;   // conn index of slot 0 of the first cell
  int64_t stride;  // cells in the segment (distance between slots of one cell)
  int64_t koff;    // offset of the pattern's master matrix (entries)
  int32_t count;   // cells in this tile (1..kTile)
  int32_t nn;      // nodes per cell of the pattern
};

// Tiles of one launch group: n_fixed8 tiles of 8-node cells, then n_mixed tiles of larger cells.
struct TileRange {
  int64_t first;
  int64_t n_fixed8;
  int64_t n_mixed;
};

struct LoadParams {
  int32_t kind;
  int32_t cycles;
  double t1;
  double P0;
};

struct ElementArgs {
  const Tile* tiles;
  const double* u;
  double* f;
  const int32_t* conn;
  const uint8_t* orient;
  const uint8_t* level;
  const uint8_t* material;
  const double* matE;
  double h0;
  const double* K64;
  const float* K32;
};

hipError_t launch_ebe(const ElementArgs& a, const TileRange& r, bool fp32, bool atomic, hipStream_t s);
hipError_t launch_load(double* f, const int64_t* idx, const double* val, int64_t nnz, const LoadParams& L,
                       double t, hipStream_t s);
hipError_t launch_update(const double* un, double* unm1, double* f, const double* minv, int64_t ndof,
                         double dt2, double c, hipStream_t s);
hipError_t launch_fill(double* a, int64_t n, double v, hipStream_t s);
hipError_t launch_finite(const double* a, int64_t n, int32_t* flag, hipStream_t s);

}  // namespace sbfem
